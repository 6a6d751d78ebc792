"""Checkpointed adjoint through the C ABI against the FP64 gradient reference.

FP64 device runs must match the autograd reference to ~1e-9; FP32 runs within
1e-3 relative on dL/dlog t_stop and 1e-2 relative L2 on the velocity-gradient
fields.  The checkpoint interval must not change a single bit.
"""
import math

import numpy as np
import pytest

from paper_1908_01682_amd import inputs as I
from tests.gpu_util import HAVE_GPU, banner, needs_gpu

pytestmark = [pytest.mark.gpu, needs_gpu]

if HAVE_GPU:
    import torch
    from paper_1908_01682_amd import tfsph as T


def _prob(dim, n, seed=0, t_stop=1e-3, mass_jitter=False):
    if dim == 1:
        prob = I.dusty_wave(n_side=n, amp=1e-2, t_stop=t_stop, eps=0.8, cells_per_axis=n // 2)
    else:
        prob = I.wave_2d(n_side=n, amp=1e-2, t_stop=t_stop, eps=1.0)
    rng = np.random.default_rng(seed)
    prob.gas.v = prob.gas.v + 0.01 * rng.standard_normal(prob.gas.v.shape)
    prob.dust.v = prob.dust.v + 0.01 * rng.standard_normal(prob.dust.v.shape)
    if mass_jitter:
        prob.dust.m = prob.dust.m * rng.uniform(0.7, 1.3, prob.dust.n)
    return prob


def _relax(p):
    """The relaxation-time parameter: t_stop, 1/K when K is held constant, or t_stop_epstein."""
    if p.K > 0:
        return 1.0 / p.K
    return p.t_stop_epstein if p.t_stop_epstein > 0 else p.t_stop


def _target(orc, prob, steps):
    """Dust density by id after a twin run with the relaxation time doubled (FP64 oracle)."""
    p = prob.params
    if p.K > 0:
        p = p.replace(K=0.5 * p.K)
    elif p.t_stop_epstein > 0:
        p = p.replace(t_stop_epstein=2.0 * p.t_stop_epstein)
    else:
        p = p.replace(t_stop=2.0 * p.t_stop)
    g, d = orc.from_problem(prob)
    orc.step(p, g, d, steps)
    rho = orc.density(p, d)
    t = np.zeros(prob.dust.n)
    t[d.id] = rho
    return t


def _device_positions(runner, prob):
    """FP64 absolute positions (by id) of the runner's initial (cell, offset) state."""
    out = []
    p = prob.params
    D = [(p.hi[k] - p.lo[k]) / p.n_cells[k] for k in range(p.dim)]
    for ph in (runner.gas, runner.dust):
        a = ph.numpy()
        c = a["cell"].astype(np.int64)
        cs = [c % p.n_cells[0]]
        if p.dim > 1:
            cs.append((c // p.n_cells[0]) % p.n_cells[1])
        x = np.stack([p.lo[k] + cs[k] * D[k] + a["off"][k].astype(np.float64) for k in range(p.dim)], axis=1)
        out.append(x)
    return out


def _reference(orc, prob, runner, target, steps):
    from oracle import adjoint_torch as AT
    xg, xd = _device_positions(runner, prob)
    vg = np.stack([v.cpu().numpy().astype(np.float64) for v in runner.gas.vel], axis=1)
    vd = np.stack([v.cpu().numpy().astype(np.float64) for v in runner.dust.vel], axis=1)
    return AT.gradients(prob.params, xg, xd, prob.gas.m, prob.dust.m, vg, vd, _relax(prob.params), target, steps)


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("dim,n,steps,ckpt,mass,K,TE", [(2, 24, 12, 5, False, 0.0, 0.0), (1, 160, 15, 4, True, 0.0, 0.0),
                                                        (2, 20, 7, 7, True, 0.0, 0.0), (1, 160, 12, 5, True, 800.0, 0.0),
                                                        (2, 24, 9, 4, True, 1000.0, 0.0),
                                                        (1, 160, 12, 5, True, 0.0, 1.5e-3),
                                                        (2, 24, 9, 4, True, 0.0, 1e-3)])
def test_adjoint_fp64_matches_reference(orc, dim, n, steps, ckpt, mass, K, TE):
    """K > 0 holds the drag coefficient constant (the scalar is then dL/dlog(1/K)); TE > 0 selects
    the Epstein law (scalar dL/dlog T_E)."""
    prob = _prob(dim, n, seed=dim, mass_jitter=mass)
    if K > 0:
        prob.params = prob.params.replace(K=K)
    if TE > 0:
        prob.params = prob.params.replace(t_stop_epstein=TE)
    target = _target(orc, prob, steps)
    banner(f"adjoint fp64 dim={dim} n={n} steps={steps} ckpt={ckpt}")
    runner = T.AdjointRunner(prob, steps, ckpt, precision=T.TFSPH_F64)
    loss, dlogt, gv, gu = runner.run(target)
    torch.cuda.synchronize()
    ref_loss, ref_s, ref_gv, ref_gu = _reference(orc, prob, runner, target, steps)
    assert abs(float(loss) - ref_loss) <= 1e-10 * ref_loss
    assert abs(float(dlogt) - ref_s) <= 1e-8 * abs(ref_s)
    assert np.max(np.abs(gv.cpu().numpy() - ref_gv)) <= 1e-8 * np.max(np.abs(ref_gv))
    assert np.max(np.abs(gu.cpu().numpy() - ref_gu)) <= 1e-8 * np.max(np.abs(ref_gu))


@pytest.mark.parametrize("dim,n,steps,ckpt", [(2, 32, 20, 6), (1, 400, 40, 10)])
def test_adjoint_fp32_matches_reference(orc, dim, n, steps, ckpt):
    prob = _prob(dim, n, seed=5 + dim)
    target = _target(orc, prob, steps)
    banner(f"adjoint fp32 dim={dim} n={n} steps={steps} ckpt={ckpt}")
    runner = T.AdjointRunner(prob, steps, ckpt, precision=T.TFSPH_F32)
    loss, dlogt, gv, gu = runner.run(target.astype(np.float32))
    torch.cuda.synchronize()
    ref_loss, ref_s, ref_gv, ref_gu = _reference(orc, prob, runner, target.astype(np.float32).astype(np.float64),
                                                 steps)
    assert abs(float(loss) - ref_loss) <= 1e-3 * ref_loss, (float(loss), ref_loss)
    assert abs(float(dlogt) - ref_s) <= 1e-3 * abs(ref_s), (float(dlogt), ref_s)
    assert _rel_l2(gv.cpu().numpy(), ref_gv) <= 1e-2
    assert _rel_l2(gu.cpu().numpy(), ref_gu) <= 1e-2


def test_checkpoint_interval_and_rerun_are_bitwise_identical():
    prob = _prob(2, 24, seed=3)
    target = np.full(prob.dust.n, 1.0, dtype=np.float32)
    res = []
    for ckpt in (1, 4, 13, 13):
        runner = T.AdjointRunner(prob, 13, ckpt, precision=T.TFSPH_F32)
        out = runner.run(target)
        torch.cuda.synchronize()
        res.append([o.cpu().numpy() for o in out])
    for other in res[1:]:
        for a, b in zip(res[0], other):
            assert np.array_equal(a, b)


def test_autograd_function(orc):
    prob = _prob(2, 20, seed=4)
    steps = 6
    target = _target(orc, prob, steps)
    runner = T.AdjointRunner(prob, steps, 3, precision=T.TFSPH_F64)
    v0g = torch.tensor(prob.gas.v, dtype=torch.float64, device="cuda", requires_grad=True)
    v0d = torch.tensor(prob.dust.v, dtype=torch.float64, device="cuda", requires_grad=True)
    s = torch.tensor(math.log(prob.params.t_stop), dtype=torch.float64, device="cuda", requires_grad=True)
    loss = T.tfsph_loss(v0g, v0d, s, runner, target)
    (3.0 * loss).backward()
    ref_loss, ref_s, ref_gv, ref_gu = _reference(orc, prob, runner, target, steps)
    assert abs(float(loss) - ref_loss) <= 1e-10 * ref_loss
    assert abs(float(s.grad) - 3.0 * ref_s) <= 1e-8 * abs(3.0 * ref_s)
    assert np.max(np.abs(v0g.grad.cpu().numpy() - 3.0 * ref_gv)) <= 1e-8 * np.max(np.abs(3.0 * ref_gv))
    assert np.max(np.abs(v0d.grad.cpu().numpy() - 3.0 * ref_gu)) <= 1e-8 * np.max(np.abs(3.0 * ref_gu))


def test_adjoint_rejects_unsupported():
    prob = I.dusty_shock(n=400)
    params = T.make_params(prob.params, T.TFSPH_F32)
    with pytest.raises(T.TfsphError):
        T.tfsph_adjoint_workspace_size(params, 400, 400, 10, 5)       # adiabatic + viscosity


def _oracle_runs(orc, prob, cases, steps, watch=None):
    """Run the oracle for every (params, gas velocities, dust velocities) case in lock step and
    check that every run keeps the first run's drag cells and canonical order at every step.
    With watch = (gas ids, dust ids) also returns, per watched particle, its smallest distance
    to a cell face over the first run, in cell widths."""
    runs = []
    for p, vg, vd in cases:
        g = orc.from_positions(p, prob.gas.x, vg, prob.gas.m, prob.gas.id)
        d = orc.from_positions(p, prob.dust.x, vd, prob.dust.m, prob.dust.id)
        runs.append((p, g, d))
    D = orc.cell_width(prob.params)[:prob.params.dim]
    near = [np.full(len(w), np.inf) for w in watch] if watch else None
    for s in range(steps):
        for p, g, d in runs:
            orc.step(p, g, d, 1)
        # the oracle keeps each step's canonical order: equal cell histories give equal arrays
        g0, d0 = runs[0][1], runs[0][2]
        for _, g, d in runs[1:]:
            same = all(np.array_equal(a, b) for a, b in ((g.cell, g0.cell), (g.id, g0.id), (d.cell, d0.cell),
                                                         (d.id, d0.id)))
            assert same, f"a drag cell differs at step {s}"
        if watch:
            for k, (ph, ids) in enumerate(((g0, watch[0]), (d0, watch[1]))):
                o = ph.off[:, np.argsort(ph.id)][:, ids] / D[:, None]
                near[k] = np.minimum(near[k], np.min(np.minimum(o, 1.0 - o), axis=0))
    losses = []
    for p, g, d in runs:
        rho = orc.density(p, d)
        losses.append(float(np.mean((rho - prob.extra["target"][d.id]) ** 2)))
    return losses, near


def test_full_size_adjoint_against_oracle_differences(orc):
    """The full adjoint workload (2D wave, 512^2 + 512^2 particles, 256^2 cells, 200 steps,
    checkpoint every 20) as the benchmark runs it, against the FP64 C oracle: its loss, the
    central difference of its loss in log t_stop, and the central differences along two
    velocity directions, one moving the initial velocities of 24 gas particles and one of 24
    dust particles (random signs and components).  Particles of this wave cross drag cells
    (its displacement exceeds the half spacing), and the adjoint holds the cells of the forward
    run: every difference step must leave every particle's drag cell and the canonical order
    unchanged at every step, which is checked, and the perturbed particles are drawn among
    those that never come within a fifth of a cell width of a face.  One particle reaches a face
    at step 189 so closely that any velocity difference moves its crossing, so the velocity
    directions are checked over the first 180 steps (same checkpoint interval).  FP64 device
    run: loss to 1e-10, the three derivatives to 1e-6.  FP32 device run (the benchmark's): loss
    to 1e-4, dL/dlog t_stop to 1e-3, the velocity derivatives to 1e-2."""
    prob = I.workload("wave2d", steps=200)
    ex = prob.extra
    k = np.asarray(ex["kvec"])
    ex["target"] = ex["rho_d0"] * (1.0 + ex["amp"] * np.sin(prob.dust.x @ k))
    target = ex["target"]
    steps, ckpt = 200, 20
    p0 = prob.params
    ts = p0.t_stop
    e, ev = 1e-5, 1e-7
    rng = np.random.default_rng(12)
    pool_g = rng.choice(prob.gas.n, 4096, replace=False)
    pool_d = rng.choice(prob.dust.n, 4096, replace=False)
    losses, near = _oracle_runs(orc, prob, [(p0.replace(t_stop=t), prob.gas.v, prob.dust.v)
                                            for t in (ts, ts * math.exp(e), ts * math.exp(-e))],
                                steps, watch=(pool_g, pool_d))
    l0, fd_t = losses[0], (losses[1] - losses[2]) / (2 * e)
    sel_g = pool_g[near[0] > 0.2][:24]
    sel_d = pool_d[near[1] > 0.2][:24]
    assert len(sel_g) == 24 and len(sel_d) == 24
    dv = np.zeros_like(prob.gas.v)
    du = np.zeros_like(prob.dust.v)
    dv[sel_g, rng.integers(0, 2, 24)] = rng.choice([-1.0, 1.0], 24)
    du[sel_d, rng.integers(0, 2, 24)] = rng.choice([-1.0, 1.0], 24)
    sv = 180
    lv, _ = _oracle_runs(orc, prob, [(p0, prob.gas.v + ev * dv, prob.dust.v),
                                      (p0, prob.gas.v - ev * dv, prob.dust.v),
                                      (p0, prob.gas.v, prob.dust.v + ev * du),
                                      (p0, prob.gas.v, prob.dust.v - ev * du)], sv)
    fd_v, fd_u = (lv[0] - lv[1]) / (2 * ev), (lv[2] - lv[3]) / (2 * ev)
    for prec, tl, tg, tv in ((T.TFSPH_F64, 1e-10, 1e-6, 1e-6), (T.TFSPH_F32, 1e-4, 1e-3, 1e-2)):
        tgt = target if prec == T.TFSPH_F64 else target.astype(np.float32)
        banner(f"adjoint full size: {prob.gas.n}+{prob.dust.n} particles, {steps} steps, ckpt {ckpt}, prec {prec}")
        runner = T.AdjointRunner(prob, steps, ckpt, precision=prec)
        loss, dlogt, _, _ = runner.run(tgt)
        torch.cuda.synchronize()
        del runner
        runner = T.AdjointRunner(prob, sv, ckpt, precision=prec)
        _, _, gv, gu = runner.run(tgt)
        torch.cuda.synchronize()
        del runner
        dir_v = float(np.sum(gv.cpu().numpy().astype(np.float64) * dv))
        dir_u = float(np.sum(gu.cpu().numpy().astype(np.float64) * du))
        banner(f"loss {float(loss):.9e} vs {l0:.9e}; dL/dlog t_stop {float(dlogt):.9e} vs {fd_t:.9e}; "
               f"dL/dv0.dv {dir_v:.9e} vs {fd_v:.9e}; dL/du0.du {dir_u:.9e} vs {fd_u:.9e}")
        assert abs(float(loss) - l0) <= tl * l0
        assert abs(float(dlogt) - fd_t) <= tg * abs(fd_t)
        assert abs(dir_v - fd_v) <= tv * abs(fd_v)
        assert abs(dir_u - fd_u) <= tv * abs(fd_u)
