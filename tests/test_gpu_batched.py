"""Batched forms (the persistent kernel and the flattened launches) and hipGraph replay.

Every instance of a batch must evolve bitwise as it does alone through
tfsph_step, in either form; results must not depend on the launch shape or
the form; graph replays must equal eager launches on every replay.
"""
import numpy as np
import pytest

from paper_1908_01682_amd import inputs as I
from tests.gpu_util import HAVE_GPU, banner, by_id, compare_states, needs_gpu, oracle_phase

pytestmark = [pytest.mark.gpu, needs_gpu]

if HAVE_GPU:
    import torch
    from paper_1908_01682_amd import tfsph as T

KEYS = ("cell", "id", "off", "vel", "rho")


def _batch_1d(seed=11, n_inst=6):
    probs = I.batched_waves(n_inst=n_inst, n_min=500, n_max=3000, seed=seed, amp=1e-2)
    probs.append(I.dusty_wave(n_side=41, amp=1e-2, t_stop=3e-4, eps=0.2, cells_per_axis=20))   # tiny, odd N
    return probs


def _batch_1d_kmode(seed=21):
    """Instances with the drag coefficient K held constant and with the Epstein law next to
    constant-t_stop ones."""
    probs = I.batched_waves(n_inst=6, n_min=600, n_max=2500, seed=seed, amp=1e-2)
    for i, p in enumerate(probs):
        if i % 3 == 0:
            p.params = p.params.replace(K=float(200.0 * (i + 1)))
        elif i % 3 == 1:
            p.params = p.params.replace(t_stop_epstein=float(1e-3 * (i + 1)))
    return probs


def _batch_2d():
    rng = np.random.default_rng(3)
    out = []
    for n in (24, 40, 32):
        p = I.wave_2d(n_side=n, amp=1e-2, t_stop=float(10 ** rng.uniform(-4, -2)), eps=float(10 ** rng.uniform(-1, 1)))
        out.append(p)
    return out


def _same(a, b):
    A, B = by_id(a), by_id(b)
    for k in KEYS:
        if A[k] is None:
            continue
        assert np.array_equal(A[k], B[k]), k


FORMS = {"persistent": 0, "flat": 1, "mixed": 2}


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("dim,precision,kmode", [(1, 0, False), (1, 1, False), (2, 0, False), (1, 0, True)])
def test_batched_equals_plain_bitwise(dim, precision, kmode, form):
    """Both forms, and a call of each in turn (the second call counts from the arrays the first
    left), against tfsph_step on each instance alone."""
    probs = _batch_1d_kmode() if kmode else (_batch_1d() if dim == 1 else _batch_2d())
    banner(f"batched dim={dim} precision={precision} n_inst={len(probs)} form={form}")
    f0 = T.TFSPH_BATCH_PERSISTENT if form == "persistent" else T.TFSPH_BATCH_FLAT
    f1 = T.TFSPH_BATCH_PERSISTENT if form != "flat" else T.TFSPH_BATCH_FLAT
    bs = T.BatchedSimulation(probs, precision=precision, form=f0)
    bs.step(7)
    bs.set_tuning(256, f1)
    bs.step(13)
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        sim = T.Simulation(p, precision=precision)
        sim.step(20)
        torch.cuda.synchronize()
        g, d = bs.instance(i)
        _same(g, sim.gas.numpy())
        _same(d, sim.dust.numpy())
        sim.close()
    flags, _ = bs.flags()
    bs.close()
    assert not (flags & T.TFSPH_FLAG_NONFINITE)


def _batch_1d_viscous(all_viscous):
    """Instances with artificial viscosity (the general force loop), on every instance or on
    every other one next to the isothermal loop without viscosity."""
    probs = I.batched_waves(n_inst=5, n_min=600, n_max=2500, seed=31, amp=1e-2)
    for i, p in enumerate(probs):
        if all_viscous or i % 2 == 0:
            p.params = p.params.replace(av_alpha=1.0, av_beta=2.0)
    return probs


@pytest.mark.parametrize("form", ["persistent", "flat"])
@pytest.mark.parametrize("all_viscous", [True, False], ids=["all_viscous", "mixed"])
def test_batched_force_kinds_equal_plain_bitwise(all_viscous, form):
    """The flattened force launch is specialised on a force loop that every instance shares
    and picks each instance's loop at run time otherwise: either way every instance equals
    tfsph_step on it alone, bitwise."""
    probs = _batch_1d_viscous(all_viscous)
    banner(f"batched force kinds all_viscous={all_viscous} form={form}")
    bs = T.BatchedSimulation(probs, precision=0, form=FORMS[form])
    bs.step(12)
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        sim = T.Simulation(p, precision=0)
        sim.step(12)
        torch.cuda.synchronize()
        g, d = bs.instance(i)
        _same(g, sim.gas.numpy())
        _same(d, sim.dust.numpy())
        sim.close()
    flags, _ = bs.flags()
    bs.close()
    assert not (flags & T.TFSPH_FLAG_NONFINITE)


def test_batched_matches_oracle(orc):
    probs = _batch_1d(seed=5, n_inst=3)
    bs = T.BatchedSimulation(probs, precision=0)
    # oracle from the batched initial state
    init = [bs.instance(i) for i in range(len(probs))]
    bs.step(5)
    torch.cuda.synchronize()
    for i, p in enumerate(probs):
        for ph, src in ((init[i][0], p.gas), (init[i][1], p.dust)):
            ph["mass"] = src.m[ph["id"]]        # packed batches carry per-instance masses in the descriptor
        og, od = oracle_phase(orc, init[i][0], 1), oracle_phase(orc, init[i][1], 1)
        orc.step(p.params, og, od, 5)
        g, d = bs.instance(i)
        g["mass"], d["mass"] = p.gas.m[g["id"]], p.dust.m[d["id"]]
        err = compare_states(p.params, g, d, og, od, p.params.c_s)
        assert all(v <= 5e-5 for v in err.values()), (i, err)
    bs.close()


def test_batched_launch_shape_invariance():
    probs = _batch_1d(seed=8, n_inst=5)
    res = []
    for blk in (64, 256, 1024):
        bs = T.BatchedSimulation(probs, precision=0, block=blk)
        bs.step(15)
        torch.cuda.synchronize()
        res.append([bs.instance(i) for i in range(len(probs))])
        bs.close()
    for other in res[1:]:
        for (g0, d0), (g1, d1) in zip(res[0], other):
            _same(g0, g1)
            _same(d0, d1)


@pytest.mark.parametrize("form", [0, 1], ids=["persistent", "flat"])
def test_batched_graph_replays_equal_eager(form):
    probs = _batch_1d(seed=9, n_inst=4)
    eager = T.BatchedSimulation(probs, precision=0, form=form)
    graph = T.BatchedSimulation(probs, precision=0, form=form)
    for rep in range(4):
        eager.step(6)
        graph.step_graph(6)
        torch.cuda.synchronize()
        # eager host work and a synchronisation between replays
        ge = [eager.instance(i) for i in range(len(probs))]
        gg = [graph.instance(i) for i in range(len(probs))]
        for (a0, a1), (b0, b1) in zip(ge, gg):
            _same(a0, b0)
            _same(a1, b1)
    eager.close()
    graph.close()


@pytest.mark.parametrize("chunk", [1, 8])
def test_step_graph_equals_eager(chunk):
    prob = I.dusty_shock(n=6000, t_stop=1e-3)
    a = T.Simulation(prob, precision=0)
    b = T.Simulation(prob, precision=0)
    for rep in range(3):
        a.step(19)
        b.step_graph(19, chunk=chunk)
        torch.cuda.synchronize()
        _same(a.gas.numpy(), b.gas.numpy())
        _same(a.dust.numpy(), b.dust.numpy())
        e = a.gas.numpy()["energy"]
        assert np.array_equal(e, b.gas.numpy()["energy"])
    a.close()
    b.close()


def test_batched_rejects_bad_desc():
    probs = _batch_1d(seed=1, n_inst=2)
    bs = T.BatchedSimulation(probs, precision=0)
    other = T.BatchedSimulation(probs, precision=0)
    with pytest.raises(T.TfsphError):
        T.tfsph_step_batched(bs.handle, other.state, 1)       # state not bound to this batch
    with pytest.raises(T.TfsphError):
        bs.set_block(100)                                       # not a multiple of 64
    bs.close()
    other.close()


def test_autotuner_picks_a_shape_and_caches(tmp_path):
    from paper_1908_01682_amd import autotune as A
    probs = _batch_1d(seed=12, n_inst=4)
    bs = T.BatchedSimulation(probs, precision=0)
    path = str(tmp_path / "tune.json")
    before = [bs.instance(i) for i in range(len(probs))]
    r1 = A.tune(bs, steps=4, blocks=(256, 512, 1024), path=path, graph=True)
    assert r1["bitwise_identical"] and not r1["cached"]
    assert set(r1["ms_per_step"]) == {"persistent/256", "persistent/512", "persistent/1024",
                                      *(f"flat/{c}" for c in A.CANDIDATE_FLAT_CELLS)}
    assert (r1["form"], r1["block"], r1["cells_per_block"]) in (
        [(A.PERSISTENT, b, 0) for b in (256, 512, 1024)] + [(A.FLAT, 256, c) for c in A.CANDIDATE_FLAT_CELLS])
    after = [bs.instance(i) for i in range(len(probs))]      # state restored
    for (g0, d0), (g1, d1) in zip(before, after):
        for k in ("cell", "id", "off", "vel"):
            assert np.array_equal(g0[k], g1[k]) and np.array_equal(d0[k], d1[k])
    r2 = A.tune(bs, steps=4, blocks=(256, 512, 1024), path=path, graph=True)
    assert r2["cached"] and (r2["form"], r2["block"], r2["cells_per_block"]) == \
        (r1["form"], r1["block"], r1["cells_per_block"])
    assert (bs.form, bs.block, bs.cells_per_block) == (r1["form"], r1["block"], r1["cells_per_block"])
    bs.close()


def test_flat_cells_per_block_invariance():
    """The flattened form at several cells per update workgroup, changed between calls and
    across graph replays (a graph captured with another block table is dropped), gives
    bitwise the state of the default shape."""
    probs = _batch_1d(seed=9, n_inst=5)
    ref = T.BatchedSimulation(probs, precision=0, form=T.TFSPH_BATCH_FLAT)
    ref.step(12)
    torch.cuda.synchronize()
    want = [ref.instance(i) for i in range(len(probs))]
    ref.close()
    bs = T.BatchedSimulation(probs, precision=0, form=T.TFSPH_BATCH_FLAT, cells_per_block=16)
    bs.step_graph(3)
    bs.set_tuning(256, T.TFSPH_BATCH_FLAT, 200)
    bs.step_graph(3)
    bs.set_tuning(256, T.TFSPH_BATCH_FLAT, 16)
    bs.step_graph(3)                 # the same key as the first capture, with the table rebuilt
    bs.set_tuning(256, T.TFSPH_BATCH_FLAT, 1)
    bs.step(3)
    torch.cuda.synchronize()
    for i, (g, d) in enumerate(want):
        g1, d1 = bs.instance(i)
        _same(g, g1)
        _same(d, d1)
    with pytest.raises(T.TfsphError):
        bs.set_tuning(256, T.TFSPH_BATCH_FLAT, 257)
    bs.close()


def test_full_size_batched_equals_plain_on_sampled_instances(tmp_path):
    """The full batched workload (256 uneven 1D waves, 5.4M particles, 500 steps) in the launch
    configuration the benchmark times (form and workgroup size autotuned on graph replays,
    hipGraph replay), and in the other form: sampled instances, the largest and the smallest
    among them, are bitwise what tfsph_step gives alone."""
    from paper_1908_01682_amd import autotune as A
    probs = I.batched_waves()
    steps = probs[0].steps
    sizes = [p.gas.n + p.dust.n for p in probs]
    rng = np.random.default_rng(17)
    sample = sorted({int(np.argmax(sizes)), int(np.argmin(sizes)), *rng.integers(0, len(probs), 2).tolist()})
    banner(f"batched full size: {len(probs)} instances, {sum(sizes)} particles, {steps} steps, sample {sample}")
    bs = T.BatchedSimulation(probs, precision=T.TFSPH_F32)
    A.tune(bs, steps=4, path=str(tmp_path / "tune.json"), graph=True)
    other = T.BatchedSimulation(probs, precision=T.TFSPH_F32, block=512,
                                form=T.TFSPH_BATCH_PERSISTENT if bs.form == T.TFSPH_BATCH_FLAT else T.TFSPH_BATCH_FLAT)
    banner(f"batched full size: tuned form {bs.form} block {bs.block}, other form {other.form}")
    bs.step_graph(steps)
    other.step_graph(steps)
    torch.cuda.synchronize()
    for b in (bs, other):
        flags, _ = b.flags()
        assert not (flags & T.TFSPH_FLAG_NONFINITE)
    for i in sample:
        sim = T.Simulation(probs[i], precision=T.TFSPH_F32)
        sim.step(steps)
        torch.cuda.synchronize()
        for b in (bs, other):
            g, d = b.instance(i)
            _same(g, sim.gas.numpy())
            _same(d, sim.dust.numpy())
        sim.close()
    bs.close()
    other.close()
