"""Pins of the oracle's second-order IMEX step (ARS(2,2,2), Ascher, Ruuth & Spiteri 1997, with
the drag in cell of Section 2.3 as its implicit part and the SPH terms, gravity and the drift as
its explicit part).

Each check compares the oracle with a fact fixed independently of its code: the scheme's linear
stability function, worked out by hand from the published tableau; exact parabolic trajectories
(the explicit pair integrates a constant acceleration exactly); conservation of momentum; the
stiff limit of the drag; and the observed order of accuracy (halving tau divides the error by
about 4, where the first-order step divides it by about 2).
"""
import math

import numpy as np
import pytest

from paper_1908_01682_amd import inputs as I

GAM = 1.0 - 1.0 / math.sqrt(2.0)


def _R(z):
    """ARS(2,2,2) on y' = -lambda y (all implicit), z = tau lambda:
    Y2 = y / (1 + gamma z); Y3 (1 + gamma z) = y - (1 - gamma) z Y2, so
    R(z) = (1 + (2 gamma - 1) z) / (1 + gamma z)^2 = 1 - z + z^2 / 2 + O(z^3)."""
    return (1.0 + (2.0 * GAM - 1.0) * z) / (1.0 + GAM * z) ** 2


def _uniform_mixture(eps, v0, u0, n=64, **kw):
    prob = I.dusty_wave(n_side=n, dim=1, amp=0.0, eps=eps, h_over_dx=2.0, cells_per_axis=n // 2)
    prob.gas.v[:] = v0
    prob.dust.v[:] = u0
    prob.params = prob.params.replace(scheme=1, **kw)
    return prob


def test_stability_function_is_second_order():
    """The hand-derived R(z) matches exp(-z) to second order and is L-stable."""
    for z in (1e-2, 2e-2):
        assert abs(_R(z) - math.exp(-z)) < 0.1 * z ** 3
    assert abs(_R(1e8)) < 1e-7


@pytest.mark.parametrize("eps", [1.0, 0.3, 7.0])
@pytest.mark.parametrize("z", [0.05, 1.0, 30.0, 1e4])
def test_uniform_mixture_decays_by_the_stability_function(orc, eps, z):
    """Uniform mixture, constant t_stop: per step v - u is multiplied by R(tau (1 + eps) / t_stop)
    and the barycentric velocity is unchanged."""
    prob = _uniform_mixture(eps, 0.03, -0.01)
    tau = prob.params.dt
    p = prob.params.replace(t_stop=tau * (1.0 + eps) / z)
    g, d = orc.from_problem(prob)
    bary = (0.03 + eps * -0.01) / (1 + eps)
    for s in range(1, 6):
        orc.step(p, g, d, 1)
        gi, di = g.by_id(), d.by_id()
        rel = gi.vel[0] - di.vel[0]
        assert np.max(np.abs(rel - 0.04 * _R(z) ** s)) < 1e-15
        assert np.max(np.abs((gi.vel[0] + eps * di.vel[0]) / (1 + eps) - bary)) < 1e-15


@pytest.mark.parametrize("law", ["K", "epstein"])
def test_other_drag_laws_decay_by_the_stability_function(orc, law):
    """K held constant: z = tau K (1/rho_g + 1/rho_d); Epstein t*_stop = T_E / rho*_g:
    z = tau (rho_g + rho_d) / T_E (uniform mixture, rho_g = 1, rho_d = eps)."""
    eps = 0.5
    prob = _uniform_mixture(eps, 0.03, -0.01)
    tau = prob.params.dt
    if law == "K":
        K = 400.0
        p = prob.params.replace(K=K, t_stop=float("nan"))
        z = tau * K * (1.0 + 1.0 / eps)
    else:
        TE = 3e-3
        p = prob.params.replace(t_stop_epstein=TE, t_stop=float("nan"))
        z = tau * (1.0 + eps) / TE
    g, d = orc.from_problem(prob)
    for s in range(1, 4):
        orc.step(p, g, d, 1)
        rel = g.by_id().vel[0] - d.by_id().vel[0]
        assert np.max(np.abs(rel - 0.04 * _R(z) ** s)) < 1e-15


@pytest.mark.parametrize("scheme,coef", [(1, 0.5), (0, 1.0)], ids=["imex", "first_order"])
def test_free_fall_is_an_exact_parabola(orc, scheme, coef):
    """No drag (t_stop ~ infinity) and no pressure (c_s ~ 0): every particle falls with
    v^{n+1} = v^n + tau g and x^{n+1} = x^n + tau v^n + c tau^2 g, with c = 1/2 for the IMEX pair
    ((1 - delta) gamma = 1/2) and c = 1 for the first-order step (x moves with v^{n+1})."""
    rng = np.random.default_rng(3)
    prob = I.dusty_wave(n_side=64, dim=2, amp=0.0, h_over_dx=2.0, cells_per_axis=16)
    for ph in (prob.gas, prob.dust):
        ph.v[:] = 0.05 * rng.standard_normal(ph.v.shape)
    gvec = (0.8, -1.3, 0.0)
    p = prob.params.replace(scheme=scheme, t_stop=1e30, c_s=1e-12, g=gvec)
    g, d = orc.from_problem(prob)
    x0 = [orc.positions(p, ph.by_id()) for ph in (g, d)]
    v0 = [ph.by_id().vel.T.copy() for ph in (g, d)]
    nst = 3
    orc.step(p, g, d, nst)
    tau = p.dt
    ga = np.array(gvec[:2])
    for ph, xa, va in zip((g, d), x0, v0):
        b = ph.by_id()
        T = nst * tau
        assert np.max(np.abs(b.vel.T - (va + T * ga))) < 1e-14
        # sum over the steps of tau v^n + c tau^2 g
        want = xa + T * va + (nst * (nst - 1) / 2 + nst * coef) * tau ** 2 * ga
        got = orc.positions(p, b)
        dx = (got - want + 0.5) % 1.0 - 0.5          # periodic unit box
        assert np.max(np.abs(dx)) < 1e-14


def _random_mixture(dim, n, seed, **kw):
    rng = np.random.default_rng(seed)
    nc = [12, 10, 8][:dim]
    nc3 = tuple(nc + [1] * (3 - dim))
    p = I.Params(dim=dim, n_cells=nc3, lo=(-0.3, 0.1, 0.0), hi=(0.7, 1.1, 1.0), h=[0.04, 0.04, 0.06][dim - 1],
                 dt=2e-3, c_s=1.0, scheme=1, **kw)
    xg = np.stack([rng.uniform(p.lo[k], p.hi[k], n) for k in range(dim)], axis=1)
    xd = np.stack([rng.uniform(p.lo[k], p.hi[k], n) for k in range(dim)], axis=1)
    g = I.Phase(xg, 0.1 * rng.standard_normal((n, dim)), rng.uniform(0.5, 1.5, n) / n, np.arange(n, dtype=np.int32))
    dd = I.Phase(xd, 0.1 * rng.standard_normal((n, dim)), rng.uniform(0.1, 3.0, n) / n, np.arange(n, dtype=np.int32))
    return I.Problem("mix", p, g, dd, 1)


@pytest.mark.parametrize("dim", [1, 2, 3])
@pytest.mark.parametrize("law", ["t_stop", "K"])
def test_momentum_is_conserved(orc, dim, law):
    """Pressure pair terms cancel in the sum and the drag only exchanges momentum inside a
    volume, at both implicit stages, so total momentum is conserved over an IMEX step."""
    kw = dict(t_stop=1e-3) if law == "t_stop" else dict(K=300.0, t_stop=float("nan"))
    prob = _random_mixture(dim, 1500, 70 + dim, **kw)
    g, d = orc.from_problem(prob)
    P0 = (g.mass * g.vel).sum(axis=1) + (d.mass * d.vel).sum(axis=1)
    scale = (g.mass * np.abs(g.vel)).sum() + (d.mass * np.abs(d.vel)).sum()
    orc.step(prob.params, g, d, 2)
    P1 = (g.mass * g.vel).sum(axis=1) + (d.mass * d.vel).sum(axis=1)
    assert np.max(np.abs(P1 - P0)) < 1e-14 * scale


def test_stiff_limit_common_velocity(orc):
    """t_stop -> 0: the last implicit stage leaves one velocity per volume for both phases."""
    prob = _random_mixture(2, 1500, 81, t_stop=1e-13)
    p = prob.params
    g, d = orc.from_problem(prob)
    orc.step(p, g, d, 1)
    ncell = int(np.prod(p.n_cells[:2]))
    for k in range(2):
        lo = np.full(ncell, np.inf)
        hi = np.full(ncell, -np.inf)
        for ph in (g, d):
            np.minimum.at(lo, ph.cell, ph.vel[k])
            np.maximum.at(hi, ph.cell, ph.vel[k])
        both = np.isin(np.arange(ncell), g.cell) & np.isin(np.arange(ncell), d.cell)
        assert both.sum() > ncell // 2
        assert np.max(hi[both] - lo[both]) < 1e-8


def _wave_run(orc, scheme, nsteps, T, t_stop, n=200, amp=1e-4):
    prob = I.dusty_wave(n_side=n, amp=amp, t_stop=t_stop, cells_per_axis=n // 2)
    p = prob.params.replace(scheme=scheme, dt=T / nsteps)
    g, d = orc.from_problem(prob)
    orc.step(p, g, d, nsteps)
    return np.concatenate([g.by_id().vel[0], d.by_id().vel[0]])


def test_second_order_in_time(orc):
    """Dusty wave (N = 200, t_stop = 0.01, amplitude 1e-4: no particle changes cell, so the
    semi-discrete system is smooth): successive differences of the IMEX solution fall by about 4
    per halving of tau, those of the first-order step by about 2, and the IMEX solution agrees
    with the first-order one as tau -> 0 (both discretise the same system)."""
    T, ts = 0.02, 0.01
    steps = (8, 16, 32, 64)
    imex = [_wave_run(orc, 1, s, T, ts) for s in steps]
    idic = [_wave_run(orc, 0, s, T, ts) for s in steps]
    d_imex = [np.max(np.abs(imex[i] - imex[i + 1])) for i in range(3)]
    d_idic = [np.max(np.abs(idic[i] - idic[i + 1])) for i in range(3)]
    r_imex = [d_imex[i] / d_imex[i + 1] for i in range(2)]
    r_idic = [d_idic[i] / d_idic[i + 1] for i in range(2)]
    assert all(3.5 < r < 4.6 for r in r_imex), (d_imex, r_imex)
    assert all(1.7 < r < 2.3 for r in r_idic), (d_idic, r_idic)
    fine = _wave_run(orc, 0, 2048, T, ts)
    # the first-order step at 2048 steps is within ~d_idic[-1] / 32 of the limit
    assert np.max(np.abs(imex[-1] - fine)) < d_idic[-1] / 8


def test_second_order_in_time_adiabatic(orc):
    """The same for an adiabatic gas with viscosity (the energy equation is in the explicit
    part): uniform density and a smooth periodic pressure profile p ~ 0.2 + 0.8 (1 + cos 2 pi x)/2
    on the 1D tube (N = 800), no particle changes cell over T = 0.02."""
    prob = I.dusty_shock(n=800, t_stop=1e-2, rho_r=1.0, p_r=1.0)
    x = prob.gas.x[:, 0]
    prob.gas.e = 2.5 * (0.8 * 0.5 * (1.0 + np.cos(2.0 * np.pi * x)) + 0.2)
    T = 2e-2
    outs = []
    for s in (40, 80, 160, 320):        # tau from 5e-4 (the CFL step) down
        q = prob.copy()
        p = q.params.replace(scheme=1, dt=T / s)
        g, d = orc.from_problem(q)
        orc.step(p, g, d, s)
        gi, di = g.by_id(), d.by_id()
        outs.append(np.concatenate([gi.vel[0], di.vel[0], gi.energy]))
    dd = [np.max(np.abs(outs[i] - outs[i + 1])) for i in range(3)]
    r = [dd[i] / dd[i + 1] for i in range(2)]
    assert all(3.4 < v < 4.6 for v in r), (dd, r)
