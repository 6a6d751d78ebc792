"""Pins of the FP64 gradient reference (oracle/adjoint_torch.py).

Its forward pass must reproduce the C oracle's step to rounding, and its
autograd gradients must equal central finite differences of the C oracle's
loss: d/d log t_stop directly, and d/dv0, d/du0 along random directions.
With the drag coefficient K held constant the scalar is log(1/K) instead.
"""
import math

import numpy as np
import pytest
import torch

from paper_1908_01682_amd import inputs as I


def _problem(dim, seed, per_particle_dust_mass=False, kmode=False, epstein=False):
    if dim == 1:
        prob = I.dusty_wave(n_side=120, amp=1e-2, t_stop=1e-3, eps=0.7, cells_per_axis=60)
    else:
        prob = I.wave_2d(n_side=24, amp=1e-2, t_stop=1e-3, eps=1.3)
    rng = np.random.default_rng(seed)
    prob.gas.v = prob.gas.v + 0.02 * rng.standard_normal(prob.gas.v.shape)
    prob.dust.v = prob.dust.v + 0.02 * rng.standard_normal(prob.dust.v.shape)
    if per_particle_dust_mass:
        prob.dust.m = prob.dust.m * rng.uniform(0.5, 1.5, prob.dust.n)
    if kmode:
        prob.params = prob.params.replace(K=800.0)
    if epstein:
        prob.params = prob.params.replace(t_stop_epstein=1.5e-3)
    return prob


def _relax(p):
    """The relaxation-time parameter: t_stop, 1/K when K is held constant, or t_stop_epstein."""
    if p.K > 0:
        return 1.0 / p.K
    return p.t_stop_epstein if p.t_stop_epstein > 0 else p.t_stop


def _with_relax(p, t):
    if p.K > 0:
        return p.replace(K=1.0 / t)
    return p.replace(t_stop_epstein=t) if p.t_stop_epstein > 0 else p.replace(t_stop=t)


def c_oracle_loss(orc, prob, v0g, v0d, t_stop, target, steps):
    p = _with_relax(prob.params, t_stop)
    g = orc.from_positions(p, prob.gas.x, v0g, prob.gas.m, prob.gas.id)
    d = orc.from_positions(p, prob.dust.x, v0d, prob.dust.m, prob.dust.id)
    orc.step(p, g, d, steps)
    rho = orc.density(p, d)            # sorts d
    return float(np.mean((rho - target[d.id]) ** 2)), g, d


def _target(orc, prob, steps):
    _, _, d = c_oracle_loss(orc, prob, prob.gas.v, prob.dust.v, 2.0 * _relax(prob.params), np.zeros(prob.dust.n),
                            steps)
    rho = orc.density(prob.params, d)
    t = np.zeros(prob.dust.n)
    t[d.id] = rho
    return t


@pytest.mark.parametrize("dim,law", [(1, "t"), (2, "t"), (1, "K"), (2, "K"), (1, "E"), (2, "E")])
def test_torch_forward_equals_c_oracle(orc, dim, law):
    from oracle import adjoint_torch as AT
    prob = _problem(dim, 1, per_particle_dust_mass=True, kmode=law == "K", epstein=law == "E")
    steps = 8
    target = _target(orc, prob, steps)
    p = prob.params
    loss_c, g, d = c_oracle_loss(orc, prob, prob.gas.v, prob.dust.v, _relax(p), target, steps)
    vg = torch.tensor(prob.gas.v)
    vd = torch.tensor(prob.dust.v)
    s = torch.tensor(math.log(_relax(p)), dtype=torch.float64)
    loss_t, v, u, (xg, xd), _ = AT.forward_loss(p, prob.gas.x, prob.dust.x, prob.gas.m, prob.dust.m, vg, vd, s,
                                               target, steps)
    gi, di = g.by_id(), d.by_id()
    assert np.max(np.abs(v.detach().numpy().T - gi.vel)) < 1e-13
    assert np.max(np.abs(u.detach().numpy().T - di.vel)) < 1e-13
    L = np.array([p.hi[k] - p.lo[k] for k in range(dim)])
    dx = xg.detach().numpy() - orc.positions(p, gi)
    dx -= L * np.round(dx / L)
    assert np.max(np.abs(dx)) < 1e-13
    assert abs(float(loss_t) - loss_c) <= 1e-10 * loss_c


@pytest.mark.parametrize("dim,mass,law", [(1, False, "t"), (2, False, "t"), (2, True, "t"),
                                          (1, False, "K"), (2, True, "K"), (1, True, "E"), (2, True, "E")])
def test_gradients_match_central_differences(orc, dim, mass, law):
    from oracle import adjoint_torch as AT
    prob = _problem(dim, 2 + dim, per_particle_dust_mass=mass, kmode=law == "K", epstein=law == "E")
    steps = 6
    p = prob.params
    t0 = _relax(p)
    target = _target(orc, prob, steps)
    loss, dls, dvg, dvd = AT.gradients(p, prob.gas.x, prob.dust.x, prob.gas.m, prob.dust.m, prob.gas.v,
                                       prob.dust.v, t0, target, steps)
    # d/d log t_stop (d/d log(1/K) with K held constant)
    e = 1e-5
    lp, _, _ = c_oracle_loss(orc, prob, prob.gas.v, prob.dust.v, t0 * math.exp(e), target, steps)
    lm, _, _ = c_oracle_loss(orc, prob, prob.gas.v, prob.dust.v, t0 * math.exp(-e), target, steps)
    fd = (lp - lm) / (2 * e)
    assert abs(dls - fd) <= 1e-6 * abs(fd) + 1e-12 * loss, (dls, fd)
    assert abs(fd) > 1e-3 * loss / 1.0       # the derivative is not trivially zero
    # directional derivatives in v0 and u0
    rng = np.random.default_rng(7)
    for which in ("gas", "dust"):
        dirn = rng.standard_normal(prob.gas.v.shape if which == "gas" else prob.dust.v.shape)
        h = 1e-6
        vg_p, vd_p = prob.gas.v.copy(), prob.dust.v.copy()
        vg_m, vd_m = prob.gas.v.copy(), prob.dust.v.copy()
        if which == "gas":
            vg_p += h * dirn
            vg_m -= h * dirn
            ana = float(np.sum(dvg * dirn))
        else:
            vd_p += h * dirn
            vd_m -= h * dirn
            ana = float(np.sum(dvd * dirn))
        lp, _, _ = c_oracle_loss(orc, prob, vg_p, vd_p, t0, target, steps)
        lm, _, _ = c_oracle_loss(orc, prob, vg_m, vd_m, t0, target, steps)
        fd = (lp - lm) / (2 * h)
        assert abs(ana - fd) <= 1e-5 * abs(fd) + 1e-9 * loss, (which, ana, fd)
