"""Pins of the oracle's two comparison schemes: the Monaghan-Kocharyan explicit pairwise drag
(Section 2.1, eqs. 8-10) and the semi-implicit ISPH drag with SPH interpolation (Section 2.2,
eqs. 11-16), and of all three schemes against the paper's own printed errors (Tables 1-2).

Each check compares the oracle with something it does not compute itself: the values the
paper prints for its runs, the exact relaxation of a uniform mixture on a lattice where SPH
interpolation is exact, the drag-free and stiff limits, exact momentum conservation, and the
linear dusty-wave solution.
"""
import numpy as np
import pytest

from paper_1908_01682_amd import inputs as I
from tests import paper_tables as PT

MK, ISPH, IDIC = 2, 3, 0


def _uniform(eps, v0, u0, scheme, n=64, **kw):
    """Gas and dust on the same 1D lattice, h = 2 dx: SPH sums and interpolation are exact."""
    prob = I.dusty_wave(n_side=n, dim=1, amp=0.0, eps=eps, t_stop=1e-3, h_over_dx=2.0, cells_per_axis=n // 2)
    prob.gas.v[:] = v0
    prob.dust.v[:] = u0
    prob.params = prob.params.replace(scheme=scheme, **kw)
    return prob


# ---------------------------------------------------------------------------
# the paper's printed errors
# ---------------------------------------------------------------------------

def _close_to_printed(ours, printed, rel):
    digits = len(repr(printed).split(".")[1].lstrip("0")) if "." in repr(printed) else 1
    half_unit = 0.5 * 10.0 ** (np.floor(np.log10(printed)) - (digits - 1))
    return abs(ours - printed) <= max(rel * printed, half_unit)


@pytest.mark.parametrize("row", PT.printed("table1_dustywave.txt"), ids=["h0.01", "h0.02"])
def test_table1_dustywave_errors_are_the_papers(orc, row):
    """Table 1: the L2 error of the dust velocity at t = 0.5 (RMS over the amplitude of the
    exact wave at that time).  MK and ISPH, which have no cells, give 0.0423 / 0.0338 and
    0.150 / 0.081 against 0.0417 / 0.0332 and 0.1486 / 0.079 printed: within 4 %.  IDIC with
    drag cells one particle spacing wide gives 3.6e-4 and 1.5e-3 against 0.0003 and 0.0012,
    printed with one and two digits: within 30 %, two orders of magnitude below the others."""
    h, tau, want = row
    got = {}
    for m in ("MK", "ISPH", "IDIC"):
        prob = PT.wave_problem(h, tau, m)
        x, u = PT.run_oracle(orc, prob)
        got[m] = PT.wave_error(prob, x, u)
    for m, rel in (("MK", 0.04), ("ISPH", 0.04), ("IDIC", 0.3)):
        assert _close_to_printed(got[m], want[m], rel), (m, got, want)
    assert got["IDIC"] < got["ISPH"] / 50 and got["ISPH"] < got["MK"], got
    stored = PT.stored_oracle_errors()
    for m in got:
        assert abs(got[m] - stored[("wave", h, tau, m)]) <= 1e-9 * got[m], (m, got[m])


@pytest.mark.parametrize("row", PT.printed("table2_dustyshock.txt"), ids=["h0.01", "h0.02"])
def test_table2_dustyshock_ranking_and_size(orc, row):
    """Table 2: IDIC < MK < ISPH for the Dustyshock at t = 0.2, as printed.  The norm is not
    defined in the paper; with the RMS over |x| < 0.25 against the stiff-limit solution IDIC
    and MK are within 10 % of the printed values and ISPH within 30 % (it comes out lower)."""
    h, tau, want = row
    got = {}
    for m in ("MK", "ISPH", "IDIC"):
        prob = PT.shock_problem(h, tau, m)
        x, u = PT.run_oracle(orc, prob)
        got[m] = PT.shock_error(prob, x, u)
    assert got["IDIC"] < got["MK"] < got["ISPH"], got
    for m, rel in (("IDIC", 0.1), ("MK", 0.1), ("ISPH", 0.3)):
        assert abs(got[m] - want[m]) <= rel * want[m], (m, got, want)
    stored = PT.stored_oracle_errors()
    for m in got:
        assert abs(got[m] - stored[("shock", h, tau, m)]) <= 1e-9 * got[m], (m, got[m])


# ---------------------------------------------------------------------------
# ISPH
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("eps", [1.0, 0.3, 7.0])
@pytest.mark.parametrize("law", ["t_stop", "K", "epstein"])
def test_isph_uniform_mixture_decays_like_the_implicit_solve(orc, eps, law):
    """On a lattice where SPH interpolation is exact, every particle's two-velocity system of
    eqs. (12)-(15) is the cell system of IDIC with the continuum densities: v - u shrinks by
    exactly 1 / (1 + tau K (1/rho_g + 1/rho_d)) per step and the barycentre stays."""
    kw = dict(t_stop=dict(), K=dict(K=800.0), epstein=dict(t_stop_epstein=2e-3))[law]
    prob = _uniform(eps, 0.3, -0.1, ISPH, **kw)
    p = prob.params
    rho_g, rho_d = 1.0, eps
    K = dict(t_stop=rho_d / p.t_stop, K=800.0, epstein=rho_g * rho_d / 2e-3)[law]
    D = 1.0 + p.dt * K * (1.0 / rho_g + 1.0 / rho_d)
    bary = (0.3 * rho_g + -0.1 * rho_d) / (rho_g + rho_d)
    g, d = orc.from_problem(prob)
    for s in range(1, 5):
        orc.step(p, g, d, 1)
        gi, di = g.by_id(), d.by_id()
        assert np.max(np.abs(gi.vel[0] - di.vel[0] - 0.4 / D ** s)) < 1e-14
        assert np.max(np.abs((rho_g * gi.vel[0] + rho_d * di.vel[0]) / (rho_g + rho_d) - bary)) < 1e-14


def test_isph_stiff_limit_is_the_barycentre(orc):
    prob = _uniform(3.0, 0.5, -0.2, ISPH, t_stop=1e-13)
    g, d = orc.from_problem(prob)
    orc.step(prob.params, g, d, 1)
    bary = (0.5 + 3.0 * -0.2) / 4.0
    assert np.max(np.abs(g.vel[0] - bary)) < 1e-9 and np.max(np.abs(d.vel[0] - bary)) < 1e-9


def _random_mixture(dim, n, seed, **kw):
    rng = np.random.default_rng(seed)
    nside = int(round(n ** (1.0 / dim)))
    if dim == 1:
        prob = I.dusty_shock(n=n, t_stop=1e-3, seed=seed)
    else:
        prob = I.dusty_wave(n_side=nside, dim=dim, amp=1e-2, h_over_dx=1.0, cells_per_axis=nside // 2,
                            kvec=[2 * np.pi] * dim)
        for ph in (prob.gas, prob.dust):
            ph.x = np.mod(ph.x + rng.uniform(-0.2, 0.2, ph.x.shape) / nside, 1.0)
            ph.v = ph.v + rng.normal(0.0, 0.05, ph.v.shape)
            ph.m = ph.m * rng.uniform(0.5, 1.5, ph.m.shape)
    prob.params = prob.params.replace(**kw)
    return prob


@pytest.mark.parametrize("scheme", [MK, ISPH])
@pytest.mark.parametrize("dim", [1, 2])
def test_drag_free_limit_is_the_idic_drag_free_step(orc, scheme, dim):
    """With no drag (t_stop -> infinity) MK and ISPH are SPH gas plus free-streaming dust, like
    IDIC in the same limit: the three give the same state (they share the SPH sums)."""
    prob = _random_mixture(dim, 400, 5, t_stop=1e300, g=(0.2, -0.1, 0.0))
    ref = prob.copy()
    ref.params = ref.params.replace(scheme=IDIC)
    prob.params = prob.params.replace(scheme=scheme)
    g, d = orc.from_problem(prob)
    g0, d0 = orc.from_problem(ref)
    orc.step(prob.params, g, d, 3)
    orc.step(ref.params, g0, d0, 3)
    for a, b in ((g, g0), (d, d0)):
        a, b = a.by_id(), b.by_id()
        assert np.max(np.abs(a.vel - b.vel)) < 1e-14 and np.array_equal(a.cell, b.cell)
        assert np.max(np.abs(a.off - b.off)) < 1e-16


# ---------------------------------------------------------------------------
# MK
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("dim", [1, 2, 3])
def test_mk_conserves_total_momentum(orc, dim):
    """Section 2.1: the drag a gas particle loses is what the dust gains, pair by pair, and the
    pressure sum is antisymmetric: total momentum changes only by tau g (M_g + M_d)."""
    n = {1: 800, 2: 900, 3: 1000}[dim]
    prob = _random_mixture(dim, n, 11, t_stop=2e-3, scheme=MK, g=(0.3, -0.2, 0.1))
    p = prob.params
    g, d = orc.from_problem(prob)
    def mom():
        return g.vel @ g.mass + d.vel @ d.mass
    m0 = mom()
    orc.step(p, g, d, 1)
    gv = np.asarray(p.g[:dim]) * p.dt * (g.mass.sum() + d.mass.sum())
    scale = np.abs(g.vel).max() * g.mass.sum() + np.abs(d.vel).max() * d.mass.sum()
    assert np.max(np.abs(mom() - m0 - gv)) < 1e-13 * scale


@pytest.mark.parametrize("dim", [1, 2])
def test_mk_uniform_relaxation_is_the_continuum_drag(orc, dim):
    """A uniform mixture with the dust lattice staggered half a spacing from the gas: one MK
    step multiplies v - u by 1 - tau K (1/rho_g + 1/rho_d) S, where S is the kernel average of
    sigma r r / (r^2 + eta^2).  With sigma = dim, S = 1 minus at most eta^2 / r_min^2 (1D,
    where the lattice sum of W is exactly one) and within 1 % of 1 in 2D; a missing sigma
    would give S = 1/2 in 2D."""
    n = 64 if dim == 1 else 32
    h_over_dx = 2.0 if dim == 1 else 1.0
    prob = I.dusty_wave(n_side=n, dim=dim, amp=0.0, eps=1.0, h_over_dx=h_over_dx,
                        cells_per_axis=n // 2, kvec=[2 * np.pi] * dim)
    dx = 1.0 / n
    prob.dust.x = np.mod(prob.dust.x + 0.5 * dx, 1.0)
    prob.gas.v[:] = 0.2 / np.sqrt(dim)
    prob.dust.v[:] = -0.1 / np.sqrt(dim)
    K = 300.0
    prob.params = prob.params.replace(scheme=MK, K=K)
    p = prob.params
    g, d = orc.from_problem(prob)
    orc.step(p, g, d, 1)
    rel = (g.vel[0].mean() - d.vel[0].mean()) / (0.3 / np.sqrt(dim))
    S = (1.0 - rel) / (p.dt * K * 2.0)
    eta2 = 0.001 * p.h ** 2
    r_min = 0.5 * dx * np.sqrt(dim)
    if dim == 1:
        assert 1.0 - eta2 / r_min ** 2 <= S <= 1.0, S
    else:
        assert abs(S - 1.0) < 0.01, S
    assert np.std(g.vel[0]) < 1e-12 and np.std(d.vel[0]) < 1e-12


# ---------------------------------------------------------------------------
# both: the mild-drag dusty wave converges (h < c_s t_stop, the regime the paper says they need)
# ---------------------------------------------------------------------------

def test_isph_mild_drag_wave_converges(orc):
    """h < c_s t_stop, the regime where the paper says the fully Lagrangian schemes work: the
    ISPH error against the linear solution falls under refinement (h / dx fixed)."""
    scheme = ISPH
    errs = []
    for n in (100, 200, 400):
        prob = I.dusty_wave(n_side=n, dim=1, amp=1e-4, t_stop=0.05, h_over_dx=2.0, cells_per_axis=n // 2)
        prob.params = prob.params.replace(scheme=scheme, dt=0.1 * prob.params.h)
        prob.steps = int(round(0.3 / prob.params.dt))
        x, u = PT.run_oracle(orc, prob)
        from oracle.analytic import dusty_wave_linear
        ref = dusty_wave_linear(prob.extra, 0.05, prob.steps * prob.params.dt, x)
        errs.append(np.sqrt(np.mean((u - ref[3]) ** 2)) / 1e-4)
    assert errs[0] < 0.05 and errs[1] < 0.7 * errs[0] and errs[2] < 0.7 * errs[1], errs


def test_mk_co_located_pair_carries_no_drag(orc):
    """The pair term of eq. (8) is along r_ja, so a dust particle sitting on a gas particle
    exerts no drag on it: with both phases on one 1D lattice (h = 2 dx) the uniform-mixture
    relaxation loses the r = 0 term of the kernel average, W(0) dx = 1/3, and S = 2/3 up to the
    eta^2 clipping of the other pairs (at most eta^2 / dx^2 = 0.004)."""
    n = 64
    prob = I.dusty_wave(n_side=n, dim=1, amp=0.0, eps=1.0, h_over_dx=2.0, cells_per_axis=n // 2)
    prob.gas.v[:] = 0.2
    prob.dust.v[:] = -0.1
    K = 300.0
    prob.params = prob.params.replace(scheme=MK, K=K)
    p = prob.params
    g, d = orc.from_problem(prob)
    orc.step(p, g, d, 1)
    S = (1.0 - (g.vel[0].mean() - d.vel[0].mean()) / 0.3) / (p.dt * K * 2.0)
    assert (2.0 / 3.0) * (1 - 0.004) <= S <= 2.0 / 3.0, S
