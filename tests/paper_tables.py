"""The paper's comparison runs of Section 3 (Tables 1 and 2) for the tests: the printed
values, the problems, and the error measures.

* Table 1 (Dustywave): L2 = RMS over the dust particles of (u - u_exact) divided by the
  amplitude of u_exact at that time (sqrt(2) times its RMS on the lattice), u_exact the linear
  two-fluid solution at the particle positions.
* Table 2 (Dustyshock): L2 = RMS of (u - u_exact) over the dust particles with |x| < 0.25,
  u_exact the stiff-drag limit: the Riemann problem of one fluid of density (1 + eps) rho_g.
The paper defines neither norm; these reproduce its printed values (see the tests).
"""
import os

import numpy as np

from oracle.analytic import dusty_wave_linear, exact_riemann
from paper_1908_01682_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
SCHEMES = {"MK": 2, "ISPH": 3, "IDIC": 0}


def printed(name):
    """Rows (h, tau, {method: value}) of tests/golden/<name>.txt."""
    rows = []
    for line in open(os.path.join(HERE, "golden", name)):
        line = line.split("#")[0].split()
        if line:
            h, tau, mk, isph, idic = map(float, line)
            rows.append((h, tau, dict(MK=mk, ISPH=isph, IDIC=idic)))
    return rows


def stored_oracle_errors():
    """{(kind, h, tau, method): error} from tests/golden/tables_oracle.txt (written by
    tests/golden/make_tables_oracle.py from the oracle alone)."""
    out = {}
    for line in open(os.path.join(HERE, "golden", "tables_oracle.txt")):
        line = line.split("#")[0].split()
        if line:
            kind, h, tau, m, err = line
            out[(kind, float(h), float(tau), m)] = float(err)
    return out


def wave_problem(h, tau, method):
    return I.paper_dustywave(h=h, dt=tau, scheme=SCHEMES[method])


def shock_problem(h, tau, method):
    return I.paper_dustyshock(h=h, dt=tau, scheme=SCHEMES[method])


def wave_error(prob, x, u):
    """x: (n, 1) absolute dust positions, u: dust velocities, both by id, at t = steps * tau."""
    p = prob.params
    ref = dusty_wave_linear(prob.extra, prob.extra["rho_d0"] / p.K, prob.steps * p.dt, x)
    return float(np.sqrt(np.mean((u - ref[3]) ** 2) / (2.0 * np.mean(ref[3] ** 2))))


def shock_error(prob, x, u):
    p = prob.params
    ex = prob.extra
    t = prob.steps * p.dt
    x = np.asarray(x).reshape(-1)
    sel = np.abs(x) < 0.25
    e1 = 1.0 + ex["eps"]
    _, uref, _ = exact_riemann(e1 * ex["rho_l"], 0.0, ex["p_l"], e1 * ex["rho_r"], 0.0, ex["p_r"], ex["gamma"],
                               x[sel] / t)
    return float(np.sqrt(np.mean((u[sel] - uref) ** 2)))


def run_oracle(orc, prob):
    """Dust positions (n, dim) and the velocity along x, by id, after prob.steps steps."""
    g, d = orc.from_problem(prob)
    orc.step(prob.params, g, d, prob.steps)
    di = d.by_id()
    return orc.positions(prob.params, di), di.vel[0]
