"""Reference solutions the paper's test problems are measured against (Section 3) --
TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``.

* ``dusty_wave_linear``: the linearised isothermal two-fluid equations (1)-(3) for one Fourier
  mode, integrated exactly with a matrix exponential (the Dustywave problem's reference).
* ``exact_riemann``: the exact solution of the ideal-gas Riemann problem (textbook two-wave
  construction).  With the densities scaled by (1 + eps) it is the stiff-drag limit of the
  Dustyshock problem: gas and dust move as one fluid of density (1 + eps) rho_g carrying the
  gas pressure.
"""
import math

import numpy as np
from scipy.linalg import expm


def dusty_wave_linear(extra, t_stop, t, x):
    """Linearised two-fluid equations (1)-(3), isothermal: y' = M y for the Fourier
    amplitudes (rho_g, v, rho_d, u) of exp(i k.x); returns the four fields at x."""
    rg, rd, c, A = extra["rho_g0"], extra["rho_d0"], extra["c_s"], extra["amp"]
    kv = np.asarray(extra["kvec"])
    k = np.linalg.norm(kv)
    K = rd / t_stop
    M = np.array([[0, -1j * k * rg, 0, 0], [-1j * k * c * c / rg, -K / rg, 0, K / rg],
                  [0, 0, 0, -1j * k * rd], [0, K / rd, 0, -K / rd]], dtype=complex)
    y = expm(M * t) @ np.array([rg * A, A * c, rd * A, A * c], dtype=complex)
    ph = np.exp(1j * (np.atleast_2d(x) @ kv[: np.atleast_2d(x).shape[1]]))
    return [np.imag(y[i] * ph) for i in range(4)]


def exact_riemann(rl, ul, pl, rr, ur, pr, gamma, xi):
    """Exact solution of the ideal-gas Riemann problem sampled at xi = x / t (textbook
    two-wave construction with Newton iteration for the star pressure)."""
    g = gamma
    cl, cr = math.sqrt(g * pl / rl), math.sqrt(g * pr / rr)

    def fk(p, rk, pk, ck):
        if p > pk:
            A, B = 2 / ((g + 1) * rk), (g - 1) / (g + 1) * pk
            f = (p - pk) * math.sqrt(A / (p + B))
            df = math.sqrt(A / (B + p)) * (1 - (p - pk) / (2 * (B + p)))
        else:
            f = 2 * ck / (g - 1) * ((p / pk) ** ((g - 1) / (2 * g)) - 1)
            df = 1 / (rk * ck) * (p / pk) ** (-(g + 1) / (2 * g))
        return f, df

    p = 0.5 * (pl + pr)
    for _ in range(100):
        fl, dfl = fk(p, rl, pl, cl)
        fr, dfr = fk(p, rr, pr, cr)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        p = max(p - dp, 1e-12)
        if abs(dp) < 1e-14 * p:
            break
    fl, _ = fk(p, rl, pl, cl)
    fr, _ = fk(p, rr, pr, cr)
    us = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    rho = np.empty_like(xi)
    vel = np.empty_like(xi)
    prs = np.empty_like(xi)
    for i, s in enumerate(xi):
        if s < us:   # left of contact
            if p > pl:
                sl = ul - cl * math.sqrt((g + 1) / (2 * g) * p / pl + (g - 1) / (2 * g))
                if s < sl:
                    rho[i], vel[i], prs[i] = rl, ul, pl
                else:
                    rho[i] = rl * (p / pl + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * p / pl + 1)
                    vel[i], prs[i] = us, p
            else:
                cls = cl * (p / pl) ** ((g - 1) / (2 * g))
                if s < ul - cl:
                    rho[i], vel[i], prs[i] = rl, ul, pl
                elif s > us - cls:
                    rho[i], vel[i], prs[i] = rl * (p / pl) ** (1 / g), us, p
                else:
                    c = 2 / (g + 1) * (cl + (g - 1) / 2 * (ul - s))
                    vel[i] = 2 / (g + 1) * (cl + (g - 1) / 2 * ul + s)
                    rho[i] = rl * (c / cl) ** (2 / (g - 1))
                    prs[i] = pl * (c / cl) ** (2 * g / (g - 1))
        else:
            if p > pr:
                sr = ur + cr * math.sqrt((g + 1) / (2 * g) * p / pr + (g - 1) / (2 * g))
                if s > sr:
                    rho[i], vel[i], prs[i] = rr, ur, pr
                else:
                    rho[i] = rr * (p / pr + (g - 1) / (g + 1)) / ((g - 1) / (g + 1) * p / pr + 1)
                    vel[i], prs[i] = us, p
            else:
                crs = cr * (p / pr) ** ((g - 1) / (2 * g))
                if s > ur + cr:
                    rho[i], vel[i], prs[i] = rr, ur, pr
                elif s < us + crs:
                    rho[i], vel[i], prs[i] = rr * (p / pr) ** (1 / g), us, p
                else:
                    c = 2 / (g + 1) * (cr - (g - 1) / 2 * (ur - s))
                    vel[i] = 2 / (g + 1) * (-cr + (g - 1) / 2 * ur + s)
                    rho[i] = rr * (c / cr) ** (2 / (g - 1))
                    prs[i] = pr * (c / cr) ** (2 * g / (g - 1))
    return rho, vel, prs
