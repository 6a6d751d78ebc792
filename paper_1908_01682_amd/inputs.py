"""Seeded synthetic workloads for the two-fluid SPH step (gas + dust particles).

This module only *generates inputs*: particle positions, velocities, masses,
energies and ids, plus the run parameters.  It contains none of the method's
arithmetic (no kernel sums, no binning, no drag); both the HIP path and the
FP64 oracle read its output, so it is the only code the two sides share.

Every array is float64 / int32 numpy, positions are absolute (N, d) arrays in
the periodic box [lo, hi).  Random numbers come from numpy's PCG64
(``numpy.random.default_rng(seed)``).

Workloads (the paper's two test problems, Section 3, plus larger synthetic
stand-ins of the same structure):

* ``dusty_wave``   -- linear sound wave in an isothermal gas-dust mixture
  (the "Dustywave" problem), 1D or 2D, cell-centred lattice displaced so that
  density follows rho0 (1 + A sin k.x).
* ``dusty_shock``  -- Sod-type shock tube in a coupled mixture ("Dustyshock"),
  mirrored periodic tube on [-0.5, 0.5), jittered lattice with per-particle
  mass m = rho(x) dx.
* ``dusty_box``    -- 3D periodic box, jittered lattice, Gaussian random
  velocity field, dust-to-gas ratio log-uniform per region.
* ``batched_waves``-- many independent 1D dusty waves of uneven size.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

ISOTHERMAL = 0
ADIABATIC = 1


@dataclasses.dataclass
class Phase:
    """One particle species.  ``x`` and ``v`` are (N, d) float64."""
    x: np.ndarray
    v: np.ndarray
    m: np.ndarray               # (N,) per-particle mass
    id: np.ndarray              # (N,) int32
    e: Optional[np.ndarray] = None   # (N,) specific internal energy (gas, adiabatic only)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def copy(self) -> "Phase":
        return Phase(self.x.copy(), self.v.copy(), self.m.copy(), self.id.copy(),
                     None if self.e is None else self.e.copy())

    def uniform_mass(self) -> Optional[float]:
        """The common particle mass if every particle has the same mass."""
        if self.n and np.all(self.m == self.m[0]):
            return float(self.m[0])
        return None


@dataclasses.dataclass
class Params:
    """Run parameters; names follow the paper's symbols."""
    dim: int
    n_cells: tuple            # drag cells per axis (length 3, unused axes = 1)
    lo: tuple                 # box lower corner (length 3)
    hi: tuple                 # box upper corner (length 3)
    h: float                  # smoothing length
    c_s: float = 1.0          # sound speed (isothermal) / unused for adiabatic
    t_stop: float = 1e-3      # velocity relaxation time
    dt: float = 1e-3          # time step tau
    eos: int = ISOTHERMAL
    gamma: float = 1.4
    g: tuple = (0.0, 0.0, 0.0)
    av_alpha: float = 0.0
    av_beta: float = 0.0
    K: float = 0.0            # > 0: drag coefficient K = rho_d / t_stop of eq. (7) held constant
                              # (t_stop then varies per cell as rho*_d / K; t_stop above is unused)
    t_stop_epstein: float = 0.0   # > 0: t*_stop = t_stop_epstein / rho*_g per cell (Epstein drag with
                                  # fixed grain size and sound speed); t_stop and K unused
    scheme: int = 0           # 0: first-order IDIC step; 1: second-order IMEX step, ARS(2,2,2) with
                              # the drag in cell as its implicit part
    cfl: float = 0.0          # > 0: Courant number of eq. (4) checked after every step (flag only)

    def cell_width(self):
        return tuple((self.hi[k] - self.lo[k]) / self.n_cells[k] for k in range(3))

    def replace(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class Problem:
    name: str
    params: Params
    gas: Phase
    dust: Phase
    steps: int
    extra: dict = dataclasses.field(default_factory=dict)

    def copy(self) -> "Problem":
        return Problem(self.name, self.params, self.gas.copy(), self.dust.copy(), self.steps,
                       dict(self.extra))


def _pad3(t, fill):
    t = list(t)
    return tuple(t + [fill] * (3 - len(t)))


def _wrap(x, lo, hi):
    """Map coordinates into [lo, hi) (periodic box)."""
    L = hi - lo
    y = lo + np.mod(x - lo, L)
    y = np.where(y >= hi, y - L, y)
    return y


# ----------------------------------------------------------------------------
# Dusty wave (1D / 2D)
# ----------------------------------------------------------------------------

def _wave_lattice(n_side, dim, amp, kvec, rho0, seed_jitter=None):
    """Cell-centred lattice q = (i + 1/2) dx displaced along k by (A/|k|) cos(k.q).

    With equal masses this makes the density rho0 (1 + A sin k.x) to first order
    in A.  Returns positions (N, d) in [0, 1)^d and the unit wave vector.
    """
    dx = 1.0 / n_side
    idx = np.arange(n_side ** dim)
    q = (np.stack([(idx // n_side ** a) % n_side for a in range(dim)], axis=1) + 0.5) * dx
    k = np.asarray(kvec, dtype=np.float64)
    kn = float(np.linalg.norm(k))
    khat = k / kn
    phase = q @ k
    x = q + np.outer((amp / kn) * np.cos(phase), khat)
    x = _wrap(x, 0.0, 1.0)
    return x, q, khat, kn


def dusty_wave(n_side: int = 200, dim: int = 1, amp: float = 1e-4, rho_g0: float = 1.0,
               eps: float = 1.0, c_s: float = 1.0, t_stop: float = 1e-3, h_over_dx: float = 2.0,
               cells_per_axis: Optional[int] = None, cfl: float = 0.25, steps: int = 1000,
               kvec=None, name: str = "dusty_wave") -> Problem:
    """Isothermal dusty sound wave (the Dustywave problem of Section 3).

    Both phases sit on the same displaced lattice (n_side per axis), densities
    rho_g0 (1 + A sin k.x) and eps rho_g0 (1 + A sin k.x), both velocities
    A c_s sin(k.x) along k.  Periodic unit box.
    """
    if kvec is None:
        kvec = [2.0 * math.pi] + [0.0] * (dim - 1) if dim == 1 else [2.0 * math.pi] * dim
    x, q, khat, kn = _wave_lattice(n_side, dim, amp, kvec, rho_g0)
    n = x.shape[0]
    dx = 1.0 / n_side
    h = h_over_dx * dx
    vol = 1.0 / n
    k = np.asarray(kvec, dtype=np.float64)
    s = np.sin(x @ k)
    vel = np.outer(amp * c_s * s, khat)
    if cells_per_axis is None:
        cells_per_axis = int(round(1.0 / (2.0 * h))) if dim > 1 else int(round(1.0 / h))
    gas = Phase(x=x.copy(), v=vel.copy(), m=np.full(n, rho_g0 * vol), id=np.arange(n, dtype=np.int32))
    dust = Phase(x=x.copy(), v=vel.copy(), m=np.full(n, eps * rho_g0 * vol), id=np.arange(n, dtype=np.int32))
    dt = cfl * h / max(float(np.max(np.abs(vel))) if n else 0.0, c_s)
    params = Params(dim=dim, n_cells=_pad3([cells_per_axis] * dim, 1), lo=(0.0, 0.0, 0.0),
                    hi=(1.0, 1.0, 1.0), h=h, c_s=c_s, t_stop=t_stop, dt=dt)
    extra = dict(amp=amp, kvec=tuple(k.tolist()), rho_g0=rho_g0, rho_d0=eps * rho_g0, c_s=c_s, eps=eps)
    return Problem(name, params, gas, dust, steps, extra)


# ----------------------------------------------------------------------------
# Dusty shock (1D)
# ----------------------------------------------------------------------------

def dusty_shock(n: int = 100_000, t_stop: float = 1e-3, eps: float = 1.0, gamma: float = 1.4,
                rho_l: float = 1.0, p_l: float = 1.0, rho_r: float = 0.125, p_r: float = 0.1,
                jitter: float = 0.1, h_over_dx: float = 2.0, cfl: float = 0.25, steps: int = 2000,
                seed: int = 2, av_alpha: float = 1.0, av_beta: float = 2.0,
                cells: Optional[int] = None, K: float = 0.0) -> Problem:
    """Sod-type shock tube in a coupled gas-dust mixture (the Dustyshock problem).

    Mirrored periodic tube [-0.5, 0.5): left state for x < 0, right state for
    x >= 0, so there are jumps at 0 and at the periodic seam +-0.5.  Both
    phases use a uniform lattice with spacing dx = 1/n, jittered by
    U(-jitter, jitter) dx, and per-particle masses m = rho(x_lattice) dx
    (dust: eps * rho).  Gas is adiabatic with gamma; velocities start at zero.
    K > 0 holds the drag coefficient K = rho_d / t_stop fixed instead of t_stop
    (the paper's shock test: K = 500, so t_stop is 0.002 on the left and
    0.00025 on the right of the tube).
    """
    rng = np.random.default_rng(seed)
    dx = 1.0 / n
    q = -0.5 + (np.arange(n) + 0.5) * dx
    left = q < 0.0
    rho = np.where(left, rho_l, rho_r)
    p = np.where(left, p_l, p_r)
    xg = q + rng.uniform(-jitter, jitter, n) * dx
    xd = q + rng.uniform(-jitter, jitter, n) * dx
    xg = _wrap(xg, -0.5, 0.5)[:, None]
    xd = _wrap(xd, -0.5, 0.5)[:, None]
    e = p / ((gamma - 1.0) * rho)
    gas = Phase(x=xg, v=np.zeros((n, 1)), m=rho * dx, id=np.arange(n, dtype=np.int32), e=e)
    dust = Phase(x=xd, v=np.zeros((n, 1)), m=eps * rho * dx, id=np.arange(n, dtype=np.int32))
    h = h_over_dx * dx
    if cells is None:
        cells = int(round(1.0 / h))
    c_max = math.sqrt(gamma * p_l / rho_l)
    dt = cfl * h / c_max
    params = Params(dim=1, n_cells=(cells, 1, 1), lo=(-0.5, 0.0, 0.0), hi=(0.5, 1.0, 1.0), h=h,
                    c_s=c_max, t_stop=t_stop, dt=dt, eos=ADIABATIC, gamma=gamma,
                    av_alpha=av_alpha, av_beta=av_beta, K=K)
    extra = dict(rho_l=rho_l, p_l=p_l, rho_r=rho_r, p_r=p_r, eps=eps, gamma=gamma)
    name = f"dusty_shock_K{K:g}" if K > 0 else f"dusty_shock_tstop{t_stop:g}"
    return Problem(name, params, gas, dust, steps, extra)


# ----------------------------------------------------------------------------
# 3D dusty box
# ----------------------------------------------------------------------------

def _random_velocity_field(x, rng, n_modes=64, kmax=4, rms=0.1):
    """Sum of n_modes Fourier modes with integer k in [-kmax, kmax]^3 \\ {0}.

    Mode amplitudes are N(0, I_3), phases U[0, 2 pi); every component is then
    rescaled to the requested rms over the particles.
    """
    ks = np.array([(i, j, k) for i in range(-kmax, kmax + 1) for j in range(-kmax, kmax + 1)
                   for k in range(-kmax, kmax + 1) if (i, j, k) != (0, 0, 0)], dtype=np.float64)
    sel = rng.choice(len(ks), size=n_modes, replace=False)
    kv = ks[sel] * (2.0 * math.pi)
    amps = rng.standard_normal((n_modes, 3))
    phases = rng.uniform(0.0, 2.0 * math.pi, n_modes)
    v = np.zeros_like(x)
    chunk = 1 << 13   # small enough that the (chunk, n_modes) temporaries are reused, not re-faulted
    for s in range(0, x.shape[0], chunk):
        arg = x[s:s + chunk] @ kv.T + phases[None, :]
        v[s:s + chunk] = np.cos(arg) @ amps
    std = np.sqrt(np.mean(v * v, axis=0))
    std = np.where(std > 0, std, 1.0)
    return v * (rms / std)


def dusty_box(n_side: int = 128, cells_per_axis: int = 64, regions_per_axis: int = 8, t_stop: float = 1e-4,
              c_s: float = 1.0, sigma_v: float = 0.1, jitter: float = 0.1, cfl: float = 0.25,
              steps: int = 200, seed: int = 3, eps_range=(-2.0, 1.0)) -> Problem:
    """3D periodic dusty box: jittered lattice, random velocity field, per-region dust/gas ratio.

    h = dx = 1/n_side.  Gas and dust share the lattice (independent jitter);
    gas velocities use a field drawn with ``seed``, dust an independent field
    drawn with ``seed + 1``.  Dust mass is eps_r * m_g with eps_r = 10^U(eps_range)
    drawn per region (regions_per_axis^3 regions).
    """
    rng = np.random.default_rng(seed)
    dx = 1.0 / n_side
    ax = (np.arange(n_side) + 0.5) * dx
    zz, yy, xx = np.meshgrid(ax, ax, ax, indexing="ij")
    q = np.stack([xx.reshape(-1), yy.reshape(-1), zz.reshape(-1)], axis=1)
    n = q.shape[0]
    xg = _wrap(q + rng.uniform(-jitter, jitter, q.shape) * dx, 0.0, 1.0)
    xd = _wrap(q + rng.uniform(-jitter, jitter, q.shape) * dx, 0.0, 1.0)
    eps_r = 10.0 ** rng.uniform(eps_range[0], eps_range[1], regions_per_axis ** 3)
    vg = _random_velocity_field(xg, np.random.default_rng(seed), rms=sigma_v * c_s)
    vd = _random_velocity_field(xd, np.random.default_rng(seed + 1), rms=sigma_v * c_s)
    reg = np.minimum((q * regions_per_axis).astype(np.int64), regions_per_axis - 1)
    rid = reg[:, 0] + regions_per_axis * (reg[:, 1] + regions_per_axis * reg[:, 2])
    m_g = 1.0 / n
    gas = Phase(x=xg, v=vg, m=np.full(n, m_g), id=np.arange(n, dtype=np.int32))
    dust = Phase(x=xd, v=vd, m=m_g * eps_r[rid], id=np.arange(n, dtype=np.int32))
    h = dx
    vmax = max(float(np.max(np.abs(vg))), float(np.max(np.abs(vd))))
    dt = cfl * h / max(vmax, c_s)
    params = Params(dim=3, n_cells=(cells_per_axis,) * 3, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                    h=h, c_s=c_s, t_stop=t_stop, dt=dt)
    return Problem("dusty_box_3d", params, gas, dust, steps, dict(eps_r=eps_r))


# ----------------------------------------------------------------------------
# Batched 1D waves
# ----------------------------------------------------------------------------

def batched_waves(n_inst: int = 256, n_min: int = 500, n_max: int = 20000, steps: int = 500,
                  amp: float = 1e-4, cfl: float = 0.25, seed: int = 4,
                  tstop_range=(-5.0, -1.0), eps_range=(-2.0, 1.0)):
    """Many independent 1D dusty waves of uneven size.

    Per instance: N ~ U{n_min..n_max} particles per phase on [0, 1), h = 2/N,
    floor(N/2) drag cells, tau = cfl h / c_s, t_stop = 10^U(tstop_range),
    dust/gas ratio eps = 10^U(eps_range), rho_g0 = 1, amplitude ``amp``.
    Returns a list of Problems.
    """
    rng = np.random.default_rng(seed)
    ns = rng.integers(n_min, n_max + 1, n_inst)
    tst = 10.0 ** rng.uniform(tstop_range[0], tstop_range[1], n_inst)
    eps = 10.0 ** rng.uniform(eps_range[0], eps_range[1], n_inst)
    out = []
    for i in range(n_inst):
        n = int(ns[i])
        p = dusty_wave(n_side=n, dim=1, amp=amp, eps=float(eps[i]), t_stop=float(tst[i]),
                       h_over_dx=2.0, cells_per_axis=n // 2, cfl=cfl, steps=steps,
                       name=f"batched_wave_{i}")
        # tau = cfl h / c_s (the wave velocity amplitude is far below c_s)
        p.params = p.params.replace(dt=cfl * p.params.h / p.params.c_s)
        out.append(p)
    return out


# ----------------------------------------------------------------------------
# The paper's own comparison runs (Section 3, Tables 1 and 2)
# ----------------------------------------------------------------------------

def paper_dustywave(h: float = 0.01, dt: float = 0.00025, n: int = 600, K: float = 500.0, eps: float = 1.0,
                    amp: float = 1e-4, t_end: float = 0.5, scheme: int = 0) -> Problem:
    """The Dustywave runs of Table 1: N = 2 x 600 particles on [0, 1), K = 500 held constant
    (eq. 22, dust/gas ratio 1, so t_stop = 0.002), c_s = 1, the given h and tau, to t = 0.5.
    Drag cells are one particle spacing wide, so each holds one gas and one dust particle.
    The amplitude is not printed; 1e-4 keeps the wave linear."""
    prob = dusty_wave(n_side=n, dim=1, amp=amp, eps=eps, c_s=1.0, t_stop=eps / K, h_over_dx=h * n,
                      cells_per_axis=n, steps=int(round(t_end / dt)), name=f"paper_dustywave_h{h:g}")
    prob.params = prob.params.replace(dt=dt, K=K, scheme=scheme)
    return prob


def paper_dustyshock(h: float = 0.01, dt: float = 0.000025, n_left: int = 880, n_right: int = 110,
                     K: float = 500.0, eps: float = 1.0, gamma: float = 1.4, t_end: float = 0.2,
                     av_alpha: float = 1.0, av_beta: float = 2.0, scheme: int = 0) -> Problem:
    """The Dustyshock runs of Table 2: N = 2 x 990 = 2 x (880 + 110) particles of equal mass, so
    the spacing jumps 8:1 with the Sod densities 1 | 0.125 (pressures 1 | 0.1), on the mirrored
    periodic tube [-0.5, 0.5) (left state on [-0.5, 0)); gas and dust share the lattice; K = 500
    held constant (t_stop = 0.002 | 0.00025), the given h and tau, to t = 0.2.  Drag cells are
    one left-state spacing wide.  Adiabatic gas with Monaghan-Gingold viscosity."""
    rho_l, p_l, rho_r, p_r = 1.0, 1.0, 0.125, 0.1
    dxl, dxr = 0.5 / n_left, 0.5 / n_right
    x = np.concatenate([-0.5 + (np.arange(n_left) + 0.5) * dxl, (np.arange(n_right) + 0.5) * dxr])[:, None]
    n = x.shape[0]
    left = x[:, 0] < 0.0
    rho = np.where(left, rho_l, rho_r)
    pres = np.where(left, p_l, p_r)
    m = np.full(n, rho_l * dxl)
    e = pres / ((gamma - 1.0) * rho)
    ids = np.arange(n, dtype=np.int32)
    gas = Phase(x=x.copy(), v=np.zeros((n, 1)), m=m.copy(), id=ids.copy(), e=e)
    dust = Phase(x=x.copy(), v=np.zeros((n, 1)), m=eps * m, id=ids.copy())
    c_max = math.sqrt(gamma * p_l / rho_l)
    params = Params(dim=1, n_cells=(2 * n_left, 1, 1), lo=(-0.5, 0.0, 0.0), hi=(0.5, 1.0, 1.0), h=h,
                    c_s=c_max, t_stop=eps * rho_r / K, dt=dt, eos=ADIABATIC, gamma=gamma,
                    av_alpha=av_alpha, av_beta=av_beta, K=K, scheme=scheme)
    extra = dict(rho_l=rho_l, p_l=p_l, rho_r=rho_r, p_r=p_r, eps=eps, gamma=gamma)
    return Problem(f"paper_dustyshock_h{h:g}", params, gas, dust, int(round(t_end / dt)), extra)


# ----------------------------------------------------------------------------
# Named workloads
# ----------------------------------------------------------------------------

def wave_2d(n_side: int = 512, amp: float = 1e-2, t_stop: float = 1e-3, eps: float = 1.0,
            steps: int = 200) -> Problem:
    """2D periodic dusty wave, k = 2 pi (1, 1), h = dx, drag cells of width 2h."""
    p = dusty_wave(n_side=n_side, dim=2, amp=amp, eps=eps, t_stop=t_stop, h_over_dx=1.0,
                   cells_per_axis=n_side // 2, steps=steps, kvec=[2 * math.pi, 2 * math.pi],
                   name="dusty_wave_2d")
    p.params = p.params.replace(dt=0.25 * p.params.h / p.params.c_s)
    return p


def workload(name: str, **kw) -> Problem:
    """The five standard workloads by short name.

    wave1d   -- 1D dusty wave, 200 + 200 particles, 100 cells, t_stop 1e-3, 1000 steps (FP64 sized)
    shock1d  -- 1D dusty shock, 1e5 + 1e5 particles, 5e4 cells, 2000 steps
    box3d    -- 3D dusty box, 128^3 + 128^3 particles, 64^3 cells, t_stop 1e-4, 200 steps
    wave2d   -- 2D dusty wave, 512^2 + 512^2 particles, 256^2 cells, t_stop 1e-3, 200 steps
    """
    if name == "wave1d":
        return dusty_wave(n_side=200, dim=1, amp=1e-4, t_stop=1e-3, h_over_dx=2.0, cells_per_axis=100,
                          cfl=0.25, steps=1000, **kw)
    if name == "shock1d":
        return dusty_shock(**kw)
    if name == "box3d":
        return dusty_box(**kw)
    if name == "wave2d":
        return wave_2d(**kw)
    raise KeyError(name)
