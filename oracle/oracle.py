"""Python access to the FP64 oracle (``tfsph_oracle.c``) -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the CPU-baseline leg of the
benchmark may import this module.  It shares no code with the HIP library:
the C oracle is compiled with gcc into ``oracle/_liboracle.so`` and driven
through ctypes here.

Besides the C step this module holds ``bin_reference``, the plain numpy
definition of the binning (cell carry rule, lexicographic (cell, id) order,
per-cell counts), evaluated in a caller-chosen precision so that integer
decisions are taken in the same precision as the kernel under test.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tfsph_oracle.c")
_LIB = os.path.join(_HERE, "_liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("nc", ctypes.c_int32 * 3), ("lo", ctypes.c_double * 3),
                ("hi", ctypes.c_double * 3), ("h", ctypes.c_double), ("eos", ctypes.c_int32),
                ("cs", ctypes.c_double), ("gamma", ctypes.c_double), ("tstop", ctypes.c_double),
                ("g", ctypes.c_double * 3), ("dt", ctypes.c_double), ("av_alpha", ctypes.c_double),
                ("av_beta", ctypes.c_double), ("K", ctypes.c_double), ("tse", ctypes.c_double)]


class _Phase(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("cell", ctypes.c_void_p), ("off", ctypes.c_void_p),
                ("vel", ctypes.c_void_p), ("mass", ctypes.c_void_p), ("rho", ctypes.c_void_p),
                ("energy", ctypes.c_void_p), ("id", ctypes.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P, PH = ctypes.POINTER(_Params), ctypes.POINTER(_Phase)
        L.orc_step.argtypes = [P, PH, PH, ctypes.c_int32, ctypes.c_void_p]
        L.orc_step.restype = ctypes.c_int64
        L.orc_step_imex.argtypes = [P, PH, PH, ctypes.c_int32]
        L.orc_step_imex.restype = ctypes.c_int64
        L.orc_step_mk.argtypes = [P, PH, PH, ctypes.c_int32]
        L.orc_step_mk.restype = None
        L.orc_step_isph.argtypes = [P, PH, PH, ctypes.c_int32]
        L.orc_step_isph.restype = ctypes.c_int64
        L.orc_phase_density.argtypes = [P, PH, ctypes.c_void_p]
        L.orc_phase_forces.argtypes = [P, PH, ctypes.c_void_p, ctypes.c_void_p]
        L.orc_canonicalize.argtypes = [P, PH]
        L.orc_sort.argtypes = [P, PH]
        L.orc_kernel_w.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.orc_kernel_w.restype = ctypes.c_double
        L.orc_kernel_dw.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.orc_kernel_dw.restype = ctypes.c_double
        L.orc_num_threads.restype = ctypes.c_int
        L.orc_set_num_threads.argtypes = [ctypes.c_int]
        _lib = L
    return _lib


def params_struct(p) -> _Params:
    """``p``: any object with the attributes of ``inputs.Params``."""
    s = _Params()
    s.dim = p.dim
    for k in range(3):
        s.nc[k] = int(p.n_cells[k])
        s.lo[k] = float(p.lo[k])
        s.hi[k] = float(p.hi[k])
        s.g[k] = float(p.g[k])
    s.h, s.eos, s.cs, s.gamma = float(p.h), int(p.eos), float(p.c_s), float(p.gamma)
    s.tstop, s.dt, s.av_alpha, s.av_beta = float(p.t_stop), float(p.dt), float(p.av_alpha), float(p.av_beta)
    s.K = float(getattr(p, "K", 0.0))
    s.tse = float(getattr(p, "t_stop_epstein", 0.0))
    return s


@dataclasses.dataclass
class OPhase:
    """FP64 oracle state of one phase in (cell, offset) form.  off/vel are (dim, n)."""
    cell: np.ndarray
    off: np.ndarray
    vel: np.ndarray
    mass: np.ndarray
    id: np.ndarray
    rho: np.ndarray
    energy: Optional[np.ndarray] = None

    @property
    def n(self):
        return int(self.cell.shape[0])

    def copy(self):
        return OPhase(self.cell.copy(), self.off.copy(), self.vel.copy(), self.mass.copy(), self.id.copy(),
                      self.rho.copy(), None if self.energy is None else self.energy.copy())

    def _struct(self):
        for a in ("cell", "off", "vel", "mass", "id", "rho"):
            arr = getattr(self, a)
            assert arr.flags.c_contiguous, a
        s = _Phase()
        s.n = self.n
        s.cell = self.cell.ctypes.data
        s.off = self.off.ctypes.data
        s.vel = self.vel.ctypes.data
        s.mass = self.mass.ctypes.data
        s.rho = self.rho.ctypes.data
        s.energy = self.energy.ctypes.data if self.energy is not None else None
        s.id = self.id.ctypes.data
        return s

    def by_id(self):
        """Arrays reordered by particle id."""
        o = np.argsort(self.id, kind="stable")
        return OPhase(self.cell[o], self.off[:, o], self.vel[:, o], self.mass[o], self.id[o], self.rho[o],
                      None if self.energy is None else self.energy[o])


def cell_width(p):
    return np.array([(p.hi[k] - p.lo[k]) / p.n_cells[k] for k in range(3)])


def from_positions(p, x, v, m, ids, e=None) -> OPhase:
    """Absolute FP64 positions (n, d) -> (cell, offset) with cell = floor((x - lo)/Delta)."""
    x = np.asarray(x, dtype=np.float64)
    n, d = x.shape
    D = cell_width(p)
    c = np.zeros((n, 3), dtype=np.int64)
    off = np.zeros((d, n))
    for k in range(d):
        rel = x[:, k] - p.lo[k]
        ck = np.floor(rel / D[k]).astype(np.int64)
        o = rel - ck * D[k]
        c[:, k] = ck
        off[k] = o
    lin = c[:, 0] % p.n_cells[0]
    if d > 1:
        lin = lin + p.n_cells[0] * (c[:, 1] % p.n_cells[1])
    if d > 2:
        lin = lin + p.n_cells[0] * p.n_cells[1] * (c[:, 2] % p.n_cells[2])
    # every array is a fresh copy: the oracle steps and sorts its state in place
    ph = OPhase(cell=lin.astype(np.int32), off=np.array(off, dtype=np.float64, order="C", copy=True),
                vel=np.array(np.asarray(v, dtype=np.float64).T.reshape(d, n), order="C", copy=True),
                mass=np.array(m, dtype=np.float64, order="C", copy=True),
                id=np.array(ids, dtype=np.int32, order="C", copy=True), rho=np.zeros(n),
                energy=None if e is None else np.array(e, dtype=np.float64, order="C", copy=True))
    lib().orc_canonicalize(ctypes.byref(params_struct(p)), ctypes.byref(ph._struct()))
    return ph


def from_problem(prob):
    g, d = prob.gas, prob.dust
    return (from_positions(prob.params, g.x, g.v, g.m, g.id, g.e),
            from_positions(prob.params, d.x, d.v, d.m, d.id, None))


def positions(p, ph: OPhase) -> np.ndarray:
    """Absolute positions (n, dim) of an oracle phase."""
    D = cell_width(p)
    dim = p.dim
    lin = ph.cell.astype(np.int64)
    cs = [lin % p.n_cells[0]]
    if dim > 1:
        cs.append((lin // p.n_cells[0]) % p.n_cells[1])
    if dim > 2:
        cs.append(lin // (p.n_cells[0] * p.n_cells[1]))
    return np.stack([p.lo[k] + cs[k] * D[k] + ph.off[k] for k in range(dim)], axis=1)


SCHEME_IDIC, SCHEME_IMEX2, SCHEME_MK, SCHEME_ISPH = 0, 1, 2, 3


def step(p, gas: OPhase, dust: OPhase, nsteps: int = 1, cell_diag: Optional[np.ndarray] = None) -> int:
    """Advance both phases ``nsteps`` steps in place.  ``p.scheme``:
    0: the first-order IDIC step (returns the one-phase-cell count summed over the drag solves);
    1: the second-order IMEX step (ARS(2,2,2) with the drag in cell as its implicit part; the same
       count over both solves; ``cell_diag`` is not filled);
    2: the explicit Monaghan-Kocharyan pairwise drag of Section 2.1 (returns 0);
    3: the semi-implicit ISPH drag of Section 2.2 (returns the number of particles with no particle
       of the other phase within 2h, summed over the steps).
    On exit the dust ``rho`` holds the dust summation density of the last step for schemes 2 and 3."""
    sg, sd = gas._struct(), dust._struct()
    scheme = getattr(p, "scheme", 0)
    if scheme != SCHEME_IDIC and cell_diag is not None:
        raise ValueError("cell_diag is only filled by the first-order IDIC step")
    if scheme == SCHEME_IMEX2:
        r = lib().orc_step_imex(ctypes.byref(params_struct(p)), ctypes.byref(sg), ctypes.byref(sd), int(nsteps))
        return int(r)
    if scheme == SCHEME_MK:
        lib().orc_step_mk(ctypes.byref(params_struct(p)), ctypes.byref(sg), ctypes.byref(sd), int(nsteps))
        return 0
    if scheme == SCHEME_ISPH:
        r = lib().orc_step_isph(ctypes.byref(params_struct(p)), ctypes.byref(sg), ctypes.byref(sd), int(nsteps))
        return int(r)
    ptr = cell_diag.ctypes.data if cell_diag is not None else None
    r = lib().orc_step(ctypes.byref(params_struct(p)), ctypes.byref(sg), ctypes.byref(sd), int(nsteps), ptr)
    return int(r)


def density(p, ph: OPhase) -> np.ndarray:
    """Summation density of a phase over itself (sorts the phase in place)."""
    out = np.zeros(ph.n)
    lib().orc_phase_density(ctypes.byref(params_struct(p)), ctypes.byref(ph._struct()), out.ctypes.data)
    return out


def gas_forces(p, gas: OPhase):
    """(A (dim, n), de/dt (n)) of the explicit gas terms; sorts the phase, fills rho."""
    acc = np.zeros((p.dim, gas.n))
    dedt = np.zeros(gas.n)
    lib().orc_phase_forces(ctypes.byref(params_struct(p)), ctypes.byref(gas._struct()), acc.ctypes.data,
                           dedt.ctypes.data if gas.energy is not None else None)
    return acc, dedt


def kernel_w(dim, h, r):
    return lib().orc_kernel_w(dim, h, r)


def kernel_dw(dim, h, r):
    return lib().orc_kernel_dw(dim, h, r)


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_num_threads(n: int) -> None:
    lib().orc_set_num_threads(int(n))


# ---------------------------------------------------------------------------
# Binning reference in a chosen precision (numpy)
# ---------------------------------------------------------------------------

def bin_reference(p, cell, off, ids, dtype=np.float32):
    """Plain definition of the binning step.

    Carry rule per axis in ``dtype`` arithmetic (while off < 0: off += Delta,
    c -= 1; then while off >= Delta: off -= Delta, c += 1; c wraps periodically),
    linear index cx + nx (cy + ny cz), permutation = lexsort by (cell, id),
    per-cell counts and exclusive offsets.

    ``off`` is (dim, n).  Returns dict(cell, off, perm, count, start).
    """
    dim = p.dim
    D = np.array([dtype((p.hi[k] - p.lo[k]) / p.n_cells[k]) for k in range(dim)], dtype=dtype)
    lin = np.asarray(cell, dtype=np.int64)
    c = [lin % p.n_cells[0]]
    if dim > 1:
        c.append((lin // p.n_cells[0]) % p.n_cells[1])
    if dim > 2:
        c.append(lin // (p.n_cells[0] * p.n_cells[1]))
    o = np.array(off, dtype=dtype, copy=True)
    for k in range(dim):
        ok = o[k]
        ck = c[k].copy()
        while True:
            m = ok < 0
            if not m.any():
                break
            ok[m] = (ok[m] + D[k]).astype(dtype)
            ck[m] -= 1
        while True:
            m = ok >= D[k]
            if not m.any():
                break
            ok[m] = (ok[m] - D[k]).astype(dtype)
            ck[m] += 1
        c[k] = np.mod(ck, p.n_cells[k])
        o[k] = ok
    new = c[0].copy()
    if dim > 1:
        new += p.n_cells[0] * c[1]
    if dim > 2:
        new += p.n_cells[0] * p.n_cells[1] * c[2]
    ncell = int(np.prod(p.n_cells[:dim]))
    perm = np.lexsort((np.asarray(ids), new))
    count = np.bincount(new, minlength=ncell)
    start = np.concatenate([[0], np.cumsum(count)[:-1]])
    return dict(cell=new.astype(np.int32), off=o, perm=perm, count=count.astype(np.int64),
                start=start.astype(np.int64))
