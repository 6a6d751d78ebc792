"""Thin Python binding of ``libtfsph.so`` (C ABI in ``include/tfsph.h``).

Only argument marshalling lives here: every step of the method runs in the
HIP kernels behind the C ABI.  PyTorch supplies device memory (tensors) and
the HIP stream (``torch.cuda.current_stream()``).  If the compiled library is
missing, every entry point raises -- there is no fallback path.

Low-level functions carry the C names (``tfsph_init``, ``tfsph_step``, ...);
``Simulation`` bundles a state, its workspace and a context.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtfsph.so")

TFSPH_OK = 0
TFSPH_F32, TFSPH_F64 = 0, 1
TFSPH_FLAG_NONFINITE = 1
TFSPH_FLAG_EMPTY_PHASE_CELL = 2
TFSPH_FLAG_BAD_CELL = 4
TFSPH_FLAG_CELL_OVERFLOW = 8
TFSPH_FLAG_CFL = 16
TFSPH_SCHEME_IDIC, TFSPH_SCHEME_IMEX2, TFSPH_SCHEME_MK, TFSPH_SCHEME_ISPH = 0, 1, 2, 3

STATUS = {0: "TFSPH_OK", -1: "TFSPH_E_INVALID_ARG", -2: "TFSPH_E_WORKSPACE", -3: "TFSPH_E_HIP",
          -4: "TFSPH_E_UNSUPPORTED", -5: "TFSPH_E_STATE"}


class TfsphError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        super().__init__(f"{where}: {STATUS.get(status, status)}: {detail}")
        self.status = status


class Params(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int32), ("n_cells", ctypes.c_int32 * 3), ("box_lo", ctypes.c_double * 3),
                ("box_hi", ctypes.c_double * 3), ("h", ctypes.c_double), ("eos", ctypes.c_int32),
                ("c_s", ctypes.c_double), ("gamma", ctypes.c_double), ("t_stop", ctypes.c_double),
                ("g", ctypes.c_double * 3), ("dt", ctypes.c_double), ("av_alpha", ctypes.c_double),
                ("av_beta", ctypes.c_double), ("precision", ctypes.c_int32), ("K", ctypes.c_double),
                ("t_stop_epstein", ctypes.c_double), ("scheme", ctypes.c_int32), ("cfl", ctypes.c_double)]


class PhaseC(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("cell", ctypes.c_void_p), ("off", ctypes.c_void_p * 3),
                ("vel", ctypes.c_void_p * 3), ("mass", ctypes.c_void_p), ("mass_uniform", ctypes.c_double),
                ("rho", ctypes.c_void_p), ("energy", ctypes.c_void_p), ("id", ctypes.c_void_p)]


class StateC(ctypes.Structure):
    _fields_ = [("gas", PhaseC), ("dust", PhaseC)]


class BatchDesc(ctypes.Structure):
    _fields_ = [("n_inst", ctypes.c_int32), ("params", ctypes.POINTER(Params)),
                ("gas_offset", ctypes.POINTER(ctypes.c_int64)), ("dust_offset", ctypes.POINTER(ctypes.c_int64)),
                ("mass_gas", ctypes.POINTER(ctypes.c_double)), ("mass_dust", ctypes.POINTER(ctypes.c_double))]


class BatchTuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("form", ctypes.c_int32), ("cells_per_block", ctypes.c_int32)]


TFSPH_BATCH_PERSISTENT, TFSPH_BATCH_FLAT = 0, 1


_lib = None


def lib():
    """Load the compiled library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1908_01682_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        vp, P = ctypes.c_void_p, ctypes.POINTER(Params)
        L.tfsph_status_string.restype = ctypes.c_char_p
        L.tfsph_status_string.argtypes = [ctypes.c_int]
        L.tfsph_last_error.restype = ctypes.c_char_p
        L.tfsph_validate.argtypes = [P]
        L.tfsph_workspace_size.argtypes = [P, ctypes.c_int64, ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
        L.tfsph_init.argtypes = [ctypes.POINTER(vp), P, ctypes.POINTER(StateC), vp, ctypes.c_size_t, vp]
        L.tfsph_step.argtypes = [vp, ctypes.POINTER(StateC), ctypes.c_int32, vp]
        L.tfsph_density.argtypes = [vp, ctypes.POINTER(StateC), ctypes.c_int32, vp]
        L.tfsph_get_flags.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_int64)]
        L.tfsph_signal_speed.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
        L.tfsph_cfl_dt.argtypes = [P, ctypes.c_double, ctypes.POINTER(ctypes.c_double)]
        L.tfsph_step_noalloc.argtypes = [P, ctypes.POINTER(StateC), ctypes.c_int32, vp, vp, vp]
        L.tfsph_destroy.argtypes = [vp]
        L.tfsph_positions_to_cells.argtypes = [P, ctypes.c_int64, vp, vp, ctypes.c_void_p * 3, vp]
        L.tfsph_cells_to_positions.argtypes = [P, ctypes.c_int64, vp, ctypes.c_void_p * 3, vp, vp]
        L.tfsph_profile.argtypes = [vp, ctypes.c_int32]
        L.tfsph_profile_sampled.argtypes = [vp, ctypes.c_int32]
        L.tfsph_set_kernel_variant.argtypes = [vp, ctypes.c_int32]
        L.tfsph_set_cells_per_block.argtypes = [vp, ctypes.c_int32]
        L.tfsph_profile_read.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(ctypes.c_double),
                                         ctypes.POINTER(ctypes.c_int64)]
        L.tfsph_step_graph.argtypes = [vp, ctypes.POINTER(StateC), ctypes.c_int32, ctypes.c_int32, vp]
        BD, BT, ST = ctypes.POINTER(BatchDesc), ctypes.POINTER(BatchTuning), ctypes.POINTER(StateC)
        L.tfsph_batch_workspace_size.argtypes = [BD, ctypes.POINTER(ctypes.c_size_t)]
        L.tfsph_batch_init.argtypes = [ctypes.POINTER(vp), BD, ST, BT, vp, ctypes.c_size_t, vp]
        L.tfsph_batch_set_tuning.argtypes = [vp, BT]
        L.tfsph_step_batched.argtypes = [vp, ST, ctypes.c_int32, vp]
        L.tfsph_step_batched_graph.argtypes = [vp, ST, ctypes.c_int32, vp]
        L.tfsph_batch_get_flags.argtypes = [vp, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_int64)]
        L.tfsph_batch_destroy.argtypes = [vp]
        L.tfsph_adjoint_workspace_size.argtypes = [P, ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                                   ctypes.POINTER(ctypes.c_size_t)]
        L.tfsph_step_adjoint.argtypes = [P, ST, ctypes.c_int32, ctypes.c_int32, vp, ctypes.c_void_p * 3,
                                         ctypes.c_void_p * 3, vp, vp, vp, ctypes.c_size_t, vp]
        for name in ("tfsph_validate", "tfsph_workspace_size", "tfsph_init", "tfsph_step", "tfsph_density",
                     "tfsph_get_flags", "tfsph_signal_speed", "tfsph_cfl_dt", "tfsph_step_noalloc", "tfsph_destroy", "tfsph_positions_to_cells", "tfsph_cells_to_positions",
                     "tfsph_profile", "tfsph_profile_sampled", "tfsph_profile_read", "tfsph_set_kernel_variant", "tfsph_set_cells_per_block", "tfsph_step_graph", "tfsph_batch_workspace_size",
                     "tfsph_batch_init", "tfsph_batch_set_tuning", "tfsph_step_batched", "tfsph_step_batched_graph",
                     "tfsph_batch_get_flags", "tfsph_batch_destroy", "tfsph_adjoint_workspace_size",
                     "tfsph_step_adjoint"):
            getattr(L, name).restype = ctypes.c_int
        _lib = L
    return _lib


def _check(status: int, where: str):
    if status != TFSPH_OK:
        raise TfsphError(status, where, lib().tfsph_last_error().decode())


def _stream_handle(stream=None) -> int:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _ptr(t) -> Optional[int]:
    return None if t is None else int(t.data_ptr())


# ----------------------------------------------------------------------------
# C-named entry points
# ----------------------------------------------------------------------------

def make_params(p, precision: int = TFSPH_F32) -> Params:
    """``p``: an ``inputs.Params``-like object."""
    c = Params()
    c.dim = int(p.dim)
    for k in range(3):
        c.n_cells[k] = int(p.n_cells[k]) if k < p.dim else 1
        c.box_lo[k] = float(p.lo[k])
        c.box_hi[k] = float(p.hi[k])
        c.g[k] = float(p.g[k])
    c.h, c.eos, c.c_s, c.gamma = float(p.h), int(p.eos), float(p.c_s), float(p.gamma)
    c.t_stop, c.dt = float(p.t_stop), float(p.dt)
    c.av_alpha, c.av_beta = float(p.av_alpha), float(p.av_beta)
    c.precision = int(precision)
    c.K = float(getattr(p, "K", 0.0))
    c.t_stop_epstein = float(getattr(p, "t_stop_epstein", 0.0))
    c.scheme = int(getattr(p, "scheme", TFSPH_SCHEME_IDIC))
    c.cfl = float(getattr(p, "cfl", 0.0))
    return c


def tfsph_validate(params: Params) -> None:
    _check(lib().tfsph_validate(ctypes.byref(params)), "tfsph_validate")


def tfsph_workspace_size(params: Params, n_gas: int, n_dust: int) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().tfsph_workspace_size(ctypes.byref(params), int(n_gas), int(n_dust), ctypes.byref(out)),
           "tfsph_workspace_size")
    return int(out.value)


def tfsph_init(params: Params, state: StateC, workspace, ws_bytes: int, stream=None) -> ctypes.c_void_p:
    ctx = ctypes.c_void_p()
    _check(lib().tfsph_init(ctypes.byref(ctx), ctypes.byref(params), ctypes.byref(state), _ptr(workspace),
                            int(ws_bytes), _stream_handle(stream)), "tfsph_init")
    return ctx


def tfsph_step(ctx, state: StateC, n_steps: int, stream=None) -> None:
    _check(lib().tfsph_step(ctx, ctypes.byref(state), int(n_steps), _stream_handle(stream)), "tfsph_step")


def tfsph_step_graph(ctx, state: StateC, n_steps: int, chunk: int, stream=None) -> None:
    _check(lib().tfsph_step_graph(ctx, ctypes.byref(state), int(n_steps), int(chunk), _stream_handle(stream)),
           "tfsph_step_graph")


def tfsph_density(ctx, state: StateC, phase: int, stream=None) -> None:
    _check(lib().tfsph_density(ctx, ctypes.byref(state), int(phase), _stream_handle(stream)), "tfsph_density")


def tfsph_get_flags(ctx):
    f = ctypes.c_uint32(0)
    n = ctypes.c_int64(0)
    _check(lib().tfsph_get_flags(ctx, ctypes.byref(f), ctypes.byref(n)), "tfsph_get_flags")
    return int(f.value), int(n.value)


def tfsph_signal_speed(ctx) -> float:
    """Largest max(|v|, c) since the last call (eq. 4); synchronises."""
    out = ctypes.c_double(0.0)
    _check(lib().tfsph_signal_speed(ctx, ctypes.byref(out)), "tfsph_signal_speed")
    return float(out.value)


def tfsph_cfl_dt(params: Params, signal_speed: float) -> float:
    """Time step of the Courant bound of eq. (4) (host only)."""
    out = ctypes.c_double(0.0)
    _check(lib().tfsph_cfl_dt(ctypes.byref(params), float(signal_speed), ctypes.byref(out)), "tfsph_cfl_dt")
    return float(out.value)


def tfsph_step_noalloc(params: Params, state: StateC, n_steps: int, flags_out=None, one_phase_out=None,
                       stream=None) -> None:
    """tfsph_init + tfsph_step(n_steps) on the library's static workspace (no allocation);
    flags_out / one_phase_out: optional device tensors (uint32 / int64, one element)."""
    _check(lib().tfsph_step_noalloc(ctypes.byref(params), ctypes.byref(state), int(n_steps), _ptr(flags_out),
                                    _ptr(one_phase_out), _stream_handle(stream)), "tfsph_step_noalloc")


TFSPH_KERNEL_UPDATE, TFSPH_KERNEL_DENSITY, TFSPH_KERNEL_BIN, TFSPH_KERNEL_FORCE = 0, 1, 2, 3


TFSPH_VARIANT_AUTO, TFSPH_VARIANT_GLOBAL, TFSPH_VARIANT_LDS_BRICKS = 0, 1, 2


def tfsph_set_kernel_variant(ctx, variant: int) -> None:
    _check(lib().tfsph_set_kernel_variant(ctx, int(variant)), "tfsph_set_kernel_variant")


def tfsph_set_cells_per_block(ctx, cells: int) -> None:
    _check(lib().tfsph_set_cells_per_block(ctx, int(cells)), "tfsph_set_cells_per_block")


def tfsph_profile(ctx, enable, rotate: bool = False, every: int = 1) -> None:
    """Start (enable true) or stop kernel timing; with rotate, one kernel kind is timed in every
    `every`-th step, the kinds in turn."""
    if enable and rotate and every != 1:
        _check(lib().tfsph_profile_sampled(ctx, int(every)), "tfsph_profile_sampled")
        return
    mode = 0 if not enable else (2 if rotate else 1)
    _check(lib().tfsph_profile(ctx, mode), "tfsph_profile")


def tfsph_profile_read(ctx, kernel: int):
    """(total_ms, launches) of one kernel kind since profiling was enabled."""
    ms = ctypes.c_double(0.0)
    n = ctypes.c_int64(0)
    _check(lib().tfsph_profile_read(ctx, int(kernel), ctypes.byref(ms), ctypes.byref(n)), "tfsph_profile_read")
    return float(ms.value), int(n.value)


def tfsph_destroy(ctx) -> None:
    if ctx:
        _check(lib().tfsph_destroy(ctx), "tfsph_destroy")


def tfsph_positions_to_cells(params: Params, x, cell, off, stream=None) -> None:
    offs = (ctypes.c_void_p * 3)(*[_ptr(o) for o in off] + [None] * (3 - len(off)))
    n = int(cell.numel())
    _check(lib().tfsph_positions_to_cells(ctypes.byref(params), n, _ptr(x), _ptr(cell), offs,
                                          _stream_handle(stream)), "tfsph_positions_to_cells")


def tfsph_cells_to_positions(params: Params, cell, off, x, stream=None) -> None:
    offs = (ctypes.c_void_p * 3)(*[_ptr(o) for o in off] + [None] * (3 - len(off)))
    n = int(cell.numel())
    _check(lib().tfsph_cells_to_positions(ctypes.byref(params), n, _ptr(cell), offs, _ptr(x),
                                          _stream_handle(stream)), "tfsph_cells_to_positions")


# ----------------------------------------------------------------------------
# device state held in torch tensors
# ----------------------------------------------------------------------------

class DevicePhase:
    """SoA device arrays of one phase (torch tensors)."""

    def __init__(self, n, dim, dtype, device, mass_array: bool, energy: bool, rho: bool):
        import torch
        self.n, self.dim = n, dim
        self.cell = torch.zeros(n, dtype=torch.int32, device=device)
        self.off = [torch.zeros(n, dtype=dtype, device=device) for _ in range(dim)]
        self.vel = [torch.zeros(n, dtype=dtype, device=device) for _ in range(dim)]
        self.mass = torch.zeros(n, dtype=dtype, device=device) if mass_array else None
        self.mass_uniform = 0.0
        self.rho = torch.zeros(n, dtype=dtype, device=device) if rho else None
        self.energy = torch.zeros(n, dtype=dtype, device=device) if energy else None
        self.id = torch.zeros(n, dtype=torch.int32, device=device)

    def cstruct(self) -> PhaseC:
        c = PhaseC()
        c.n = self.n
        c.cell = _ptr(self.cell)
        for d in range(3):
            c.off[d] = _ptr(self.off[d]) if d < self.dim else None
            c.vel[d] = _ptr(self.vel[d]) if d < self.dim else None
        c.mass = _ptr(self.mass)
        c.mass_uniform = float(self.mass_uniform)
        c.rho = _ptr(self.rho)
        c.energy = _ptr(self.energy)
        c.id = _ptr(self.id)
        return c

    def numpy(self) -> dict:
        """Host copy: cell, off (dim, n), vel (dim, n), mass, rho, energy, id (current order)."""
        out = dict(cell=self.cell.cpu().numpy(), id=self.id.cpu().numpy(),
                   off=np.stack([o.cpu().numpy() for o in self.off]) if self.dim else None,
                   vel=np.stack([v.cpu().numpy() for v in self.vel]) if self.dim else None)
        out["mass"] = self.mass.cpu().numpy() if self.mass is not None else np.full(self.n, self.mass_uniform)
        out["rho"] = self.rho.cpu().numpy() if self.rho is not None else None
        out["energy"] = self.energy.cpu().numpy() if self.energy is not None else None
        return out

    def load(self, cell, off, vel, ids, mass=None, energy=None):
        """Copy host arrays (cell-relative form) into the device tensors."""
        import torch
        self.cell.copy_(torch.as_tensor(np.asarray(cell, dtype=np.int32)))
        self.id.copy_(torch.as_tensor(np.asarray(ids, dtype=np.int32)))
        for d in range(self.dim):
            self.off[d].copy_(torch.as_tensor(np.asarray(off[d])).to(self.off[d].dtype))
            self.vel[d].copy_(torch.as_tensor(np.asarray(vel[d])).to(self.vel[d].dtype))
        if mass is not None and self.mass is not None:
            self.mass.copy_(torch.as_tensor(np.asarray(mass)).to(self.mass.dtype))
        if energy is not None and self.energy is not None:
            self.energy.copy_(torch.as_tensor(np.asarray(energy)).to(self.energy.dtype))


def _torch_dtype(precision):
    import torch
    return torch.float64 if precision == TFSPH_F64 else torch.float32


class DeviceState:
    """Both phases of one problem in device arrays (torch tensors), in the cell-relative form
    of the C ABI, with the C structs pointing at them.  No workspace and no context."""

    def __init__(self, prob, precision: int = TFSPH_F32, device="cuda", stream=None, dust_rho: bool = True):
        import torch
        self.prob = prob
        self.precision = precision
        self.device = torch.device(device)
        self.stream = stream
        p = prob.params
        self.params = make_params(p, precision)
        tfsph_validate(self.params)
        dt = _torch_dtype(precision)
        self.dtype = dt
        g, d = prob.gas, prob.dust
        mg, md = g.uniform_mass(), d.uniform_mass()
        self.gas = DevicePhase(g.n, p.dim, dt, self.device, mg is None, g.e is not None, True)
        self.dust = DevicePhase(d.n, p.dim, dt, self.device, md is None, False, dust_rho)
        for ph, src, mu in ((self.gas, g, mg), (self.dust, d, md)):
            ph.mass_uniform = mu if mu is not None else 0.0
            self._upload(ph, src)
        self.state = StateC(self.gas.cstruct(), self.dust.cstruct())

    def _upload(self, ph: DevicePhase, src):
        import torch
        x = torch.as_tensor(np.ascontiguousarray(src.x.T), dtype=torch.float64).to(self.device)
        tfsph_positions_to_cells(self.params, x, ph.cell, ph.off, self.stream)
        for k in range(ph.dim):
            ph.vel[k].copy_(torch.as_tensor(src.v[:, k]).to(ph.vel[k].dtype))
        ph.id.copy_(torch.as_tensor(src.id.astype(np.int32)))
        if ph.mass is not None:
            ph.mass.copy_(torch.as_tensor(src.m).to(ph.mass.dtype))
        if ph.energy is not None:
            ph.energy.copy_(torch.as_tensor(src.e).to(ph.energy.dtype))


class Simulation(DeviceState):
    """A state + workspace + context for one problem on one GPU."""

    def __init__(self, prob, precision: int = TFSPH_F32, device="cuda", stream=None, dust_rho: bool = True):
        import torch
        super().__init__(prob, precision, device, stream, dust_rho)
        g, d = prob.gas, prob.dust
        self.ws_bytes = tfsph_workspace_size(self.params, g.n, d.n)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        base = self.workspace.data_ptr()
        self._ws_off = (-base) % 256
        self._ws = self.workspace[self._ws_off:]
        self.ctx = tfsph_init(self.params, self.state, self._ws, self.ws_bytes, stream)

    def step(self, n: int = 1) -> None:
        tfsph_step(self.ctx, self.state, n, self.stream)

    def density(self, phase: int) -> None:
        tfsph_density(self.ctx, self.state, phase, self.stream)

    def signal_speed(self) -> float:
        return tfsph_signal_speed(self.ctx)

    def flags(self):
        return tfsph_get_flags(self.ctx)

    def positions(self, phase: int = 0) -> np.ndarray:
        import torch
        ph = self.gas if phase == 0 else self.dust
        x = torch.empty(ph.dim * ph.n, dtype=torch.float64, device=self.device)
        tfsph_cells_to_positions(self.params, ph.cell, ph.off, x, self.stream)
        return x.view(ph.dim, ph.n).cpu().numpy().T

    def close(self):
        if getattr(self, "ctx", None):
            tfsph_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def step_graph(self, n: int, chunk: int = 16) -> None:
        tfsph_step_graph(self.ctx, self.state, n, chunk, self.stream)


# ----------------------------------------------------------------------------
# batched form
# ----------------------------------------------------------------------------

def tfsph_batch_workspace_size(desc: BatchDesc) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().tfsph_batch_workspace_size(ctypes.byref(desc), ctypes.byref(out)), "tfsph_batch_workspace_size")
    return int(out.value)


def tfsph_batch_init(desc: BatchDesc, state: StateC, tuning: Optional[BatchTuning], workspace, ws_bytes: int,
                     stream=None):
    b = ctypes.c_void_p()
    _check(lib().tfsph_batch_init(ctypes.byref(b), ctypes.byref(desc), ctypes.byref(state),
                                  ctypes.byref(tuning) if tuning is not None else None, _ptr(workspace),
                                  int(ws_bytes), _stream_handle(stream)), "tfsph_batch_init")
    return b


def tfsph_batch_set_tuning(b, tuning: BatchTuning) -> None:
    _check(lib().tfsph_batch_set_tuning(b, ctypes.byref(tuning)), "tfsph_batch_set_tuning")


def tfsph_step_batched(b, state: StateC, n_steps: int, stream=None) -> None:
    _check(lib().tfsph_step_batched(b, ctypes.byref(state), int(n_steps), _stream_handle(stream)),
           "tfsph_step_batched")


def tfsph_step_batched_graph(b, state: StateC, n_steps: int, stream=None) -> None:
    _check(lib().tfsph_step_batched_graph(b, ctypes.byref(state), int(n_steps), _stream_handle(stream)),
           "tfsph_step_batched_graph")


def tfsph_batch_get_flags(b):
    f = ctypes.c_uint32(0)
    n = ctypes.c_int64(0)
    _check(lib().tfsph_batch_get_flags(b, ctypes.byref(f), ctypes.byref(n)), "tfsph_batch_get_flags")
    return int(f.value), int(n.value)


def tfsph_batch_destroy(b) -> None:
    if b:
        _check(lib().tfsph_batch_destroy(b), "tfsph_batch_destroy")


class BatchedSimulation:
    """Many independent problems (same dim, isothermal) in packed device arrays,
    advanced together: one persistent launch per call (form TFSPH_BATCH_PERSISTENT) or
    six launches per step over every instance (TFSPH_BATCH_FLAT)."""

    def __init__(self, probs, precision: int = TFSPH_F32, device="cuda", block: int = 0, stream=None,
                 form: int = TFSPH_BATCH_PERSISTENT, cells_per_block: int = 0):
        import torch
        self.probs = list(probs)
        self.precision = precision
        self.device = torch.device(device)
        self.stream = stream
        dim = self.probs[0].params.dim
        dt = _torch_dtype(precision)
        ng = [p.gas.n for p in self.probs]
        nd = [p.dust.n for p in self.probs]
        self.goff = np.concatenate([[0], np.cumsum(ng)]).astype(np.int64)
        self.doff = np.concatenate([[0], np.cumsum(nd)]).astype(np.int64)
        self.gas = DevicePhase(int(self.goff[-1]), dim, dt, self.device, False, False, True)
        self.dust = DevicePhase(int(self.doff[-1]), dim, dt, self.device, False, False, True)
        n = len(self.probs)
        self._params = (Params * n)(*[make_params(p.params, precision) for p in self.probs])
        self._goff = (ctypes.c_int64 * (n + 1))(*self.goff.tolist())
        self._doff = (ctypes.c_int64 * (n + 1))(*self.doff.tolist())
        mg = [p.gas.uniform_mass() for p in self.probs]
        md = [p.dust.uniform_mass() for p in self.probs]
        if any(m is None for m in mg + md):
            raise ValueError("batched instances need a uniform mass per phase")
        self._mg = (ctypes.c_double * n)(*mg)
        self._md = (ctypes.c_double * n)(*md)
        self.desc = BatchDesc(n, self._params, self._goff, self._doff, self._mg, self._md)
        for i, p in enumerate(self.probs):
            for ph, src, o in ((self.gas, p.gas, self.goff), (self.dust, p.dust, self.doff)):
                a, b = int(o[i]), int(o[i + 1])
                if b == a:
                    continue
                x = torch.as_tensor(np.ascontiguousarray(src.x.T), dtype=torch.float64).to(self.device)
                tfsph_positions_to_cells(self._params[i], x, ph.cell[a:b], [t[a:b] for t in ph.off], stream)
                for k in range(dim):
                    ph.vel[k][a:b].copy_(torch.as_tensor(src.v[:, k]).to(dt))
                ph.id[a:b].copy_(torch.as_tensor(src.id.astype(np.int32)))
        self.state = StateC(self.gas.cstruct(), self.dust.cstruct())
        self.ws_bytes = tfsph_batch_workspace_size(self.desc)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:]
        self.block, self.form, self.cells_per_block = block, form, cells_per_block
        self.handle = tfsph_batch_init(self.desc, self.state, BatchTuning(block, form, cells_per_block), self._ws,
                                       self.ws_bytes, stream)

    def set_tuning(self, block: int, form: int = TFSPH_BATCH_PERSISTENT, cells_per_block: int = 0) -> None:
        """Launch shape: workgroup size of the persistent form, the form, and the cells per
        workgroup of the flattened form's update launch (0 = default).  Results do not change."""
        tfsph_batch_set_tuning(self.handle, BatchTuning(block, form, cells_per_block))
        self.block, self.form, self.cells_per_block = block, form, cells_per_block

    def set_block(self, block: int) -> None:
        self.set_tuning(block, TFSPH_BATCH_PERSISTENT)

    def step(self, n: int) -> None:
        tfsph_step_batched(self.handle, self.state, n, self.stream)

    def step_graph(self, n: int) -> None:
        tfsph_step_batched_graph(self.handle, self.state, n, self.stream)

    def flags(self):
        return tfsph_batch_get_flags(self.handle)

    def instance(self, i: int) -> tuple:
        """(gas, dust) numpy dicts of instance i (current order)."""
        out = []
        for ph, o in ((self.gas, self.goff), (self.dust, self.doff)):
            a, b = int(o[i]), int(o[i + 1])
            d = ph.numpy()
            out.append({k: (None if v is None else (v[..., a:b] if k in ("off", "vel") else v[a:b]))
                        for k, v in d.items()})
        return tuple(out)

    def close(self):
        if getattr(self, "handle", None):
            tfsph_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------
# adjoint
# ----------------------------------------------------------------------------

def tfsph_adjoint_workspace_size(params: Params, n_gas: int, n_dust: int, n_steps: int, ckpt_every: int) -> int:
    out = ctypes.c_size_t(0)
    _check(lib().tfsph_adjoint_workspace_size(ctypes.byref(params), int(n_gas), int(n_dust), int(n_steps),
                                              int(ckpt_every), ctypes.byref(out)), "tfsph_adjoint_workspace_size")
    return int(out.value)


def tfsph_step_adjoint(params: Params, state: StateC, n_steps: int, ckpt_every: int, target, dv0, du0, dlogt, loss,
                       workspace, ws_bytes: int, stream=None) -> None:
    g = (ctypes.c_void_p * 3)(*[_ptr(t) for t in dv0] + [None] * (3 - len(dv0)))
    d = (ctypes.c_void_p * 3)(*[_ptr(t) for t in du0] + [None] * (3 - len(du0)))
    _check(lib().tfsph_step_adjoint(ctypes.byref(params), ctypes.byref(state), int(n_steps), int(ckpt_every),
                                    _ptr(target), g, d, _ptr(dlogt), _ptr(loss), _ptr(workspace), int(ws_bytes),
                                    _stream_handle(stream)), "tfsph_step_adjoint")


class AdjointRunner:
    """Initial state of a problem on the device plus the adjoint workspace.

    ``run(target)`` returns (loss, dL/dlog t_stop, dL/dv0, dL/du0) with the
    velocity gradients as (n, dim) tensors indexed by particle id (with the
    drag coefficient K held constant the scalar is dL/dlog(1/K)).  The initial
    arrays stay in id order, so ``set_velocities`` takes (n, dim) by id.
    """

    def __init__(self, prob, n_steps: int, ckpt_every: int, precision: int = TFSPH_F32, device="cuda",
                 stream=None):
        import torch
        self.prob = prob
        self.n_steps, self.ckpt_every = int(n_steps), int(ckpt_every)
        self.precision = precision
        self.device = torch.device(device)
        self.stream = stream
        p = prob.params
        self.dim = p.dim
        self.params = make_params(p, precision)
        tfsph_validate(self.params)
        self.dtype = _torch_dtype(precision)
        g, d = prob.gas, prob.dust
        if not (np.array_equal(g.id, np.arange(g.n)) and np.array_equal(d.id, np.arange(d.n))):
            raise ValueError("AdjointRunner expects particles given in id order 0..n-1")
        mg, md = g.uniform_mass(), d.uniform_mass()
        self.gas = DevicePhase(g.n, p.dim, self.dtype, self.device, mg is None, False, True)
        self.dust = DevicePhase(d.n, p.dim, self.dtype, self.device, md is None, False, True)
        for ph, src, mu in ((self.gas, g, mg), (self.dust, d, md)):
            ph.mass_uniform = mu if mu is not None else 0.0
            x = torch.as_tensor(np.ascontiguousarray(src.x.T), dtype=torch.float64).to(self.device)
            tfsph_positions_to_cells(self.params, x, ph.cell, ph.off, stream)
            for k in range(ph.dim):
                ph.vel[k].copy_(torch.as_tensor(src.v[:, k]).to(self.dtype))
            ph.id.copy_(torch.as_tensor(src.id.astype(np.int32)))
            if ph.mass is not None:
                ph.mass.copy_(torch.as_tensor(src.m).to(self.dtype))
        self.state = StateC(self.gas.cstruct(), self.dust.cstruct())
        self.ws_bytes = tfsph_adjoint_workspace_size(self.params, g.n, d.n, self.n_steps, self.ckpt_every)
        self.workspace = torch.empty(self.ws_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self.workspace.data_ptr()) % 256
        self._ws = self.workspace[off:]
        self.dv0 = [torch.zeros(g.n, dtype=self.dtype, device=self.device) for _ in range(p.dim)]
        self.du0 = [torch.zeros(d.n, dtype=self.dtype, device=self.device) for _ in range(p.dim)]
        self.out = torch.zeros(2, dtype=torch.float64, device=self.device)

    def set_t_stop(self, t_stop: float) -> None:
        """Relaxation-time parameter: t_stop, or 1/K when the drag coefficient K is held
        constant (the scalar gradient of ``run`` is then dL/dlog(1/K)), or t_stop_epstein."""
        if self.params.K > 0:
            self.params.K = 1.0 / float(t_stop)
        elif self.params.t_stop_epstein > 0:
            self.params.t_stop_epstein = float(t_stop)
        else:
            self.params.t_stop = float(t_stop)

    def set_velocities(self, v0g=None, v0d=None) -> None:
        for ph, v in ((self.gas, v0g), (self.dust, v0d)):
            if v is None:
                continue
            for k in range(self.dim):
                ph.vel[k].copy_(v[:, k].to(self.dtype))

    def run(self, target):
        import torch
        t = torch.as_tensor(target).to(device=self.device, dtype=self.dtype).contiguous()
        tfsph_step_adjoint(self.params, self.state, self.n_steps, self.ckpt_every, t, self.dv0, self.du0,
                           self.out[1:2], self.out[0:1], self._ws, self.ws_bytes, self.stream)
        out = self.out.clone()
        return (out[0], out[1], torch.stack(self.dv0, dim=1).clone(), torch.stack(self.du0, dim=1).clone())


def _make_loss_function():
    import torch

    class TFSPHLoss(torch.autograd.Function):
        """loss = TFSPHLoss.apply(v0_gas, v0_dust, log_t_stop, runner, target).

        The forward call runs the C-ABI adjoint once (its forward sweep gives the
        loss, its reverse sweep the gradients); backward scales the stored
        gradients by the incoming scalar gradient."""

        @staticmethod
        def forward(ctx, v0g, v0d, log_tstop, runner, target):
            runner.set_velocities(v0g.detach(), v0d.detach())
            runner.set_t_stop(float(torch.exp(log_tstop.detach())))
            loss, dlogt, gv, gu = runner.run(target)
            ctx.save_for_backward(gv.to(v0g.dtype), gu.to(v0d.dtype), dlogt.to(log_tstop.dtype))
            return loss.to(log_tstop.dtype)

        @staticmethod
        def backward(ctx, gout):
            gv, gu, dlogt = ctx.saved_tensors
            return gout * gv, gout * gu, gout * dlogt, None, None

    return TFSPHLoss


_loss_fn = None


def tfsph_loss(v0g, v0d, log_tstop, runner: AdjointRunner, target):
    """Differentiable dust-density misfit of ``runner``'s problem (see TFSPHLoss)."""
    global _loss_fn
    if _loss_fn is None:
        _loss_fn = _make_loss_function()
    return _loss_fn.apply(v0g, v0d, log_tstop, runner, target)
