"""Host-only checks of the C ABI: symbols, parameter validation, workspace sizing.

No device call is made here, so these run on a machine without a GPU.
"""
import ctypes
import os
import re

import pytest

from paper_1908_01682_amd import inputs as I
from paper_1908_01682_amd import tfsph as T

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for hdr in os.listdir(os.path.join(ROOT, "include")):
        if not hdr.endswith(".h"):
            continue
        src = open(os.path.join(ROOT, "include", hdr)).read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        names |= set(re.findall(r"^[A-Za-z_][\w \*]*?\b(tfsph_\w+)\s*\(", src, flags=re.M))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(T.LIB_PATH):
        from paper_1908_01682_amd import build
        build.build(verbose=False)
    return T.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert len(names) >= 10, names
    for n in names:
        assert hasattr(lib, n), n


def test_no_cpu_fallback_symbols_or_torch_in_abi():
    src = open(os.path.join(ROOT, "include", "tfsph.h")).read()
    assert "torch" not in src.lower() and "at::" not in src


def _good(dim=1, precision=T.TFSPH_F32):
    prob = I.workload("wave1d") if dim == 1 else I.wave_2d(n_side=64)
    return T.make_params(prob.params, precision)


def _status(p):
    return T.lib().tfsph_validate(ctypes.byref(p))


def test_validate_accepts_workloads(lib):
    for prob in (I.workload("wave1d"), I.dusty_shock(n=2000), I.wave_2d(n_side=64),
                 I.dusty_box(n_side=16, cells_per_axis=8)):
        assert _status(T.make_params(prob.params)) == 0, T.lib().tfsph_last_error()


@pytest.mark.parametrize("field,value", [
    ("dim", 0), ("dim", 4), ("h", 0.0), ("h", float("nan")), ("t_stop", 0.0), ("t_stop", -1.0),
    ("dt", 0.0), ("dt", float("inf")), ("c_s", 0.0), ("eos", 7), ("precision", 3), ("av_alpha", -1.0),
])
def test_validate_rejects_bad_scalars(lib, field, value):
    p = _good()
    setattr(p, field, value)
    assert _status(p) == -1
    assert len(T.lib().tfsph_last_error()) > 0


def test_validate_rejects_bad_geometry(lib):
    p = _good()
    p.n_cells[1] = 2            # unused axis must be 1
    assert _status(p) == -1
    p = _good()
    p.box_hi[0] = p.box_lo[0]
    assert _status(p) == -1
    p = _good()
    p.n_cells[0], p.h = 4, 0.2  # 2h / Delta = 1.6: window of 2 cells needs >= 5 cells
    assert _status(p) == -1
    p.n_cells[0] = 5
    assert _status(p) == 0
    p = _good()
    p.h = 0.5                   # 2h spans 100 cells: window too large
    assert _status(p) == -1
    p = _good()
    p.eos, p.gamma = 1, 1.0
    assert _status(p) == -1


def test_workspace_size(lib):
    p = _good()
    a = T.tfsph_workspace_size(p, 200, 200)
    b = T.tfsph_workspace_size(p, 400, 400)
    assert 0 < a < b
    p64 = _good(precision=T.TFSPH_F64)
    assert T.tfsph_workspace_size(p64, 200, 200) > a
    assert T.tfsph_workspace_size(p, 0, 0) > 0
    with pytest.raises(T.TfsphError):
        T.tfsph_workspace_size(p, -1, 5)


def test_init_rejects_bad_arguments_before_any_device_work(lib):
    p = _good()
    st = T.StateC()
    st.gas.n = 10
    st.dust.n = 10
    ctx = ctypes.c_void_p()
    # NULL arrays
    r = T.lib().tfsph_init(ctypes.byref(ctx), ctypes.byref(p), ctypes.byref(st), None, 0, None)
    assert r == -1 and not ctx.value
    # NULL state
    r = T.lib().tfsph_init(ctypes.byref(ctx), ctypes.byref(p), None, None, 0, None)
    assert r == -1
    # NULL ctx pointer for step
    assert T.lib().tfsph_step(None, ctypes.byref(st), 1, None) == -1
    assert T.lib().tfsph_status_string(-2) == b"TFSPH_E_WORKSPACE"


def test_tuning_calls_reject_null_context(lib):
    """The tuning entry points validate on the host and never touch a device without a context."""
    L = T.lib()
    assert L.tfsph_set_kernel_variant(None, 0) == -1
    assert L.tfsph_set_cells_per_block(None, 32) == -1
    assert L.tfsph_profile(None, 1) == -1
    assert L.tfsph_profile_sampled(None, 4) == -1


def test_workspace_holds_neighbour_masks(lib):
    """AUTO keeps 8 bytes per gas particle and pair of opposite window rows for the neighbour
    masks: 9 rows, so 5 masks, in 3D with a one-cell window (h = dx, cells of 2h); 1000 more gas
    particles need at least 40 kB."""
    p = T.make_params(I.dusty_box(n_side=16, cells_per_axis=8).params)
    a = T.tfsph_workspace_size(p, 4096, 4096)
    b = T.tfsph_workspace_size(p, 5096, 4096)
    assert b - a >= 1000 * 8 * 5


def test_validate_drag_coefficient_mode(lib):
    """K > 0 holds the drag coefficient constant and leaves t_stop unused; K must be finite and
    non-negative, and with K = 0 t_stop must be positive."""
    p = _good()
    p.K, p.t_stop = 500.0, 0.0
    assert _status(p) == 0, T.lib().tfsph_last_error()
    for bad in (-1.0, float("nan"), float("inf")):
        p.K = bad
        assert _status(p) == -1
    p.K, p.t_stop = 0.0, 0.0
    assert _status(p) == -1
    p.t_stop_epstein = 2e-3                     # Epstein law: t_stop unused
    assert _status(p) == 0, T.lib().tfsph_last_error()
    p.K = 500.0                                 # two drag laws at once
    assert _status(p) == -1
    p.K, p.t_stop_epstein = 0.0, -1.0
    assert _status(p) == -1


def test_validate_scheme(lib):
    """scheme selects the first-order IDIC step (0), the second-order IMEX step (1), or one of
    the paper's comparison schemes, MK (2) and ISPH (3); anything else is rejected on the host."""
    p = _good()
    for ok in (T.TFSPH_SCHEME_IDIC, T.TFSPH_SCHEME_IMEX2, T.TFSPH_SCHEME_MK, T.TFSPH_SCHEME_ISPH):
        p.scheme = ok
        assert _status(p) == 0, T.lib().tfsph_last_error()
    for bad in (-1, 4, 7):
        p.scheme = bad
        assert _status(p) == -1


def test_imex_workspace_holds_the_stage_data(lib):
    """The IMEX step keeps, per gas particle, a second sorted copy with its level-n index, the
    stage predictor (cell, id, offsets, velocity) and the stage data (two accelerations, the
    stage-2 velocity and its drag increment): in FP32 3D at least 4 + 8 + 24 + 48 bytes more."""
    prob = I.dusty_box(n_side=16, cells_per_axis=8)
    p1 = T.make_params(prob.params)
    p2 = T.make_params(prob.params.replace(scheme=1))
    n = 4096
    a = T.tfsph_workspace_size(p1, n, n)
    b = T.tfsph_workspace_size(p2, n, n)
    assert b - a >= n * (4 + 8 + 24 + 48)


def test_validate_cfl(lib):
    """cfl = 0 turns the Courant check off; a positive finite value turns it on; negative or
    non-finite values are rejected on the host."""
    p = _good()
    for ok in (0.0, 0.25, 0.9):
        p.cfl = ok
        assert _status(p) == 0, T.lib().tfsph_last_error()
    for bad in (-0.1, float("nan"), float("inf")):
        p.cfl = bad
        assert _status(p) == -1


def test_cfl_dt_is_the_courant_bound(lib):
    """Eq. (4): tau = CFL h / max(v, c).  Isothermal: c_s is a floor of the signal speed;
    adiabatic: the signal speed is taken as given (it holds each gas particle's sound speed)."""
    p = _good()                                   # 1D wave, isothermal, c_s = 1, h = 0.01
    p.cfl = 0.25
    assert T.tfsph_cfl_dt(p, 0.0) == pytest.approx(0.25 * p.h / p.c_s, rel=1e-15)
    assert T.tfsph_cfl_dt(p, 0.5) == pytest.approx(0.25 * p.h / p.c_s, rel=1e-15)
    assert T.tfsph_cfl_dt(p, 4.0) == pytest.approx(0.25 * p.h / 4.0, rel=1e-15)
    # the wave generator computes its own tau the same way
    prob = I.workload("wave1d")
    q = T.make_params(prob.params)
    q.cfl = 0.25
    vmax = float(abs(prob.gas.v).max())
    assert T.tfsph_cfl_dt(q, vmax) == pytest.approx(prob.params.dt, rel=1e-15)
    a = T.make_params(I.dusty_shock(n=2000).params)
    a.cfl = 0.1
    assert T.tfsph_cfl_dt(a, 2.0) == pytest.approx(0.1 * a.h / 2.0, rel=1e-15)
    with pytest.raises(T.TfsphError):
        T.tfsph_cfl_dt(a, 0.0)                    # no floor for the adiabatic EOS: infinite bound
    for bad_speed in (-1.0, float("nan"), float("inf")):
        with pytest.raises(T.TfsphError):
            T.tfsph_cfl_dt(p, bad_speed)
    p.cfl = 0.0
    with pytest.raises(T.TfsphError):
        T.tfsph_cfl_dt(p, 1.0)
