"""Host-side figures bench.py prices the kernels with, checked by brute force on small inputs."""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
from paper_1908_01682_amd import inputs as I  # noqa: E402


def _cells(prob):
    p = prob.params
    d = p.dim
    lo, hi = np.array(p.lo[:d]), np.array(p.hi[:d])
    nc = np.array(p.n_cells[:d])
    delta = (hi - lo) / nc
    c = np.minimum(np.floor(np.mod(prob.gas.x - lo, hi - lo) / delta).astype(int), nc - 1)
    win = np.ceil(2.0 * p.h / delta - 1e-12).astype(int)
    return c, nc, win


@pytest.mark.parametrize("make", [
    lambda: I.dusty_box(n_side=12, cells_per_axis=6, regions_per_axis=1),
    lambda: I.wave_2d(n_side=20, amp=1e-2),
    lambda: I.dusty_shock(n=400),
])
def test_window_candidates_brute_force(make):
    prob = make()
    c, nc, win = _cells(prob)
    d = (c[None, :, :] - c[:, None, :]) % nc                # wrapped cell offset of every pair
    d = np.where(d > nc // 2, d - nc, d)
    total = int(np.all(np.abs(d) <= win, axis=-1).sum())
    assert bench.window_candidates(prob) == total


@pytest.mark.parametrize("make", [
    lambda: I.dusty_box(n_side=10, cells_per_axis=5, regions_per_axis=1),
    lambda: I.wave_2d(n_side=24, amp=1e-2),
])
def test_support_pairs_brute_force(make):
    prob = make()
    p = prob.params
    d = p.dim
    L = np.array(p.hi[:d]) - np.array(p.lo[:d])
    x = prob.gas.x
    r = x[:, None, :] - x[None, :, :]
    r -= L * np.round(r / L)
    dist = np.sqrt((r ** 2).sum(-1))
    # lattice pairs at exactly 2h (where W = 0) are not counted: the cut sits 1e-12 below 2h
    assert bench.support_pairs(prob) == int((dist < 2.0 * p.h * (1.0 - 1e-12)).sum())


@pytest.mark.parametrize("make", [
    lambda: I.dusty_box(n_side=10, cells_per_axis=5, regions_per_axis=1),
    lambda: I.wave_2d(n_side=24, amp=1e-2),
    lambda: I.dusty_shock(n=400),
])
def test_cross_phase_counts_brute_force(make):
    """Gas-dust candidates and pairs (the comparison schemes' pair kernels): every gas particle
    against every dust particle, in both directions."""
    prob = make()
    p = prob.params
    d = p.dim
    lo, hi = np.array(p.lo[:d]), np.array(p.hi[:d])
    L = hi - lo
    nc = np.array(p.n_cells[:d])
    delta = L / nc
    win = np.ceil(2.0 * p.h / delta - 1e-12).astype(int)
    cell = lambda x: np.minimum(np.floor(np.mod(x - lo, L) / delta).astype(int), nc - 1)
    cg, cd = cell(prob.gas.x), cell(prob.dust.x)
    off = (cd[None, :, :] - cg[:, None, :]) % nc
    off = np.where(off > nc // 2, off - nc, off)
    cand = int(np.all(np.abs(off) <= win, axis=-1).sum())
    r = prob.gas.x[:, None, :] - prob.dust.x[None, :, :]
    r -= L * np.round(r / L)
    pairs = int((np.sqrt((r ** 2).sum(-1)) < 2.0 * p.h * (1.0 - 1e-12)).sum())
    assert bench.window_candidates(prob, "gas", "dust") == cand == bench.window_candidates(prob, "dust", "gas")
    assert bench.support_pairs(prob, "gas", "dust") == pairs == bench.support_pairs(prob, "dust", "gas")


def test_step_bytes_counts_state_keys_density_and_cells():
    prob = I.dusty_box(n_side=8, cells_per_axis=4, regions_per_axis=1)
    g, s = prob.gas, prob.dust
    per_gas = 16 * 3 + 8 + 8 + (8 if g.uniform_mass() is None else 0)
    per_dust = 16 * 3 + 8 + (8 if s.uniform_mass() is None else 0)
    assert bench.step_bytes(prob) == g.n * per_gas + s.n * per_dust + 32 * 4 ** 3


def test_more_than_one_gpu_is_refused(capsys):
    """bench.py measures one GPU: --gpus above 1 exits with a message before touching a device."""
    assert bench.main(["--gpus", "2"]) == 2
    assert "one GPU only" in capsys.readouterr().err
