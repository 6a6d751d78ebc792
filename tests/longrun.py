"""Long runs of the full-size workloads against stored oracle end states.

The FP32 device state of a workload is built here on the host, in numpy, from the
generator's absolute positions (cell = floor, then the carry rule in FP32 arithmetic, as
the binning defines it), so the oracle run that wrote the stored end state and the device
run start from the same bits.  The stored file holds a sample of the oracle's end state
(every ``STRIDE``-th particle id of each phase); the device run is compared on that sample.

Errors are reported as the relative L2 norm of each field over the sample: for velocities,
density and energy ``||q - q_ref|| / ||q_ref - mean(q_ref)||``; for positions the difference
is taken against the reference's displacement from the initial position
(``||x - x_ref|| / ||x_ref - x0||``, periodic), not against the box.
"""
from __future__ import annotations

import os

import numpy as np

from oracle import oracle as O
from paper_1908_01682_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")

# name -> (problem maker, steps, id stride of the stored sample)
RUNS = {
    "shock1d_ts1e-1": (lambda: I.dusty_shock(n=100_000, t_stop=1e-1), 2000, 32),
    "shock1d_ts1e-3": (lambda: I.dusty_shock(n=100_000, t_stop=1e-3), 2000, 32),
    "shock1d_ts1e-5": (lambda: I.dusty_shock(n=100_000, t_stop=1e-5), 2000, 32),
    "box3d": (lambda: I.dusty_box(), 200, 256),
}


def golden_path(name: str) -> str:
    return os.path.join(GOLDEN, f"longrun_{name}.npz")


def fp32_phase(p, ph):
    """FP32 (cell, offset) form of a generator phase: cell = floor((x - lo)/Delta) in FP64,
    offset rounded to FP32, then the carry rule in FP32 (an offset that rounds up to Delta
    moves to the next cell).  Returns a dict of host arrays (cell, off, vel, mass, id, energy)."""
    o64 = O.from_positions(p, ph.x, ph.v, ph.m, ph.id, ph.e)
    ref = O.bin_reference(p, o64.cell, o64.off.astype(np.float32), o64.id, np.float32)
    return dict(cell=ref["cell"].astype(np.int32), off=np.ascontiguousarray(ref["off"], dtype=np.float32),
                vel=np.ascontiguousarray(o64.vel, dtype=np.float32), mass=o64.mass.astype(np.float32),
                id=o64.id.astype(np.int32),
                energy=None if o64.energy is None else o64.energy.astype(np.float32))


def fp32_state(prob):
    p = prob.params
    return fp32_phase(p, prob.gas), fp32_phase(p, prob.dust)


def nudged(st) -> dict:
    """The same FP32 state with every offset moved one ulp toward zero (offsets stay in
    [0, Delta)): the smallest change of the state."""
    out = dict(st)
    out["off"] = np.nextafter(st["off"], np.float32(0)).astype(np.float32)
    return out


def to_oracle(st) -> "O.OPhase":
    """FP64 oracle phase holding exactly the FP32 values of ``st``."""
    n = st["cell"].shape[0]
    return O.OPhase(cell=st["cell"].copy(), off=np.ascontiguousarray(st["off"].astype(np.float64)),
                    vel=np.ascontiguousarray(st["vel"].astype(np.float64)),
                    mass=st["mass"].astype(np.float64), id=st["id"].copy(), rho=np.zeros(n),
                    energy=None if st["energy"] is None else st["energy"].astype(np.float64))


def absolute(p, cell, off):
    """Absolute FP64 positions (dim, n) of (cell, offset) arrays."""
    D = O.cell_width(p)
    lin = np.asarray(cell, dtype=np.int64)
    cs = [lin % p.n_cells[0], (lin // p.n_cells[0]) % p.n_cells[1], lin // (p.n_cells[0] * p.n_cells[1])]
    return np.stack([p.lo[k] + cs[k] * D[k] + np.asarray(off[k], dtype=np.float64) for k in range(p.dim)])


def sample(ph: dict, stride: int) -> dict:
    """Fields of the particles whose id is a multiple of ``stride``, ordered by id."""
    ids = np.asarray(ph["id"])
    sel = np.nonzero(ids % stride == 0)[0]
    sel = sel[np.argsort(ids[sel], kind="stable")]
    out = {}
    for k, v in ph.items():
        if v is None:
            continue
        v = np.asarray(v)
        out[k] = v[:, sel] if v.ndim == 2 else v[sel]
    return out


def field_errors(p, got_g: dict, got_d: dict, ref: dict, x0_g, x0_d) -> dict:
    """Relative L2 of every field (module docstring) of sampled device phases against the
    stored oracle sample ``ref`` (keys g_*, d_*); x0_* are the sampled initial positions."""
    L = np.array([p.hi[k] - p.lo[k] for k in range(p.dim)])[:, None]
    wrap = lambda d: d - L * np.round(d / L)

    def rel(a, b):
        den = np.linalg.norm(b - np.mean(b, axis=-1, keepdims=True))
        return float(np.linalg.norm(a - b) / max(den, 1e-300))

    err = {}
    for tag, got, x0 in (("gas", got_g, x0_g), ("dust", got_d, x0_d)):
        pre = tag[0] + "_"
        assert np.array_equal(got["id"], ref[pre + "id"]), tag
        x = absolute(p, got["cell"], got["off"])
        xr = absolute(p, ref[pre + "cell"], ref[pre + "off"])
        err[f"x_{tag}"] = float(np.linalg.norm(wrap(x - xr)) / max(np.linalg.norm(wrap(xr - x0)), 1e-300))
        err[f"v_{tag}"] = rel(got["vel"].astype(np.float64), ref[pre + "vel"])
    err["rho_gas"] = rel(got_g["rho"].astype(np.float64), ref["g_rho"])
    if "g_energy" in ref:
        err["e_gas"] = rel(got_g["energy"].astype(np.float64), ref["g_energy"])
    return err
