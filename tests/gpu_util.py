"""Helpers shared by the GPU tests: read the device state back and compare
with the FP64 oracle under the stated tolerances."""
import numpy as np
import pytest

try:
    import torch
    HAVE_GPU = torch.cuda.is_available()
except Exception:       # pragma: no cover
    HAVE_GPU = False

needs_gpu = pytest.mark.skipif(not HAVE_GPU, reason="no HIP device")


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)


def oracle_phase(orc, dev: dict, dim):
    """Promote a device phase (numpy dict from DevicePhase.numpy()) to an FP64 oracle phase."""
    n = dev["cell"].shape[0]
    return orc.OPhase(cell=dev["cell"].astype(np.int32).copy(),
                      off=np.ascontiguousarray(dev["off"].astype(np.float64).reshape(dim, n)),
                      vel=np.ascontiguousarray(dev["vel"].astype(np.float64).reshape(dim, n)),
                      mass=np.ascontiguousarray(dev["mass"].astype(np.float64)),
                      id=dev["id"].astype(np.int32).copy(),
                      rho=np.zeros(n),
                      energy=None if dev["energy"] is None else dev["energy"].astype(np.float64).copy())


def by_id(dev: dict):
    o = np.argsort(dev["id"], kind="stable")
    out = {}
    for k, v in dev.items():
        if v is None:
            out[k] = None
        elif v.ndim == 2:
            out[k] = v[:, o]
        else:
            out[k] = v[o]
    return out


def position_error(p, cell_a, off_a, cell_b, off_b):
    """Max over particles and axes of |x_a - x_b| (periodic), in units of the cell width."""
    dim = p.dim
    D = np.array([(p.hi[k] - p.lo[k]) / p.n_cells[k] for k in range(3)])
    nc = p.n_cells

    def split(c):
        c = c.astype(np.int64)
        cs = [c % nc[0]]
        if dim > 1:
            cs.append((c // nc[0]) % nc[1])
        if dim > 2:
            cs.append(c // (nc[0] * nc[1]))
        return cs

    ca, cb = split(cell_a), split(cell_b)
    worst = 0.0
    for k in range(dim):
        dc = ca[k] - cb[k]
        dc = (dc + nc[k] // 2) % nc[k] - nc[k] // 2
        dx = dc * D[k] + (off_a[k].astype(np.float64) - off_b[k])
        worst = max(worst, float(np.max(np.abs(dx)) / D[k]) if dx.size else 0.0)
    return worst


def compare_states(p, gpu_g, gpu_d, orc_g, orc_d, c_s):
    """Normalised max errors (A21 reading): velocities by max(c_s, max|v|), density by
    max rho, positions by the cell width.  All inputs matched by id."""
    G, D = by_id(gpu_g), by_id(gpu_d)
    og, od = orc_g.by_id(), orc_d.by_id()
    assert np.array_equal(G["id"], og.id) and np.array_equal(D["id"], od.id)
    sv = max(c_s, float(np.max(np.abs(og.vel))) if og.vel.size else 0.0,
             float(np.max(np.abs(od.vel))) if od.vel.size else 0.0)
    err = {}
    err["v_gas"] = float(np.max(np.abs(G["vel"] - og.vel))) / sv if og.n else 0.0
    err["v_dust"] = float(np.max(np.abs(D["vel"] - od.vel))) / sv if od.n else 0.0
    err["x_gas"] = position_error(p, G["cell"], G["off"], og.cell, og.off) if og.n else 0.0
    err["x_dust"] = position_error(p, D["cell"], D["off"], od.cell, od.off) if od.n else 0.0
    if og.n:
        err["rho_gas"] = float(np.max(np.abs(G["rho"] - og.rho))) / float(np.max(og.rho))
    if G.get("energy") is not None and og.energy is not None:
        err["e_gas"] = float(np.max(np.abs(G["energy"] - og.energy))) / float(np.max(np.abs(og.energy)))
    return err
