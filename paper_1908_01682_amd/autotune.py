"""Launch-shape autotuners.

Batched step (``tune``): the candidates are the persistent form (one workgroup per
instance) at several workgroup sizes and the flattened form (six launches per step over
every instance) at several cells per workgroup of its update launch.  For a batch signature (device name, dim, precision, instance count,
size distribution) it times every candidate on the real batch.

Plain step (``tune_plain``): the candidates are the cells owned by one block of the
update kernel (cell sums, 2x2 solve, particle update), for a problem signature (device
name, dim, precision, particle and cell counts).

Both check that every candidate leaves a bitwise-identical state (the method's sums are
evaluated in a fixed order, so the launch shape must not change a single bit) and cache
the fastest in a JSON file.

Cache path: $TFSPH_AUTOTUNE_CACHE, else ~/.cache/tfsph/autotune.json.
"""
from __future__ import annotations

import hashlib
import json
import os
import time
from typing import Iterable, Optional

import numpy as np

CANDIDATE_BLOCKS = (256, 512, 768, 1024)
CANDIDATE_CELLS_PER_BLOCK = (16, 32, 64, 128, 256)
CANDIDATE_FLAT_CELLS = (64, 128, 256)
PERSISTENT, FLAT = 0, 1


def cache_path() -> str:
    return os.environ.get("TFSPH_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "tfsph", "autotune.json"))


def signature(device_name: str, probs, precision: int) -> str:
    """Key of a batch: device, dim, precision, instance count and a coarse size histogram."""
    ns = np.array([p.gas.n + p.dust.n for p in probs], dtype=np.int64)
    hist = np.histogram(np.log2(np.maximum(ns, 1)), bins=8, range=(0, 32))[0]
    raw = json.dumps(dict(dev=device_name, dim=int(probs[0].params.dim), prec=int(precision), n=int(len(ns)),
                          hist=hist.tolist(), nmax=int(ns.max())), sort_keys=True)
    return hashlib.sha1(raw.encode()).hexdigest()[:16]


def load_cache(path: Optional[str] = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store(key: str, entry: dict, path: Optional[str] = None) -> None:
    path = path or cache_path()
    data = load_cache(path)
    data[key] = entry
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _snapshot(bs):
    return [t.clone() for ph in (bs.gas, bs.dust) for t in [ph.cell, ph.id] + ph.off + ph.vel]


def _restore(bs, snap):
    live = [t for ph in (bs.gas, bs.dust) for t in [ph.cell, ph.id] + ph.off + ph.vel]
    for dst, src in zip(live, snap):
        dst.copy_(src)


def _digest(bs) -> str:
    h = hashlib.sha1()
    for ph in (bs.gas, bs.dust):
        for t in [ph.cell, ph.id] + ph.off + ph.vel + ([ph.rho] if ph.rho is not None else []):
            h.update(t.cpu().numpy().tobytes())
    return h.hexdigest()


def tune(bs, steps: int = 20, blocks: Iterable[int] = CANDIDATE_BLOCKS, use_cache: bool = True,
         path: Optional[str] = None, flat: bool = True, graph: bool = False,
         flat_cells: Iterable[int] = CANDIDATE_FLAT_CELLS) -> dict:
    """Pick the fastest launch shape for BatchedSimulation ``bs`` and apply it: the persistent
    form at each workgroup size in ``blocks`` and, with ``flat``, the flattened form at each
    number of cells per update workgroup in ``flat_cells``.  With ``graph`` every candidate is
    timed as a replayed hipGraph of ``steps`` steps (captured before the timing), as the caller
    will run it.

    Returns {"form": f, "block": b, "cells_per_block": c, "ms_per_step": {...},
    "bitwise_identical": True, "cached": bool}; the timing keys are "persistent/<block>" and
    "flat/<cells>".  The batch state is restored to its entry value before returning.
    """
    import torch
    dev = torch.cuda.get_device_name(bs.device)
    key = signature(dev, bs.probs, bs.precision)
    cands = [(PERSISTENT, int(b), 0) for b in blocks] + ([(FLAT, 256, int(c)) for c in flat_cells] if flat else [])
    if use_cache:
        hit = load_cache(path).get(key)
        if hit and (int(hit.get("form", PERSISTENT)), int(hit.get("block", 0)),
                    int(hit.get("cells_per_block", 0))) in cands:
            bs.set_tuning(int(hit["block"]), int(hit.get("form", PERSISTENT)), int(hit.get("cells_per_block", 0)))
            return dict(hit, cached=True)
    snap = _snapshot(bs)
    timings, digests = {}, {}
    for form, blk, cpb in cands:
        name = f"flat/{cpb}" if form == FLAT else f"persistent/{blk}"
        _restore(bs, snap)
        bs.set_tuning(blk, form, cpb)
        run = bs.step_graph if graph else bs.step
        run(steps if graph else 1)  # capture, or load the code objects, outside the timing
        _restore(bs, snap)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        run(steps)
        torch.cuda.synchronize()
        timings[name] = 1e3 * (time.perf_counter() - t0) / steps
        digests[name] = _digest(bs)
    _restore(bs, snap)
    identical = len(set(digests.values())) == 1
    if not identical:
        raise RuntimeError(f"launch shapes disagree bitwise: {digests}")
    best = min(timings, key=timings.get)
    if best.startswith("flat/"):
        form, blk, cpb = FLAT, 256, int(best.split("/")[1])
    else:
        form, blk, cpb = PERSISTENT, int(best.split("/")[1]), 0
    bs.set_tuning(blk, form, cpb)
    entry = {"form": form, "block": blk, "cells_per_block": cpb, "ms_per_step": timings,
             "bitwise_identical": identical, "device": dev, "steps": steps}
    store(key, entry, path)
    return dict(entry, cached=False)


def plain_signature(device_name: str, sim) -> str:
    """Key of a single problem: device, dim, precision, particle and cell counts, scheme."""
    p = sim.prob.params
    raw = json.dumps(dict(dev=device_name, dim=int(p.dim), prec=int(sim.precision), ng=int(sim.gas.n),
                          nd=int(sim.dust.n), cells=[int(c) for c in p.n_cells[:p.dim]],
                          scheme=int(getattr(p, "scheme", 0)), kind="plain"), sort_keys=True)
    return hashlib.sha1(raw.encode()).hexdigest()[:16]


def _plain_tensors(sim):
    out = []
    for ph in (sim.gas, sim.dust):
        out += [ph.cell, ph.id] + list(ph.off) + list(ph.vel)
        out += [t for t in (ph.mass, ph.energy, ph.rho) if t is not None]
    return out


def tune_plain(sim, steps: int = 20, cells: Iterable[int] = CANDIDATE_CELLS_PER_BLOCK, use_cache: bool = True,
               path: Optional[str] = None) -> dict:
    """Pick the fastest cells-per-block of the update kernel for Simulation ``sim`` and apply it
    (``tfsph_set_cells_per_block``).  Every candidate runs ``steps`` steps from the same state and
    must leave it bitwise identical.  Returns {"cells_per_block": c, "ms_per_step": {c: ms},
    "bitwise_identical": True, "cached": bool}; the state is restored to its entry value."""
    import torch
    from . import tfsph as T
    dev = torch.cuda.get_device_name(sim.device)
    key = plain_signature(dev, sim)
    cands = [int(c) for c in cells]
    if use_cache:
        hit = load_cache(path).get(key)
        if hit and int(hit.get("cells_per_block", 0)) in cands:
            T.tfsph_set_cells_per_block(sim.ctx, int(hit["cells_per_block"]))
            return dict(hit, cached=True)
    live = _plain_tensors(sim)
    snap = [t.clone() for t in live]

    def restore():
        for dst, src in zip(live, snap):
            dst.copy_(src)

    timings, digests = {}, {}
    for c in cands:
        T.tfsph_set_cells_per_block(sim.ctx, c)
        restore()
        sim.step(1)                 # loads the code objects outside the timing
        restore()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        timings[str(c)] = 1e3 * (time.perf_counter() - t0) / steps
        h = hashlib.sha1()
        for t in live:
            h.update(t.cpu().numpy().tobytes())
        digests[str(c)] = h.hexdigest()
    restore()
    identical = len(set(digests.values())) == 1
    if not identical:
        raise RuntimeError(f"cells per block change the state: {digests}")
    best = int(min(timings, key=timings.get))
    T.tfsph_set_cells_per_block(sim.ctx, best)
    entry = {"cells_per_block": best, "ms_per_step": timings, "bitwise_identical": identical, "device": dev,
             "steps": steps}
    store(key, entry, path)
    return dict(entry, cached=False)
