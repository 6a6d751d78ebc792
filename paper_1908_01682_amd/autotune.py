"""Launch-shape autotuner for the batched persistent kernel.

For a batch signature (device name, dim, precision, instance count, size
distribution) it times every candidate workgroup size on the real batch,
checks that every candidate leaves a bitwise-identical state (the method's
sums are evaluated in a fixed order, so the launch shape must not change a
single bit), and caches the fastest in a JSON file.

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
         path: Optional[str] = None) -> dict:
    """Pick the fastest workgroup size for BatchedSimulation ``bs`` and apply it.

    Returns {"block": b, "ms_per_step": {...}, "bitwise_identical": True, "cached": bool}.
    The batch state is restored to its entry value before returning.
    """
    import torch
    dev = torch.cuda.get_device_name(bs.device)
    key = signature(dev, bs.probs, bs.precision)
    if use_cache:
        hit = load_cache(path).get(key)
        if hit and hit.get("block") in tuple(blocks):
            bs.set_block(int(hit["block"]))
            return dict(hit, cached=True)
    snap = _snapshot(bs)
    timings, digests = {}, {}
    for blk in blocks:
        _restore(bs, snap)
        bs.set_block(blk)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        bs.step(steps)
        torch.cuda.synchronize()
        timings[int(blk)] = 1e3 * (time.perf_counter() - t0) / steps
        digests[int(blk)] = _digest(bs)
    _restore(bs, snap)
    identical = len(set(digests.values())) == 1
    if not identical:
        raise RuntimeError(f"launch shapes disagree bitwise: {digests}")
    best = min(timings, key=timings.get)
    bs.set_block(best)
    entry = {"block": best, "ms_per_step": timings, "bitwise_identical": identical, "device": dev,
             "steps": steps}
    store(key, entry, path)
    return dict(entry, cached=False)
