"""Throughput of the IDIC two-fluid SPH step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload box3d|shock1d|wave2d]

Prints ONE JSON line: gas+dust particle-steps/s of whole IDIC steps
(bin -> density -> force + predictor + cell solve + update) with inputs
resident in HBM, the HBM roofline of the dominant kernel (its launches timed
with HIP events on the stream they run on), and the FP64 CPU oracle timed on
the host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "gas+dust particle-steps/s per GPU (% HBM roofline); adjoint/forward time ratio"

WORKLOADS = {
    "box3d": "3D periodic dusty box, 128^3 gas + 128^3 dust, 64^3 cells, t_stop 1e-4, FP32",
    "shock1d": "1D dusty shock, 1e5 gas + 1e5 dust, 5e4 cells, t_stop 1e-3, FP32",
    "wave2d": "2D periodic dusty wave, 512^2 gas + 512^2 dust, 256^2 cells, t_stop 1e-3, FP32",
}


def update_kernel_bytes(prob) -> float:
    """Algorithmic HBM bytes of one launch of the update kernel.

    Per particle it must read its position (dim x 4 B) and velocity (dim x 4 B)
    and write both back (16 dim B in total) and write its cell key (4 B);
    a gas particle also reads its density across the global density -> force
    dependency (4 B); a per-particle mass is read once (4 B).
    """
    d = prob.params.dim
    g, s = prob.gas, prob.dust
    gas_b = 16 * d + 4 + 4 + (4 if g.uniform_mass() is None else 0) + (8 if g.e is not None else 0)
    dust_b = 16 * d + 4 + (4 if s.uniform_mass() is None else 0)
    return float(g.n * gas_b + s.n * dust_b)


def measured_traffic(workload: str):
    """HBM bytes per launch of k_update from the committed FETCH_SIZE / WRITE_SIZE summary,
    or None when the kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"k_update_{workload}_hbm_counters.md")
    if not os.path.exists(path):
        return None
    h = hashlib.sha1()
    for f in ("common.hpp", "sph.hpp", "binning.hpp", "enqueue.hpp"):
        with open(os.path.join(ROOT, "paper_1908_01682_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    rec = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.split(":")[0] in ("kernel_source_sha1", "traffic_bytes_per_launch"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    if rec.get("kernel_source_sha1") != h.hexdigest()[:16]:
        return None
    return float(rec["traffic_bytes_per_launch"])


def adjoint_ratio(I, T, torch, steps=200, ckpt=20):
    """Adjoint / forward time on the 2D dusty wave (512^2 + 512^2, 256^2 cells).

    Forward = n plain steps + the dust density of the misfit; adjoint = one
    tfsph_step_adjoint call (its own forward sweep with checkpoints, the
    replays and the reverse steps).  Target: the analytic initial dust profile.
    """
    prob = I.workload("wave2d", steps=steps)
    ex = prob.extra
    k = np.asarray(ex["kvec"])
    target = (ex["rho_d0"] * (1.0 + ex["amp"] * np.sin(prob.dust.x @ k))).astype(np.float32)
    sim = T.Simulation(prob, precision=T.TFSPH_F32)
    sim.step(2)
    sim.density(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    sim.density(1)
    torch.cuda.synchronize()
    fwd = time.perf_counter() - t0
    sim.close()
    runner = T.AdjointRunner(prob, steps, ckpt, precision=T.TFSPH_F32)
    runner.run(target)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss, dlogt, _, _ = runner.run(target)
    torch.cuda.synchronize()
    adj = time.perf_counter() - t0
    return {"ratio": adj / fwd, "forward_ms": 1e3 * fwd, "adjoint_ms": 1e3 * adj, "steps": steps,
            "ckpt_every": ckpt, "workload": WORKLOADS["wave2d"], "loss": float(loss), "dL_dlog_tstop": float(dlogt),
            "workspace_MiB": runner.ws_bytes / 2 ** 20}


def batched_throughput(I, T, torch, steps=500, plain_steps=20):
    """256 uneven 1D dusty waves in one persistent launch (autotuned, hipGraph replay),
    against the same instances through the plain path one at a time."""
    from paper_1908_01682_amd import autotune as A
    probs = I.batched_waves(steps=steps)
    n_part = sum(p.gas.n + p.dust.n for p in probs)
    bs = T.BatchedSimulation(probs, precision=T.TFSPH_F32)
    tune = A.tune(bs, steps=10)
    bs.step_graph(steps)           # capture + first replay
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bs.step_graph(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    flags, _ = bs.flags()
    bs.close()
    plain_t, plain_ps = 0.0, 0
    for p in probs:
        sim = T.Simulation(p, precision=T.TFSPH_F32)
        sim.step_graph(plain_steps, chunk=plain_steps)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step_graph(plain_steps, chunk=plain_steps)
        torch.cuda.synchronize()
        plain_t += time.perf_counter() - t0
        plain_ps += (p.gas.n + p.dust.n) * plain_steps
        sim.close()
    value = n_part * steps / wall
    plain = plain_ps / plain_t
    return {"value": value, "unit": "particle-steps/s", "ms_per_step": 1e3 * wall / steps, "steps": steps,
            "instances": len(probs), "particles": n_part, "block": tune["block"],
            "plain_path_value": plain, "vs_plain": value / plain, "nonfinite": bool(flags & 1)}


def cpu_baseline(prob, steps: int):
    from oracle import oracle as O
    O.build()
    g, d = O.from_problem(prob)
    t0 = time.perf_counter()
    O.step(prob.params, g, d, steps)
    dt = time.perf_counter() - t0
    n = prob.gas.n + prob.dust.n
    return {"value": n * steps / dt, "unit": "particle-steps/s", "cores": O.num_threads(), "kind": "oracle",
            "sample": f"{steps} steps of the full {prob.name} workload ({n} particles), FP64, "
                      f"{dt:.2f} s wall"}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="box3d", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-steps", type=int, default=4)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the adjoint and batched measurements")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy a 256 MiB device buffer 3 times (reference for HBM byte counters)")
    a = ap.parse_args(argv)
    if a.gpus != 1:
        print(f"bench.py measures one GPU only (asked for --gpus {a.gpus}); this build has no multi-GPU path.",
              file=sys.stderr)
        return 2
    import torch
    if not torch.cuda.is_available():
        print("no HIP device", file=sys.stderr)
        return 2
    from paper_1908_01682_amd import inputs as I
    from paper_1908_01682_amd import tfsph as T

    if a.copy_calibration:
        src = torch.ones(64 * 2 ** 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: 3 x {src.numel() * 4} bytes read and written", file=sys.stderr, flush=True)
    print(f"[bench] generating {a.workload}", file=sys.stderr, flush=True)
    prob = I.workload(a.workload)
    n_part = prob.gas.n + prob.dust.n
    sim = T.Simulation(prob, precision=T.TFSPH_F32)
    stream = torch.cuda.current_stream()
    sim.step(a.warmup)
    torch.cuda.synchronize()
    print(f"[bench] warmup done, timing {a.steps} steps", file=sys.stderr, flush=True)

    T.tfsph_profile(sim.ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(a.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    T.tfsph_profile(sim.ctx, False)
    upd_ms, upd_n = T.tfsph_profile_read(sim.ctx, T.TFSPH_KERNEL_UPDATE)
    den_ms, den_n = T.tfsph_profile_read(sim.ctx, T.TFSPH_KERNEL_DENSITY)
    bin_ms, bin_n = T.tfsph_profile_read(sim.ctx, T.TFSPH_KERNEL_BIN)
    flags, _ = sim.flags()
    sim.close()
    if flags & T.TFSPH_FLAG_NONFINITE:
        print("[bench] non-finite state", file=sys.stderr)
        return 1

    ms_per_step = 1e3 * wall / a.steps
    value = n_part * a.steps / wall
    upd_avg_s = upd_ms / max(upd_n, 1) * 1e-3
    alg = update_kernel_bytes(prob)
    achieved = alg / upd_avg_s / 1e9
    result = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOADS[a.workload], "particles": n_part,
                   "cells": int(np.prod(prob.params.n_cells[:prob.params.dim])), "dim": prob.params.dim},
        "roofline": {"bound": "hbm", "kernel": "k_update", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(a.workload),
                     "algorithmic_bytes_per_launch": alg, "avg_launch_ms": upd_avg_s * 1e3},
        "kernel_ms_per_step": {"update": upd_ms / max(upd_n, 1), "density": den_ms / max(den_n, 1),
                               "bin": bin_ms / max(bin_n, 1)},
        "adjoint_forward_ratio": None,
    }
    if not a.no_extras:
        print("[bench] adjoint / forward ratio (2D wave)", file=sys.stderr, flush=True)
        adj = adjoint_ratio(I, T, torch)
        result["adjoint_forward_ratio"] = adj["ratio"]
        result["adjoint"] = adj
        print("[bench] batched 1D waves", file=sys.stderr, flush=True)
        result["batched"] = batched_throughput(I, T, torch)
    if not a.no_cpu_baseline:
        print(f"[bench] oracle on host cores, {a.cpu_steps} steps", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(prob, a.cpu_steps)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
