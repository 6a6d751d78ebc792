"""Throughput of the IDIC two-fluid SPH step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload box3d|shock1d|wave2d]

Prints ONE JSON line: gas+dust particle-steps/s of whole IDIC steps
(bin -> density -> force + predictor -> cell solve + update) with inputs
resident in HBM; the roofline of the dominant kernel (its launches timed with
HIP events on the stream they run on, one kernel kind in every few steps, the
kinds in turn, inside the timed steps; the pair kernels are bound by vector
ALU work, priced in algorithmic flops against the FP32 vector peak, the update
kernel by HBM bytes); the whole step's algorithmic HBM bytes against the HBM
peak; and the FP64 CPU oracle timed on the host cores on a bounded sample of
the same workload.  Extras (skipped with --no-extras): the adjoint / forward
time ratio, the batched 1D waves, the second-order IMEX step, and the paper's
three drag schemes (IDIC, ISPH, MK) side by side on the same workload.
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
FP32_PEAK_TFLOPS = 157.3      # MI355X vector FP32 (packed); FP64 vector 78.6
FP64_PEAK_TFLOPS = 78.6
# FP32 vector without packed instructions, which the build disables: 256 CUs x 4 SIMDs x 16 lanes
# x 2 (FMA) x 2.4 GHz
FP32_NONPACKED_TFLOPS = 78.6
METRIC = "gas+dust particle-steps/s per GPU (% HBM roofline); adjoint/forward time ratio"

WORKLOADS = {
    "box3d": "3D periodic dusty box, 128^3 gas + 128^3 dust, 64^3 cells, t_stop 1e-4, FP32",
    "shock1d": "1D dusty shock, 1e5 gas + 1e5 dust, 5e4 cells, t_stop 1e-3, FP32",
    "wave2d": "2D periodic dusty wave, 512^2 gas + 512^2 dust, 256^2 cells, t_stop 1e-3, FP32",
}

# floating-point operations the method needs, per unit (see the roofline notes in bench output)
FLOPS_PER_CANDIDATE = 8       # r^2 of a window candidate: 3 sub + 3 mul + 2 add
FLOPS_PER_DENSITY_PAIR = 13   # q = sqrt(r^2)/h (2), f(q) (9), m f accumulated (2)
FLOPS_PER_FORCE_PAIR = 28     # r^2 (8), r and 1/r (2), q (1), f'(q) (7), m (P_a+P_b) f'/r (4), 3 fma (6)


def _cell_counts(prob, x):
    p = prob.params
    d = p.dim
    nc = np.array(p.n_cells[:d])
    lo, hi = np.array(p.lo[:d]), np.array(p.hi[:d])
    delta = (hi - lo) / nc
    cell = np.floor((np.mod(x - lo, hi - lo)) / delta).astype(np.int64)
    cell = np.minimum(cell, nc - 1)
    counts = np.zeros(tuple(nc), dtype=np.int64)
    np.add.at(counts, tuple(cell.T), 1)
    return counts, np.ceil(2.0 * p.h / delta - 1e-12).astype(int)


def window_candidates(prob, phase: str = "gas", other: str = "gas") -> int:
    """Sum over the particles of ``phase`` of the population of ``other`` in their
    neighbour-cell window (the candidates a cell-list search must test), from the initial
    cell counts."""
    import itertools
    d = prob.params.dim
    counts, win = _cell_counts(prob, getattr(prob, phase).x)
    others = counts if other == phase else _cell_counts(prob, getattr(prob, other).x)[0]
    wsum = np.zeros_like(others)
    for off in itertools.product(*[range(-w, w + 1) for w in win]):
        wsum += np.roll(others, shift=tuple(-o for o in off), axis=tuple(range(d)))
    return int((counts * wsum).sum())


def support_pairs(prob, phase: str = "gas", other: str = "gas") -> int:
    """Sum over the particles of ``phase`` of the particles of ``other`` within 2h (a particle
    counts itself when both are the same phase), periodic."""
    from scipy.spatial import cKDTree
    p = prob.params
    d = p.dim
    lo, hi = np.array(p.lo[:d]), np.array(p.hi[:d])
    x = np.mod(getattr(prob, phase).x - lo, hi - lo)
    y = x if other == phase else np.mod(getattr(prob, other).x - lo, hi - lo)
    tree = cKDTree(y, boxsize=hi - lo)
    n = tree.query_ball_point(x, r=2.0 * p.h * (1.0 - 1e-12), return_length=True, workers=-1)
    return int(np.sum(n))


def update_kernel_bytes(prob) -> float:
    """Algorithmic HBM bytes of one launch of the update kernel (cell sums, implicit solve,
    particle update): per particle it must read its position (dim x 4 B) and velocity
    (dim x 4 B) and write both back (16 dim B in total) and write its cell key (4 B); a gas
    particle also reads its density across the global density -> force dependency (4 B); a
    per-particle mass is read once (4 B)."""
    d = prob.params.dim
    g, s = prob.gas, prob.dust
    gas_b = 16 * d + 4 + 4 + (4 if g.uniform_mass() is None else 0) + (8 if g.e is not None else 0)
    dust_b = 16 * d + 4 + (4 if s.uniform_mass() is None else 0)
    return float(g.n * gas_b + s.n * dust_b)


def step_bytes(prob) -> float:
    """Algorithmic HBM bytes of one whole step: every particle reads and writes its state
    (16 dim B), writes and reads its cell key (8 B) and, when per-particle, its mass (8 B);
    gas writes and reads its density across the density -> force dependency (8 B) and its
    energy when adiabatic (8 B); per cell both phases write and read count and offset (32 B)."""
    p = prob.params
    d = p.dim
    g, s = prob.gas, prob.dust
    gas_b = 16 * d + 8 + 8 + (8 if g.uniform_mass() is None else 0) + (8 if g.e is not None else 0)
    dust_b = 16 * d + 8 + (8 if s.uniform_mass() is None else 0)
    return float(g.n * gas_b + s.n * dust_b + 32 * int(np.prod(p.n_cells[:d])))


COUNTER_SOURCES = ("common.hpp", "sph.hpp", "binning.hpp", "enqueue.hpp", "host.hpp")


def kernel_source_sha() -> str:
    import hashlib
    h = hashlib.sha1()
    for f in COUNTER_SOURCES:
        with open(os.path.join(ROOT, "paper_1908_01682_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_valu_share(workload: str):
    """Share of the chip's non-packed VALU issue slots each kernel used, from the committed
    SQ-counter summary, or None when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", f"pair_kernels_{workload}_valu_counters.md")
    if not os.path.exists(path):
        return None
    out, sha = {}, None
    with open(path) as fh:
        for line in fh:
            if line.startswith("kernel_source_sha1:"):
                sha = line.split(":", 1)[1].strip()
            cols = [c.strip() for c in line.strip().strip("|").split("|")]
            if len(cols) == 7 and cols[0].startswith("k_"):
                try:
                    out[cols[0]] = float(cols[6])
                except ValueError:
                    pass
    return out if sha == kernel_source_sha() and out else None


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of a kernel from the committed FETCH_SIZE / WRITE_SIZE summary,
    or None when the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_hbm_counters.md")
    if not os.path.exists(path):
        return None
    rec = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and line.split(":")[0] in ("kernel_source_sha1", "traffic_bytes_per_launch"):
                k, v = line.split(":", 1)
                rec[k.strip()] = v.strip()
    if rec.get("kernel_source_sha1") != kernel_source_sha() or "traffic_bytes_per_launch" not in rec:
        return None
    return float(rec["traffic_bytes_per_launch"])


def adjoint_ratio(I, T, torch, steps=200, ckpt=20):
    """Adjoint / forward time on the 2D dusty wave (512^2 + 512^2, 256^2 cells).

    Forward = n plain steps + the dust density of the misfit; adjoint = one
    tfsph_step_adjoint call (its own forward sweep with checkpoints, the
    replays and the reverse steps); each the best of repeated timings.  Target:
    the analytic initial dust profile.
    """
    prob = I.workload("wave2d", steps=steps)
    ex = prob.extra
    k = np.asarray(ex["kvec"])
    target = (ex["rho_d0"] * (1.0 + ex["amp"] * np.sin(prob.dust.x @ k))).astype(np.float32)
    sim = T.Simulation(prob, precision=T.TFSPH_F32)
    sim.step(2)
    sim.density(1)
    torch.cuda.synchronize()
    fwd = float("inf")
    for _ in range(3):            # best of three: one 200-step pass is short enough to be noisy
        t0 = time.perf_counter()
        sim.step(steps)
        sim.density(1)
        torch.cuda.synchronize()
        fwd = min(fwd, time.perf_counter() - t0)
    sim.close()
    runner = T.AdjointRunner(prob, steps, ckpt, precision=T.TFSPH_F32)
    runner.run(target)
    torch.cuda.synchronize()
    adj = float("inf")
    for _ in range(2):
        t0 = time.perf_counter()
        loss, dlogt, _, _ = runner.run(target)
        torch.cuda.synchronize()
        adj = min(adj, time.perf_counter() - t0)
    return {"ratio": adj / fwd, "forward_ms": 1e3 * fwd, "adjoint_ms": 1e3 * adj, "steps": steps,
            "ckpt_every": ckpt, "workload": WORKLOADS["wave2d"], "loss": float(loss), "dL_dlog_tstop": float(dlogt),
            "workspace_MiB": runner.ws_bytes / 2 ** 20}


# per gas-dust pair within 2h of the comparison schemes' pair kernels (Sections 2.1-2.2)
FLOPS_MK_PAIR = 33            # q (2), W(q) (9), (v_a - u_j).r (8), m K / (rho_a rho_j) (v.r) / (r^2 + eta^2) W (8), 3 fma (6)
FLOPS_ISPH_GAS_PAIR = 20      # q (2), W(q) (9), m W and m W / rho (2), density sum (1), velocity sums (6)
FLOPS_ISPH_DUST_PAIR = 47     # r, q (2), m W, m W / rho, density sum (12), pressure sum (4), velocity sums (6),
#                               1/r and m W'(q) / r (10), the two gradient sums (13)
SCHEME_T_STOP = 0.05          # about 25 steps of the 3D box: the explicit MK drag is stable there


def drag_schemes(prob, I, T, torch, steps=100, warmup=50, cpu_steps=0, counts=None):
    """The paper's three drag schemes on the same workload with t_stop = SCHEME_T_STOP: IDIC, and
    the comparison schemes MK (explicit pairwise drag, eqs. 8-10) and ISPH (interpolated
    two-velocity solve, eqs. 11-16), whose step keeps IDIC's binning and explicit gas pass and
    replaces the cell solve by one thread per gas particle (the dust window) and one per dust
    particle (the gas window).  Per scheme: whole-step time, per-kind launch times, the drag
    kernels priced in algorithmic flops against the FP32 vector peak, and (cpu_steps > 0) the
    oracle on the host cores."""
    counts = dict(counts or {})
    if "cross_candidates" not in counts:
        counts["cross_candidates"] = window_candidates(prob, "gas", "dust")
        counts["cross_pairs"] = support_pairs(prob, "gas", "dust")
    if "gas_pairs" not in counts:
        counts["gas_pairs"] = support_pairs(prob)
    cand, cross = counts["cross_candidates"], counts["cross_pairs"]
    press = FLOPS_PER_FORCE_PAIR * (counts["gas_pairs"] - prob.gas.n)
    # k_pair_gas and k_pair_dust run back to back inside one timed kind
    work = {
        "MK": {"k_gas_predict": press,
               "k_pair_gas_and_dust": 2 * (FLOPS_PER_CANDIDATE * cand + FLOPS_MK_PAIR * cross)},
        "ISPH": {"k_gas_predict": press,
                 "k_pair_gas_and_dust": 2 * FLOPS_PER_CANDIDATE * cand
                 + (FLOPS_ISPH_GAS_PAIR + FLOPS_ISPH_DUST_PAIR) * cross},
    }
    kinds = (T.TFSPH_KERNEL_BIN, T.TFSPH_KERNEL_DENSITY, T.TFSPH_KERNEL_FORCE, T.TFSPH_KERNEL_UPDATE)
    n_part = prob.gas.n + prob.dust.n
    out = {"t_stop": SCHEME_T_STOP, "steps": steps, "warmup": warmup, **counts}
    for name, scheme in (("IDIC", T.TFSPH_SCHEME_IDIC), ("ISPH", T.TFSPH_SCHEME_ISPH), ("MK", T.TFSPH_SCHEME_MK)):
        q = prob.copy()
        q.params = q.params.replace(t_stop=SCHEME_T_STOP, scheme=scheme)
        sim = T.Simulation(q, precision=T.TFSPH_F32)
        sim.step(warmup)
        T.tfsph_profile(sim.ctx, True, rotate=steps >= 4, every=max(1, steps // 48))
        torch.cuda.synchronize()
        sim.step(steps)
        torch.cuda.synchronize()
        T.tfsph_profile(sim.ctx, False)
        names = (("binning", "k_density", "k_gas_predict", "k_update") if name == "IDIC" else
                 ("binning", "k_density_gas_and_dust", "k_gas_predict", "k_pair_gas_and_dust"))
        kms = {}
        for k, kind in zip(names, kinds):
            ms, n = T.tfsph_profile_read(sim.ctx, kind)
            kms[k] = ms / n if n else 0.0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        flags, _ = sim.flags()
        sim.close()
        rec = {"ms_per_step": 1e3 * wall / steps, "value": n_part * steps / wall, "unit": "particle-steps/s",
               "kernel_ms_per_step": kms, "nonfinite": bool(flags & T.TFSPH_FLAG_NONFINITE)}
        if name in work:
            per = {}
            for k, flops in work[name].items():
                t = kms[k] * 1e-3
                ach = flops / t / 1e12 if t > 0 else 0.0
                per[k] = {"bound": "alu", "achieved": ach, "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                          "frac": ach / FP32_PEAK_TFLOPS, "avg_launch_ms": kms[k],
                          "algorithmic_flops_per_launch": flops}
            rec["roofline"] = per[max(per, key=lambda k: kms[k])] | {"kernel": max(per, key=lambda k: kms[k])}
            rec["kernels"] = per
        if cpu_steps > 0:
            from oracle import oracle as O
            O.build()
            g, d = O.from_problem(q)
            t0 = time.perf_counter()
            O.step(q.params, g, d, cpu_steps)
            dt = time.perf_counter() - t0
            rec["cpu_baseline"] = {"value": n_part * cpu_steps / dt, "unit": "particle-steps/s",
                                   "cores": O.num_threads(), "kind": "oracle",
                                   "sample": f"{cpu_steps} steps of the same workload, FP64, {dt:.2f} s wall"}
        out[name] = rec
    base = out["IDIC"]["ms_per_step"]
    for name in ("ISPH", "MK"):
        out[name]["time_vs_idic"] = out[name]["ms_per_step"] / base
    return out


def batched_throughput(I, T, torch, steps=500, plain_steps=20, cpu_steps=0):
    """256 uneven 1D dusty waves advanced together (form and workgroup size autotuned among the
    persistent kernel and the flattened launches, hipGraph replay), against the same instances
    through the plain path one at a time; with cpu_steps > 0 also the oracle on every instance,
    one after the other, on the host cores."""
    from paper_1908_01682_amd import autotune as A
    probs = I.batched_waves(steps=steps)
    n_part = sum(p.gas.n + p.dust.n for p in probs)
    bs = T.BatchedSimulation(probs, precision=T.TFSPH_F32)
    tune = A.tune(bs, steps=10, graph=True)
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
    cpu = None
    if cpu_steps > 0:
        from oracle import oracle as O
        O.build()
        states = [O.from_problem(p) for p in probs]
        t0 = time.perf_counter()
        for p, (g, d) in zip(probs, states):
            O.step(p.params, g, d, cpu_steps)
        dt = time.perf_counter() - t0
        cpu = {"value": n_part * cpu_steps / dt, "unit": "particle-steps/s", "cores": O.num_threads(),
               "kind": "oracle", "sample": f"{cpu_steps} step(s) of every instance, FP64, {dt:.2f} s wall"}
    return {"cpu_baseline": cpu, "value": value, "unit": "particle-steps/s", "ms_per_step": 1e3 * wall / steps,
            "steps": steps,
            "instances": len(probs), "particles": n_part, "block": tune["block"],
            "form": "flat" if tune["form"] == A.FLAT else "persistent", "cells_per_block": tune["cells_per_block"],
            "tuner_ms_per_step": tune["ms_per_step"],
            "plain_path_value": plain, "vs_plain": value / plain, "nonfinite": bool(flags & 1)}


def imex_throughput(prob, T, torch, steps=100, warmup=100, cpu_steps=0):
    """The same workload with the second-order IMEX step (three binnings, two density and force
    passes, two drag solves per step); with cpu_steps > 0 also the oracle's IMEX step on the host
    cores."""
    q = prob.copy()
    q.params = q.params.replace(scheme=T.TFSPH_SCHEME_IMEX2)
    sim = T.Simulation(q, precision=T.TFSPH_F32)
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    flags, _ = sim.flags()
    sim.close()
    n = q.gas.n + q.dust.n
    rec = {"ms_per_step": 1e3 * wall / steps, "value": n * steps / wall, "unit": "particle-steps/s",
           "steps": steps, "nonfinite": bool(flags & T.TFSPH_FLAG_NONFINITE)}
    if cpu_steps > 0:
        from oracle import oracle as O
        O.build()
        g, d = O.from_problem(q)
        t0 = time.perf_counter()
        O.step(q.params, g, d, cpu_steps)
        dt = time.perf_counter() - t0
        rec["cpu_baseline"] = {"value": n * cpu_steps / dt, "unit": "particle-steps/s", "cores": O.num_threads(),
                               "kind": "oracle", "sample": f"{cpu_steps} IMEX step(s) of the same workload, FP64, "
                                                           f"{dt:.2f} s wall"}
    return rec


def cpu_baseline(prob, steps: int, steps_1t: int = 1):
    """The FP64 oracle on the host cores (all threads, then one thread) on a bounded sample."""
    from oracle import oracle as O
    O.build()
    n = prob.gas.n + prob.dust.n
    cores = O.num_threads()
    g, d = O.from_problem(prob)
    t0 = time.perf_counter()
    O.step(prob.params, g, d, steps)
    dt = time.perf_counter() - t0
    O.set_num_threads(1)
    g, d = O.from_problem(prob)
    t0 = time.perf_counter()
    O.step(prob.params, g, d, steps_1t)
    dt1 = time.perf_counter() - t0
    O.set_num_threads(cores)
    return {"value": n * steps / dt, "unit": "particle-steps/s", "cores": cores, "kind": "oracle",
            "sample": f"{steps} steps of the full {prob.name} workload ({n} particles), FP64, {dt:.2f} s wall "
                      f"on {cores} threads; {steps_1t} step on 1 thread, {dt1:.2f} s",
            "value_1_thread": n * steps_1t / dt1}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=200,
                    help="untimed steps first: the first few hundred steps after start-up run slower")
    ap.add_argument("--workload", default="box3d", choices=sorted(WORKLOADS))
    ap.add_argument("--cpu-steps", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the adjoint, batched, IMEX and drag-scheme measurements")
    ap.add_argument("--scheme", default="idic", choices=("idic", "imex"),
                    help="time step timed: the paper's first-order step (default) or the second-order IMEX step")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy a 256 MiB device buffer 3 times (reference for HBM byte counters)")
    ap.add_argument("--scheme-cpu-steps", type=int, default=1,
                    help="oracle steps timed per drag scheme in the scheme comparison, and for the IMEX step")
    ap.add_argument("--only", choices=("adjoint", "batched", "schemes"),
                    help="run only that extra measurement and print its record as the JSON line "
                         "(for profiling it on its own; not the benchmark line)")
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

    if a.only:
        print(f"[bench] {a.only} only", file=sys.stderr, flush=True)
        if a.only == "schemes":
            rec = drag_schemes(I.workload(a.workload), I, T, torch, cpu_steps=0)
        else:
            rec = (adjoint_ratio if a.only == "adjoint" else batched_throughput)(I, T, torch)
        print(json.dumps({"only": a.only, **rec}), flush=True)
        return 0

    if a.copy_calibration:
        src = torch.ones(64 * 2 ** 20, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] copy calibration: 3 x {src.numel() * 4} bytes read and written", file=sys.stderr, flush=True)
    print(f"[bench] generating {a.workload}", file=sys.stderr, flush=True)
    prob = I.workload(a.workload)
    imex_main = a.scheme == "imex"
    if imex_main:
        prob.params = prob.params.replace(scheme=T.TFSPH_SCHEME_IMEX2)
    n_part = prob.gas.n + prob.dust.n
    sim = T.Simulation(prob, precision=T.TFSPH_F32)
    stream = torch.cuda.current_stream()
    # cells per block of the update kernel, timed on this problem (the results do not depend on it)
    from paper_1908_01682_amd import autotune as A
    tuning = A.tune_plain(sim, steps=20, use_cache=False)
    print(f"[bench] update kernel: {tuning['cells_per_block']} cells per block", file=sys.stderr, flush=True)
    sim.step(a.warmup)
    torch.cuda.synchronize()
    print(f"[bench] warmup done, timing {a.steps} steps", file=sys.stderr, flush=True)

    # HIP events around one kernel kind in every `every`-th step, the kinds in turn, so that few
    # events sit between the timed launches; each kind still gets about 12 timed steps of 200
    every = max(1, a.steps // 48)
    T.tfsph_profile(sim.ctx, True, rotate=a.steps >= 4, every=every)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(a.steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    T.tfsph_profile(sim.ctx, False)
    kernel_ms = {}
    # per launch of the kind; with the IMEX step the force and update kinds cover the stage kernels
    names = (("k_density", "k_gas_predict", "k_update", "binning") if not imex_main else
             ("k_density", "imex_force_stages", "imex_update_stages", "binning"))
    for name, kind in zip(names, (T.TFSPH_KERNEL_DENSITY, T.TFSPH_KERNEL_FORCE, T.TFSPH_KERNEL_UPDATE,
                                  T.TFSPH_KERNEL_BIN)):
        ms, n = T.tfsph_profile_read(sim.ctx, kind)
        kernel_ms[name] = ms / n if n else 0.0
    # the same steps without the timing events (throughput as an application sees it)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(a.steps)
    torch.cuda.synchronize()
    wall_plain = time.perf_counter() - t0
    flags, _ = sim.flags()
    sim.close()
    if flags & T.TFSPH_FLAG_NONFINITE:
        print("[bench] non-finite state", file=sys.stderr)
        return 1

    ms_per_step = 1e3 * wall / a.steps
    value = n_part * a.steps / wall
    print("[bench] counting window candidates and support pairs", file=sys.stderr, flush=True)
    cand = window_candidates(prob)
    pairs = support_pairs(prob)
    peak_tf = FP32_PEAK_TFLOPS
    work = {
        "k_density": ("alu", FLOPS_PER_CANDIDATE * cand + FLOPS_PER_DENSITY_PAIR * pairs, peak_tf, "TFLOP/s"),
        "k_gas_predict": ("alu", FLOPS_PER_FORCE_PAIR * (pairs - prob.gas.n), peak_tf, "TFLOP/s"),
        "k_update": ("hbm", update_kernel_bytes(prob), HBM_PEAK_GBS, "GB/s"),
    }
    if imex_main:   # the density kernel is the same launch; the other kinds mix several stage kernels
        work = {"k_density": work["k_density"]}
    per_kernel = {}
    for k, (bound, amount, peak, unit) in work.items():
        t = kernel_ms[k] * 1e-3
        ach = amount / t / (1e12 if unit == "TFLOP/s" else 1e9) if t > 0 else 0.0
        per_kernel[k] = {"bound": bound, "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak,
                         "avg_launch_ms": kernel_ms[k],
                         ("algorithmic_flops_per_launch" if bound == "alu" else "algorithmic_bytes_per_launch"): amount}
        if bound == "alu":
            per_kernel[k]["frac_of_nonpacked_peak"] = ach / FP32_NONPACKED_TFLOPS
    dom = max(work, key=lambda k: kernel_ms[k])
    roof = dict(per_kernel[dom])
    roof = {"bound": roof.pop("bound"), "achieved": roof.pop("achieved"), "peak": roof.pop("peak"),
            "unit": roof.pop("unit"), "frac": roof.pop("frac"), "traffic": measured_traffic(dom, a.workload),
            "kernel": dom, **roof}
    sbytes = step_bytes(prob)
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
        "config": {"workload": WORKLOADS[a.workload] + (", second-order IMEX step" if imex_main else ""),
                   "scheme": a.scheme, "particles": n_part,
                   "cells": int(np.prod(prob.params.n_cells[:prob.params.dim])), "dim": prob.params.dim},
        "roofline": roof,
        "hbm_roofline_step": None if imex_main else {
            "algorithmic_bytes_per_step": sbytes, "achieved_GBs": sbytes / (ms_per_step * 1e-3) / 1e9,
            "frac": sbytes / (ms_per_step * 1e-3) / 1e9 / HBM_PEAK_GBS},
        "kernels": per_kernel,
        "kernel_ms_per_step": kernel_ms,
        "tuning": {"cells_per_block": tuning["cells_per_block"], "ms_per_step": tuning["ms_per_step"]},
        "valu_issue_share": measured_valu_share(a.workload),
        "window_candidates": cand,
        "support_pairs": pairs,
        "uninstrumented": {"ms_per_step": 1e3 * wall_plain / a.steps, "value": n_part * a.steps / wall_plain},
        "adjoint_forward_ratio": None,
    }
    if not a.no_extras:
        print("[bench] adjoint / forward ratio (2D wave)", file=sys.stderr, flush=True)
        adj = adjoint_ratio(I, T, torch)
        result["adjoint_forward_ratio"] = adj["ratio"]
        result["adjoint"] = adj
        print("[bench] batched 1D waves", file=sys.stderr, flush=True)
        result["batched"] = batched_throughput(I, T, torch, cpu_steps=0 if a.no_cpu_baseline else 1)
        if not imex_main:
            print("[bench] second-order IMEX step on the same workload", file=sys.stderr, flush=True)
            imex = imex_throughput(prob, T, torch, cpu_steps=0 if a.no_cpu_baseline else a.scheme_cpu_steps)
            imex["cost_vs_first_order"] = imex["ms_per_step"] / result["uninstrumented"]["ms_per_step"]
            result["imex"] = imex
            print(f"[bench] the three drag schemes at t_stop {SCHEME_T_STOP}", file=sys.stderr, flush=True)
            result["drag_schemes"] = drag_schemes(prob, I, T, torch, counts={"gas_pairs": pairs},
                                                  cpu_steps=0 if a.no_cpu_baseline else a.scheme_cpu_steps)
    if not a.no_cpu_baseline:
        print(f"[bench] oracle on host cores, {a.cpu_steps} steps", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(prob, a.cpu_steps)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
