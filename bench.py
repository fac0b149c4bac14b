"""Benchmark of the VDS hot path on one MI355X.

A step is one implicit Euler step of the particle scheme on the 4-bead
Hookean chain under shear (P = 20000 particles, D = 9, h = 0.4, dt = 1e-3):
centring and operand packing, the two O(P^2) kernel passes per fixed-point
iteration, drift, update and convergence test, and the FP64 stress.  The
headline value is pair-evaluations per second over the timed steps (one
pair-evaluation is one ordered (I, J) in one pass).

Prints ONE JSON line.  Inputs are resident in HBM before the timed region.
The roofline object covers the dominant kernel (the pair pass): algorithmic
FLOP per launch / average launch time measured with HIP events on the
launching stream, against the MI355X dense FP32 matrix peak.  The CPU baseline
is the FP64 oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3   # MI355X dense FP32 (matrix and packed vector), AMD datasheet
PEAK_HBM_GBS = 8000.0


def flops_per_pair(D: int) -> int:
    # dot product 2D, norm combine + clamp + scale 4, accumulate S 1, accumulate sum e x_J 2D - 1
    return 4 * D + 4


def cpu_baseline(cfg, sample_rows: int, threads: int):
    from oracle import vds as ovds
    import workloads as wl
    q = wl.f32_as_f64(wl.to_f32(cfg["q0"]))
    x = ovds.particle_major(q)
    P = cfg["P"]
    w = ovds.uniform_weights(P)
    rows = np.arange(sample_rows)
    S_rows = ovds.density_sums(x, w, cfg["h"], rows=rows, threads=threads)   # warm the pool / caches
    S_all = np.concatenate([S_rows, np.ones(P - sample_rows)])                # pass B weights (values irrelevant to timing)
    t0 = time.perf_counter()
    ovds.brownian_terms(x, w, cfg["h"], rows=rows, S_all=S_all, threads=threads)
    dt = time.perf_counter() - t0
    pairs = 2.0 * sample_rows * P
    return dict(value=pairs / dt, unit="pair-evals/s", cores=threads, kind="oracle",
                sample=f"both kernel passes (term1 and term2) for {sample_rows} of {P} rows of the "
                       f"P={P}, D=9 chain state, FP64 NumPy with {threads} threads: {pairs:.3g} pair-evals in {dt:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--P", type=int, default=20000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-rows", type=int, default=6000)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--t-end", action="store_true", help="also time the full 500-step run to t_end")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the particle rows would shard by block with an all-gather of S between passes).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_2603_12550_amd as pkg
    from paper_2603_12550_amd import _vds
    import workloads as wl

    torch.cuda.set_device(0)
    cfg = wl.chain4_shear(P=args.P)
    P, D = cfg["P"], 9
    ctx = pkg.Context(3, P, cfg["h"], H=cfg["H"], G=cfg["G"], dt=cfg["dt"], scheme="implicit",
                      picard_rtol=1e-6, picard_max=50, picard_batch=3)
    q0 = torch.from_numpy(wl.to_f32(cfg["q0"])).cuda()
    if not args.no_autotune:
        ctx.autotune(q0)
    tune = ctx.get_tuning()
    q = q0.clone()

    for _ in range(args.warmup):
        ctx.step(q)
    torch.cuda.synchronize()

    ctx.timing_enable(True)
    iters = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        d = ctx.step(q)
        iters += d["last_iters"]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tim = ctx.timing_read(_vds.VDS_TIMER_PAIR)
    ctx.timing_enable(False)

    pairs = 2.0 * P * P * iters
    value = pairs / elapsed
    avg_ms = tim["ms"] / max(1, tim["launches"])
    flop_launch = P * P * flops_per_pair(D)
    achieved = flop_launch / (avg_ms * 1e-3) / 1e12

    out = {
        "metric": "kernel pair-evals/s (% FP32 peak); wall time to t_end vs plain VDS at <=1e-2 stress err",
        "value": value,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: 4-bead chain bonds drawn N(0, I/3), seed 2",
        "config": {"workload": f"chain4_shear: 4-bead Hookean chain, P={P}, D=9, h=0.4, shear rate 1, "
                               f"implicit Euler dt=1e-3, fixed-point rtol 1e-6",
                   "P": P, "D": D, "pair_tuning": tune,
                   "fixed_point_iterations": iters},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS, "traffic": None,
                     "kernel": "k_pair_mfma" if tune["impl"] == 0 else "k_pair_valu",
                     "avg_launch_ms": avg_ms, "launches": tim["launches"],
                     "flop_per_launch": flop_launch, "flop_per_pair": flops_per_pair(D)},
    }

    if args.t_end:
        qt = q0.clone()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        d = ctx.step(qt, nsteps=cfg["steps"])
        torch.cuda.synchronize()
        out["t_end"] = {"steps": cfg["steps"], "seconds": time.perf_counter() - t1, "iterations": d["iters"],
                        "tau": d["tau"].tolist()}

    if not args.no_cpu:
        threads = min(16, len(os.sched_getaffinity(0)))
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_rows, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
