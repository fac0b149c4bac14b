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
    """Algorithmic FLOP of one pair-evaluation: 2D for the distance dot product,
    2 to combine the norms and scale, 2(D + 1) to accumulate e w and e w x_J
    (plus one exp, not counted)."""
    return 4 * D + 4


def cpu_baseline(cfg, threads: int):
    """One implicit step of the FP64 oracle on the same state (all rows), timed."""
    from oracle import vds as ovds
    import workloads as wl
    q = wl.f32_as_f64(wl.to_f32(cfg["q0"]))
    P = cfg["P"]
    w = ovds.uniform_weights(P)
    prob = ovds.problem_from(cfg)
    t0 = time.perf_counter()
    _, iters = ovds.step_implicit(q, w, prob, threads=threads)
    dt = time.perf_counter() - t0
    pairs = 2.0 * P * P * iters
    return dict(value=pairs / dt, unit="pair-evals/s", cores=threads, kind="oracle",
                sample=f"one implicit step (fixed-point tolerance 1e-13, {iters} iterations, both kernel "
                       f"passes per iteration over all rows) of the P={P}, D=9 chain workload, FP64 NumPy "
                       f"row blocks on {threads} threads: {pairs:.3g} pair-evals in {dt:.1f} s")


def kernel_source_hash() -> str:
    import hashlib
    src = os.path.join(ROOT, "paper_2603_12550_amd", "csrc", "pair_kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


def measured_traffic(kernel: str, tuning: dict, P: int):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC summary,
    if it was taken on the current kernel source and the same launch shape."""
    path = os.path.join(ROOT, "profiles", "pair_pass_chain4_P20000_traffic.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("pair_kernels_sha256_16") != kernel_source_hash() or rec.get("kernel") != kernel \
            or rec.get("tuning") != tuning or rec.get("P") != P:
        return None
    return rec.get("hbm_bytes_per_launch")


def copy_calibration(nbytes: int = 1 << 29, reps: int = 5):
    """A plain device copy of known size, for scaling FETCH_SIZE / WRITE_SIZE."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--P", type=int, default=20000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--tuning", type=str, default="", help="impl,rows_per_wave,col_splits (skips the autotuner)")
    ap.add_argument("--copy-calibration", action="store_true", help="only run a plain copy of known size")
    ap.add_argument("--sweep", action="store_true", help="only time every pair-kernel tuning and print a table")
    ap.add_argument("--t-end", action="store_true", help="also time the full 500-step run to t_end")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the particle rows would shard by block with an all-gather of S between passes).",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return

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
    if args.sweep:
        for impl, rbs in ((0, (1, 2, 4)), (1, (1,))):
            for rb in rbs:
                for sp in (1, 2, 4, 8, 16, 32):
                    ctx.set_tuning(impl, rb, sp)
                    q = q0.clone()
                    ctx.step(q, nsteps=2)
                    ctx.timing_enable(True)
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    d = ctx.step(q, nsteps=5)
                    torch.cuda.synchronize()
                    el = time.perf_counter() - t0
                    tim = ctx.timing_read(_vds.VDS_TIMER_PAIR)
                    ctx.timing_enable(False)
                    print(json.dumps({"impl": impl, "rows_per_wave": rb, "col_splits": sp,
                                      "pair_avg_ms": tim["ms"] / max(1, tim["launches"]),
                                      "step_ms": el * 1e3 / 5, "iters": d["iters"]}), flush=True)
        return
    if args.tuning:
        ctx.set_tuning(*[int(v) for v in args.tuning.split(",")])
    else:
        ctx.autotune(q0)
    tune = ctx.get_tuning()
    q = q0.clone()

    if args.warmup:
        ctx.step(q, nsteps=args.warmup)
    torch.cuda.synchronize()

    ctx.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d = ctx.step(q, nsteps=args.steps)
    torch.cuda.synchronize()
    iters = d["iters"]
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
        "roofline": {"bound": "mfma" if tune["impl"] == 0 else "alu", "achieved": achieved,
                     "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic("k_pair_mfma" if tune["impl"] == 0 else "k_pair_valu", tune, P),
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
        out["cpu_baseline"] = cpu_baseline(cfg, threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
