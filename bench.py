"""Benchmark of the VDS hot path on one MI355X.

A step is one implicit Euler step of the particle scheme on the 4-bead
Hookean chain under shear (P = 20000 particles, D = 9, h = 0.4, dt = 1e-3):
centring and operand packing, the two O(P^2) kernel passes per fixed-point
iteration, drift, update and convergence test, and the FP64 stress.  The
headline value is pair-evaluations per second over the timed steps (one
pair-evaluation is one ordered (I, J) in one pass), computed in FP32 on the
FP32 matrix cores.

Output: one JSON line per extra measurement and one for the FP16-split pair
form (a separate, labelled arithmetic), then the headline as the LAST line
(under 2 KB).  Inputs are resident in HBM before the timed region.  The
headline's roofline object covers the dominant kernel (the pair pass):
algorithmic FLOP per launch / average launch time measured with HIP events on
the launching stream, against the MI355X dense FP32 matrix peak.  The CPU
baseline is the FP64 oracle timed on a bounded sample of the same workload.
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
LEARNED_INPUT_NOISE = 10.0  # training input noise, in increment standard deviations
TIMING_STRIDE = 5          # event-timed pair launches: every 5th, odd so that passes A and B are both sampled
PEAK_HBM_GBS = 8000.0


def flops_per_pair(D: int) -> int:
    """Algorithmic FLOP of one pair-evaluation: 2D for the distance dot product,
    2 to combine the norms and scale, 2(D + 1) to accumulate e w and e w x_J
    (plus one exp, not counted)."""
    return 4 * D + 4


def cpu_baseline(cfg, threads: int):
    """One implicit step of the FP64 oracle on the same state (all rows), timed
    on `threads` host threads; then both kernel passes of the same oracle over
    a sample of rows on one thread."""
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
    # one core: passes A and B for 1000 rows against all P columns (S of every
    # column from the threaded run's own routine, untimed)
    x = ovds.particle_major(q)
    S_all = ovds.density_sums(x, w, prob.h, threads=threads)
    rows = np.arange(1000)
    t1 = time.perf_counter()
    ovds.brownian_terms(x, w, prob.h, rows=rows, S_all=S_all, threads=1)
    dt1 = time.perf_counter() - t1
    pairs1 = 2.0 * len(rows) * P
    return dict(value=pairs / dt, unit="pair-evals/s", cores=threads, kind="oracle",
                sample=f"one implicit step of the P={P}, D=9 chain (fixed-point tol 1e-13, {iters} iterations, "
                       f"both passes over all rows), FP64 NumPy row blocks on {threads} threads: "
                       f"{pairs:.3g} pair-evals in {dt:.1f} s",
                one_core={"value": pairs1 / dt1, "cores": 1,
                          "sample": f"passes A and B of 1000 rows x {P} columns on one thread: "
                                    f"{pairs1:.3g} pair-evals in {dt1:.2f} s"})


def kernel_source_hash() -> str:
    import hashlib
    src = os.path.join(ROOT, "paper_2603_12550_amd", "csrc", "pair_kernels.hip")
    return hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]


PAIR_KERNEL = {0: "k_pair_mfma", 1: "k_pair_valu", 2: "k_pair_mfma16", 3: "k_pair_mfma16", 4: "k_pair_mfma32"}
PAIR_ARITHMETIC = {
    0: "fp32: pair products on FP32 MFMA 16x16x4, FP32 exponentials",
    1: "fp32: pair products as FP32 vector FMAs, FP32 exponentials",
    2: "fp16 hi/lo split (~22-bit) sums: distances on FP32 MFMA, kernel-weighted sums on FP16 MFMA with split "
       "factors, FP32 accumulation",
    3: "fp16 hi/lo split (~22-bit): both pair products on FP16 MFMA with every factor split into high and low "
       "halves, FP32 accumulation and exponentials",
    4: "fp32: distances on FP32 MFMA 32x32x2, kernel-weighted sums on FP32 MFMA 4x4x1, FP32 exponentials",
}
# v_exp_f32 issues 8 lanes per cycle per SIMD (measured: 8 cycles per wave64 instruction)
EXP_PER_S = 256 * 4 * 8 * 2.4e9
PEAK_FP16_TFLOPS = 2500.0


def issued_mfma_flop_per_pair(impl: int, D: int) -> float:
    """FLOP the matrix cores issue per pair-eval (padding included)."""
    if impl == 4:
        kp = (D + 2) & ~1
        ng = (D + 4) // 4
        return 2.0 * kp + 2.0 * 4 * ng
    if impl == 0:
        kk = (D + 2 + 3) // 4
        return 2.0 * 4 * kk + 2.0 * 16
    if impl in (2, 3):
        slices = (3 * D + 2 + 31) // 32 if impl == 3 else 0
        return (1.5 + slices) * 16 * 16 * 32 * 2 / 256
    return 0.0


def secondary_ceilings(impl: int, D: int, pairs_per_s: float):
    """Ceilings besides the algorithmic FP32 rate: one exp per pair-eval on the
    transcendental unit, and the matrix-core rate of the MFMA work each
    pair-eval issues (FP32 for the FP32 forms, FP16 for the split ones)."""
    out = {"exp_unit": {"pair_evals_per_s": EXP_PER_S, "frac": pairs_per_s / EXP_PER_S}}
    f = issued_mfma_flop_per_pair(impl, D)
    if f:
        peak = PEAK_FP16_TFLOPS if impl in (2, 3) else PEAK_FP32_TFLOPS
        out["issued_mfma"] = {"dtype": "fp16" if impl in (2, 3) else "fp32", "flop_per_pair": f,
                              "tflops": pairs_per_s * f / 1e12, "frac": pairs_per_s * f / (peak * 1e12)}
    return out


def _compact(o, sig=4):
    """Floats rounded to `sig` significant digits, for the JSON lines."""
    if isinstance(o, float):
        return float(f"{o:.{sig}g}")
    if isinstance(o, dict):
        return {k: _compact(v, sig) for k, v in o.items()}
    if isinstance(o, (list, tuple)):
        return [_compact(v, sig) for v in o]
    return o


def measured_traffic(kernel: str, tuning: dict, P: int):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 PMC summary,
    if it was taken on the current kernel source and the same launch shape."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_chain4_P{P}_traffic.json")
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


def _timer_rate(ctx, which):
    from paper_2603_12550_amd import _vds
    t = ctx.timing_read(which)
    return t["ms"], t["launches"], t["work"]


def measure_pod_rom(pkg, wl, torch, P):
    """POD-reduced chain: reference run of 2000 implicit steps collecting 300
    snapshots over steps 0..1000, rank-180 basis, 2000 reduced explicit steps
    with freezes every 300; errors of the reduced state and stress at t_end."""
    from paper_2603_12550_amd import _vds
    cfg = wl.pod_chain4(P=P)
    ctx = pkg.Context(3, P, cfg["h"], H=cfg["H"], G=cfg["G"], dt=cfg["dt"], scheme="implicit")
    q0 = torch.from_numpy(wl.to_f32(cfg["q0"])).cuda()
    snaps = [int(v) for v in wl.snapshot_steps(cfg["snapshots"], cfg["snap_until"])]
    X = torch.empty((len(snaps) * 3, 3 * P), dtype=torch.float32, device="cuda")
    # the stress of both runs is compared every `out_every` steps (err_MOR of
    # Section 3.1 at each output; the Table 4 protocol compares at t_end)
    out_every = 100
    stops = sorted(set(snaps) | set(range(out_every, cfg["steps"] + 1, out_every)))
    snap_pos = {s: i for i, s in enumerate(snaps)}
    tau_ref_hist = []
    q = q0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    for s in stops:
        if s > done:
            ctx.step(q, nsteps=s - done)
            done = s
        if s in snap_pos:
            li = snap_pos[s]
            X[3 * li:3 * li + 3].copy_(q.reshape(3, 3 * P))
        if s % out_every == 0:
            tau_ref_hist.append(ctx.stress(q))
    torch.cuda.synchronize()
    T_ref = time.perf_counter() - t0
    tau_ref = ctx.stress(q)
    ctx.timing_enable(True)
    t1 = time.perf_counter()
    U, eig = ctx.pod_basis(X, cfg["R"])
    torch.cuda.synchronize()
    T_pod = time.perf_counter() - t1
    gemm = _timer_rate(ctx, _vds.VDS_TIMER_GEMM)
    ctx.timing_enable(False)
    rom = pkg.Rom(ctx, U)
    p = ctx.pod_project(U, q0)
    rom.run(p.clone(), 300, 300)          # warm-up
    ctx.timing_enable(True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    tau_rom_hist = rom.run(p, cfg["rom_steps"], cfg["freeze_every"], output_every=out_every)
    torch.cuda.synchronize()
    T_rom = time.perf_counter() - t2
    tau_rom = tau_rom_hist[-1]
    err_hist = [float(np.linalg.norm(a - b) / np.linalg.norm(b)) for a, b in zip(tau_rom_hist, tau_ref_hist)]
    kg = _timer_rate(ctx, _vds.VDS_TIMER_KGEMM)
    ctx.timing_enable(False)
    q_rom = ctx.pod_reconstruct(U, p)
    err_mor = float((q_rom - q).norm() / q.norm())
    # the same windows integrated exactly, then with windows chosen by the energy law
    exact = {}
    for label, adaptive in (("exact_windows", False), ("adaptive_windows", True)):
        pe = ctx.pod_project(U, q0)
        rom.run_exact(pe.clone(), 300, 300, adaptive=adaptive, energy_tol=0.1)  # warm-up
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        tau_e, windows, wstats = rom.run_exact(pe, cfg["rom_steps"], cfg["freeze_every"], adaptive=adaptive,
                                               energy_tol=0.1)
        torch.cuda.synchronize()
        T_e = time.perf_counter() - t3
        exact[label] = {"T_s": T_e, "T_over_T_ref": T_e / T_ref,
                        "err_mor_t_end": float((ctx.pod_reconstruct(U, pe) - q).norm() / q.norm()),
                        "stress_rel_err_vs_plain": float(np.linalg.norm(tau_e - tau_ref) / np.linalg.norm(tau_ref)),
                        **wstats, "window_lengths": [round(w_, 6) for w_ in windows]}
    # shorter freeze intervals: the freeze error dominates the reduced run's
    # error (the basis itself reproduces the final state's stress to 0.4 %)
    freeze_sweep = {}
    for fe in (100, 50, 25):
        pf = ctx.pod_project(U, q0)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        tau_f = rom.run(pf, cfg["rom_steps"], fe)
        torch.cuda.synchronize()
        T_f = time.perf_counter() - t4
        freeze_sweep[f"freeze_every_{fe}"] = {
            "T_s": T_f, "T_over_T_ref": T_f / T_ref,
            "err_mor_t_end": float((ctx.pod_reconstruct(U, pf) - q).norm() / q.norm()),
            "stress_rel_err_vs_plain": float(np.linalg.norm(tau_f - tau_ref) / np.linalg.norm(tau_ref))}
    midpoint_sweep, extrapolated_sweep = {}, {}
    for mode, sweep, fes in ((True, midpoint_sweep, (300, 200, 150, 100)),
                             ("extrapolated", extrapolated_sweep, (300, 200, 150, 100, 50))):
        for fe in fes:
            pf = ctx.pod_project(U, q0)
            torch.cuda.synchronize()
            t4 = time.perf_counter()
            tau_f = rom.run(pf, cfg["rom_steps"], fe, midpoint=mode)
            torch.cuda.synchronize()
            T_f = time.perf_counter() - t4
            sweep[f"freeze_every_{fe}"] = {
                "T_s": T_f, "T_over_T_ref": T_f / T_ref,
                "err_mor_t_end": float((ctx.pod_reconstruct(U, pf) - q).norm() / q.norm()),
                "stress_rel_err_vs_plain": float(np.linalg.norm(tau_f - tau_ref) / np.linalg.norm(tau_ref))}
    qp = ctx.pod_reconstruct(U, ctx.pod_project(U, q))
    projection_floor = {"state": float((qp - q).norm() / q.norm()),
                        "stress": float(np.linalg.norm(ctx.stress(qp) - tau_ref) / np.linalg.norm(tau_ref))}
    lam = np.asarray(eig)
    return {
        "workload": f"POD-reduced 4-bead chain, P={P}: reference 2000 implicit steps, 300 snapshots over "
                    f"steps 0-1000 (900 columns), R=180, 2000 reduced explicit steps, freeze every 300",
        "T_ref_s": T_ref, "T_rom_s": T_rom, "T_rom_over_T_ref": T_rom / T_ref, "T_pod_offline_s": T_pod,
        "err_mor_t_end": err_mor,
        "stress_rel_err_vs_plain": float(np.linalg.norm(tau_rom - tau_ref) / np.linalg.norm(tau_ref)),
        "stress_rel_err_at_outputs": {"every_steps": out_every, "errors": err_hist, "max": max(err_hist)},
        "tau_ref": tau_ref.tolist(), "tau_rom": tau_rom.tolist(),
        "eig_head": lam[:8].tolist(),
        # tail eigenvalues of the FP32 Gram matrix below its rounding level come out
        # of either sign: the remaining energy counts the positive ones, and the
        # largest negative one gives the level below which it cannot be resolved
        "remaining_energy_at_R": float(np.clip(lam[cfg["R"]:], 0, None).sum() / np.clip(lam, 0, None).sum()),
        "gram_rounding_level": float(max(0.0, -lam.min()) / np.clip(lam, 0, None).sum()),
        "gemm_ms": gemm[0], "gemm_tflops": gemm[2] / (gemm[0] * 1e-3) / 1e12 if gemm[0] else None,
        "kernel_gemm_ms_per_freeze": kg[0] / max(1, kg[1]),
        **exact,
        "kernel_gemm_tflops": kg[2] / (kg[0] * 1e-3) / 1e12 if kg[0] else None,
        "freeze_sweep": freeze_sweep,
        "midpoint_freeze_sweep": midpoint_sweep,
        "extrapolated_midpoint_freeze_sweep": extrapolated_sweep,
        "projection_floor_t_end": projection_floor,
    }


def pod_best_within(e: dict, bar: float = 1e-2):
    """The fastest reduced-run schedule of a POD measurement (`measure_pod_rom`'s
    result) whose stress error against the plain scheme at t_end is within
    `bar`: {"time_ratio", "stress_err", "schedule"}, or None if none is."""
    cands = [("start freezes every 300", e["T_rom_over_T_ref"], e["stress_rel_err_vs_plain"])]
    for key, label in (("freeze_sweep", "start freezes"), ("midpoint_freeze_sweep", "midpoint freezes"),
                       ("extrapolated_midpoint_freeze_sweep", "extrapolated-midpoint freezes")):
        for k, v in (e.get(key) or {}).items():  # k = "freeze_every_<steps>"
            cands.append((f"{label} every {k.rsplit('_', 1)[-1]}", v["T_over_T_ref"], v["stress_rel_err_vs_plain"]))
    for key, label in (("exact_windows", "exact windows every 300"), ("adaptive_windows", "adaptive exact windows")):
        v = e.get(key)
        if v:
            cands.append((label, v["T_over_T_ref"], v["stress_rel_err_vs_plain"]))
    ok = [c for c in cands if c[2] <= bar]
    if not ok:
        return None
    label, ratio, err = min(ok, key=lambda c: c[1])
    return {"time_ratio": ratio, "stress_err": err, "schedule": label}


def measure_batched(pkg, wl, torch, steps):
    """512 ensembles, explicit Euler, one graph-captured step replayed, to t_end
    (`steps` steps); then a sample of ensembles run one by one on plain
    contexts from the same states over the same steps: stress error of the
    batched form at t_end against them, and the speedup."""
    ens = wl.ensembles()
    G = np.stack([wl.shear_gradient(r) for r in ens["rate"]])
    b = pkg.Batch(ens["P"], ens["h"], G)
    states = [torch.from_numpy(wl.to_f32(wl.ensemble_state(ens, e))).cuda() for e in range(ens["n_ens"])]
    q0 = b.pack(states)
    tune = b.autotune(q0)
    q = q0.clone()
    b.step(q, nsteps=2)
    q = q0.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tau = b.step(q, nsteps=steps, stress=True)
    torch.cuda.synchronize()
    T_b = time.perf_counter() - t0
    pairs = 2.0 * float((ens["P"].astype(np.float64) ** 2).sum()) * steps
    # plain single-ensemble contexts on a sample, same steps from the same start
    rng = np.random.default_rng(11)
    sample = rng.choice(ens["n_ens"], 12, replace=False)
    t_plain, pairs_plain, errs = 0.0, 0.0, []
    for e in sample:
        e = int(e)
        ctx = pkg.Context(3, int(ens["P"][e]), ens["h"][e], G=G[e], dt=ens["dt"], scheme="explicit")
        qe = states[e].clone()
        ctx.autotune(qe)
        ctx.step(qe, nsteps=1)
        qe = states[e].clone()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ctx.step(qe, nsteps=steps)
        torch.cuda.synchronize()
        t_plain += time.perf_counter() - t1
        pairs_plain += 2.0 * float(ens["P"][e]) ** 2 * steps
        tp = ctx.stress(qe)
        errs.append(float(np.linalg.norm(tau[e] - tp) / np.linalg.norm(tp)))
    rate_b, rate_p = pairs / T_b, pairs_plain / t_plain
    return {
        "workload": f"{ens['n_ens']} independent 4-bead ensembles, P_b in [2000, 16000] (sum {int(ens['P'].sum())}), "
                    f"shear rate log-uniform [0.1, 10], h_b = 0.4 (P_b/20000)^(-1/13), explicit dt=1e-3, {steps} steps",
        "tuning": tune, "seconds_to_t_end": T_b, "pair_evals_per_s": rate_b,
        "plain_single_ensemble_pair_evals_per_s": rate_p, "speedup_vs_plain_single": rate_b / rate_p,
        "plain_sample": [int(v) for v in sample],
        "max_stress_rel_err_vs_plain_at_t_end": max(errs),
        "tau_mean_trace": float(np.mean([np.trace(t) for t in tau])),
    }


def _learned_rollout_vs_plain(torch, ctx, m, U, q0, rate, rollout_steps):
    """Plain-scheme run and checked learned rollout from q0 over rollout_steps
    steps: (T_plain, tau_ref, T_rollout, rollout stats)."""
    import math
    q = q0.clone()
    ctx.step(q.clone(), nsteps=2)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.step(q, nsteps=rollout_steps)
    torch.cuda.synchronize()
    T_plain = time.perf_counter() - t1
    tau_ref = ctx.stress(q)
    # what the basis alone can reach: the plain final state projected and reconstructed
    qp = ctx.pod_reconstruct(U, ctx.pod_project(U, q))
    floor = float(np.linalg.norm(ctx.stress(qp) - tau_ref) / np.linalg.norm(tau_ref))
    p = ctx.pod_project(U, q0)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    st = m.rollout(ctx, U, p, math.log(rate), nsteps=rollout_steps, check_every=50, resid_tol=0.2, energy_tol=0.5)
    torch.cuda.synchronize()
    st["projection_floor_stress"] = floor
    return T_plain, tau_ref, time.perf_counter() - t2, st


LEARNED_LR, LEARNED_LR_FINAL = 2e-3, 1e-4  # half-cosine decay of the Adam step over the epochs


def _train_learned(pkg, wl, torch, mk, q0, nb, R, rates, n_snap_runs, run_steps, epochs, seed=3):
    """POD basis from the snapshots (every 10 steps) of the first n_snap_runs
    runs, training pairs from the projected trajectories of every run, and the
    trained network; returns (U, m, pairs, losses)."""
    import math
    from paper_2603_12550_amd import learned
    states = []
    for r in rates[:n_snap_runs]:
        states += learned.run_states(mk(r), q0, run_steps, 10)
    U, _ = mk(rates[0]).pod_basis(learned.snapshot_matrix(states), R)
    del states
    trajs = [(learned.reduced_trajectory(mk(r), U, q0, run_steps), math.log(r)) for r in rates]
    nin, nout = nb * R + 1, nb * R
    m = pkg.Mlp(nin, 128, nout, 256)
    init = np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in wl.mlp_init(9, [nin, 128, 128, nout])])
    m.set_params(torch.from_numpy(wl.to_f32(init)).cuda())
    X, T = learned.training_set(m, trajs)
    del trajs
    losses = learned.train(m, X, T, epochs=epochs, batch=64, lr=LEARNED_LR, seed=seed, input_noise=LEARNED_INPUT_NOISE,
                           lr_final=LEARNED_LR_FINAL)
    return U, m, int(X.shape[0]), losses


def measure_learned(pkg, wl, torch, P, n_runs, n_snap_runs, run_steps, epochs, rollout_steps, seed=3):
    """Learned reduced step on the 4-bead chain (R = 180, input 541, width 128):
    explicit runs at log-uniform shear rates in [0.1, 10], then a checked rollout
    at a held-out rate against the plain scheme and against the POD-Galerkin
    reduced model (the method without the network)."""
    R, h, rate = 180, 0.4, 1.0
    rates = wl.mlp_shear_rates(n_runs)
    q0 = torch.from_numpy(wl.to_f32(wl.gaussian_bonds(2, 3, P, 1 / 3))).cuda()
    mk = lambda r: pkg.Context(3, P, h, G=wl.shear_gradient(r), dt=1e-3, scheme="explicit")
    t0 = time.perf_counter()
    U, m, pairs, losses = _train_learned(pkg, wl, torch, mk, q0, 3, R, rates, n_snap_runs, run_steps, epochs, seed)
    torch.cuda.synchronize()
    T_offline = time.perf_counter() - t0
    ctx = mk(rate)
    T_plain, tau_ref, T_roll, st = _learned_rollout_vs_plain(torch, ctx, m, U, q0, rate, rollout_steps)
    rom = pkg.Rom(ctx, U)
    pg = ctx.pod_project(U, q0)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    tau_gal = rom.run(pg, rollout_steps, 50)
    torch.cuda.synchronize()
    T_gal = time.perf_counter() - t3
    err = lambda t: float(np.linalg.norm(t - tau_ref) / np.linalg.norm(tau_ref))
    return {
        "workload": f"learned reduced step, 4-bead chain P={P}, R={R} (input {3 * R + 1}, width 128, SiLU), "
                    f"{n_runs} training runs x {run_steps} explicit steps at shear rates log-uniform [0.1, 10] "
                    f"({pairs} pairs; basis from the snapshots of the first {n_snap_runs} runs), {epochs} epochs of "
                    f"batch 64 at lr {LEARNED_LR:g} falling to {LEARNED_LR_FINAL:g} (half cosine), input noise {LEARNED_INPUT_NOISE} increment standard deviations; rollout "
                    f"{rollout_steps} steps at the held-out rate {rate}, checked every 50 steps (increment residual "
                    f"<= 0.2, energy-law gap <= 0.5)",
        "offline_s": T_offline, "final_loss": float(losses[-1]), "first_loss": float(losses[0]),
        "T_plain_s": T_plain, "T_rollout_s": T_roll, "speedup_vs_plain": T_plain / T_roll,
        "stress_rel_err_vs_plain": err(st["tau"]), "checks": st["checks"], "fallbacks": st["fallbacks"],
        "max_resid": st["max_resid"], "max_energy_gap": st["max_energy_gap"],
        "projection_floor_stress": st["projection_floor_stress"],
        "without_network_pod_galerkin": {"T_s": T_gal, "stress_rel_err_vs_plain": err(tau_gal),
                                         "speedup_vs_plain": T_plain / T_gal},
    }


def measure_learned_fene(pkg, wl, torch, n_runs, R, run_steps, epochs, rollout_steps):
    """The learned reduced step re-instantiated on the 6-bead FENE chain (D = 15,
    P = 50000): its own basis (R per bond), network and training runs at
    log-uniform shear rates in [0.3, 3], and a checked rollout at the held-out
    rate 1 against the plain scheme.  The POD-Galerkin model has no FENE form
    (its reduced spring term is exact only for linear springs), so the plain
    scheme is the method without the network here."""
    import math
    cfg = wl.fene_chain6()
    P, rate = cfg["P"], 1.0
    rates = wl.mlp_shear_rates(n_runs, log10_range=(math.log10(0.3), math.log10(3.0)))
    q0 = torch.from_numpy(wl.to_f32(cfg["q0"])).cuda()
    mk = lambda r: pkg.Context(5, P, cfg["h"], G=wl.shear_gradient(r), dt=cfg["dt"], scheme="explicit",
                               potential="fene", b_max=cfg["b_max"])
    t0 = time.perf_counter()
    U, m, pairs, losses = _train_learned(pkg, wl, torch, mk, q0, 5, R, rates, n_runs, run_steps, epochs)
    torch.cuda.synchronize()
    T_offline = time.perf_counter() - t0
    T_plain, tau_ref, T_roll, st = _learned_rollout_vs_plain(torch, mk(rate), m, U, q0, rate, rollout_steps)
    err = float(np.linalg.norm(st["tau"] - tau_ref) / np.linalg.norm(tau_ref))
    return {
        "workload": f"learned reduced step, 6-bead FENE chain P={P}, D=15, b_max={cfg['b_max']}, R={R} per bond "
                    f"(input {5 * R + 1}, width 128, SiLU), {n_runs} training runs x {run_steps} explicit steps at "
                    f"shear rates log-uniform [0.3, 3] ({pairs} pairs), {epochs} epochs of batch 64 at lr {LEARNED_LR:g} falling to {LEARNED_LR_FINAL:g}, input "
                    f"noise {LEARNED_INPUT_NOISE}; rollout {rollout_steps} steps at the held-out rate {rate}, checked "
                    f"every 50 steps (increment residual <= 0.2, energy-law gap <= 0.5)",
        "offline_s": T_offline, "final_loss": float(losses[-1]), "first_loss": float(losses[0]),
        "T_plain_s": T_plain, "T_rollout_s": T_roll, "speedup_vs_plain": T_plain / T_roll,
        "stress_rel_err_vs_plain": err, "checks": st["checks"], "fallbacks": st["fallbacks"],
        "max_resid": st["max_resid"], "max_energy_gap": st["max_energy_gap"],
        "projection_floor_stress": st["projection_floor_stress"],
    }


def measure_appendix_a(pkg, wl, torch):
    """Accuracy study of the reference dynamics (Appendix A) at the paper's
    settings: 4-bead chain, P = 1000, t = 6, dt in {1e-2 .. 5e-4} for both
    schemes, and P in {100 .. 5000} at dt = 1e-3; median-rule bandwidths."""
    from paper_2603_12550_amd import accuracy
    grid = torch.from_numpy(wl.to_f32(wl.density_grid(9))).cuda()
    t0 = time.perf_counter()
    res = accuracy.time_step_study(wl.appendix_a_chain4(P=1000), grid)
    res["particles"] = accuracy.particle_study(lambda P: wl.appendix_a_chain4(P=P, seed=30 + P), grid)
    res["seconds"] = time.perf_counter() - t0
    res["paper"] = {"dt_1e-3_error": "about 1e-4",
                    "explicit_vs_implicit_dt_5e-4": {"position_l2": 9.51e-5, "position_linf": 1.01e-4,
                                                     "density_l2": 1.17e-4, "density_linf": 1.80e-4,
                                                     "stress_fro": 9.56e-5},
                    "P_1000_vs_5000": "about 5-10 %"}
    return res


def measure_paper_tables(pkg, wl, torch):
    """Tables 1-6 (Sections 3.2, 3.3) at the paper's sizes: reference run,
    POD basis, and the POD-Galerkin run for every reduced rank, with
    T_mor / T_ref and err_MOR(t = 6) next to the paper's CPU values."""
    from paper_2603_12550_amd import tables
    out = {}
    for name in wl.PAPER_TABLES:
        case = wl.paper_table_case(name)
        out[name] = tables.run_table(case, wl.snapshot_steps(case["snapshots"], case["snap_until"]))
    return out


def measure_predictor(pkg, wl, torch, P, steps):
    """Implicit steps of the headline workload started from 2 q^n - q^(n-1)
    (picard_predictor = 1) against the default start from q^n: time per step,
    fixed-point iterations and the stress difference after the same steps."""
    cfg = wl.chain4_shear(P=P)
    q0 = torch.from_numpy(wl.to_f32(cfg["q0"])).cuda()
    out = {"workload": f"chain4_shear P={P}, {steps} implicit steps in one call, rtol 1e-6"}
    taus = {}
    for name, pred in (("from_q", 0), ("predictor", 1)):
        ctx = pkg.Context(3, P, cfg["h"], H=cfg["H"], G=cfg["G"], dt=cfg["dt"], scheme="implicit",
                          picard_rtol=1e-6, picard_max=50, picard_batch=3, picard_predictor=pred)
        ctx.step(q0.clone(), nsteps=3)
        q = q0.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        d = ctx.step(q, nsteps=steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        taus[name] = d["tau"]
        out[name] = {"ms_per_step": el * 1e3 / steps, "iterations_per_step": d["iters"] / steps,
                     "pair_evals_per_s": 2.0 * P * P * d["iters"] / el}
    out["stress_rel_diff"] = float(np.linalg.norm(taus["predictor"] - taus["from_q"]) / np.linalg.norm(taus["from_q"]))
    out["speedup"] = out["from_q"]["ms_per_step"] / out["predictor"]["ms_per_step"]
    return out


def measure_fene(pkg, wl, torch, steps):
    """6-bead FENE chain (D = 15), P = 50000, explicit steps of the plain scheme."""
    from paper_2603_12550_amd import _vds
    cfg = wl.fene_chain6()
    P = cfg["P"]
    ctx = pkg.Context(5, P, cfg["h"], G=cfg["G"], dt=cfg["dt"], scheme="explicit", potential="fene",
                      b_max=cfg["b_max"])
    q = torch.from_numpy(wl.to_f32(cfg["q0"])).cuda()
    tune = ctx.autotune(q)
    ctx.step(q, nsteps=2)
    ctx.timing_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.step(q, nsteps=steps)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    ms, n, work = _timer_rate(ctx, _vds.VDS_TIMER_PAIR)
    ctx.timing_enable(False)
    avg = ms / max(1, n)
    return {"workload": f"6-bead FENE chain, D=15, P={P}, b_max=50, explicit dt=1e-3, {steps} steps",
            "tuning": tune, "pair_evals_per_s": 2.0 * P * P * steps / T,
            "pair_kernel_avg_ms": avg,
            "pair_kernel_tflops": P * P * flops_per_pair(15) / (avg * 1e-3) / 1e12,
            "tau": ctx.stress(q).tolist()}


def _timed_steps(torch, ctx, q0, steps, warmup):
    """`warmup` untimed steps, then `steps` timed implicit steps with HIP events
    (no system fence) around every TIMING_STRIDE-th pair launch."""
    from paper_2603_12550_amd import _vds
    q = q0.clone()
    if warmup:
        ctx.step(q, nsteps=warmup)
    torch.cuda.synchronize()
    ctx.timing_enable(True, stride=TIMING_STRIDE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    d = ctx.step(q, nsteps=steps)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tim = ctx.timing_read(_vds.VDS_TIMER_PAIR)
    ctx.timing_enable(False)
    return d, elapsed, tim


def _pair_roofline(tune, P, D, iters, tim):
    avg_ms = tim["ms"] / max(1, tim["launches"])
    # every queued pair launch ran (none returned early past convergence), so
    # the sampled average is that of full passes
    all_ran = (2 * iters + TIMING_STRIDE - 1) // TIMING_STRIDE == tim["launches"]
    flop_launch = P * P * flops_per_pair(D)
    achieved = flop_launch / (avg_ms * 1e-3) / 1e12
    return avg_ms, all_ran, flop_launch, achieved


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--P", type=int, default=20000)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--tuning", type=str, default="",
                    help="impl,rows_per_wave,col_splits of the FP32 pair kernel (default: the library's default)")
    ap.add_argument("--fp16-tuning", type=str, default="3,2,8",
                    help="impl,rows_per_wave,col_splits of the FP16-split line ('' skips it)")
    ap.add_argument("--autotune", action="store_true", help="let the library's autotuner pick the pair shape")
    ap.add_argument("--no-t-end", action="store_true", help="skip the plain run to t_end (500 steps)")
    ap.add_argument("--copy-calibration", action="store_true", help="only run a plain copy of known size")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the POD-reduced, batched, learned and FENE measurements")
    ap.add_argument("--extras", type=str, default="", help="comma-separated subset of the extra measurements")
    ap.add_argument("--batched-steps", type=int, default=200)
    ap.add_argument("--learned-runs", type=int, default=334, help="training runs (300 steps each: 1e5 pairs)")
    ap.add_argument("--learned-snapshot-runs", type=int, default=48, help="runs whose snapshots make the basis")
    ap.add_argument("--learned-run-steps", type=int, default=300)
    ap.add_argument("--learned-epochs", type=int, default=60)
    ap.add_argument("--fene-learned-runs", type=int, default=48)
    ap.add_argument("--learned-seed", type=int, default=3, help="seed of the training order and input noise")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the particle rows would shard by block with an all-gather of S between passes).",
              file=sys.stderr)
        sys.exit(2)

    if args.copy_calibration:
        copy_calibration()
        return

    import torch
    import paper_2603_12550_amd as pkg
    import workloads as wl

    torch.cuda.set_device(0)
    cfg = wl.chain4_shear(P=args.P)
    P, D = cfg["P"], 9
    mk = lambda: pkg.Context(3, P, cfg["h"], H=cfg["H"], G=cfg["G"], dt=cfg["dt"], scheme="implicit",
                             picard_rtol=1e-6, picard_max=50, picard_batch=3)
    q0 = torch.from_numpy(wl.to_f32(cfg["q0"])).cuda()

    # the FP16-split pair form: a different arithmetic, reported on its own line
    if args.fp16_tuning:
        c16 = mk()
        c16.set_tuning(*[int(v) for v in args.fp16_tuning.split(",")])
        t16 = c16.get_tuning()
        d16, el16, tim16 = _timed_steps(torch, c16, q0, args.steps, args.warmup)
        avg16, ran16, _, ach16 = _pair_roofline(t16, P, D, d16["iters"], tim16)
        sec16 = secondary_ceilings(t16["impl"], D, P * P / (avg16 * 1e-3))
        print(json.dumps(_compact({
            "line": "fp16_split_pair_form", "dtype": "fp16 hi/lo split, ~22-bit",
            "arithmetic": PAIR_ARITHMETIC[t16["impl"]], "tuning": t16,
            "value": 2.0 * P * P * d16["iters"] / el16, "unit": "pair-evals/s", "ms_per_step": el16 * 1e3 / args.steps,
            "pair_kernel": PAIR_KERNEL[t16["impl"]], "pair_avg_launch_ms": avg16, "all_timed_launches_ran": ran16,
            "algorithmic_fp32_tflops": ach16,
            "fp16_mfma": {"peak_tflops": PEAK_FP16_TFLOPS, **sec16["issued_mfma"]},
            "exp_unit_frac": sec16["exp_unit"]["frac"]})), flush=True)
        del c16

    ctx = mk()
    if args.autotune:
        ctx.autotune(q0)
    elif args.tuning:
        ctx.set_tuning(*[int(v) for v in args.tuning.split(",")])
    tune = ctx.get_tuning()
    if tune["impl"] not in (0, 1, 4):
        print("bench.py: the headline runs an FP32 pair form (impl 0, 1 or 4)", file=sys.stderr)
        sys.exit(2)
    d, elapsed, tim = _timed_steps(torch, ctx, q0, args.steps, args.warmup)
    iters = d["iters"]
    avg_ms, all_ran, flop_launch, achieved = _pair_roofline(tune, P, D, iters, tim)
    sec = secondary_ceilings(tune["impl"], D, P * P / (avg_ms * 1e-3))

    # plain GPU VDS to t_end (the configuration's 500 steps), same context
    t_end = None
    if not args.no_t_end:
        qt = q0.clone()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dte = ctx.step(qt, nsteps=cfg["steps"])
        torch.cuda.synchronize()
        t_end = {"steps": cfg["steps"], "s": time.perf_counter() - t1, "iters": dte["iters"]}

    extras = {}
    if not args.no_extras:
        for name, fn in (("pod_reduced", lambda: measure_pod_rom(pkg, wl, torch, P)),
                         ("batched", lambda: measure_batched(pkg, wl, torch, args.batched_steps)),
                         ("learned", lambda: measure_learned(pkg, wl, torch, P, args.learned_runs,
                                                            args.learned_snapshot_runs, args.learned_run_steps,
                                                            args.learned_epochs, 300, args.learned_seed)),
                         ("learned_fene", lambda: measure_learned_fene(pkg, wl, torch, args.fene_learned_runs, 108,
                                                                       300, 200, 300)),
                         ("implicit_predictor", lambda: measure_predictor(pkg, wl, torch, P, 100)),
                         ("fene_chain6", lambda: measure_fene(pkg, wl, torch, 20)),
                         ("appendix_a", lambda: measure_appendix_a(pkg, wl, torch)),
                         ("paper_tables", lambda: measure_paper_tables(pkg, wl, torch))):
            if args.extras and name not in args.extras.split(","):
                continue
            t0 = time.perf_counter()
            extras[name] = fn()
            print(json.dumps(_compact({"extra": name, "seconds": time.perf_counter() - t0, **extras[name]})),
                  flush=True)

    out = {
        "metric": "kernel pair-evals/s (% FP32 peak); wall time to t_end vs plain VDS at <=1e-2 stress err",
        "value": 2.0 * P * P * iters / elapsed,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic: 4-bead chain bonds drawn N(0, I/3), seed 2",
        "config": {"workload": f"4-bead Hookean chain P={P} D=9 h=0.4 shear 1, implicit Euler dt=1e-3, "
                               f"fixed-point rtol 1e-6",
                   "pair_arithmetic": PAIR_ARITHMETIC[tune["impl"]],
                   "tuning": [tune["impl"], tune["rows_per_wave"], tune["col_splits"]],
                   "iters_per_step": iters / max(1, args.steps)},
        "roofline": {"bound": "mfma", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_FP32_TFLOPS,
                     "traffic": measured_traffic(PAIR_KERNEL[tune["impl"]], tune, P),
                     "kernel": PAIR_KERNEL[tune["impl"]], "avg_launch_ms": avg_ms, "launches": tim["launches"],
                     "all_timed_launches_ran": bool(all_ran), "flop_per_pair": flops_per_pair(D),
                     "issued_mfma_frac": sec.get("issued_mfma", {}).get("frac"),
                     "exp_unit_frac": sec["exp_unit"]["frac"]},
        "t_end": t_end,
    }
    vs = {}
    if "pod_reduced" in extras:
        e = extras["pod_reduced"]
        vs["pod_rom"] = {"time_ratio": e["T_rom_over_T_ref"], "stress_err": e["stress_rel_err_vs_plain"]}
        best = pod_best_within(e, 1e-2)
        if best is not None:
            vs["pod_rom_within_1e-2"] = best
    if "batched" in extras:
        e = extras["batched"]
        vs["batched"] = {"speedup": e["speedup_vs_plain_single"], "stress_err": e["max_stress_rel_err_vs_plain_at_t_end"]}
    if "learned" in extras:
        e = extras["learned"]
        vs["learned"] = {"speedup": e["speedup_vs_plain"], "stress_err": e["stress_rel_err_vs_plain"]}
    if vs:
        out["vs_plain_at_t_end"] = vs
    if not args.no_cpu:
        threads = min(16, len(os.sched_getaffinity(0)))
        out["cpu_baseline"] = cpu_baseline(cfg, threads)
    print(json.dumps(_compact(out)), flush=True)


if __name__ == "__main__":
    main()
