"""The paper's POD-MOR experiments (Sections 3.2, 3.3, Tables 1-6) at the
paper's sizes on the GPU path: one reference run of the particle scheme
collecting snapshots, the POD basis, and for every reduced rank R the
POD-Galerkin run with its wall time against the reference run's and the
relative L2 position error at t = 6.  Every computation is a call into libvds;
this module only orders the calls, times them and forms the error norms.
"""
from __future__ import annotations

import time

import numpy as np
import torch

from ._vds import Context, Rom


def _sync():
    torch.cuda.synchronize()


def run_table(case: dict, snapshot_steps) -> dict:
    """case: a setting from workloads.paper_table_case; snapshot_steps: the
    step indices of the snapshots (uniform over [0, snap_until])."""
    nb, P = case["nb"], case["P"]
    m = 3 * P
    q0 = torch.from_numpy(np.ascontiguousarray(case["q0"], dtype=np.float32)).cuda()
    # median-rule bandwidth of the initial state (eq. model_bandwidth), then fixed
    probe = Context(nb, P, 1.0, H=case["H"], G=case["G"], dt=case["dt"], scheme="explicit")
    med, h = probe.median_bandwidth(q0)
    ctx = Context(nb, P, h, H=case["H"], G=case["G"], dt=case["dt"], scheme="explicit", kT=case["kT"],
                  zeta=case["zeta"], n=case["n"])
    # reference run: timed without snapshots, then repeated collecting them
    q = q0.clone()
    ctx.step(q.clone(), nsteps=2)
    _sync()
    t0 = time.perf_counter()
    ctx.step(q, nsteps=case["steps"])
    _sync()
    T_ref = time.perf_counter() - t0
    q_ref = q
    snaps = [int(s) for s in snapshot_steps]
    X = torch.empty((len(snaps) * nb, m), dtype=torch.float32, device="cuda")
    qs, done = q0.clone(), 0
    for li, s in enumerate(snaps):
        if s > done:
            ctx.step(qs, nsteps=s - done)
            done = s
        X[nb * li:nb * li + nb].copy_(qs.reshape(nb, m))
    Rmax = max(case["R"])
    _sync()
    t1 = time.perf_counter()
    U_all, eig = ctx.pod_basis(X, Rmax)
    _sync()
    T_pod = time.perf_counter() - t1
    lam = np.clip(np.asarray(eig), 0.0, None)
    rows = []
    for R in case["R"]:
        U = U_all[:R].contiguous()
        rom = Rom(ctx, U)
        p = ctx.pod_project(U, q0)
        rom.run(p.clone(), 300, 300)  # warm-up
        _sync()
        t2 = time.perf_counter()
        rom.run(p, case["steps"], case["freeze_every"])
        _sync()
        T_mor = time.perf_counter() - t2
        q_mor = ctx.pod_reconstruct(U, p)
        err = float((q_mor - q_ref).norm() / q_ref.norm())
        rows.append({"R": R, "T_mor_s": T_mor, "T_mor_over_T_ref": T_mor / T_ref, "err_mor_t6": err,
                     "remaining_energy": float(lam[R:].sum() / lam.sum())})
    paper = case["paper"]
    return {"beads": nb + 1, "P": P, "h": h, "median": med, "snapshots": len(snaps), "T_ref_s": T_ref,
            "T_pod_s": T_pod, "rows": rows,
            "paper": {"T_ref_s": paper["T_ref_s"], "time_pct": list(paper["time_pct"]),
                      "err_pct": list(paper["err_pct"])}}
