"""Accuracy study of the reference dynamics (Appendix A) on the GPU path:
time-step and particle-number convergence of the particle scheme, measured by
the relative position, density and stress errors the appendix defines.  Every
computation is a call into libvds (steps, stress, density at the grid points,
the median-rule bandwidth); this module only orders the calls and forms the
norms of the differences.
"""
from __future__ import annotations

import math

import numpy as np
import torch

from ._vds import Context


def _rel(a: np.ndarray, b: np.ndarray, ord_):
    a, b = np.asarray(a, np.float64).ravel(), np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b, ord_) / np.linalg.norm(b, ord_))


def run_to_end(cfg: dict, q0: torch.Tensor, h: float, dt: float, scheme: str, grid: torch.Tensor):
    """Runs the chain of `cfg` from q0 to t_end with step dt; returns the final
    state (host FP64), the density at the grid points and the stress."""
    nsteps = int(round(cfg["t_end"] / dt))
    ctx = Context(cfg["nb"], cfg["P"], h, H=cfg["H"], G=cfg["G"], dt=dt, scheme=scheme, kT=cfg["kT"],
                  zeta=cfg["zeta"], n=cfg["n"])
    q = q0.clone()
    ctx.step(q, nsteps=nsteps)
    f = ctx.density_at(q, grid).cpu().numpy().astype(np.float64)
    tau = ctx.stress(q)
    return q.cpu().numpy().astype(np.float64), f, tau


def errors(a, b) -> dict:
    """Appendix A's relative errors of run a against the benchmark run b
    (each (q, f, tau)); positions only when both have the same particles."""
    out = {}
    if a[0].shape == b[0].shape:
        out["position_l2"] = _rel(a[0], b[0], 2)
        out["position_linf"] = _rel(a[0], b[0], np.inf)
    out["density_l2"] = _rel(a[1], b[1], 2)
    out["density_linf"] = float(np.max(np.abs(a[1] - b[1])) / np.max(np.abs(b[1])))
    out["stress_fro"] = _rel(a[2], b[2], 2)
    return out


def median_h(cfg: dict, q0: torch.Tensor) -> float:
    ctx = Context(cfg["nb"], cfg["P"], 1.0, H=cfg["H"], G=cfg["G"], dt=cfg["dt"])
    return ctx.median_bandwidth(q0)[1]


def time_step_study(cfg: dict, grid: torch.Tensor, dts=(1e-2, 5e-3, 2e-3, 1e-3, 5e-4), schemes=("explicit", "implicit")):
    """Errors of each dt against the smallest one, per scheme, and of the two
    schemes against each other at the smallest dt."""
    q0 = torch.from_numpy(np.ascontiguousarray(cfg["q0"], dtype=np.float32)).cuda()
    h = median_h(cfg, q0)
    dt0 = min(dts)
    res = {"h": h, "P": cfg["P"], "t_end": cfg["t_end"], "dts": list(dts)}
    bench = {}
    for scheme in schemes:
        runs = {dt: run_to_end(cfg, q0, h, dt, scheme, grid) for dt in dts}
        bench[scheme] = runs[dt0]
        res[scheme] = {f"{dt:g}": errors(runs[dt], runs[dt0]) for dt in dts if dt != dt0}
    if len(schemes) == 2:
        res["explicit_vs_implicit"] = errors(bench[schemes[0]], bench[schemes[1]])
    return res


def particle_study(make_cfg, grid: torch.Tensor, Ps=(100, 200, 500, 1000, 5000), dt=1e-3, scheme="explicit"):
    """Density and stress errors of each P against the largest one; each P
    draws its own initial sample and median-rule bandwidth."""
    P0 = max(Ps)
    runs = {}
    for P in Ps:
        cfg = make_cfg(P)
        q0 = torch.from_numpy(np.ascontiguousarray(cfg["q0"], dtype=np.float32)).cuda()
        runs[P] = run_to_end(cfg, q0, median_h(cfg, q0), dt, scheme, grid)
    return {"P0": P0, "dt": dt, **{str(P): errors(runs[P], runs[P0]) for P in Ps if P != P0}}
