"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and names parameter sets; it holds none
of the particle scheme's arithmetic.  Every array it returns is float64; the
GPU path receives the float32 cast and the oracle the same float32 values
promoted back to float64, so input rounding never counts as kernel error.

Parameter values follow the paper's experiment setup (Section 3.1): friction
zeta = 4, k_B T = 1, number density n = 1, Hookean springs H_k = 1 (or
H_k = k for the inhomogeneous chain), thermal-equilibrium Gaussian starts, and
simple shear whose only nonzero velocity-gradient entry drives q_1 by q_2.
"""
from __future__ import annotations

import numpy as np

D_SPACE = 3  # spatial dimension d (Section 2.1)


def shear_gradient(rate: float) -> np.ndarray:
    """G = (grad u)^T for simple shear: dq_1/dt gains rate * q_2."""
    G = np.zeros((3, 3))
    G[0, 1] = rate
    return G


def gaussian_bonds(seed: int, nb: int, P: int, var) -> np.ndarray:
    """q[k][I][alpha] ~ N(0, var_k), i.i.d. (Section 3.1 initial condition).

    `var` is a scalar or a per-bond sequence of variances.
    """
    rng = np.random.default_rng(seed)
    var = np.broadcast_to(np.asarray(var, dtype=np.float64), (nb,))
    q = rng.standard_normal((nb, P, D_SPACE))
    return q * np.sqrt(var)[:, None, None]


def truncated_gaussian_bonds(seed: int, nb: int, P: int, var: float, r2max: float) -> np.ndarray:
    """Gaussian bonds redrawn until every |q_k|^2 < r2max (FENE domain)."""
    rng = np.random.default_rng(seed)
    q = rng.standard_normal((nb, P, D_SPACE)) * np.sqrt(var)
    bad = (q * q).sum(-1) >= r2max
    while bad.any():
        q[bad] = rng.standard_normal((int(bad.sum()), D_SPACE)) * np.sqrt(var)
        bad = (q * q).sum(-1) >= r2max
    return q


def random_weights(seed: int, P: int) -> np.ndarray:
    """Positive weights summing to one (weighted-particle variant)."""
    rng = np.random.default_rng(seed)
    w = rng.uniform(0.5, 1.5, size=P)
    return w / w.sum()


def to_f32(a: np.ndarray) -> np.ndarray:
    """The float32 values both sides consume."""
    return np.ascontiguousarray(a, dtype=np.float32)


def f32_as_f64(a: np.ndarray) -> np.ndarray:
    return np.asarray(np.asarray(a, dtype=np.float32), dtype=np.float64)


# ---------------------------------------------------------------------------
# Named workloads.  Plain parameter records; both sides translate them into
# their own problem descriptions.
# ---------------------------------------------------------------------------

def dumbbell_shear(P: int = 2000, seed: int = 1, steps: int = 100):
    """3D Hookean dumbbell, N(0, I) start, shear rate 1 (Wi = 1), h = 0.3,
    implicit dt = 1e-3."""
    return dict(name=f"dumbbell_shear_P{P}", nb=1, P=P, kT=1.0, zeta=4.0, n=1.0,
                h=0.3, dt=1e-3, G=shear_gradient(1.0), H=np.ones(1),
                potential="hookean", b_max=0.0, scheme="implicit", steps=steps,
                q0=gaussian_bonds(seed, 1, P, 1.0))


def chain4_shear(P: int = 20000, seed: int = 2, steps: int = 500, inhomogeneous: bool = False):
    """4-bead Hookean chain (3 bonds, D = 9), N(0, I/3) per bond, shear rate 1,
    h = 0.4, implicit dt = 1e-3."""
    H = np.arange(1, 4, dtype=np.float64) if inhomogeneous else np.ones(3)
    return dict(name=f"chain4_shear_P{P}", nb=3, P=P, kT=1.0, zeta=4.0, n=1.0,
                h=0.4, dt=1e-3, G=shear_gradient(1.0), H=H,
                potential="hookean", b_max=0.0, scheme="implicit", steps=steps,
                q0=gaussian_bonds(seed, 3, P, 1.0 / 3.0))


def pod_chain4(P: int = 20000, seed: int = 2, ref_steps: int = 2000, snapshots: int = 300,
               snap_until: int = 1000, R: int = 180, rom_steps: int = 2000, freeze_every: int = 300):
    """POD-reduced 4-bead chain: the chain4_shear state run `ref_steps` as the
    reference, `snapshots` uniform snapshots over steps [0, snap_until]."""
    base = chain4_shear(P=P, seed=seed, steps=ref_steps)
    base.update(name=f"pod_chain4_P{P}_R{R}", snapshots=snapshots, snap_until=snap_until,
                R=R, rom_steps=rom_steps, freeze_every=freeze_every)
    return base


def snapshot_steps(snapshots: int, snap_until: int) -> np.ndarray:
    """Uniformly spaced integer step indices 0 = s_0 < ... < s_{L} = snap_until."""
    return np.unique(np.round(np.linspace(0, snap_until, snapshots)).astype(np.int64))


def ensembles(n_ens: int = 512, seed: int = 4, p_lo: int = 2000, p_hi: int = 16000,
              h_ref: float = 0.4, p_ref: int = 20000, D: int = 9):
    """Independent micro-macro ensembles of 4-bead chains.

    P_b ~ U{p_lo..p_hi}; shear rate log-uniform in [0.1, 10];
    h_b = h_ref * (P_b / p_ref)^(-1/(D+4)); q ~ N(0, I/3) with seed 1000*seed + b.
    """
    rng = np.random.default_rng(seed)
    P = rng.integers(p_lo, p_hi + 1, size=n_ens)
    rate = 10.0 ** rng.uniform(-1.0, 1.0, size=n_ens)
    h = h_ref * (P / p_ref) ** (-1.0 / (D + 4))
    return dict(name=f"ensembles_{n_ens}", n_ens=n_ens, P=P.astype(np.int64), rate=rate, h=h,
                nb=3, kT=1.0, zeta=4.0, n=1.0, dt=1e-3, H=np.ones(3), seed=seed)


def ensemble_state(ens: dict, b: int) -> np.ndarray:
    return gaussian_bonds(1000 * ens["seed"] + b, ens["nb"], int(ens["P"][b]), 1.0 / 3.0)


def fene_chain6(P: int = 50000, seed: int = 5, b_max: float = 50.0):
    """6-bead FENE chain (5 bonds, D = 15), shear rate 1, b_max = 50,
    h = 0.4 (P/20000)^(-1/19), start N(0, kT/H) truncated to the FENE domain."""
    h = 0.4 * (P / 20000.0) ** (-1.0 / 19.0)
    return dict(name=f"fene_chain6_P{P}", nb=5, P=P, kT=1.0, zeta=4.0, n=1.0, h=h, dt=1e-3,
                G=shear_gradient(1.0), H=np.ones(5), potential="fene", b_max=b_max,
                scheme="explicit", steps=200,
                q0=truncated_gaussian_bonds(seed, 5, P, 1.0, 0.9 * b_max))


def appendix_a_chain4(P: int = 1000, seed: int = 21, rate: float = 1.0):
    """Accuracy study of the reference dynamics (Appendix A): 4-bead Hookean
    chain in simple shear, thermal-equilibrium start N(0, kT/H) = N(0, I) per
    bond, zeta = 4, up to t = 6; the bandwidth follows the median rule of the
    initial state (computed by the caller)."""
    return dict(name=f"appendix_a_chain4_P{P}", nb=3, P=P, kT=1.0, zeta=4.0, n=1.0, dt=1e-3,
                G=shear_gradient(rate), H=np.ones(3), potential="hookean", b_max=0.0, t_end=6.0,
                q0=gaussian_bonds(seed, 3, P, 1.0))


# Tables 1-6 (Sections 3.2, 3.3): beads, P, flow, inhomogeneous springs, reduced ranks, and
# the paper's own T_mor / T_ref and err_MOR(t = 6) (in percent) on its CPU.
PAPER_TABLES = {
    "table1_noflow_2bead": dict(beads=2, P=1000, rate=0.0, H_k=False, R=(1, 2, 3, 4, 5, 10, 20, 40),
                                T_ref_s=394, time_pct=(0.360, 0.605, 0.819, 1.08, 1.43, 3.66, 11.8, 43.3),
                                err_pct=(4.76, 2.34, 1.04, 0.635, 0.595, 0.816, 0.843, 0.865)),
    "table2_noflow_3bead": dict(beads=3, P=1000, rate=0.0, H_k=False, R=(1, 2, 3, 4, 5, 10, 20, 40),
                                T_ref_s=533, time_pct=(0.441, 0.612, 0.758, 0.955, 1.23, 2.82, 8.90, 32.1),
                                err_pct=(70.8, 12.8, 7.50, 4.47, 2.72, 1.82, 1.98, 1.98)),
    "table3_shear_2bead": dict(beads=2, P=1000, rate=1.0, H_k=False, R=(10, 15, 20, 25, 30, 40),
                               T_ref_s=385, time_pct=(3.77, 7.31, 12.2, 18.4, 26.0, 44.9),
                               err_pct=(10.5, 9.47, 8.76, 8.41, 8.23, 8.08)),
    "table4_shear_4bead_P1000": dict(beads=4, P=1000, rate=1.0, H_k=False, R=(10, 15, 20, 25, 30, 40),
                                     T_ref_s=704, time_pct=(2.30, 4.24, 6.89, 10.3, 14.4, 24.8),
                                     err_pct=(12.5, 6.67, 5.67, 5.00, 4.42, 3.72)),
    "table5_shear_4bead_P10000": dict(beads=4, P=10000, rate=1.0, H_k=False, R=(10, 15, 20, 25, 30, 40),
                                      T_ref_s=70104, time_pct=(2.31, 4.30, 6.90, 10.5, 14.8, 25.4),
                                      err_pct=(13.2, 6.60, 5.99, 5.59, 5.41, 5.18)),
    "table6_shear_4bead_Hk": dict(beads=4, P=1000, rate=1.0, H_k=True, R=(10, 15, 20, 25, 30, 40),
                                  T_ref_s=673, time_pct=(2.39, 4.43, 7.20, 10.8, 15.1, 25.8),
                                  err_pct=(18.3, 11.1, 9.55, 8.36, 7.93, 7.02)),
}


def paper_table_case(name: str, seed: int = 40):
    """Setting of one of the paper's tables (Section 3.1): thermal-equilibrium
    start N(0, kT/H_k), zeta = 4, explicit dt = 1e-3 to t = 6, snapshots at
    L + 1 uniform times in [0, 3] with L = P d / (N - 1) capped at the 3000 steps
    available, freezes every 300 steps."""
    t = PAPER_TABLES[name]
    nb, P = t["beads"] - 1, t["P"]
    H = np.arange(1, nb + 1, dtype=np.float64) if t["H_k"] else np.ones(nb)
    L = min(P * D_SPACE // nb, 3000)
    return dict(name=name, nb=nb, P=P, kT=1.0, zeta=4.0, n=1.0, dt=1e-3, G=shear_gradient(t["rate"]), H=H,
                steps=6000, snap_until=3000, snapshots=L + 1, freeze_every=300, R=t["R"],
                q0=gaussian_bonds(seed, nb, P, 1.0 / H), paper=t)


def density_grid(D: int, values=(-2.0, 0.0, 2.0)) -> np.ndarray:
    """All points of values^D (Appendix A evaluates the density on {-2, 0, 2}^D)."""
    axes = np.meshgrid(*[np.asarray(values, dtype=np.float64)] * D, indexing="ij")
    return np.stack([a.reshape(-1) for a in axes], axis=1)


def mlp_shear_rates(n_runs: int, seed: int = 5, log10_range=(-1.0, 1.0)) -> np.ndarray:
    """Shear rates of the learned-model training runs, log-uniform in
    [10^lo, 10^hi] (default [0.1, 10])."""
    rng = np.random.default_rng(seed)
    return 10.0 ** rng.uniform(log10_range[0], log10_range[1], size=n_runs)


def mlp_init(seed: int, sizes) -> list:
    """He-uniform initial weights for an MLP with layer sizes `sizes`;
    returns [(W[out][in], b[out]), ...] in float64."""
    rng = np.random.default_rng(seed)
    layers = []
    for fan_in, fan_out in zip(sizes[:-1], sizes[1:]):
        lim = np.sqrt(6.0 / fan_in)
        layers.append((rng.uniform(-lim, lim, size=(fan_out, fan_in)), np.zeros(fan_out)))
    return layers
