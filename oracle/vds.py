"""FP64 oracle of the VDS particle scheme.  TEST INFRASTRUCTURE ONLY (see the
package docstring): the GPU library neither imports nor links this.

State layout follows the paper's bond-major index k(I alpha) (Section 2.2):
q has shape [nb][P][d], bond k, particle I, spatial component alpha.  The
particle-major view x[I] = (q_{1,I}, ..., q_{nb,I}) in R^D, D = nb*d, is the
point the Gaussian blob kernel acts on.

Weights: the paper uses the uniform empirical measure 1/P (eq. model_DeteParAppr).
The weighted form used here comes from the blob energy
Phi_w = sum_K w_K log sum_J w_J K_h(x_K - x_J); its scaled gradient
(1/w_I) dPhi_w/dx_I is exactly the bracket of eq. model_DymRepPar when every
w_I = 1/P, because the kernel's normalisation and a common weight cancel in both
ratios.
"""
from __future__ import annotations

import math
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    """Physical and numerical parameters (Sections 2.1, 2.2 and 3.1)."""
    nb: int                      # bonds N-1
    h: float                     # kernel bandwidth
    dt: float = 1e-3
    kT: float = 1.0              # k_B T
    zeta: float = 4.0            # friction
    n: float = 1.0               # polymer number density in the stress
    G: np.ndarray = field(default_factory=lambda: np.zeros((3, 3)))  # (grad u)^T
    H: np.ndarray | None = None  # spring constants H_j, default ones
    potential: str = "hookean"   # or "fene" (Bird et al. force law, not in the paper)
    b_max: float = 0.0           # FENE extensibility
    d: int = 3

    def __post_init__(self):
        self.G = np.asarray(self.G, dtype=np.float64).reshape(3, 3)
        self.H = np.ones(self.nb) if self.H is None else np.asarray(self.H, dtype=np.float64)

    @property
    def D(self) -> int:
        return self.nb * self.d


def problem_from(cfg: dict) -> Problem:
    return Problem(nb=cfg["nb"], h=cfg["h"], dt=cfg["dt"], kT=cfg["kT"], zeta=cfg["zeta"],
                   n=cfg["n"], G=cfg["G"], H=cfg["H"], potential=cfg["potential"],
                   b_max=cfg["b_max"])


# ---------------------------------------------------------------------------
# Model pieces (Section 2.1)
# ---------------------------------------------------------------------------

def rouse_matrix(nb: int) -> np.ndarray:
    """A_jk = 2 [j = k] - [|j - k| = 1]."""
    A = np.zeros((nb, nb))
    for j in range(nb):
        for k in range(nb):
            if j == k:
                A[j, k] = 2.0
            elif abs(j - k) == 1:
                A[j, k] = -1.0
    return A


def grad_potential(q: np.ndarray, prob: Problem) -> np.ndarray:
    """grad_{q_j} Psi for every bond: Hookean H_j q_j (eq. model_Hookean);
    FENE H_j q_j / (1 - |q_j|^2 / b_max)."""
    Hq = prob.H[:, None, None] * q
    if prob.potential == "hookean":
        return Hq
    r2 = (q * q).sum(-1, keepdims=True)
    return Hq / (1.0 - r2 / prob.b_max)


def potential(q: np.ndarray, prob: Problem) -> np.ndarray:
    """Psi(q_I) per particle, summed over bonds."""
    r2 = (q * q).sum(-1)                                  # [nb][P]
    if prob.potential == "hookean":
        psi = 0.5 * prob.H[:, None] * r2
    else:
        psi = -0.5 * prob.H[:, None] * prob.b_max * np.log(1.0 - r2 / prob.b_max)
    return psi.sum(0)


def particle_major(q: np.ndarray) -> np.ndarray:
    """[nb][P][d] -> x[P][nb*d]."""
    nb, P, d = q.shape
    return np.ascontiguousarray(q.transpose(1, 0, 2).reshape(P, nb * d))


def bond_major(x: np.ndarray, nb: int, d: int = 3) -> np.ndarray:
    P = x.shape[0]
    return np.ascontiguousarray(x.reshape(P, nb, d).transpose(1, 0, 2))


def uniform_weights(P: int) -> np.ndarray:
    return np.full(P, 1.0 / P)


# ---------------------------------------------------------------------------
# Kernel sums (eq. model_DeteParAppr, the Gaussian K_h, eq. model_DymRepPar)
# ---------------------------------------------------------------------------

def _row_blocks(nrows: int, ncols: int, D: int):
    B = max(1, min(nrows, int(6e6 // max(1, ncols * D))))
    return [(s, min(nrows, s + B)) for s in range(0, nrows, B)]


def _weighted_sums(xr: np.ndarray, xc: np.ndarray, wc: np.ndarray, h: float, threads: int):
    """For each row point y: s(y) = sum_J wc_J exp(-|y - xc_J|^2 / 2h^2) and
    a(y) = sum_J wc_J exp(...) (y - xc_J), by direct differences."""
    D = xr.shape[1]
    s = np.empty(xr.shape[0])
    a = np.empty_like(xr)

    def work(blk):
        lo, hi = blk
        diff = xr[lo:hi, None, :] - xc[None, :, :]           # y - x_J
        r2 = (diff * diff).sum(-1)
        kw = np.exp(-r2 / (2.0 * h * h)) * wc[None, :]
        s[lo:hi] = kw.sum(1)
        a[lo:hi] = np.einsum("ij,ijd->id", kw, diff)

    blocks = _row_blocks(xr.shape[0], xc.shape[0], D)
    if threads > 1 and len(blocks) > 1:
        with ThreadPoolExecutor(threads) as ex:
            list(ex.map(work, blocks))
    else:
        for b in blocks:
            work(b)
    return s, a


def density_sums(x: np.ndarray, w: np.ndarray, h: float, rows=None, threads: int = 1) -> np.ndarray:
    """S_I = sum_J w_J exp(-|x_I - x_J|^2 / 2h^2), the unnormalised mollified
    density at the particles (J = I included)."""
    xr = x if rows is None else x[rows]
    s, _ = _weighted_sums(xr, x, w, h, threads)
    return s


def brownian_terms(x: np.ndarray, w: np.ndarray, h: float, rows=None, S_all=None, threads: int = 1):
    """The two kernel terms of eq. model_DymRepPar (weighted form).

    term1_I = sum_J w_J grad K_h(x_I - x_J) / sum_J w_J K_h(x_I - x_J)
    term2_I = sum_K (w_K / S_K) grad K_h(x_I - x_K),   S_K = sum_J w_J K_h(x_K - x_J)

    with grad K_h(y) = -(y / h^2) K_h(y); the normalisation of K_h cancels.
    Returns (S[rows], term1[rows], term2[rows]).  Pass B needs S at every
    particle, computed here unless `S_all` is given.
    """
    xr = x if rows is None else x[rows]
    s_r, a1 = _weighted_sums(xr, x, w, h, threads)
    if S_all is None:
        S_all = s_r if rows is None else density_sums(x, w, h, threads=threads)
    _, a2 = _weighted_sums(xr, x, w / S_all, h, threads)
    term1 = -a1 / (h * h * s_r[:, None])
    term2 = -a2 / (h * h)
    return s_r, term1, term2


def blob_energy(x: np.ndarray, w: np.ndarray, h: float) -> float:
    """Phi_w = sum_K w_K log sum_J w_J K(x_K - x_J) (unnormalised kernel)."""
    return float((w * np.log(density_sums(x, w, h))).sum())


# ---------------------------------------------------------------------------
# Drift, velocity and time stepping (eq. model_DymRepPar, Appendix A)
# ---------------------------------------------------------------------------

def thermo_force(q: np.ndarray, w: np.ndarray, prob: Problem, threads: int = 1):
    """g_{j,I} = k_B T (term1 + term2)_{j,I} + grad_{q_j} Psi(q_I), plus S."""
    x = particle_major(q)
    S, t1, t2 = brownian_terms(x, w, prob.h, threads=threads)
    b = bond_major(t1 + t2, prob.nb, prob.d)
    return prob.kT * b + grad_potential(q, prob), S


def flow_term(q: np.ndarray, prob: Problem) -> np.ndarray:
    """(G q_{k,I}) for every bond and particle."""
    return np.einsum("ab,kib->kia", prob.G, q)


def rouse_apply(A: np.ndarray, g: np.ndarray) -> np.ndarray:
    """(A (x) I_d) g: sum_j A_kj g_{j,I}."""
    return np.einsum("kj,jia->kia", A, g)


def velocity(q: np.ndarray, w: np.ndarray, prob: Problem, threads: int = 1) -> np.ndarray:
    """dq_{k,I}/dt = G q_{k,I} - (1/zeta) sum_j A_kj [k_B T b_{j,I} + grad_j Psi(q_I)]
    (eq. model_DymRepPar with the convection term dropped, Section 3.1)."""
    g, _ = thermo_force(q, w, prob, threads)
    return flow_term(q, prob) - rouse_apply(rouse_matrix(prob.nb), g) / prob.zeta


def step_explicit(q: np.ndarray, w: np.ndarray, prob: Problem, threads: int = 1) -> np.ndarray:
    """First-order explicit Euler (Appendix A): q+ = q + dt v(q)."""
    return q + prob.dt * velocity(q, w, prob, threads)


def step_implicit(q: np.ndarray, w: np.ndarray, prob: Problem, rtol: float = 1e-13,
                  max_iter: int = 200, threads: int = 1):
    """First-order implicit Euler of Appendix A: flow term at t, kernel and
    potential terms at t+:  q+ = q* + dt u(q+),  q* = q + dt G q,
    u(x) = -(1/zeta)(A (x) I)(k_B T b(x) + grad Psi(x)).

    The paper solves this "by iteration" without naming one; this takes plain
    fixed-point (Picard) iteration from x0 = q, stopping when
    max|x_{m+1} - x_m| <= rtol * max(1, max|x_{m+1}|).
    Returns (q+, iterations)."""
    A = rouse_matrix(prob.nb)
    qstar = q + prob.dt * flow_term(q, prob)
    x = q.copy()
    for m in range(1, max_iter + 1):
        g, _ = thermo_force(x, w, prob, threads)
        xn = qstar - prob.dt * rouse_apply(A, g) / prob.zeta
        delta = np.abs(xn - x).max()
        x = xn
        if delta <= rtol * max(1.0, np.abs(x).max()):
            return x, m
    raise RuntimeError("Picard iteration did not converge")


def run(q: np.ndarray, w: np.ndarray, prob: Problem, steps: int, scheme: str = "implicit",
        threads: int = 1, callback=None):
    """Advance `steps` steps; `callback(step, q)` sees every state."""
    iters = []
    for s in range(steps):
        if scheme == "explicit":
            q = step_explicit(q, w, prob, threads)
        else:
            q, m = step_implicit(q, w, prob, threads=threads)
            iters.append(m)
        if callback is not None:
            callback(s + 1, q)
    return q, iters


# ---------------------------------------------------------------------------
# Observables (Sections 2.1 and 3.1, Appendix A; energy law from the blob energy)
# ---------------------------------------------------------------------------

def stress(q: np.ndarray, w: np.ndarray, prob: Problem) -> np.ndarray:
    """tau = n sum_I w_I sum_j q_{j,I} (x) grad Psi_j(q_{j,I})  (3x3); no
    isotropic part is subtracted, so equilibrium gives n (N-1) k_B T Id."""
    gp = grad_potential(q, prob)
    return prob.n * np.einsum("i,kia,kib->ab", w, q, gp)


def free_energy(q: np.ndarray, w: np.ndarray, prob: Problem, threads: int = 1) -> float:
    """F_h = sum_I w_I [k_B T log f_h(q_I) + Psi(q_I)],
    f_h(q_I) = (2 pi h^2)^(-D/2) sum_J w_J exp(-|q_I - q_J|^2 / 2h^2)."""
    S = density_sums(particle_major(q), w, prob.h, threads=threads)
    logf = np.log(S) - 0.5 * prob.D * math.log(2.0 * math.pi * prob.h ** 2)
    return float((w * (prob.kT * logf + potential(q, prob))).sum())


def dissipation_and_work(q: np.ndarray, w: np.ndarray, prob: Problem, threads: int = 1):
    """Dissipation (1/zeta) sum_I w_I g_I^T (A (x) I) g_I and flow work
    sum_I w_I g_I . (G q_I), so that dF_h/dt = work - dissipation."""
    g, _ = thermo_force(q, w, prob, threads)
    A = rouse_matrix(prob.nb)
    Ag = rouse_apply(A, g)
    diss = float(np.einsum("i,kia,kia->", w, g, Ag)) / prob.zeta
    work = float(np.einsum("i,kia,kia->", w, g, flow_term(q, prob)))
    return diss, work


def density_at(points: np.ndarray, q: np.ndarray, w: np.ndarray, h: float) -> np.ndarray:
    """f_h(y) = sum_I w_I K_h(y - q_I) at foreign points y[J][D] (Appendix A)."""
    x = particle_major(q)
    s, _ = _weighted_sums(np.asarray(points, dtype=np.float64), x, w, h, 1)
    return s * (2.0 * math.pi * h * h) ** (-0.5 * x.shape[1])


def median_bandwidth(q: np.ndarray) -> float:
    """h = med / sqrt(2 log P), med over all ordered pairs (J, K), J = K
    included (eq. model_bandwidth)."""
    x = particle_major(q)
    P = x.shape[0]
    diff = x[:, None, :] - x[None, :, :]
    dist = np.sqrt((diff * diff).sum(-1)).ravel()
    return float(np.median(dist) / math.sqrt(2.0 * math.log(P)))
