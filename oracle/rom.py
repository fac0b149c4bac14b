"""FP64 oracle of the POD-Galerkin reduced model (Section 2.4).  TEST
INFRASTRUCTURE ONLY; shares nothing with the GPU library.

Two independent evaluations of the reduced operators are given:

* `operators_literal` writes the paper's index sums for X^H, X^B1 and X^B2 out
  term by term (uniform weights, as in the paper); it is O(P^2 R^2 d) and meant
  for P d <= a few hundred.
* `operators` is the same algebra regrouped into products of P x R mode blocks
  U_alpha (rows (I, alpha) of U) with the kernel matrix Z, valid for any
  positive weights; with uniform weights it equals the literal sums (a test
  checks this), and it is what larger cases use.

Between freezes the reduced state follows eq. model_DymReduced with explicit
Euler (Section 3.1), or, in `rom_run_windows` (a variant beyond the paper), the
exact solution of that linear equation over each window.  The freeze reading: at steps 0, M, 2M, ... reconstruct
q~ = U p, rebuild X^B1, X^B2 from the kernel matrix at q~ with h fixed, and keep
p; X^H is built once.
"""
from __future__ import annotations

import numpy as np

from . import pod, vds


def mode_blocks(U: np.ndarray, P: int, d: int = 3) -> np.ndarray:
    """U_alpha in R^{P x R}: rows (I, alpha) of U, stacked as Ua[alpha][I][s]."""
    R = U.shape[1]
    return np.ascontiguousarray(U.reshape(P, d, R).transpose(1, 0, 2))


def hydro_literal(U: np.ndarray, G: np.ndarray, P: int, d: int = 3) -> np.ndarray:
    """X^H_st = sum_I sum_{alpha,beta} U_{(I alpha) s} G_{alpha beta} U_{(I beta) t}."""
    R = U.shape[1]
    XH = np.zeros((R, R))
    for I in range(P):
        for a in range(d):
            for b in range(d):
                if G[a, b] != 0.0:
                    XH += G[a, b] * np.outer(U[I * d + a], U[I * d + b])
    return XH


def brownian_literal(U: np.ndarray, qt: np.ndarray, h: float):
    """X^B1, X^B2 by the paper's sums with Z_IK = K_h(q~_I - q~_K) and
    Y_{IK alpha t} = U_{(I alpha) t} - U_{(K alpha) t} (uniform weights)."""
    nb, P, d = qt.shape
    R = U.shape[1]
    x = vds.particle_major(qt)
    diff = x[:, None, :] - x[None, :, :]
    Z = np.exp(-(diff * diff).sum(-1) / (2.0 * h * h))
    rowsum = Z.sum(1)       # sum_J Z_IJ
    colsum = Z.sum(0)       # sum_J Z_JK
    XB1 = np.zeros((R, R))
    XB2 = np.zeros((R, R))
    for I in range(P):
        for a in range(d):
            us = U[I * d + a]                       # U_{(I alpha) s}
            for K in range(P):
                y = U[I * d + a] - U[K * d + a]     # Y_{IK alpha t}
                XB1 += np.outer(us, Z[I, K] * y / rowsum[I])
                XB2 += np.outer(us, Z[I, K] * y / colsum[K])
    return -XB1 / h ** 2, -XB2 / h ** 2


def operators_literal(U: np.ndarray, qt: np.ndarray, prob: vds.Problem):
    P = qt.shape[1]
    XH = hydro_literal(U, prob.G, P, prob.d)
    XB1, XB2 = brownian_literal(U, qt, prob.h)
    return XH, XB1, XB2


def hydro(U: np.ndarray, G: np.ndarray, P: int, d: int = 3) -> np.ndarray:
    """X^H = sum_{alpha,beta} G_{alpha beta} U_alpha^T U_beta."""
    Ua = mode_blocks(U, P, d)
    return sum(G[a, b] * Ua[a].T @ Ua[b] for a in range(d) for b in range(d))


def brownian(U: np.ndarray, qt: np.ndarray, w: np.ndarray, h: float):
    """Weighted X^B1, X^B2 regrouped:
    X^B1 = -(1/h^2) sum_a [U_a^T U_a - U_a^T diag(1/S) Z diag(w) U_a]
    X^B2 = -(1/h^2) sum_a [U_a^T diag(T) U_a - U_a^T Z diag(w/S) U_a]
    with S = Z w and T = Z (w/S)."""
    nb, P, d = qt.shape
    x = vds.particle_major(qt)
    diff = x[:, None, :] - x[None, :, :]
    Z = np.exp(-(diff * diff).sum(-1) / (2.0 * h * h))
    S = Z @ w
    T = Z @ (w / S)
    Ua = mode_blocks(U, P, d)
    XB1 = np.zeros((U.shape[1],) * 2)
    XB2 = np.zeros_like(XB1)
    for a in range(d):
        XB1 += Ua[a].T @ Ua[a] - Ua[a].T @ ((Z @ (w[:, None] * Ua[a])) / S[:, None])
        XB2 += Ua[a].T @ (T[:, None] * Ua[a]) - Ua[a].T @ (Z @ ((w / S)[:, None] * Ua[a]))
    return -XB1 / h ** 2, -XB2 / h ** 2


def brownian_rows(U: np.ndarray, qt: np.ndarray, w: np.ndarray, h: float, block: int = 256,
                  threads: int = 1):
    """`brownian` with the kernel matrix formed one block of rows at a time, for
    sizes where Z (P x P) does not fit in memory: the same sums, grouped by row
    blocks.  S = Z w and T = Z (w/S) are row sums; the terms of X^B1 and X^B2
    are sums over rows I of U_a[I]^T (row-I quantities), so each row block
    contributes its share and the shares are added in block order."""
    from concurrent.futures import ThreadPoolExecutor
    nb, P, d = qt.shape
    R = U.shape[1]
    x = vds.particle_major(qt)
    Ua = mode_blocks(U, P, d)
    blocks = [(lo, min(P, lo + block)) for lo in range(0, P, block)]

    def zrows(lo, hi):
        # |x_I - x_J|^2 by direct differences, one component at a time
        r2 = np.zeros((hi - lo, P))
        for a in range(x.shape[1]):
            diff = x[lo:hi, a, None] - x[None, :, a]
            r2 += diff * diff
        return np.exp(-r2 / (2.0 * h * h))

    def pmap(fn):
        if threads > 1:
            # one BLAS thread per worker: the workers already fill the cores
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1, user_api="blas"), ThreadPoolExecutor(threads) as ex:
                return list(ex.map(fn, blocks))
        return [fn(b) for b in blocks]

    S = np.concatenate(pmap(lambda b: zrows(*b) @ w))
    T = np.concatenate(pmap(lambda b: zrows(*b) @ (w / S)))
    wU = [w[:, None] * Ua[a] for a in range(d)]
    wsU = [(w / S)[:, None] * Ua[a] for a in range(d)]

    def share(b):
        lo, hi = b
        Z = zrows(lo, hi)
        X1 = np.zeros((R, R))
        X2 = np.zeros((R, R))
        for a in range(d):
            Ub = Ua[a][lo:hi]
            X1 += Ub.T @ Ub - Ub.T @ ((Z @ wU[a]) / S[lo:hi, None])
            X2 += Ub.T @ (T[lo:hi, None] * Ub) - Ub.T @ (Z @ wsU[a])
        return X1, X2

    XB1 = np.zeros((R, R))
    XB2 = np.zeros((R, R))
    for X1, X2 in pmap(share):
        XB1 += X1
        XB2 += X2
    return -XB1 / h ** 2, -XB2 / h ** 2


def reduced_rhs(p: np.ndarray, XH: np.ndarray, XB: np.ndarray, prob: vds.Problem) -> np.ndarray:
    """Right side of eq. model_DymReduced for p[k][s]:
    dp_k/dt = X^H p_k - (1/zeta)[k_B T sum_j A_kj (X^B1 + X^B2) p_j + sum_j H_j A_kj p_j]."""
    A = vds.rouse_matrix(prob.nb)
    return (p @ XH.T - (prob.kT / prob.zeta) * (A @ (p @ XB.T))
            - (A @ (prob.H[:, None] * p)) / prob.zeta)


def rom_run(U: np.ndarray, q0: np.ndarray, w: np.ndarray, prob: vds.Problem, steps: int,
            freeze_every: int, callback=None, midpoint=False):
    """Reduced explicit Euler from p(0) = U^T q(0) with the freeze schedule
    above.  `callback(step, p)` sees every reduced state.  Returns p(steps).

    With `midpoint` (an addition, not in the paper) the operators of a window
    of n steps are rebuilt at the state predicted for its midpoint: n // 2
    steps from the window's start with the start's operators (none when
    n = 1), then the window is taken from its start with the new operators.
    With `midpoint="extrapolated"` (also an addition) every window after the
    first takes its operators at the midpoint state extrapolated on the line
    through the previous window's start state and its own, i.e.
    p + (n // 2) / n_prev (p - p_prev) for a previous window of n_prev steps;
    the first window predicts as with `midpoint`."""
    if prob.potential != "hookean":
        raise ValueError("the reduced spring term is exact only for Hookean springs")
    extrapolated = midpoint == "extrapolated"
    nb, P, d = q0.shape
    p = pod.project(U, q0)
    XH = hydro(U, prob.G, P, d)

    def operators_at(pp):
        XB1, XB2 = brownian(U, pod.reconstruct(U, pp, P, d), w, prob.h)
        return XB1 + XB2

    XB = None
    p_prev, n_prev = None, 0
    for s in range(steps):
        if s % freeze_every == 0:
            n = min(freeze_every, steps - s)
            half = n // 2
            if extrapolated and n_prev > 0 and half > 0:
                XB = operators_at(p + (half / n_prev) * (p - p_prev))
            else:
                XB = operators_at(p)
                if midpoint and half > 0:
                    pm = p
                    for _ in range(half):
                        pm = pm + prob.dt * reduced_rhs(pm, XH, XB, prob)
                    XB = operators_at(pm)
            if extrapolated:
                p_prev, n_prev = p, n
        p = p + prob.dt * reduced_rhs(p, XH, XB, prob)
        if callback is not None:
            callback(s + 1, p)
    return p


def reduced_generator(XH: np.ndarray, XB: np.ndarray, prob: vds.Problem, R: int) -> np.ndarray:
    """Matrix of the linear map p -> reduced_rhs(p) on vec(p) (index k R + s),
    assembled column by column from unit states."""
    n = prob.nb * R
    L = np.empty((n, n))
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        L[:, i] = reduced_rhs(e.reshape(prob.nb, R), XH, XB, prob).reshape(-1)
    return L


def rom_run_windows(U: np.ndarray, q0: np.ndarray, w: np.ndarray, prob: vds.Problem, windows) -> np.ndarray:
    """The reduced model integrated exactly between freezes: for each window of
    length dt_w (times, in order) freeze at the current p as above, then
    p <- exp(dt_w L) p with L the constant generator of eq. model_DymReduced over
    the window (matrix exponential by scipy).  Returns p at the end."""
    from scipy.linalg import expm
    if prob.potential != "hookean":
        raise ValueError("the reduced spring term is exact only for Hookean springs")
    nb, P, d = q0.shape
    p = pod.project(U, q0)
    R = p.shape[1]
    XH = hydro(U, prob.G, P, d)
    for dtw in windows:
        qt = pod.reconstruct(U, p, P, d)
        XB1, XB2 = brownian(U, qt, w, prob.h)
        L = reduced_generator(XH, XB1 + XB2, prob, R)
        p = (expm(dtw * L) @ p.reshape(-1)).reshape(nb, R)
    return p


def reduced_stress(U: np.ndarray, p: np.ndarray, w: np.ndarray, prob: vds.Problem, P: int) -> np.ndarray:
    """Stress of the reconstructed state q~ = U p (plain definition)."""
    return vds.stress(pod.reconstruct(U, p, P, prob.d), w, prob)
