"""FP64 oracle of the POD offline phase and the POD maps.  TEST INFRASTRUCTURE
ONLY; shares nothing with the GPU library.

The basis comes from the singular value decomposition of the snapshot matrix
itself (Section 1.3: POD is the best rank-R approximation, equivalently the SVD
of X), which is a different route from the GPU's Gram matrix plus symmetric
eigensolve, so the two check each other.
"""
from __future__ import annotations

import numpy as np


def snapshot_matrix(states) -> np.ndarray:
    """X in R^{Pd x (L+1)(N-1)}: column (l, k) is the bond-k slice q_{k:}(t_l)
    flattened over (I, alpha) (Section 3.1).  `states` is a sequence of
    [nb][P][d] arrays; columns are ordered snapshot-major, bond-minor."""
    cols = []
    for q in states:
        for k in range(q.shape[0]):
            cols.append(np.asarray(q[k], dtype=np.float64).reshape(-1))
    return np.stack(cols, axis=1)


def pod_basis(X: np.ndarray, R: int):
    """U = first R left singular vectors of X; returns (U, lambda) where
    lambda_i = sigma_i^2 are the eigenvalues of X X^T (and of X^T X)."""
    Uh, sig, _ = np.linalg.svd(X, full_matrices=False)
    return Uh[:, :R], sig ** 2


def remaining_energy(lam: np.ndarray) -> np.ndarray:
    """1 - sum_{j<=i} lambda_j / sum_all lambda (Section 3.3, eigenvalue figure)."""
    lam = np.asarray(lam, dtype=np.float64)
    return 1.0 - np.cumsum(lam) / lam.sum()


def project(U: np.ndarray, q: np.ndarray) -> np.ndarray:
    """p_{k:} = U^T q_{k:} for every bond (eq. model_pq)."""
    nb = q.shape[0]
    return np.stack([U.T @ q[k].reshape(-1) for k in range(nb)])


def reconstruct(U: np.ndarray, p: np.ndarray, P: int, d: int = 3) -> np.ndarray:
    """q~_{k:} = U p_{k:} (eq. model_pq), returned as [nb][P][d]."""
    return np.stack([(U @ p[k]).reshape(P, d) for k in range(p.shape[0])])


def subspace_distance(U1: np.ndarray, U2: np.ndarray) -> float:
    """Spectral norm of U1 U1^T - U2 U2^T for orthonormal column sets of equal
    size: the sine of the largest principal angle, ||(I - U1 U1^T) U2||_2."""
    E = U2 - U1 @ (U1.T @ U2)
    return float(np.linalg.norm(E, 2)) if E.size else 0.0
