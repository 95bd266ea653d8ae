"""Brute-force symmetric eigensolver for small dense matrices (n <= 200).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Cyclic-by-row Jacobi (Golub and Van Loan, Matrix Computations, section 8.5):
sweep over all (p, q) with p < q and annihilate a_pq with a plane rotation until
the off-diagonal Frobenius norm is below tol * ||A||_F.  It shares nothing with
LAPACK's eigh, so it pins the oracle's Rayleigh-Ritz independently.
"""

from __future__ import annotations

import numpy as np


def jacobi_eigh(A: np.ndarray, tol: float = 1e-15, max_sweeps: int = 60):
    """Eigenvalues (ascending) and orthonormal eigenvectors of symmetric A."""
    A = np.array(A, dtype=np.float64, copy=True)
    n = A.shape[0]
    V = np.eye(n)
    fro = np.linalg.norm(A)
    if fro == 0.0:
        return np.zeros(n), V
    for _sweep in range(max_sweeps):
        off = np.sqrt(max(np.sum(A * A) - np.sum(np.diag(A) ** 2), 0.0))
        if off <= tol * fro:
            break
        for p in range(n - 1):
            for q in range(p + 1, n):
                apq = A[p, q]
                if apq == 0.0:
                    continue
                # Symmetric Schur decomposition of the 2x2 block (GVL Alg. 8.5.1).
                tau = (A[q, q] - A[p, p]) / (2.0 * apq)
                t = (1.0 if tau >= 0 else -1.0) / (abs(tau) + np.sqrt(1.0 + tau * tau))
                c = 1.0 / np.sqrt(1.0 + t * t)
                s = t * c
                # A <- J^T A J with J = rotation in the (p, q) plane.
                ap, aq = A[:, p].copy(), A[:, q].copy()
                A[:, p] = c * ap - s * aq
                A[:, q] = s * ap + c * aq
                ap, aq = A[p, :].copy(), A[q, :].copy()
                A[p, :] = c * ap - s * aq
                A[q, :] = s * ap + c * aq
                A[p, q] = A[q, p] = 0.0
                vp, vq = V[:, p].copy(), V[:, q].copy()
                V[:, p] = c * vp - s * vq
                V[:, q] = s * vp + c * vq
    w = np.diag(A).copy()
    order = np.argsort(w)
    return w[order], V[:, order]


def jacobi_eigh_pencil(A: np.ndarray, B: np.ndarray, **kw):
    """Generalised problem A x = lambda B x via B = L L^T and L^-1 A L^-T."""
    L = np.linalg.cholesky(B)
    Li = np.linalg.inv(L)
    w, Y = jacobi_eigh(Li @ A @ Li.T, **kw)
    return w, Li.T @ Y
