"""Gradients of eigenpairs with respect to the stored values of A (B = I).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

First-order perturbation theory of a symmetric matrix with simple eigenvalues:
  d lambda_i = x_i^T dA x_i,
  d x_i = sum_{j != i} x_j (x_j^T dA x_i) / (lambda_i - lambda_j).
For a loss L(lambda, X) with adjoints lambda_bar, X_bar this gives
  dL = sum_i lambda_bar_i x_i^T dA x_i + sum_i y_i^T dA x_i,
  y_i = -sum_{j != i} x_j (x_j^T xbar_i) / (lambda_j - lambda_i).
For a symmetric perturbation of the stored pair (r, c), (c, r) the gradient is
  g_rc = sum_i lambda_bar_i x_i(r) x_i(c) + 1/2 sum_i (y_i(r) x_i(c) + x_i(r) y_i(c)).

dense_gradient() uses every eigenvector (full eigh, small n).  The large-n
form splits y_i into the part inside the computed block X (a k x k sum) and the
part outside it, which solves the projected shifted system
  (I - X X^T)(A - lambda_i I)(I - X X^T) z_i = -(I - X X^T) xbar_i,  z_i _|_ X,
by conjugate gradients (block_adjoint()).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def gradient_on_pattern(A, X, lam_bar, Y):
    """g over the stored nonzeros of CSR A (same order as A.data / A.indices)."""
    A = sp.csr_matrix(A)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    cols = A.indices
    g = np.zeros(A.nnz)
    for i in range(X.shape[1]):
        g += lam_bar[i] * X[rows, i] * X[cols, i]
        g += 0.5 * (Y[rows, i] * X[cols, i] + X[rows, i] * Y[cols, i])
    return g


def dense_gradient(A, k, lam_bar, X_bar):
    """Reference gradient from a full eigendecomposition of dense A (n small).

    Eigenvector signs follow numpy's eigh; the gradient is sign-invariant when
    the loss is (X_bar then flips with x_i).  Returns (g, lam, X) with g on the
    stored pattern of A.
    """
    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    lam_all, V = np.linalg.eigh(Ad)
    n = Ad.shape[0]
    X = V[:, :k]
    Y = np.zeros((n, k))
    for i in range(k):
        c = V.T @ X_bar(X)[:, i] if callable(X_bar) else V.T @ X_bar[:, i]
        denom = lam_all - lam_all[i]
        coef = np.zeros(n)
        mask = np.arange(n) != i
        coef[mask] = c[mask] / denom[mask]
        Y[:, i] = -V @ coef
    return gradient_on_pattern(A, X, lam_bar, Y), lam_all[:k], X


def in_block_part(lam, X, X_bar):
    """y_i^in = -sum_{j != i, j <= k} x_j (x_j^T xbar_i) / (lambda_j - lambda_i)."""
    k = X.shape[1]
    G = X.T @ X_bar  # G[j, i] = x_j^T xbar_i
    coef = np.zeros((k, k))
    for i in range(k):
        for j in range(k):
            if j != i:
                coef[j, i] = -G[j, i] / (lam[j] - lam[i])
    return X @ coef


def projected_cg(A, X, lam, rhs, tol=1e-12, maxit=5000):
    """Solve (I-XX^T)(A - lam_i I)(I-XX^T) z_i = rhs_i, z_i _|_ X, column by column.

    Plain conjugate gradients (Hestenes-Stiefel) on each column, started from
    zero, stopped when ||r_i|| <= tol * ||rhs_i||.  rhs must already be
    orthogonal to X.
    """
    A = sp.csr_matrix(A)
    proj = lambda V: V - X @ (X.T @ V)
    n, k = rhs.shape
    Z = np.zeros((n, k))
    iters = np.zeros(k, dtype=int)
    for i in range(k):
        b = rhs[:, i]
        bn = np.linalg.norm(b)
        if bn == 0.0:
            continue
        z = np.zeros(n)
        r = b.copy()
        p = r.copy()
        rr = r @ r
        for it in range(maxit):
            Ap = proj(A @ p - lam[i] * p)
            alpha = rr / (p @ Ap)
            z += alpha * p
            r -= alpha * Ap
            rr_new = r @ r
            iters[i] = it + 1
            if np.sqrt(rr_new) <= tol * bn:
                break
            p = r + (rr_new / rr) * p
            rr = rr_new
        Z[:, i] = proj(z)
    return Z, iters


def block_adjoint(A, lam, X, lam_bar, X_bar, tol=1e-12, maxit=5000):
    """Gradient on the pattern of A from the k computed eigenpairs (lam, X)."""
    Yin = in_block_part(lam, X, X_bar)
    rhs = -(X_bar - X @ (X.T @ X_bar))
    Yout, iters = projected_cg(A, X, lam, rhs, tol=tol, maxit=maxit)
    return gradient_on_pattern(A, X, lam_bar, Yin + Yout), iters
