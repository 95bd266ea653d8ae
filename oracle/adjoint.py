"""Gradients of eigenpairs with respect to the stored values of A (and of B).

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

Generalised pencil A x = lambda B x with X^T B X = I (the *_generalized
functions).  Perturbing (A, B) gives
  d lambda_i = x_i^T (dA - lambda_i dB) x_i,
  d x_i = sum_{j != i} x_j x_j^T (dA - lambda_i dB) x_i / (lambda_i - lambda_j)
          - 1/2 x_i (x_i^T dB x_i)        (the last term keeps x_i^T B x_i = 1),
so with the same y_i (now over B-orthonormal eigenvectors)
  dL = sum_i lambda_bar_i x_i^T (dA - lambda_i dB) x_i + sum_i y_i^T (dA - lambda_i dB) x_i
       - 1/2 sum_i (xbar_i^T x_i) x_i^T dB x_i,
i.e. the A gradient has the form above and the B gradient is
  g^B_rc = sum_i a_i x_i(r) x_i(c) + 1/2 sum_i b_i (y_i(r) x_i(c) + x_i(r) y_i(c)),
  a_i = -(lambda_bar_i lambda_i + 1/2 xbar_i^T x_i),  b_i = -lambda_i.
Outside the computed block y_i solves, with Pi = I - X X^T B (the B-orthogonal
projector onto the complement of span X),
  Pi^T (A - lambda_i B) Pi z_i = -Pi^T xbar_i,  y_i = Pi z_i,
because sum_{j > k} x_j x_j^T = B^-1 - X X^T.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def gradient_on_pattern(A, X, lam_bar, Y, ycoef=None):
    """g over the stored nonzeros of CSR A (same order as A.data / A.indices):
    g_rc = sum_i lam_bar_i x_i(r) x_i(c) + 1/2 sum_i ycoef_i (y_i(r) x_i(c) + x_i(r) y_i(c)),
    ycoef = 1 by default."""
    A = sp.csr_matrix(A)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    cols = A.indices
    g = np.zeros(A.nnz)
    for i in range(X.shape[1]):
        b = 1.0 if ycoef is None else ycoef[i]
        g += lam_bar[i] * X[rows, i] * X[cols, i]
        g += 0.5 * b * (Y[rows, i] * X[cols, i] + X[rows, i] * Y[cols, i])
    return g


def b_coefficients(lam, lam_bar, X, X_bar):
    """(a_i, b_i) of the B gradient: a_i = -(lambda_bar_i lambda_i + 1/2 xbar_i^T x_i),
    b_i = -lambda_i."""
    xx = np.einsum("ij,ij->j", X_bar, X) if X_bar is not None else np.zeros(len(lam))
    return -(lam_bar * lam + 0.5 * xx), -np.asarray(lam, dtype=np.float64)


def dense_gradient_generalized(A, B, k, lam_bar, X_bar):
    """Reference gradients (g_A, g_B) from a full generalised eigendecomposition of
    the dense pencil (n small); eigenvectors B-orthonormal.  Returns (gA, gB, lam, X)
    with gA on A's stored pattern and gB on B's."""
    import scipy.linalg as sla

    Ad = A.toarray() if sp.issparse(A) else np.asarray(A)
    Bd = B.toarray() if sp.issparse(B) else np.asarray(B)
    lam_all, V = sla.eigh(Ad, Bd)
    n = Ad.shape[0]
    X = V[:, :k]
    Xb = X_bar(X) if callable(X_bar) else X_bar
    Y = np.zeros((n, k))
    for i in range(k):
        c = V.T @ Xb[:, i]
        denom = lam_all - lam_all[i]
        coef = np.zeros(n)
        mask = np.arange(n) != i
        coef[mask] = c[mask] / denom[mask]
        Y[:, i] = -V @ coef
    lam = lam_all[:k]
    gA = gradient_on_pattern(A, X, lam_bar, Y)
    a, b = b_coefficients(lam, lam_bar, X, Xb)
    gB = gradient_on_pattern(B, X, a, Y, ycoef=b)
    return gA, gB, lam, X


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


def projected_cg_generalized(A, B, X, lam, rhs, tol=1e-12, maxit=5000):
    """Solve Pi^T (A - lam_i B) Pi z_i = rhs_i (Pi = I - X X^T B) column by column by
    plain conjugate gradients from zero; returns y_i = Pi z_i.  rhs must satisfy
    X^T rhs = 0 (it lies in the range of Pi^T)."""
    A = sp.csr_matrix(A)
    B = sp.csr_matrix(B)
    BX = B @ X
    Pi = lambda v: v - X @ (BX.T @ v)
    PiT = lambda v: v - BX @ (X.T @ v)
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
            q = Pi(p)
            Ap = PiT(A @ q - lam[i] * (B @ q))
            alpha = rr / (p @ Ap)
            z += alpha * p
            r -= alpha * Ap
            rr_new = r @ r
            iters[i] = it + 1
            if np.sqrt(rr_new) <= tol * bn:
                break
            p = r + (rr_new / rr) * p
            rr = rr_new
        Z[:, i] = Pi(z)
    return Z, iters


def block_adjoint_generalized(A, B, lam, X, lam_bar, X_bar, tol=1e-12, maxit=5000):
    """(g_A, g_B) from the k computed B-orthonormal eigenpairs (lam, X) of (A, B)."""
    B = sp.csr_matrix(B)
    Yin = in_block_part(lam, X, X_bar)
    rhs = -(X_bar - (B @ X) @ (X.T @ X_bar))
    Yout, iters = projected_cg_generalized(A, B, X, lam, rhs, tol=tol, maxit=maxit)
    Y = Yin + Yout
    gA = gradient_on_pattern(A, X, lam_bar, Y)
    a, b = b_coefficients(lam, lam_bar, X, X_bar)
    gB = gradient_on_pattern(B, X, a, Y, ycoef=b)
    return gA, gB, iters


def block_adjoint(A, lam, X, lam_bar, X_bar, tol=1e-12, maxit=5000):
    """Gradient on the pattern of A from the k computed eigenpairs (lam, X)."""
    Yin = in_block_part(lam, X, X_bar)
    rhs = -(X_bar - X @ (X.T @ X_bar))
    Yout, iters = projected_cg(A, X, lam, rhs, tol=tol, maxit=maxit)
    return gradient_on_pattern(A, X, lam_bar, Yin + Yout), iters
