"""Pins of the adjoint oracle: dense reference vs finite differences, and the
block projected solve vs the dense reference."""

import numpy as np
import scipy.sparse as sp

from oracle import adjoint as ADJ
from paper_1704_07458_amd import problems as P


def _loss_parts(seed, n, k):
    rng = np.random.default_rng(seed + 2000)
    w = rng.uniform(0.0, 1.0, k)
    m = rng.uniform(0.0, 1.0, n)
    return w, m


def _loss(lam, X, w, m):
    # sum_i w_i lambda_i + sum_i ||x_i o m||^2   (sign-invariant in x_i)
    return float(w @ lam + np.sum((X * m[:, None]) ** 2))


def _grads(lam, X, w, m):
    return w.copy(), 2.0 * X * (m ** 2)[:, None]


def test_dense_gradient_matches_central_differences():
    L = P.laplacian_3d(4)
    V = P.potential(0, L.n, 0.0, 4.0)
    A = P.add_diagonal(L, V).to_scipy()
    n, k = A.shape[0], 5
    w, m = _loss_parts(0, n, k)
    lam0, V0 = np.linalg.eigh(A.toarray())
    lb, xb = _grads(lam0[:k], V0[:, :k], w, m)
    g, _, _ = ADJ.dense_gradient(A, k, lb, xb)
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    cols = A.indices
    rng = np.random.default_rng(1)
    picks = rng.choice(A.nnz, 25, replace=False)
    h = 1e-5
    for p in picks:
        r, c = rows[p], cols[p]
        E = sp.lil_matrix(A.shape)
        if r == c:
            E[r, c] = 1.0
        else:
            E[r, c] = 0.5
            E[c, r] = 0.5
        vals = []
        for sgn in (1.0, -1.0):
            lam, Vv = np.linalg.eigh((A + sgn * h * E).toarray())
            vals.append(_loss(lam[:k], Vv[:, :k], w, m))
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(fd - g[p]) <= 1e-6 * max(1.0, abs(fd)), (p, fd, g[p])


def test_block_adjoint_matches_dense_reference_8cubed():
    L = P.laplacian_3d(8)
    V = P.potential(0, L.n, 0.0, 4.0)
    A = P.add_diagonal(L, V).to_scipy()
    n, k = A.shape[0], 16
    w, m = _loss_parts(0, n, k)
    lam, Vd = np.linalg.eigh(A.toarray())
    X = Vd[:, :k]
    lb, xb = _grads(lam[:k], X, w, m)
    g_ref, _, _ = ADJ.dense_gradient(A, k, lb, xb)
    g_blk, iters = ADJ.block_adjoint(A, lam[:k], X, lb, xb, tol=1e-13)
    assert np.linalg.norm(g_blk - g_ref) <= 1e-9 * np.linalg.norm(g_ref)
    assert iters.max() < 5000


def test_eigenvalue_part_is_x_dA_x():
    """With X_bar = 0 the gradient is sum_i lambda_bar_i x_i(r) x_i(c)."""
    A = P.laplacian_2d_dirichlet(6).to_scipy()
    n, k = A.shape[0], 3
    lam, Vd = np.linalg.eigh(A.toarray())
    lb = np.array([1.0, 0.0, 0.0])
    g, _, _ = ADJ.dense_gradient(A, k, lb, np.zeros((n, k)))
    x = Vd[:, 0]
    dense = np.outer(x, x)
    rows = np.repeat(np.arange(n), np.diff(A.indptr))
    assert np.allclose(g, dense[rows, A.indices], atol=1e-14)
    # the diagonal entries sum to ||x_1||^2 = 1: d lambda_1 / d(shift) = 1
    diag = rows == A.indices
    assert abs(g[diag].sum() - 1.0) < 1e-13


# ------------------------------------------------------- generalised pencil (B != I)
def _random_pencil(N, seed):
    """Q1 stiffness + random diagonal and mass + random diagonal on N^3: a
    symmetric-definite pencil with distinct eigenvalues (the plain tensor-product
    pencil has degenerate ones, where eigenvector derivatives are not defined)."""
    K, M = P.fem_q1_pencil(N)
    K, M = K.to_scipy(), M.to_scipy()
    rng = np.random.default_rng(seed)
    n = K.shape[0]
    A = (K + sp.diags(rng.uniform(0.0, 4.0, n) * K.diagonal().mean())).tocsr()
    B = (M + sp.diags(rng.uniform(0.0, 1.0, n) * M.diagonal().mean())).tocsr()
    A.sort_indices()
    B.sort_indices()
    return A, B


def _sym_unit(shape, r, c):
    E = sp.lil_matrix(shape)
    if r == c:
        E[r, c] = 1.0
    else:
        E[r, c] = 0.5
        E[c, r] = 0.5
    return E


def test_generalized_dense_gradient_matches_central_differences():
    import scipy.linalg as sla

    A, B = _random_pencil(4, 3)
    n, k = A.shape[0], 5
    w, m = _loss_parts(1, n, k)
    gA, gB, lam0, X0 = ADJ.dense_gradient_generalized(A, B, k, w, lambda X: 2.0 * X * (m ** 2)[:, None])
    rng = np.random.default_rng(4)
    for M_, g, name in ((A, gA, "A"), (B, gB, "B")):
        rows = np.repeat(np.arange(n), np.diff(M_.indptr))
        cols = M_.indices
        h = 1e-6 * abs(M_.data).max()
        for p in rng.choice(M_.nnz, 15, replace=False):
            E = _sym_unit(M_.shape, rows[p], cols[p])
            vals = []
            for sgn in (1.0, -1.0):
                Ap = (A + sgn * h * E) if name == "A" else A
                Bp = (B + sgn * h * E) if name == "B" else B
                lam, V = sla.eigh(Ap.toarray(), Bp.toarray())
                vals.append(_loss(lam[:k], V[:, :k], w, m))
            fd = (vals[0] - vals[1]) / (2 * h)
            scale = max(abs(fd), 1e-3 * np.abs(g).max())
            assert abs(fd - g[p]) <= 1e-5 * scale, (name, p, fd, g[p])


def test_generalized_gradient_euler_identities():
    """Homogeneity pins of the B term's signs: lambda(cA, B) = c lambda and X(cA, B) = X;
    lambda(A, cB) = lambda / c and X(A, cB) = X / sqrt(c).  Euler's theorem then gives
    sum_p gA_p A_p = sum_i lbar_i lambda_i and
    sum_p gB_p B_p = -sum_i lbar_i lambda_i - 1/2 sum_i xbar_i^T x_i."""
    A, B = _random_pencil(4, 5)
    n, k = A.shape[0], 6
    w, m = _loss_parts(2, n, k)
    xb_fn = lambda X: 2.0 * X * (m ** 2)[:, None]
    gA, gB, lam, X = ADJ.dense_gradient_generalized(A, B, k, w, xb_fn)
    xb = xb_fn(X)
    assert abs(gA @ A.data - w @ lam) <= 1e-10 * abs(w @ lam)
    expect = -(w @ lam) - 0.5 * np.sum(xb * X)
    assert abs(gB @ B.data - expect) <= 1e-10 * abs(expect)


def test_generalized_gradient_with_identity_B_is_the_standard_one():
    L = P.laplacian_3d(4)
    A = P.add_diagonal(L, P.potential(0, L.n, 0.0, 4.0)).to_scipy()
    n, k = A.shape[0], 5
    w, m = _loss_parts(0, n, k)
    xb_fn = lambda X: 2.0 * X * (m ** 2)[:, None]
    I = sp.identity(n, format="csr")
    gA, _, lam, X = ADJ.dense_gradient_generalized(A, I, k, w, xb_fn)
    g, _, _ = ADJ.dense_gradient(A, k, w, xb_fn)
    assert np.allclose(gA, g, rtol=1e-9, atol=1e-12 * np.abs(g).max())


def test_block_adjoint_generalized_matches_dense_reference():
    A, B = _random_pencil(6, 7)
    n, k = A.shape[0], 8
    w, m = _loss_parts(3, n, k)
    xb_fn = lambda X: 2.0 * X * (m ** 2)[:, None]
    gA, gB, lam, X = ADJ.dense_gradient_generalized(A, B, k, w, xb_fn)
    bA, bB, iters = ADJ.block_adjoint_generalized(A, B, lam, X, w, xb_fn(X), tol=1e-14,
                                                  maxit=2000)
    assert np.linalg.norm(bA - gA) <= 1e-9 * np.linalg.norm(gA)
    assert np.linalg.norm(bB - gB) <= 1e-9 * np.linalg.norm(gB)
