"""Pins of the oracle's complex Hermitian form of Algorithm 8.

The paper states the method for real pencils and notes that it carries over to
complex Hermitian ones with conjugate transposes (section 1).  The oracle's
complex iteration is pinned by closed-form spectra of twisted periodic
Laplacians and of a complex tensor-product pencil (Fourier modes diagonalise
every factor), by brute force on small random pencils, and by an independent
formulation: the real iteration on the embedding [Re A, -Im A; Im A, Re A] from
the J-paired start [X0, i X0] spans the same spaces, so its Ritz values come in
pairs equal to the complex iteration's after every step.
"""

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from oracle import closed_forms as cf
from oracle import lobpcg as L
from paper_1704_07458_amd import problems as P


def _embed(M):
    M = M.to_scipy() if hasattr(M, "to_scipy") else sp.csr_matrix(M)
    return sp.bmat([[M.real, -M.imag], [M.imag, M.real]]).tocsr()


def _paired(X0):
    return np.hstack([np.vstack([X0.real, X0.imag]), np.vstack([-X0.imag, X0.real])])


@pytest.mark.parametrize("N", [3, 4, 5])
def test_twisted_closed_forms_match_dense_solves(N):
    A = P.twisted_laplacian_3d(N).to_scipy().toarray()
    assert np.abs(A.imag).max() > 0.1  # genuinely complex
    assert np.allclose(A, A.conj().T)
    assert np.allclose(np.linalg.eigvalsh(A), cf.twisted_laplacian_3d(N), atol=1e-12)
    Ap, Bp = P.twisted_pencil_3d(N)
    Ad, Bd = Ap.to_scipy().toarray(), Bp.to_scipy().toarray()
    assert np.linalg.eigvalsh(Bd).min() > 0.0
    assert np.allclose(sla.eigh(Ad, Bd, eigvals_only=True), cf.twisted_pencil_3d(N), atol=1e-12)


def _host_rho(A, B, lam, X, normA, normB):
    BX = X if B is None else B @ X
    R = A @ X - BX * lam[None, :]
    return np.linalg.norm(R, axis=0) / ((normA + np.abs(lam) * normB) * np.linalg.norm(X, axis=0))


def test_complex_standard_problem_reaches_the_closed_form():
    N, k = 8, 10
    A = P.twisted_laplacian_3d(N).to_scipy()
    X0 = P.complex_initial_block(0, A.shape[0], P.block_size(k))
    r = L.lobpcg(A, X0, k, 1e-10, precond=L.jacobi_precond(A))
    assert r.converged
    lam, X = r.eigenpairs(k)
    exact = cf.twisted_laplacian_3d(N)[:k]
    assert np.max(np.abs(lam - exact) / np.abs(exact)) < 1e-12
    assert np.abs(X.conj().T @ X - np.eye(k)).max() < 1e-12
    assert _host_rho(A, None, lam, X, r.normA, r.normB).max() <= 1e-10


def test_complex_generalized_pencil_reaches_the_closed_form():
    N, k = 8, 10
    Ap, Bp = P.twisted_pencil_3d(N)
    A, B = Ap.to_scipy(), Bp.to_scipy()
    X0 = P.complex_initial_block(1, A.shape[0], P.block_size(k))
    r = L.lobpcg(A, X0, k, 1e-10, B=B, precond=L.jacobi_precond(A))
    assert r.converged
    lam, X = r.eigenpairs(k)
    exact = cf.twisted_pencil_3d(N)[:k]
    assert np.max(np.abs(lam - exact) / np.abs(exact)) < 1e-12
    assert np.abs(X.conj().T @ (B @ X) - np.eye(k)).max() < 1e-12
    assert _host_rho(A, B, lam, X, r.normA, r.normB).max() <= 1e-10


def test_complex_brute_force_on_a_random_pencil():
    rng = np.random.default_rng(7)
    n, k = 150, 6
    M = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    M[np.abs(M) < 1.6] = 0.0  # sparse-ish
    A = 0.5 * (M + M.conj().T) + np.diag(np.linspace(0.0, 20.0, n))
    G = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
    G[np.abs(G) < 2.0] = 0.0
    B = 0.05 * (G @ G.conj().T) + np.eye(n)
    X0 = P.complex_initial_block(3, n, P.block_size(k))
    r = L.lobpcg(sp.csr_matrix(A), X0, k, 1e-11, B=sp.csr_matrix(B), maxit=3000)
    assert r.converged
    exact = sla.eigh(A, B, eigvals_only=True)[:k]
    assert np.max(np.abs(r.theta[:k] - exact) / np.abs(exact).max()) < 1e-10


@pytest.mark.parametrize("its", [1, 2, 5])
def test_real_embedding_iteration_pairs_the_complex_ritz_values(its):
    N, k = 6, 8
    nx = P.block_size(k)
    A = P.twisted_laplacian_3d(N)
    X0 = P.complex_initial_block(2, A.n, nx)
    rc = L.lobpcg(A.to_scipy(), X0, k, 1e-10, precond=L.jacobi_precond(A.to_scipy()), maxit=its)
    Ae = _embed(A)
    re = L.lobpcg(Ae, _paired(X0), 2 * k, 1e-10, precond=L.jacobi_precond(Ae), maxit=its)
    th = np.sort(re.theta)
    assert np.max(np.abs(th[0::2] - th[1::2])) < 1e-12  # exact pairs up to rounding
    assert np.max(np.abs(th[0::2] - rc.theta)) < 1e-12
    # the sketch of the complex pencil is the complex form of the embedding's
    assert abs(re.normA - rc.normA) < 1e-12 * rc.normA


def test_real_embedding_of_the_generalized_pencil_converges_alike():
    N, k = 6, 8
    Ap, Bp = P.twisted_pencil_3d(N)
    X0 = P.complex_initial_block(4, Ap.n, P.block_size(k))
    rc = L.lobpcg(Ap.to_scipy(), X0, k, 1e-10, B=Bp.to_scipy(),
                  precond=L.jacobi_precond(Ap.to_scipy()))
    Ae, Be = _embed(Ap), _embed(Bp)
    re = L.lobpcg(Ae, _paired(X0), 2 * k, 1e-10, B=Be, precond=L.jacobi_precond(Ae))
    assert rc.converged and re.converged
    th = np.sort(re.theta)[: 2 * k]
    assert np.max(np.abs(th[0::2] - rc.theta[:k])) < 1e-11
    assert abs(re.iterations - rc.iterations) <= max(2, rc.iterations // 10)
