"""Complex Hermitian pencils on the GPU (lobpcg_create_hermitian and friends)
against the oracle's complex Algorithm 8 and the closed-form spectra of the
twisted periodic Laplacian and the complex tensor-product pencil."""

import numpy as np
import pytest

from oracle import closed_forms as cf
from oracle import lobpcg as L
from paper_1704_07458_amd import problems as P

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    assert torch.cuda.is_available()
    return torch


def _solver(A, k, B=None, **opts):
    from paper_1704_07458_amd import binding as Bd

    return Bd.HermitianSolver(A, k, B=B, **opts)


def _host_rho(A, B, lam, X, normA, normB):
    BX = X if B is None else B @ X
    R = A @ X - BX * lam[None, :]
    return np.linalg.norm(R, axis=0) / ((normA + np.abs(lam) * normB) * np.linalg.norm(X, axis=0))


def _sin_angle(X, Y):
    """sin of the largest principal angle between span(X) and span(Y), both with
    orthonormal columns: ||(I - Y Y^H) X||_2."""
    return np.linalg.norm(X - Y @ (Y.conj().T @ X), 2)


def _case(kind, N, k, seed):
    if kind == "std":
        A = P.twisted_laplacian_3d(N)
        Bm, exact = None, cf.twisted_laplacian_3d(N)[:k]
    else:
        A, Bm = P.twisted_pencil_3d(N)
        exact = cf.twisted_pencil_3d(N)[:k]
    X0 = P.complex_initial_block(seed, A.n, P.block_size(k))
    return A, Bm, exact, X0


@pytest.mark.parametrize("kind,N,k", [("std", 8, 10), ("std", 7, 5), ("gen", 8, 10)])
def test_hermitian_matches_the_oracle_and_the_closed_form(kind, N, k):
    _torch()
    A, Bm, exact, X0 = _case(kind, N, k, seed=11)
    As = A.to_scipy()
    Bs = Bm.to_scipy() if Bm is not None else None
    print(f"case {kind} N={N} k={k}", flush=True)
    s = _solver(A, k, B=Bm, precond="jacobi")
    info = s.solve(1e-10, X0)
    assert info["converged"], info
    lam, X, rho = s.eigpairs(k)
    lam, X, rho = lam.cpu().numpy(), X.cpu().numpy(), rho.cpu().numpy()
    ref = L.lobpcg(As, X0, k, 1e-10, B=Bs, precond=L.jacobi_precond(As))
    assert ref.converged
    # the embedding's sketch is the oracle's complex sketch (reading R17)
    assert abs(info["norm_A_est"] - ref.normA) <= 1e-12 * ref.normA
    assert abs(info["norm_B_est"] - ref.normB) <= 1e-12 * ref.normB
    err_cf = np.max(np.abs(lam - exact) / np.abs(exact))
    err_or = np.max(np.abs(lam - ref.theta[:k]) / np.abs(ref.theta[:k]))
    print(f"  GPU iterations {info['iterations']}, oracle {ref.iterations}; eigenvalue error vs "
          f"closed form {err_cf:.2e}, vs oracle {err_or:.2e}")
    assert err_cf <= 1e-10 and err_or <= 1e-10
    assert abs(info["iterations"] - ref.iterations) <= max(2, ref.iterations // 10)
    G = X.conj().T @ (X if Bs is None else Bs @ X)
    assert np.abs(G - np.eye(k)).max() <= 1e-10
    host = _host_rho(As, Bs, lam, X, ref.normA, ref.normB)
    assert host.max() <= 1e-10 * 1.01
    assert np.allclose(rho, _host_rho(As, Bs, lam, X, info["norm_A_est"], info["norm_B_est"]),
                       rtol=1e-6, atol=1e-15)


def test_hermitian_subspace_matches_the_oracle():
    _torch()
    N, k = 8, 10
    A, _, _, X0 = _case("std", N, k, seed=12)
    As = A.to_scipy()
    s = _solver(A, k, precond="jacobi")
    assert s.solve(1e-12, X0)["converged"]
    _, X, _ = s.eigpairs(k)
    X = X.cpu().numpy()
    ref = L.lobpcg(As, X0, k, 1e-12, precond=L.jacobi_precond(As))
    Y = ref.X[:, :k]
    sin = _sin_angle(X, Y)
    print(f"sin of the largest principal angle {sin:.2e}")
    assert sin <= 1e-7


@pytest.mark.parametrize("its", [1, 2, 5])
def test_hermitian_ritz_values_after_a_few_iterations(its):
    _torch()
    N, k = 7, 6
    A, _, _, X0 = _case("std", N, k, seed=13)
    As = A.to_scipy()
    s = _solver(A, k, precond="jacobi", maxit=its)
    info = s.solve(1e-14, X0)
    assert info["iterations"] == its
    lam, _, _ = s.eigpairs(k)
    ref = L.lobpcg(As, X0, k, 1e-14, precond=L.jacobi_precond(As), maxit=its)
    diff = np.max(np.abs(lam.cpu().numpy() - ref.theta[:k]) / np.abs(ref.theta[:k]))
    print(f"after {its} iterations: Ritz values vs oracle {diff:.2e}")
    assert diff <= 1e-10


def test_hermitian_largest_and_default_start():
    _torch()
    N, k = 6, 5
    A = P.twisted_laplacian_3d(N)
    top = cf.twisted_laplacian_3d(N)[::-1][:k]
    s = _solver(A, k, precond="none", largest=1)
    info = s.solve(1e-10)  # the library's seeded complex start
    assert info["converged"], info
    lam, X, _ = s.eigpairs(k)
    lam, X = lam.cpu().numpy(), X.cpu().numpy()
    assert np.all(np.diff(lam) <= 0)
    assert np.max(np.abs(lam - top) / np.abs(top)) <= 1e-10
    As = A.to_scipy()
    R = As @ X - X * lam[None, :]
    assert np.linalg.norm(R, axis=0).max() <= 1e-8 * np.abs(lam).max()


def test_hermitian_precision_split_and_device_input():
    torch = _torch()
    N, k = 8, 10
    A, Bm, exact, X0 = _case("gen", N, k, seed=14)
    dev = lambda M: {"rowptr": torch.from_numpy(M.rowptr).cuda(),
                     "colind": torch.from_numpy(M.colind).cuda(),
                     "values_re": torch.from_numpy(M.values_re).cuda(),
                     "values_im": torch.from_numpy(M.values_im).cuda()}
    s64 = _solver(dev(A), k, B=dev(Bm), precond="jacobi")
    assert s64.solve(1e-10, torch.from_numpy(X0).cuda())["converged"]
    l64 = s64.eigpairs(k)[0].cpu().numpy()
    s32 = _solver(A, k, B=Bm, precond="jacobi", precision="split")
    info = s32.solve(1e-10, X0)
    assert info["converged"], info
    l32, X, _ = s32.eigpairs(k)
    l32, X = l32.cpu().numpy(), X.cpu().numpy()
    e64 = np.max(np.abs(l64 - exact) / np.abs(exact))
    e32 = np.max(np.abs(l32 - l64) / np.abs(l64))
    print(f"FP64 vs closed form {e64:.2e}; split ({info['fp32_iterations']} FP32 + "
          f"{info['fp64_iterations']} FP64 iterations) vs FP64 {e32:.2e}")
    assert e64 <= 1e-10 and e32 <= 1e-10
    Bs = Bm.to_scipy()
    assert np.abs(X.conj().T @ (Bs @ X) - np.eye(k)).max() <= 1e-10
