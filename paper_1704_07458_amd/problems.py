"""Seeded synthetic pencils (A, B) and initial blocks for the LOBPCG path.

This module only builds inputs: sparse matrices in CSR form (full symmetric
storage, sorted column indices, int64 row pointers, int32 column indices,
float64 values), random diagonal potentials and Gaussian initial blocks.  It
holds none of the eigensolver's arithmetic, so both the HIP path and the CPU
oracle may draw their inputs from it.

Grid ordering is lexicographic with x fastest: index = x + N*y + N*N*z.

The paper's own test matrices (SuiteSparse, PARSEC, SIESTA; section 6, Table 1)
are not available here.  These pencils stand in for them: they have the same
structure (sparse symmetric A, optional SPD B, a few hundred to a thousand
wanted eigenpairs, block padding of about ten percent as in section 6) and
known spectra where a closed form exists.
"""

from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
import scipy.sparse as sp


@dataclasses.dataclass
class CSR:
    """A square sparse matrix in CSR form with sorted, unique column indices."""

    n: int
    rowptr: np.ndarray  # int64, n + 1
    colind: np.ndarray  # int32, nnz
    values: np.ndarray  # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix(
            (self.values, self.colind.astype(np.int64), self.rowptr), shape=(self.n, self.n)
        )

    def diagonal(self) -> np.ndarray:
        return self.to_scipy().diagonal()


def from_scipy(M) -> CSR:
    M = sp.csr_matrix(M, dtype=np.float64)
    M.sum_duplicates()  # keeps explicitly stored zeros
    M.sort_indices()
    return CSR(
        n=M.shape[0],
        rowptr=np.ascontiguousarray(M.indptr, dtype=np.int64),
        colind=np.ascontiguousarray(M.indices, dtype=np.int32),
        values=np.ascontiguousarray(M.data, dtype=np.float64),
    )


def _tridiag(N: int, lo: float, d: float, hi: float, periodic: bool = False):
    T = sp.diags([np.full(N - 1, lo), np.full(N, d), np.full(N - 1, hi)], [-1, 0, 1], format="lil")
    if periodic and N > 2:
        T[0, N - 1] = lo
        T[N - 1, 0] = hi
    return sp.csr_matrix(T)


def laplacian_2d_dirichlet(N: int) -> CSR:
    """5-point Laplacian on an N x N interior grid: diagonal 4, neighbours -1."""
    T = _tridiag(N, -1.0, 2.0, -1.0)
    I = sp.identity(N, format="csr")
    return from_scipy(sp.kron(I, T) + sp.kron(T, I))


def laplacian_3d(N: int, periodic: bool = False) -> CSR:
    """7-point Laplacian on an N^3 grid: diagonal 6, neighbours -1.

    Dirichlet (interior grid) by default; periodic wraps every axis.
    """
    T = _tridiag(N, -1.0, 2.0, -1.0, periodic=periodic)
    I = sp.identity(N, format="csr")
    A = sp.kron(sp.kron(I, I), T) + sp.kron(sp.kron(I, T), I) + sp.kron(sp.kron(T, I), I)
    return from_scipy(A)


def add_diagonal(A: CSR, v: np.ndarray) -> CSR:
    """A + diag(v) (every row of A must already store its diagonal entry)."""
    S = A.to_scipy() + sp.diags(np.asarray(v, dtype=np.float64))
    return from_scipy(S)


def fem_q1_pencil(N: int):
    """Trilinear Q1 stiffness K and mass M on an N^3 interior grid, h = 1/(N+1).

    Built as tensor products of the 1D pencil K1 = tridiag(-1, 2, -1)/h and
    M1 = h * tridiag(1, 4, 1)/6:  K = K1(x)M1(x)M1 + M1(x)K1(x)M1 + M1(x)M1(x)K1,
    M = M1(x)M1(x)M1.  Both are 27-point.
    """
    h = 1.0 / (N + 1)
    K1 = _tridiag(N, -1.0, 2.0, -1.0) / h
    M1 = _tridiag(N, 1.0, 4.0, 1.0) * (h / 6.0)
    kron3 = lambda a, b, c: sp.kron(sp.kron(a, b), c, format="coo")
    terms = [kron3(K1, M1, M1), kron3(M1, K1, M1), kron3(M1, M1, K1)]
    # Accumulate in COO so that the full 27-point pattern is stored: the
    # face-neighbour couplings of Q1 stiffness cancel to (nearly) zero, and an
    # assembled FEM matrix still stores them.
    rows = np.concatenate([t.row for t in terms])
    cols = np.concatenate([t.col for t in terms])
    vals = np.concatenate([t.data for t in terms])
    K = sp.coo_matrix((vals, (rows, cols)), shape=terms[0].shape).tocsr()
    M = kron3(M1, M1, M1)
    return from_scipy(K), from_scipy(M)


@dataclasses.dataclass
class ZCSR:
    """A square complex sparse matrix in CSR form with sorted, unique column
    indices; the real and imaginary parts of the values are separate float64
    arrays (the library's complex Hermitian input layout)."""

    n: int
    rowptr: np.ndarray  # int64, n + 1
    colind: np.ndarray  # int32, nnz
    values_re: np.ndarray  # float64, nnz
    values_im: np.ndarray  # float64, nnz

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def to_scipy(self) -> sp.csr_matrix:
        return sp.csr_matrix(
            (self.values_re + 1j * self.values_im, self.colind.astype(np.int64), self.rowptr),
            shape=(self.n, self.n),
        )


def zfrom_scipy(M) -> ZCSR:
    M = sp.csr_matrix(M, dtype=np.complex128)
    M.sum_duplicates()
    M.sort_indices()
    return ZCSR(
        n=M.shape[0],
        rowptr=np.ascontiguousarray(M.indptr, dtype=np.int64),
        colind=np.ascontiguousarray(M.indices, dtype=np.int32),
        values_re=np.ascontiguousarray(M.data.real, dtype=np.float64),
        values_im=np.ascontiguousarray(M.data.imag, dtype=np.float64),
    )


def _ring(N: int, d: float, off: float, phase: float):
    """Periodic 1D ring: d on the diagonal, off * e^{i phase} at (l, l-1) and
    off * e^{-i phase} at (l, l+1), cyclically (Hermitian)."""
    rows, cols, vals = [], [], []
    for l in range(N):
        rows += [l, l, l]
        cols += [(l - 1) % N, l, (l + 1) % N]
        vals += [off * np.exp(1j * phase), d, off * np.exp(-1j * phase)]
    M = sp.coo_matrix((np.array(vals), (rows, cols)), shape=(N, N)).tocsr()
    M.sum_duplicates()
    return M


def twisted_laplacian_3d(N: int, phases=(0.3, 0.7, 1.1)) -> ZCSR:
    """Complex Hermitian 7-point Laplacian on a periodic N^3 grid whose bonds
    along axis d carry the phase e^{i phases[d] 2 pi / N} (a uniform magnetic
    twist): diagonal 6, neighbours -e^{+-i phi_d}.  N >= 3."""
    I = sp.identity(N, format="csr")
    T = [_ring(N, 2.0, -1.0, f * 2.0 * np.pi / N) for f in phases]
    A = sp.kron(sp.kron(I, I), T[0]) + sp.kron(sp.kron(I, T[1]), I) + sp.kron(sp.kron(T[2], I), I)
    return zfrom_scipy(A)


def twisted_pencil_3d(N: int, phases=(0.3, 0.7, 1.1), phase_b: float = 0.5):
    """Complex Hermitian-definite pencil (A, B) on a periodic N^3 grid, built
    like the Q1 pencil from 1D rings: a_d = ring(2, -1, phi_d), b = ring(4, 1,
    psi) / 6 (positive definite), A = a_x (x) b (x) b + b (x) a_y (x) b + b (x) b (x) a_z
    in the x-fastest ordering, B = b (x) b (x) b; 27-point.  N >= 3."""
    a = [_ring(N, 2.0, -1.0, f * 2.0 * np.pi / N) for f in phases]
    b = _ring(N, 4.0 / 6.0, 1.0 / 6.0, phase_b * 2.0 * np.pi / N)
    kron3 = lambda z, y, x: sp.kron(sp.kron(z, y), x, format="csr")
    A = kron3(b, b, a[0]) + kron3(b, a[1], b) + kron3(a[2], b, b)
    B = kron3(b, b, b)
    return zfrom_scipy(A), zfrom_scipy(B)


def complex_initial_block(seed: int, n: int, ncols: int) -> np.ndarray:
    """Complex Gaussian initial block: real and imaginary parts N(0, 1) from
    default_rng(seed), real part drawn first; n x ncols, row-major."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((n, ncols))
    im = rng.standard_normal((n, ncols))
    return np.ascontiguousarray(re + 1j * im)


def tridiag_1d(N: int, lo: float, d: float, hi: float) -> CSR:
    return from_scipy(_tridiag(N, lo, d, hi))


def potential(seed: int, n: int, lo: float, hi: float) -> np.ndarray:
    """i.i.d. uniform[lo, hi] diagonal potential drawn from default_rng(seed + 1000)."""
    return np.random.default_rng(seed + 1000).uniform(lo, hi, n)


def initial_block(seed: int, n: int, ncols: int) -> np.ndarray:
    """Gaussian N(0, 1) initial block X0, n x ncols, from default_rng(seed).

    Returned row-major (C order), which is also the device layout of the path.
    """
    return np.ascontiguousarray(np.random.default_rng(seed).standard_normal((n, ncols)))


def random_sparse_spd(seed: int, n: int, density: float, shift: float = 1.0) -> CSR:
    """A random sparse symmetric matrix made diagonally dominant (SPD)."""
    rng = np.random.default_rng(seed)
    R = sp.random(n, n, density=density, random_state=rng, format="csr")
    R = R + R.T
    d = np.asarray(abs(R).sum(axis=1)).ravel() + shift
    return from_scipy(R + sp.diags(d))


def block_size(k: int) -> int:
    """Block width n_x = k + ceil(k/10): the ten percent padding of section 6."""
    return k + int(math.ceil(k / 10.0))


@dataclasses.dataclass
class Workload:
    name: str
    A: CSR
    B: Optional[CSR]
    k: int
    n_x: int
    tol: float
    precond: str  # "none" or "jacobi"
    X0: np.ndarray
    potential: Optional[np.ndarray] = None


def workload(idx: int, seed: int = 0, small: bool = False) -> Workload:
    """The five synthetic pencils used for parity and measurement.

    0: 2D 5-point Dirichlet Laplacian 32^2, B = I, k = 10, no preconditioner.
    1: 3D 7-point Dirichlet Laplacian 64^3, B = I, k = 100, Jacobi.
    2: Q1 FEM pencil (K, M) on 48^3, k = 400, Jacobi.
    3: periodic 3D 7-point Laplacian 96^3 + uniform[-8, 8] potential, k = 1000, Jacobi.
    4: 3D 7-point Dirichlet 32^3 + uniform[0, 4] potential, k = 64, Jacobi.

    small=True shrinks the grid (same structure) for quick parity runs.
    """
    if idx == 0:
        N = 32 if not small else 12
        A, B, k, pre, tol = laplacian_2d_dirichlet(N), None, 10, "none", 1e-8
        V = None
    elif idx == 1:
        N = 64 if not small else 12
        k = 100 if not small else 20
        A, B, pre, tol, V = laplacian_3d(N), None, "jacobi", 1e-8, None
    elif idx == 2:
        N = 48 if not small else 10
        k = 400 if not small else 20
        K, M = fem_q1_pencil(N)
        A, B, pre, tol, V = K, M, "jacobi", 1e-8, None
    elif idx == 3:
        N = 96 if not small else 12
        k = 1000 if not small else 20
        L = laplacian_3d(N, periodic=True)
        V = potential(seed, L.n, -8.0, 8.0)
        A, B, pre, tol = add_diagonal(L, V), None, "jacobi", 1e-8
    elif idx == 4:
        N = 32 if not small else 8
        k = 64 if not small else 16
        L = laplacian_3d(N)
        V = potential(seed, L.n, 0.0, 4.0)
        A, B, pre, tol = add_diagonal(L, V), None, "jacobi", 1e-8
    else:
        raise ValueError(f"no workload {idx}")
    n_x = block_size(k)
    X0 = initial_block(seed, A.n, n_x)
    return Workload(f"cfg{idx}{'-small' if small else ''}", A, B, k, n_x, tol, pre, X0, V)
