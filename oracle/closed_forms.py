"""Closed-form spectra of the synthetic pencils.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

The pencils are Kronecker sums / tensor products of 1D three-point operators,
so every eigenpair is a sum (or product) of 1D eigenpairs with sine modes.
"""

from __future__ import annotations

import numpy as np


def dirichlet_1d(N: int) -> np.ndarray:
    """Eigenvalues of tridiag(-1, 2, -1), N x N: 4 sin^2(i pi / (2(N+1))), i = 1..N."""
    i = np.arange(1, N + 1)
    return 4.0 * np.sin(i * np.pi / (2.0 * (N + 1))) ** 2


def periodic_1d(N: int) -> np.ndarray:
    """Eigenvalues of the periodic three-point Laplacian: 4 sin^2(pi i / N), i = 0..N-1."""
    i = np.arange(N)
    return 4.0 * np.sin(np.pi * i / N) ** 2


def sine_mode(N: int, i: int) -> np.ndarray:
    """Unit-norm eigenvector sin(i j pi/(N+1)), j = 1..N, of the 1D Dirichlet operator."""
    j = np.arange(1, N + 1)
    v = np.sin(i * j * np.pi / (N + 1))
    return v / np.linalg.norm(v)


def laplacian_2d_dirichlet(N: int) -> np.ndarray:
    s = dirichlet_1d(N)
    return np.sort((s[:, None] + s[None, :]).ravel())


def laplacian_3d_dirichlet(N: int) -> np.ndarray:
    s = dirichlet_1d(N)
    return np.sort((s[:, None, None] + s[None, :, None] + s[None, None, :]).ravel())


def laplacian_3d_periodic(N: int) -> np.ndarray:
    s = periodic_1d(N)
    return np.sort((s[:, None, None] + s[None, :, None] + s[None, None, :]).ravel())


def fem_1d(N: int) -> np.ndarray:
    """Eigenvalues of the 1D pencil K1 = tridiag(-1,2,-1)/h, M1 = h tridiag(1,4,1)/6.

    mu_i = 6 (1 - cos t_i) / (h^2 (2 + cos t_i)), t_i = i pi / (N+1), h = 1/(N+1).
    """
    h = 1.0 / (N + 1)
    t = np.arange(1, N + 1) * np.pi / (N + 1)
    return 6.0 * (1.0 - np.cos(t)) / (h * h * (2.0 + np.cos(t)))


def fem_q1_3d(N: int) -> np.ndarray:
    """Eigenvalues of the tensor-product Q1 pencil: mu_a + mu_b + mu_c."""
    m = fem_1d(N)
    return np.sort((m[:, None, None] + m[None, :, None] + m[None, None, :]).ravel())


def dirichlet_3d_modes(N: int, count: int):
    """Eigenvectors of the 3D 7-point Dirichlet Laplacian on N^3 for its `count`
    smallest eigenvalues: the tensor sine modes s_i(x) s_j(y) s_l(z) (grid index
    x + N y + N^2 z), orthonormal, with their eigenvalues e_i + e_j + e_l.  When
    count cuts a degenerate cluster the members kept are an arbitrary subset, so
    callers take count at a cluster boundary."""
    e = dirichlet_1d(N)
    lam = (e[:, None, None] + e[None, :, None] + e[None, None, :]).ravel()  # index i*N*N + j*N + l
    order = np.argsort(lam, kind="stable")[:count]
    S = np.stack([sine_mode(N, i) for i in range(1, N + 1)], axis=1)  # S[:, i-1] = s_i
    V = np.empty((N ** 3, count))
    for c, q in enumerate(order):
        i, j, l = q // (N * N), (q // N) % N, q % N
        V[:, c] = np.kron(S[:, l], np.kron(S[:, j], S[:, i]))
    return V, lam[order]


def smallest(values: np.ndarray, count: int) -> np.ndarray:
    """The `count` smallest values (full sort; for grids up to 96^3 this is cheap)."""
    return np.sort(values)[:count]


def cluster_boundary(values: np.ndarray, k: int, rel_gap: float = 1e-9) -> int:
    """Largest c <= k such that lambda_c and lambda_{c+1} are distinct clusters."""
    v = np.sort(values)
    c = k
    while c > 0 and abs(v[c] - v[c - 1]) <= rel_gap * max(abs(v[c]), 1.0):
        c -= 1
    return c


def norm2_laplacian_2d(N: int) -> float:
    return float(2.0 * dirichlet_1d(N)[-1])


def norm2_laplacian_3d(N: int) -> float:
    return float(3.0 * dirichlet_1d(N)[-1])


def _ring_eigenvalues(N: int, d: float, off: float, phase: float) -> np.ndarray:
    """The periodic ring with diagonal d and off * e^{+-i phase} on the cyclic
    neighbours is diagonalised by the Fourier modes e^{i theta_j l},
    theta_j = 2 pi j / N: eigenvalue d + 2 off cos(theta_j - phase), j = 0..N-1."""
    theta = 2.0 * np.pi * np.arange(N) / N
    return d + 2.0 * off * np.cos(theta - phase)


def twisted_laplacian_3d(N: int, phases=(0.3, 0.7, 1.1)) -> np.ndarray:
    """Spectrum of the complex Hermitian twisted periodic 7-point Laplacian
    (bond phases phases[d] * 2 pi / N): sums of the three axes' ring values."""
    e = [_ring_eigenvalues(N, 2.0, -1.0, f * 2.0 * np.pi / N) for f in phases]
    return np.sort((e[2][:, None, None] + e[1][None, :, None] + e[0][None, None, :]).ravel())


def twisted_pencil_3d(N: int, phases=(0.3, 0.7, 1.1), phase_b: float = 0.5) -> np.ndarray:
    """Spectrum of the complex tensor-product pencil A = a_x (x) b (x) b + ...,
    B = b (x) b (x) b: every factor is diagonalised by the same Fourier modes,
    so lambda = a_x/b_x + a_y/b_y + a_z/b_z over all mode triples."""
    b = _ring_eigenvalues(N, 4.0 / 6.0, 1.0 / 6.0, phase_b * 2.0 * np.pi / N)
    r = [_ring_eigenvalues(N, 2.0, -1.0, f * 2.0 * np.pi / N) / b for f in phases]
    return np.sort((r[2][:, None, None] + r[1][None, :, None] + r[0][None, None, :]).ravel())
