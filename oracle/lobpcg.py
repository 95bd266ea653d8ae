"""Plain FP64 oracle of the robust LOBPCG iteration (arXiv 1704.07458).

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the product path.

Every function follows one algorithm or equation of the paper, in the paper's
order and notation, with NumPy/SciPy/LAPACK primitives (matrix products, eigh,
Cholesky, Householder QR) as steps.  Nothing is blocked, fused or reordered,
and every Gram block and every product A*U, B*U is formed explicitly (the
conservative choice; the paper's shortcuts of section 5.2 are what the HIP path
is checked against).

Readings taken where the paper is silent or ambiguous (each is also an option
of the HIP path, with the same default):
  R1  the sketch Omega of section 4.3 is an n_x x n Gaussian matrix drawn from
      the seed by a counter-based generator (oracle/philox.py, stream 1),
      independent of the initial block, so that a warm start from converged
      vectors does not bias the estimate.
  R2  the preconditioner K^-1 of section 2 / Algorithm 1 is applied to the
      residual wherever Algorithm 8 uses R (W0 = K^-1 R).
  R3  Cholesky is declared unreliable (section 5.3) when cond_1(R)^3 * tau_skip
      > 1, with tau_skip = 10 eps, or when the factorisation fails.
  R4  tau_drop = tau_replace = 10 * n_u * eps, tau_ortho = 1e-12 (FP64),
      Frobenius norms in the orthogonality checks of Algorithm 5.
  R5  with soft locking, the P block is built from the LQ factorisation of
      Z_1(:, n_c:n_x)^T Z_1perp (the unconverged columns only); for n_c = 0
      this spans the same space as the LQ of Z_1perp (section 4.2).
  R6  n_c is the length of the leading run of columns meeting criterion (9),
      re-evaluated every iteration.
  R8  exactly zero columns are removed before the diagonal scaling of SVQB.
"""

from __future__ import annotations

import dataclasses
import time
from typing import Callable, List, Optional

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from . import philox

EPS64 = np.finfo(np.float64).eps


def _H(M: np.ndarray) -> np.ndarray:
    """Conjugate transpose (the transpose for real data): the paper states the
    method for real pencils and notes that it carries over to complex Hermitian
    ones with every transpose read as a conjugate transpose (section 1)."""
    return M.conj().T


# --------------------------------------------------------------------------
# Operators
# --------------------------------------------------------------------------
class Operator:
    """y = M u for a sparse symmetric M, or the identity when M is None."""

    def __init__(self, M=None):
        self.M = None if M is None else sp.csr_matrix(M)

    @property
    def is_identity(self) -> bool:
        return self.M is None

    def __call__(self, U: np.ndarray) -> np.ndarray:
        if self.M is None:
            return U.copy()
        return np.asarray(self.M @ U)


def _is_complex(mat) -> bool:
    if mat is None:
        return False
    if hasattr(mat, "values_im"):
        return mat.values_im is not None
    return np.iscomplexobj(mat.data if sp.issparse(mat) else mat)


def _csr(mat):
    if mat is None:
        return None
    if hasattr(mat, "to_scipy"):
        return mat.to_scipy()
    return sp.csr_matrix(mat)


# --------------------------------------------------------------------------
# Tolerances (reading R4 / R3)
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Tolerances:
    eps: float = EPS64
    drop_factor: float = 10.0  # tau_drop = drop_factor * n_u * eps
    replace_factor: float = 10.0  # tau_replace = replace_factor * n_u * eps
    tau_ortho: float = 1e-12
    skip_factor: float = 10.0  # tau_skip = skip_factor * eps

    def tau_drop(self, n_u: int) -> float:
        return self.drop_factor * max(n_u, 1) * self.eps

    def tau_replace(self, n_u: int) -> float:
        return self.replace_factor * max(n_u, 1) * self.eps

    @property
    def tau_skip(self) -> float:
        return self.skip_factor * self.eps


# --------------------------------------------------------------------------
# Section 4.3: backward-stable criterion (9) and the Gaussian norm sketch
# --------------------------------------------------------------------------
def sketch_norm(Mop: Operator, Omega_T: np.ndarray) -> float:
    """||M||_2^(Omega) = ||Omega M||_F / ||Omega||_F, a lower bound of ||M||_2.

    Omega is k x m; it is passed transposed (m x k) so that for symmetric M,
    ||Omega M||_F = ||M Omega^T||_F.
    """
    return float(np.linalg.norm(Mop(Omega_T)) / np.linalg.norm(Omega_T))


def criterion9(R: np.ndarray, X: np.ndarray, theta: np.ndarray, normA: float, normB: float):
    """rho_i = ||r_i||_2 / ((||A|| + |theta_i| ||B||) ||x_i||_2)  (eq. 9)."""
    rn = np.linalg.norm(R, axis=0)
    xn = np.linalg.norm(X, axis=0)
    return rn / ((normA + np.abs(theta) * normB) * xn)


def criterion7(R, X, theta):
    """||r_i|| / (|theta_i| ||x_i||)  (eq. 7, the relative residual of Anasazi)."""
    return np.linalg.norm(R, axis=0) / (np.abs(theta) * np.linalg.norm(X, axis=0))


def criterion8(R, X, BX, theta):
    """||r_i|| / (|theta_i| ||x_i||_B)  (eq. 8)."""
    xb = np.sqrt(np.abs(np.sum(X * BX, axis=0)))
    return np.linalg.norm(R, axis=0) / (np.abs(theta) * xb)


# --------------------------------------------------------------------------
# Algorithm 2: Rayleigh-Ritz with diagonal scaling
# --------------------------------------------------------------------------
def rayleigh_ritz(GA: np.ndarray, GB: np.ndarray):
    """C, theta with C^H GB C = I and C^H GA C = diag(theta), theta ascending.

    D = diag(GB)^-1/2; R^H R = D GB D; eigh(R^-H D GA D R^-1) = Z Theta;
    C = D R^-1 Z.  Raises numpy.linalg.LinAlgError if Cholesky fails.
    """
    d = 1.0 / np.sqrt(np.diag(GB).real)
    D = np.diag(d)
    R = _H(np.linalg.cholesky(D @ GB @ D))  # upper triangular, R^H R = D GB D
    Rinv = sla.solve_triangular(R, np.eye(R.shape[0]), lower=False)
    H = _H(Rinv) @ (D @ GA @ D) @ Rinv
    H = 0.5 * (H + _H(H))
    theta, Z = np.linalg.eigh(H)
    C = D @ Rinv @ Z
    return C, theta


# --------------------------------------------------------------------------
# Algorithm 4 (svqb) and Algorithm 6 (svqbDrop)
# --------------------------------------------------------------------------
def _drop_zero_columns(U: np.ndarray, MU: np.ndarray):
    """Reading R8: remove columns with exactly zero M-norm before scaling."""
    g = np.einsum("ij,ij->j", U.conj(), MU).real
    keep = g > 0.0
    return U[:, keep], MU[:, keep]


def svqb(Mop: Operator, U: np.ndarray, tau_replace: float) -> np.ndarray:
    """Algorithm 4: M-orthonormalise U, flooring small eigenvalues.

    G = U^T M U; D = diag(G)^-1/2; eigh(D G D) = Z Theta;
    theta_j <- max(theta_j, tau_replace * max|theta|); U <- U D Z Theta^-1/2.
    """
    U, MU = _drop_zero_columns(U, Mop(U))
    if U.shape[1] == 0:
        return U
    G = _H(U) @ MU
    G = 0.5 * (G + _H(G))
    d = 1.0 / np.sqrt(np.diag(G).real)
    theta, Z = np.linalg.eigh(d[:, None] * G * d[None, :])
    floor = tau_replace * np.max(np.abs(theta))
    theta = np.where(theta < floor, floor, theta)
    return U @ (d[:, None] * Z * (theta ** -0.5)[None, :])


def svqb_drop(Mop: Operator, U: np.ndarray, tau_drop: float) -> np.ndarray:
    """Algorithm 6: SVQB that keeps only J = {j : theta_j > tau_drop max|theta|}."""
    U, MU = _drop_zero_columns(U, Mop(U))
    if U.shape[1] == 0:
        return U
    G = _H(U) @ MU
    G = 0.5 * (G + _H(G))
    d = 1.0 / np.sqrt(np.diag(G).real)
    theta, Z = np.linalg.eigh(d[:, None] * G * d[None, :])
    J = theta > tau_drop * np.max(np.abs(theta))
    return U @ (d[:, None] * Z[:, J] * (theta[J] ** -0.5)[None, :])


def _rel_orth_error(U, MU):
    """||U^T M U - I||_F / (||MU||_F ||U||_F)  (Algorithm 5, inner test)."""
    if U.shape[1] == 0:
        return 0.0
    G = _H(U) @ MU
    return np.linalg.norm(G - np.eye(U.shape[1])) / (np.linalg.norm(MU) * np.linalg.norm(U))


def _rel_ext_error(V, MV, U):
    """||V^T M U||_F / (||MV||_F ||U||_F)  (Algorithm 5, outer test); MU = M U."""
    if U.shape[1] == 0 or V.shape[1] == 0:
        return 0.0
    return np.linalg.norm(_H(MV) @ U) / (np.linalg.norm(MV) * np.linalg.norm(U))


@dataclasses.dataclass
class OrthoStats:
    outer: int = 0
    svqb_calls: int = 0


def ortho_drop(
    Mop: Operator,
    U: np.ndarray,
    V: np.ndarray,
    MV: np.ndarray,
    tol: Tolerances,
    stats: Optional[OrthoStats] = None,
) -> np.ndarray:
    """Algorithm 5: orthoDrop(M, U, V, tau_ortho).

    Up to three outer block classical Gram-Schmidt passes U <- U - V (MV)^T U,
    each followed by up to three inner passes: the first an svqb (Algorithm 4),
    later ones svqbDrop (Algorithm 6).  M U is recomputed explicitly after every
    inner pass (no implicit products inside orthogonalisation, section 5.2).
    """
    stats = stats if stats is not None else OrthoStats()
    for _i in range(3):
        stats.outer += 1
        if V.shape[1] > 0:
            U = U - V @ (_H(MV) @ U)
        for j in range(3):
            n_u = U.shape[1]
            if j == 0:
                U = svqb(Mop, U, tol.tau_replace(n_u))
            else:
                U = svqb_drop(Mop, U, tol.tau_drop(n_u))
            stats.svqb_calls += 1
            MU = Mop(U)
            if _rel_orth_error(U, MU) <= tol.tau_ortho:
                break
        if U.shape[1] == 0 or _rel_ext_error(V, MV, U) <= tol.tau_ortho:
            break
    return U


def ortho(Mop: Operator, U: np.ndarray, V: np.ndarray, MV: np.ndarray, tol: Tolerances,
          stats: Optional[OrthoStats] = None, itmax1: int = 3, itmax2: int = 3) -> np.ndarray:
    """Algorithm 3 (Stathopoulos-Wu ortho with svqb only, no dropping).

    Used by the section 4.1 example, where it shows the failure that orthoDrop
    fixes, and by the version 2 rung of the section 6 ablation (lobpcg with
    ortho_kind="hl").
    """
    stats = stats if stats is not None else OrthoStats()
    for _i in range(itmax1):
        stats.outer += 1
        if V.shape[1] > 0:
            U = U - V @ (_H(MV) @ U)
        for _j in range(itmax2):
            U = svqb(Mop, U, tol.tau_replace(U.shape[1]))
            stats.svqb_calls += 1
            if _rel_orth_error(U, Mop(U)) <= tol.tau_ortho:
                break
        if V.shape[1] == 0 or _rel_ext_error(V, MV, U) <= tol.tau_ortho:
            break
    return U


# --------------------------------------------------------------------------
# Algorithm 7: Rayleigh-Ritz with improved basis selection
# --------------------------------------------------------------------------
@dataclasses.dataclass
class RRResult:
    Cx: np.ndarray  # n_s x n_x
    Cp: np.ndarray  # n_s x n_p
    theta_x: np.ndarray  # n_x Ritz values, ascending
    theta_p: np.ndarray  # n_p x n_p block Q^T Theta_perp Q
    theta_all: np.ndarray  # all n_s Ritz values
    use_ortho: bool
    flipped: bool
    cond_R: float


def _lq_rows(M: np.ndarray) -> np.ndarray:
    """Orthonormal rows Q of a Householder LQ factorisation M = L Q.

    Computed as the QR factorisation of M^T (LAPACK geqrf), which keeps Q
    orthonormal to working precision even if M is rank deficient.  Returns Q^T
    (columns orthonormal), of width min(M.shape).
    """
    q, _r = np.linalg.qr(_H(M), mode="reduced")
    return q


def rayleigh_ritz_modified(
    GA: np.ndarray,
    GB: np.ndarray,
    n_x: int,
    n_c: int,
    use_ortho: bool,
    tol: Tolerances,
    literal_lq: bool = False,
) -> RRResult:
    """Algorithm 7 on the projected pencil (GA, GB) = (S^T A S, S^T B S).

    Returns C_x, C_p and the block-diagonal Theta of the P block.  When the
    Cholesky factor is unreliable (reading R3) it returns flipped=True and no
    coefficients, so that the caller can orthogonalise W and call again.

    Z is partitioned as in eq. (5): rows split after the n_x rows of X,
    columns after the first n_x Ritz vectors.  Reading R5 for the P block:
    LQ-factorise Z_1(:, n_c:n_x)^T Z_1perp and take C_p = T Z_perp Q^T.
    literal_lq=True takes the first n_x - n_c rows of the LQ of Z_1perp
    instead (the literal reading of Algorithm 7's P block).
    """
    n_s = GA.shape[0]
    cond_R = 1.0
    if use_ortho:
        theta, Z = np.linalg.eigh(0.5 * (GA + _H(GA)))
        T = np.eye(n_s)
    else:
        g = np.diag(GB).real
        if not np.all(g > 0.0):
            # a column of S with zero B-norm (an exactly converged residual):
            # S^T B S is singular and has no Cholesky factor (reading R8)
            return RRResult(None, None, None, None, None, True, True, np.inf)
        d = 1.0 / np.sqrt(g)
        D = np.diag(d)
        try:
            R = _H(np.linalg.cholesky(D @ GB @ D))
        except np.linalg.LinAlgError:
            return RRResult(None, None, None, None, None, True, True, np.inf)
        Rinv = sla.solve_triangular(R, np.eye(n_s), lower=False)
        cond_R = np.linalg.norm(R, 1) * np.linalg.norm(Rinv, 1)
        if cond_R ** 3 * tol.tau_skip > 1.0:
            return RRResult(None, None, None, None, None, True, True, cond_R)
        H = _H(Rinv) @ (D @ GA @ D) @ Rinv
        theta, Z = np.linalg.eigh(0.5 * (H + _H(H)))
        T = D @ Rinv
    Z1 = Z[:n_x, :n_x]
    Z1p = Z[:n_x, n_x:]
    Zp = Z[:, n_x:]
    if n_s > n_x:
        if literal_lq:
            q = _lq_rows(Z1p)[:, : n_x - n_c]
        else:
            q = _lq_rows(_H(Z1[:, n_c:]) @ Z1p)
    else:
        q = np.zeros((0, 0))
    Cx = T @ Z[:, :n_x]
    Cp = T @ Zp @ q if q.size else np.zeros((n_s, 0))
    theta_p = _H(q) @ np.diag(theta[n_x:]) @ q if q.size else np.zeros((0, 0))
    return RRResult(Cx, Cp, theta[:n_x].copy(), theta_p, theta, use_ortho, False, cond_R)


# --------------------------------------------------------------------------
# Preconditioner (reading R2 / R10)
# --------------------------------------------------------------------------
def jacobi_diagonal(A) -> np.ndarray:
    """Diagonal used by the Jacobi preconditioner.

    diag(A) when it is positive; otherwise diag(A) - sigma with the
    Gershgorin shift sigma = min_i(a_ii - sum_{j!=i} |a_ij|) - 1e-3 * bound,
    bound = max_i sum_j |a_ij|, which makes the diagonal positive.
    """
    A = _csr(A)
    d = A.diagonal().real.astype(np.float64)
    if np.all(d > 0):
        return d
    absrow = np.asarray(abs(A).sum(axis=1)).ravel()
    off = absrow - np.abs(d)
    sigma = np.min(d - off) - 1e-3 * np.max(absrow)
    return d - sigma


# --------------------------------------------------------------------------
# Algorithm 8: robust LOBPCG
# --------------------------------------------------------------------------
@dataclasses.dataclass
class IterRecord:
    it: int
    n_c: int
    use_ortho: bool
    n_w: int
    n_p: int
    cond_R: float
    max_rho_active: float
    seconds: float = 0.0  # wall time of the iteration (instrumentation only)


@dataclasses.dataclass
class LobpcgResult:
    converged: bool
    iterations: int
    theta: np.ndarray  # all n_x current Ritz values
    X: np.ndarray  # n x n_x current Ritz vectors (B-orthonormal)
    rho: np.ndarray  # criterion (9) for every column
    n_c: int
    normA: float
    normB: float
    history: List[IterRecord]
    ortho_switch_iter: int
    ortho_stats: OrthoStats

    def eigenpairs(self, k):
        return self.theta[:k].copy(), self.X[:, :k].copy()


def lobpcg(
    A,
    X0: np.ndarray,
    k: int,
    tol: float,
    B=None,
    precond: Optional[Callable[[np.ndarray], np.ndarray]] = None,
    maxit: int = 2000,
    tols: Optional[Tolerances] = None,
    Omega_T: Optional[np.ndarray] = None,
    sketch_seed: int = 0,
    literal_lq: bool = False,
    exact_norms: Optional[tuple] = None,
    force_ortho: bool = False,
    ortho_kind: str = "drop",
    largest: bool = False,
    implicit_products: bool = False,
    callback: Optional[Callable[["IterRecord"], None]] = None,
) -> LobpcgResult:
    """Algorithm 8: the robust and efficient LOBPCG of the paper, FP64.

    A, B: sparse symmetric (B SPD, None = I).  X0: n x n_x initial block.
    k (= n_v): number of wanted eigenpairs, n_v <= n_x.  tol: tau of eq. (9).
    precond: W0 = precond(R) applies K^-1 column-wise (None = identity).
    Omega_T: n x m sketch for the norm estimate; default: the n x n_x Gaussian
    block of philox.sketch(sketch_seed, n, n_x) (reading R1).
    exact_norms: (||A||_2, ||B||_2) to use instead of the sketch.
    force_ortho, ortho_kind: the section 6 ablation of the algorithm's
    versions.  force_ortho orthogonalises W from the first iteration and never
    takes the Cholesky path of Algorithm 7 (the switch to useOrtho never fires);
    ortho_kind "drop" is orthoDrop (Algorithm 5), "hl" is ortho (Algorithm 3).
    The defaults are Algorithm 8 itself.
    largest: the k largest eigenpairs instead (section 2: the Ritz values are
    ordered the other way).  Taking them in descending order for A is taking
    them in ascending order for -A, so the iteration runs on (-A, B) and the
    Ritz values are negated on return; precond must then approximate the
    inverse of (-A) shifted, as for any pencil.
    callback: called with each iteration's record (timing and progress only;
    it takes no part in the arithmetic).
    implicit_products: section 5.2's implicit updates A X = (A S) C_x and
    A P = (A S) C_p after the basis update instead of recomputing the products
    (B = I only: the paper restricts them to that case).
    """
    if implicit_products and B is not None:
        raise ValueError("implicit product updates need B = I")
    if ortho_kind not in ("drop", "hl"):
        raise ValueError("ortho_kind must be 'drop' or 'hl'")
    orth = ortho_drop if ortho_kind == "drop" else ortho
    tols = tols or Tolerances()
    if largest:
        A = -_csr(A)
    Aop, Bop = Operator(_csr(A)), Operator(_csr(B))
    Kinv = precond if precond is not None else (lambda R: R.copy())
    X0 = np.asarray(X0)
    cplx = np.iscomplexobj(X0) or _is_complex(A) or _is_complex(B)
    X0 = X0.astype(np.complex128 if cplx else np.float64)
    n, n_x = X0.shape
    if not (1 <= k <= n_x) or 3 * n_x > n:
        raise ValueError("need 1 <= k <= n_x and 3 n_x <= n")

    # Section 4.3: norm estimates from the Gaussian sketch.
    if exact_norms is not None:
        normA, normB = exact_norms
    else:
        if Omega_T is not None:
            Om = Omega_T
        elif cplx:
            # reading R17: the complex Gaussian n x 2 n_x block whose real and
            # imaginary parts are the two halves of the real 2n x 2n_x sketch
            Om2 = philox.sketch(sketch_seed, 2 * n, 2 * n_x)
            Om = Om2[:n] + 1j * Om2[n:]
        else:
            Om = philox.sketch(sketch_seed, n, n_x)
        normA = sketch_norm(Aop, Om)
        normB = 1.0 if Bop.is_identity else sketch_norm(Bop, Om)

    # Start: initial Rayleigh-Ritz on X0.
    AX0, BX0 = Aop(X0), Bop(X0)
    C, theta = rayleigh_ritz(_H(X0) @ AX0, _H(X0) @ BX0)
    X = X0 @ C
    AX, BX = Aop(X), Bop(X)
    theta_x = theta
    R = AX - BX * theta_x[None, :]
    n_c, use_ortho = 0, bool(force_ortho)
    P = np.zeros((n, 0), dtype=X0.dtype)
    AP, BP = np.zeros((n, 0), dtype=X0.dtype), np.zeros((n, 0), dtype=X0.dtype)
    history: List[IterRecord] = []
    switch_iter = -1
    ostats = OrthoStats()
    rho = criterion9(R, X, theta_x, normA, normB)

    it = 0
    converged = False
    while it < maxit:
        it += 1
        t_it = time.perf_counter()
        # W (with reading R2): W0 = K^-1 R on the unconverged columns.
        W0 = Kinv(R[:, n_c:])
        V, MV = np.hstack([X, P]), np.hstack([BX, BP])
        if use_ortho:
            W = orth(Bop, W0, V, MV, tols, ostats)
        else:
            W = W0
        AW, BW = Aop(W), Bop(W)
        # S = [X, P, W]; every block of S^T A S and S^T B S explicit.
        S = np.hstack([X, P, W])
        AS = np.hstack([AX, AP, AW])
        BS = np.hstack([BX, BP, BW])
        GA, GB = _H(S) @ AS, _H(S) @ BS
        GA, GB = 0.5 * (GA + _H(GA)), 0.5 * (GB + _H(GB))
        # RayleighRitzModified (Algorithm 7).
        rr = rayleigh_ritz_modified(GA, GB, n_x, n_c, use_ortho, tols, literal_lq)
        if rr.flipped:
            # Cholesky rejected: switch to orthogonalised W for good.
            use_ortho = True
            switch_iter = it
            W = orth(Bop, W0, V, MV, tols, ostats)
            AW, BW = Aop(W), Bop(W)
            S = np.hstack([X, P, W])
            AS = np.hstack([AX, AP, AW])
            BS = np.hstack([BX, BP, BW])
            GA, GB = _H(S) @ AS, _H(S) @ BS
            GA, GB = 0.5 * (GA + _H(GA)), 0.5 * (GB + _H(GB))
            rr = rayleigh_ritz_modified(GA, GB, n_x, n_c, use_ortho, tols, literal_lq)
        # Basis update [X, P] = S [C_x, C_p]; products recomputed explicitly, or
        # updated implicitly from A S (section 5.2).
        X, P = S @ rr.Cx, S @ rr.Cp
        if implicit_products:
            AX, AP = AS @ rr.Cx, AS @ rr.Cp
            BX, BP = X, P
        else:
            AX, BX = Aop(X), Bop(X)
            AP, BP = Aop(P), Bop(P)
        theta_x = rr.theta_x
        # Residual.
        R = AX - BX * theta_x[None, :]
        # Converged count (reading R6): leading run of columns meeting criterion (9).
        rho = criterion9(R, X, theta_x, normA, normB)
        ok = rho <= tol
        n_c = int(np.argmin(ok)) if not np.all(ok) else n_x
        history.append(IterRecord(it, n_c, use_ortho, W.shape[1], P.shape[1], rr.cond_R,
                                  float(np.max(rho[n_c:])) if n_c < n_x else 0.0,
                                  time.perf_counter() - t_it))
        if callback is not None:
            callback(history[-1])
        if n_c >= k:
            converged = True
            break
        if W.shape[1] == 0 and P.shape[1] == 0:
            break  # the search space cannot grow any more
    theta_out = -theta_x if largest else theta_x.copy()
    return LobpcgResult(converged, it, theta_out, X, rho, n_c, normA, normB, history,
                        switch_iter, ostats)


@dataclasses.dataclass
class BasicResult:
    converged: bool
    breakdown: bool  # the Cholesky of Algorithm 2 failed
    iterations: int
    theta: np.ndarray
    X: np.ndarray
    rho: np.ndarray
    normA: float
    normB: float


def lobpcg_basic(A, X0: np.ndarray, k: int, tol: float, B=None,
                 precond: Optional[Callable[[np.ndarray], np.ndarray]] = None,
                 maxit: int = 2000, sketch_seed: int = 0) -> BasicResult:
    """Algorithm 1, the basic LOBPCG, with Algorithm 2 for every Rayleigh-Ritz.

    S = [X, W, P] with W = K^-1 R for all n_x columns (no locking), every block
    of S^T A S and S^T B S explicit, X = S C(:, 1:n_x) and
    P = S(:, n_x+1:end) C(n_x+1:end, 1:n_x).  Convergence as in lobpcg (criterion
    (9), leading run, reading R6).  When S^T B S has no Cholesky factor (a column
    of zero B-norm or an indefinite pencil in rounding) the method stops with
    breakdown = True: Algorithm 1 has no way around it, which is what
    Algorithms 5-8 add.
    """
    Aop, Bop = Operator(_csr(A)), Operator(_csr(B))
    Kinv = precond if precond is not None else (lambda R: R.copy())
    X0 = np.asarray(X0, dtype=np.float64)
    n, n_x = X0.shape
    Om = philox.sketch(sketch_seed, n, n_x)
    normA = sketch_norm(Aop, Om)
    normB = 1.0 if Bop.is_identity else sketch_norm(Bop, Om)

    def rr(S):
        AS, BS = Aop(S), Bop(S)
        GA, GB = S.T @ AS, S.T @ BS
        GA, GB = 0.5 * (GA + GA.T), 0.5 * (GB + GB.T)
        if not np.all(np.diag(GB) > 0.0):
            return None, None
        try:
            return rayleigh_ritz(GA, GB)
        except np.linalg.LinAlgError:
            return None, None

    C, theta = rr(X0)
    if C is None:
        return BasicResult(False, True, 0, np.zeros(n_x), X0, np.full(n_x, np.inf), normA, normB)
    X = X0 @ C
    thx = theta
    R = Aop(X) - Bop(X) * thx[None, :]
    P = np.zeros((n, 0))
    rho = criterion9(R, X, thx, normA, normB)
    for it in range(1, maxit + 1):
        W = Kinv(R)
        S = np.hstack([X, W, P])
        C, theta = rr(S)
        if C is None:
            return BasicResult(False, True, it, thx.copy(), X, rho, normA, normB)
        X = S @ C[:, :n_x]
        P = S[:, n_x:] @ C[n_x:, :n_x]
        thx = theta[:n_x]
        R = Aop(X) - Bop(X) * thx[None, :]
        rho = criterion9(R, X, thx, normA, normB)
        ok = rho <= tol
        n_c = int(np.argmin(ok)) if not np.all(ok) else n_x
        if n_c >= k:
            return BasicResult(True, False, it, thx.copy(), X, rho, normA, normB)
    return BasicResult(False, False, maxit, thx.copy(), X, rho, normA, normB)


def jacobi_precond(A):
    """K^-1 R for K = the (possibly shifted) diagonal of A."""
    d = jacobi_diagonal(A)
    return lambda R: R / d[:, None]
