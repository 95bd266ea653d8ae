"""Pins of the oracle's counter-based Gaussian generator and the section 4.3 sketch.

Section 4.3 only needs Omega to be Gaussian; the oracle's generator is pinned by
the published known-answer vectors of Philox-4x32-10, by that distribution and by
properties of the construction, not against itself.  The sketch estimate is pinned by its expectation: for Gaussian columns
omega, E ||A omega||^2 = ||A||_F^2 and E ||omega||^2 = n, so ||A Omega^T||_F /
||Omega^T||_F concentrates at ||A||_F / sqrt(n), the root mean square eigenvalue,
which the closed-form spectrum gives.
"""

import os

import numpy as np
import scipy.stats as st

from oracle import closed_forms as cf
from oracle import lobpcg as L
from oracle import philox as PH
from paper_1704_07458_amd import problems as P


GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def test_philox_matches_the_published_known_answer_vectors():
    rows = [ln.split() for ln in open(GOLDEN) if ln.strip() and not ln.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        w = [int(x, 16) for x in r]
        out = PH.philox4x32_10(*w[:4], *w[4:6])
        assert [int(x) for x in out] == w[6:], r


def test_gaussian_block_is_standard_normal():
    z = PH.gaussian_block(0, PH.STREAM_SKETCH, 1000, 200).ravel()
    assert abs(z.mean()) < 0.01
    assert abs(z.var() - 1.0) < 0.01
    assert st.kstest(z, "norm").pvalue > 1e-3
    # fourth moment of N(0, 1) is 3
    assert abs(np.mean(z ** 4) - 3.0) < 0.05


def test_uniforms_lie_in_their_half_open_ranges_and_are_uniform():
    q = np.arange(1 << 16, dtype=np.uint64)
    o = PH.philox4x32_10(q & PH.MASK32, q >> np.uint64(32), np.zeros_like(q), np.zeros_like(q),
                         7, 0)
    u1, u2 = PH.uniform_pair(*o)
    assert np.all(u1 > 0.0) and np.all(u1 <= 1.0)
    assert np.all(u2 >= 0.0) and np.all(u2 < 1.0)
    assert st.kstest(u1, "uniform").pvalue > 1e-3
    assert st.kstest(u2, "uniform").pvalue > 1e-3


def test_box_muller_special_values():
    # u1 = 1: radius 0; u1 = e^(-1/2): radius 1, and the angle 2 pi u2
    z0, z1 = PH.box_muller(np.array([1.0]), np.array([0.3]))
    assert z0[0] == 0.0 and z1[0] == 0.0
    z0, z1 = PH.box_muller(np.array([np.exp(-0.5)]), np.array([0.25]))
    assert abs(z0[0]) < 1e-15 and abs(z1[0] - 1.0) < 1e-15
    z0, z1 = PH.box_muller(np.array([np.exp(-2.0)]), np.array([0.5]))
    assert abs(z0[0] + 2.0) < 1e-14 and abs(z1[0]) < 1e-14


def test_philox_is_a_bijection_with_avalanche():
    """Distinct counters give distinct 128-bit outputs, and flipping one counter bit
    changes about half of the output bits (a keyed bijection that mixes fully)."""
    q = np.arange(1 << 16, dtype=np.uint64)
    z = np.zeros_like(q)
    o = PH.philox4x32_10(q & PH.MASK32, z, z, z, 12345, 678)
    words = np.stack(o, axis=1).astype(np.uint64)
    keys = (words[:, 0] << np.uint64(32)) | words[:, 1]
    keys2 = (words[:, 2] << np.uint64(32)) | words[:, 3]
    assert len(set(zip(keys.tolist(), keys2.tolist()))) == q.size
    flips = []
    for bit in range(32):
        o2 = PH.philox4x32_10((q[:256] ^ np.uint64(1 << bit)) & PH.MASK32, z[:256], z[:256],
                              z[:256], 12345, 678)
        diff = 0
        for a, b in zip(o, o2):
            x = (a[:256] ^ b).astype(np.uint64)
            diff = diff + np.array([bin(int(v)).count("1") for v in x])
        flips.append(diff.mean())
    assert 60.0 < np.mean(flips) < 68.0


def test_streams_and_seeds_are_independent():
    a = PH.gaussian_block(0, 0, 400, 50).ravel()
    b = PH.gaussian_block(0, 1, 400, 50).ravel()
    c = PH.gaussian_block(1, 0, 400, 50).ravel()
    for u, v in ((a, b), (a, c), (b, c)):
        assert abs(np.corrcoef(u, v)[0, 1]) < 0.02
    # the cosine and sine halves of one Box-Muller pair are uncorrelated
    assert abs(np.corrcoef(a[0::2], a[1::2])[0, 1]) < 0.02
    # the layout depends on the linear element index only: an odd element count
    # keeps the pairs of a longer block's prefix
    d = PH.gaussian_block(0, 0, 7, 3).ravel()
    assert np.array_equal(d, a[:21])
    assert np.array_equal(d, PH.gaussian_block(0, 0, 1, 21).ravel())


def test_sketch_norm_concentrates_at_the_rms_eigenvalue():
    N = 12
    A = P.laplacian_3d(N).to_scipy()
    lam = cf.laplacian_3d_dirichlet(N)
    rms = np.sqrt(np.mean(lam ** 2))
    est = L.sketch_norm(L.Operator(A), PH.sketch(0, A.shape[0], 22))
    assert abs(est / rms - 1.0) < 0.05
    assert est <= lam.max()


def test_oracle_solve_uses_the_seeded_sketch_not_x0():
    """The norms of criterion (9) do not depend on the initial block (reading R1)."""
    w = P.workload(0, small=True)
    A = w.A.to_scipy()
    r1 = L.lobpcg(A, w.X0, w.k, w.tol, maxit=2)
    r2 = L.lobpcg(A, P.initial_block(5, A.shape[0], w.n_x), w.k, w.tol, maxit=2)
    ref = L.sketch_norm(L.Operator(A), PH.sketch(0, A.shape[0], w.n_x))
    assert r1.normA == r2.normA == ref
    r3 = L.lobpcg(A, w.X0, w.k, w.tol, maxit=2, sketch_seed=3)
    assert r3.normA != r1.normA
