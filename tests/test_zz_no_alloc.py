"""lobpcg_gram_noalloc (the Gram step with its split-K partials in the library's
fixed device array) against lobpcg_gram (the same step with a caller workspace).

Both compute G = L^T R in the same kernels; only the number of row splits can
differ, so each result lies within the a-priori bound |fl(sum) - sum| <=
gamma_n sum |l_k r_k| of the exact product, and the two within twice that of
each other.  Two calls in a row, the second smaller, check that the shared array
keeps no state that leaks between calls.
"""

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def gamma(K, u):
    return K * u / (1.0 - K * u)


def _torch():
    import torch

    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_gram_noalloc_matches_gram_on_two_calls(lib, dtype):
    torch = _torch()
    from paper_1704_07458_amd import binding as B

    tdt = torch.float64 if dtype == "f64" else torch.float32
    u = U64 if dtype == "f64" else U32
    rng = np.random.default_rng(21)
    # (n, m, p, p1, col_offset, mirror): the bench's S^T [AW | W] shape with more
    # row splits than the scratch holds (the split count is capped), then a
    # smaller ragged product with the mirrored rows
    cases = [(262144, 330, 220, 110, 0, False), (5003, 130, 70, 40, 60, True)]
    for n, m, p, p1, off, mirror in cases:
        L = rng.standard_normal((n, m))
        R = rng.standard_normal((n, p))
        if dtype == "f32":
            L, R = L.astype(np.float32).astype(np.float64), R.astype(np.float32).astype(np.float64)
        Lt = torch.from_numpy(L).to(tdt).cuda()
        R1 = torch.from_numpy(R[:, :p1]).to(tdt).cuda()
        R2 = torch.from_numpy(R[:, p1:]).to(tdt).cuda().contiguous()
        ref = B.gram(Lt, R1, R2, col_offset=off, mirror=mirror).cpu().numpy()
        got = B.gram_noalloc(Lt, R1, R2, col_offset=off, mirror=mirror).cpu().numpy()
        exact = L.T @ R
        bound = gamma(n, u) * (np.abs(L).T @ np.abs(R))
        sub = got[:, off:off + p]
        assert np.all(np.abs(sub - exact) <= bound)
        assert np.all(np.abs(sub - ref[:, off:off + p]) <= 2 * bound)
        if mirror:
            # rows above col_offset come back transposed into the first columns
            assert np.array_equal(got[:off, off:off + p].T, got[off:off + p, :off])
    assert int(lib.lobpcg_gram_noalloc_max_bytes()) == 16 << 20


def test_gram_noalloc_rejects_products_beyond_its_scratch(lib):
    torch = _torch()
    from paper_1704_07458_amd import binding as B

    m = p = 1500  # 1500 * 1500 * 8 bytes = 18 MB > 16 MiB
    L = torch.zeros((64, m), dtype=torch.float64, device="cuda")
    with pytest.raises(B.LobpcgError) as e:
        B.gram_noalloc(L, L)
    assert e.value.code == -1 and "exceeds the fixed scratch" in str(e.value)
