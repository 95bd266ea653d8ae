"""Counter-based Gaussian numbers for the norm sketch of section 4.3.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

Section 4.3 estimates ||A||_2 from A applied to a Gaussian random matrix Omega.
The random numbers are drawn inside the solver, so they cannot be handed to it
as an input; instead both sides implement the same published counter-based
generator, Philox-4x32 with 10 rounds (Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11), and map its output to
normal deviates with the Box-Muller transform.  This module is the oracle's
own NumPy implementation, written from that paper's definition:

  state: four 32-bit counter words c0..c3 and two 32-bit key words k0, k1;
  round: (hi0, lo0) = M0 * c0, (hi1, lo1) = M1 * c2 (64-bit products),
         (c0, c1, c2, c3) <- (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0),
         then the key is bumped by the Weyl constants (W0, W1) mod 2^32;
  10 rounds, the first with the unbumped key;
  M0 = 0xD2511F53, M1 = 0xCD9E8D57, W0 = 0x9E3779B9, W1 = 0xBB67AE85.

Element layout of a generated n x m block (row-major, element e = i*m + j):
the pair of elements (2q, 2q+1) comes from the counter (q mod 2^32,
q div 2^32, stream, 0) under the key (seed mod 2^32, seed div 2^32);
u1 = ((c0 * 2^32 + c1) >> 11 + 1) * 2^-53 in (0, 1],
u2 = ((c2 * 2^32 + c3) >> 11) * 2^-53 in [0, 1),
element 2q = sqrt(-2 ln u1) cos(2 pi u2), element 2q+1 = sqrt(-2 ln u1) sin(2 pi u2).

Streams: 0 is the initial block the solver draws when none is given, 1 is
the sketch Omega of section 4.3.
"""

from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)

STREAM_INITIAL_BLOCK = 0
STREAM_SKETCH = 1


def philox4x32_10(c0, c1, c2, c3, k0: int, k1: int):
    """Ten Philox-4x32 rounds on arrays of counter words (uint32); returns 4 uint32 arrays."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) for c in (c0, c1, c2, c3))
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for _ in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0
        k0 = (k0 + W0) & 0xFFFFFFFF
        k1 = (k1 + W1) & 0xFFFFFFFF
    return tuple(c.astype(np.uint32) for c in (c0, c1, c2, c3))


def uniform_pair(c0, c1, c2, c3):
    """(u1 in (0, 1], u2 in [0, 1)) from the 53 high bits of each 64-bit half."""
    w1 = (c0.astype(np.uint64) << np.uint64(32)) | c1.astype(np.uint64)
    w2 = (c2.astype(np.uint64) << np.uint64(32)) | c3.astype(np.uint64)
    u1 = ((w1 >> np.uint64(11)).astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = (w2 >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return u1, u2


def box_muller(u1, u2):
    """Two independent N(0, 1) deviates from two uniforms (Box and Muller, 1958)."""
    r = np.sqrt(-2.0 * np.log(u1))
    a = 2.0 * np.pi * u2
    return r * np.cos(a), r * np.sin(a)


def gaussian_block(seed: int, stream: int, n: int, m: int) -> np.ndarray:
    """n x m row-major block of N(0, 1) numbers in the layout of the module docstring."""
    total = n * m
    npairs = (total + 1) // 2
    q = np.arange(npairs, dtype=np.uint64)
    c0 = q & MASK32
    c1 = q >> np.uint64(32)
    c2 = np.full(npairs, stream & 0xFFFFFFFF, dtype=np.uint64)
    c3 = np.zeros(npairs, dtype=np.uint64)
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    o = philox4x32_10(c0, c1, c2, c3, seed & 0xFFFFFFFF, seed >> 32)
    z0, z1 = box_muller(*uniform_pair(*o))
    out = np.empty(2 * npairs)
    out[0::2] = z0
    out[1::2] = z1
    return out[:total].reshape(n, m)


def sketch(seed: int, n: int, m: int) -> np.ndarray:
    """Omega^T of section 4.3 (n x m, m sketch rows): stream 1 of the generator."""
    return gaussian_block(seed, STREAM_SKETCH, n, m)
