"""Gaussian test matrix Omega for the randomized range finder.

Sec. 3 (Fig. rsvd (b1)) draws Omega with i.i.d. Gaussian entries.  The stream
is counter based so that the CPU oracle and the GPU draw the same matrix
without sharing code: Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11) turns a 256-bit counter and a
128-bit key into four 64-bit words; two words make one Box-Muller pair.

Element (i, j) of the m x k matrix (row i = column index of the two-site
matrix in its (s2, u2, c'') row-major order, column j = sketch column) has
linear index e = i*k + j and uses
    counter = (e // 4, bond, stream, pair),   key = (seed, 0),
    words w0..w3 = Philox4x64-10(counter, key),
    u(w) = ((w >> 11) + 1/2) * 2**-53 in (0, 1),
    q = (e % 4) // 2:  rad = sqrt(-2 ln u(w_{2q})), ang = 2 pi u(w_{2q+1}),
    value = rad * cos(ang) if e is even else rad * sin(ang).

Pinned by: the raw integer stream against ``numpy.random.Philox`` (an
independent implementation of the same bijection), and the normals by
moment / Kolmogorov-Smirnov checks.
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
# Philox4x64 multipliers and Weyl key increments (Salmon et al., SC'11, Table 2).
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B


def _mulhilo(a: int, b: int) -> tuple[int, int]:
    p = a * b
    return (p >> 64) & MASK64, p & MASK64


def philox4x64_10(ctr: tuple[int, int, int, int], key: tuple[int, int]) -> tuple[int, int, int, int]:
    """Ten Philox rounds: S-box by two 64x64->128 multiplies, P-box by a word
    swap, key bumped by the Weyl constants between rounds."""
    c0, c1, c2, c3 = (int(x) & MASK64 for x in ctr)
    k0, k1 = (int(x) & MASK64 for x in key)
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        hi0, lo0 = _mulhilo(PHILOX_M0, c0)
        hi1, lo1 = _mulhilo(PHILOX_M1, c2)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniform53(w: int) -> float:
    """Open-interval uniform from the top 53 bits of a 64-bit word."""
    return ((w >> 11) + 0.5) * 2.0 ** -53


def gaussian_matrix(m: int, k: int, seed: int, pair: int, stream: int, bond: int) -> np.ndarray:
    """The m x k test matrix Omega (FP64), element (i, j) as in the module
    docstring.  Pure Python loops: meant for the sizes of one bond update."""
    out = np.empty(m * k, dtype=np.float64)
    n = m * k
    key = (seed & MASK64, 0)
    for blk in range((n + 3) // 4):
        w = philox4x64_10((blk, bond, stream, pair), key)
        for q in range(2):
            u1 = uniform53(w[2 * q])
            u2 = uniform53(w[2 * q + 1])
            rad = np.sqrt(-2.0 * np.log(u1))
            ang = 2.0 * np.pi * u2
            for h, val in ((0, rad * np.cos(ang)), (1, rad * np.sin(ang))):
                e = 4 * blk + 2 * q + h
                if e < n:
                    out[e] = val
    return out.reshape(m, k)


def raw_words(n_blocks: int, bond: int, stream: int, pair: int, seed: int) -> np.ndarray:
    """Raw 64-bit words of blocks 0..n_blocks-1 of one bond's stream."""
    key = (seed & MASK64, 0)
    out = np.empty(4 * n_blocks, dtype=np.uint64)
    for blk in range(n_blocks):
        out[4 * blk:4 * blk + 4] = philox4x64_10((blk, bond, stream, pair), key)
    return out
