"""Counter-based random numbers for the randomized ID of Section 4.3 (test
infrastructure: only tests, smoke checks and the CPU baseline use the
oracle).

The paper's accelerated compression can sample ``Phi_c A_{c^N, c}`` with a
small Gaussian matrix ``Phi_c``.  So that the oracle and the library draw the
same ``Phi_c`` without sharing code or buffers, each implements the same
published generator: Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC 2011), turned into normal deviates by
the Box-Muller transform.

Philox4x32-10 maps a 128-bit counter (c0, c1, c2, c3) and a 64-bit key
(k0, k1) through ten rounds; one round multiplies c0 and c2 by two constants
into 64-bit products and returns
``(hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))``; the key
gains the Weyl increments (W0, W1) between rounds.

The sketch of a group has ``|c| + 16`` rows (``sketch_rows``).  Element
(i, t) of the sketch of group ``gid`` at level ``l`` uses the counter
``(i, t, gid, l)`` and the key ``SKETCH_KEY``; its words x0, x1 give
``u = (x + 1/2) 2^-32`` and the deviate ``sqrt(-2 ln u0) cos(2 pi u1)``.

Pinned by: the generator's published known-answer vectors, and the moments
and distribution of the deviates (tests/test_oracle_sketch.py).
"""
from __future__ import annotations

import numpy as np

M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
W0, W1 = np.uint32(0x9E3779B9), np.uint32(0xBB67AE85)
ROUNDS = 10
# the key of every sketch (any fixed value; both sides use this one)
SKETCH_KEY = (0x7F4A7C15, 0x9E3779B9)
# rows drawn beyond |c| (oversampling: the sketch of a block with up to |c|
# independent columns needs a few more rows than |c| to keep their geometry)
SKETCH_OVERSAMPLE = 16


def sketch_rows(nc: int, nn: int) -> int:
    """Rows of the sketch of a ``nn x nc`` block; ``nn`` (no sketch) when
    sampling would not shorten it."""
    return min(nn, nc + SKETCH_OVERSAMPLE)


_MASK = np.uint64(0xFFFFFFFF)
_SH = np.uint64(32)


def philox4x32(c0, c1, c2, c3, k0, k1, rounds: int = ROUNDS):
    """Vectorized Philox4x32: arrays (or scalars) of uint32 counter words
    and a key; returns the four output words as uint32 arrays."""
    c = [np.asarray(x, dtype=np.uint32).copy() for x in (c0, c1, c2, c3)]
    k0 = np.uint32(k0)
    k1 = np.uint32(k1)
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r > 0:
                k0 = np.uint32(k0 + W0)
                k1 = np.uint32(k1 + W1)
            p0 = M0 * c[0].astype(np.uint64)
            p1 = M1 * c[2].astype(np.uint64)
            hi0, lo0 = (p0 >> _SH).astype(np.uint32), (p0 & _MASK).astype(np.uint32)
            hi1, lo1 = (p1 >> _SH).astype(np.uint32), (p1 & _MASK).astype(np.uint32)
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def normal_from_words(x0, x1):
    """Box-Muller (cosine branch) on two uint32 words."""
    u0 = (np.asarray(x0, dtype=np.float64) + 0.5) * 2.0 ** -32
    u1 = (np.asarray(x1, dtype=np.float64) + 0.5) * 2.0 ** -32
    return np.sqrt(-2.0 * np.log(u0)) * np.cos(2.0 * np.pi * u1)


def sketch_matrix(level: int, gid: int, rows: int, cols: int) -> np.ndarray:
    """The ``rows x cols`` Gaussian sampling matrix of group ``gid`` at
    level ``level``."""
    i, t = np.meshgrid(np.arange(rows, dtype=np.uint32), np.arange(cols, dtype=np.uint32),
                       indexing="ij")
    g = np.full(i.shape, np.uint32(gid & 0xFFFFFFFF))
    lv = np.full(i.shape, np.uint32(level))
    x = philox4x32(i, t, g, lv, *SKETCH_KEY)
    return normal_from_words(x[0], x[1])
