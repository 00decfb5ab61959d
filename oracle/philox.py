"""Philox4x64-10 counter-based generator (oracle; test infrastructure).

Published definition: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11.  State: a 4-word
counter (x0, x1, x2, x3) and a 2-word key (k0, k1), all 64-bit.  One round
multiplies x0 and x2 by two fixed constants into 128-bit products and mixes

    x' = (hi(M1*x2) ^ x1 ^ k0,  lo(M1*x2),  hi(M0*x0) ^ x3 ^ k1,  lo(M0*x0)),

after which the key is bumped by two Weyl constants (golden ratio and
sqrt(3) - 1, as 64-bit fractions).  Ten rounds make one 4-word output block.

Two implementations: ``philox4x64_10`` on Python integers (one block) and
``philox4x64_10_np`` vectorised over numpy uint64 counter arrays with the
128-bit products built from 32-bit halves.  The paper does not name a
generator; this one is chosen so that the GPU and the oracle can draw the
same samples from a (key, counter) pair without sharing a stream of numbers.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1


def philox4x64_10(ctr, key):
    """One Philox4x64-10 block on Python ints: ctr (4 words), key (2 words)."""
    x0, x1, x2, x3 = (int(v) & MASK64 for v in ctr)
    k0, k1 = (int(v) & MASK64 for v in key)
    for _ in range(10):
        p0 = M0 * x0
        p1 = M1 * x2
        x0, x1, x2, x3 = ((p1 >> 64) ^ x1 ^ k0) & MASK64, p1 & MASK64, \
                         ((p0 >> 64) ^ x3 ^ k1) & MASK64, p0 & MASK64
        k0 = (k0 + W0) & MASK64
        k1 = (k1 + W1) & MASK64
    return (x0, x1, x2, x3)


_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def mulhilo64_np(a, b):
    """(hi, lo) 64-bit halves of the 128-bit products a*b (numpy uint64)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a0, a1 = a & _LO32, a >> _S32
    b0, b1 = b & _LO32, b >> _S32
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    with np.errstate(over="ignore"):
        lo = a * b
    return hi, lo


def philox4x64_10_np(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x64-10: counter words as uint64 arrays (broadcast)."""
    x0, x1, x2, x3 = (np.asarray(v, dtype=np.uint64) for v in np.broadcast_arrays(c0, c1, c2, c3))
    x0, x1, x2, x3 = x0.copy(), x1.copy(), x2.copy(), x3.copy()
    k0 = np.uint64(k0)
    k1 = np.uint64(k1)
    m0, m1, w0, w1 = np.uint64(M0), np.uint64(M1), np.uint64(W0), np.uint64(W1)
    with np.errstate(over="ignore"):
        for _ in range(10):
            hi0, lo0 = mulhilo64_np(m0, x0)
            hi1, lo1 = mulhilo64_np(m1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
            k0 = k0 + w0
            k1 = k1 + w1
    return x0, x1, x2, x3
