"""Philox4x32-10 counter-based random numbers, vectorised over numpy arrays.

Definition: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11, section 4 (the Philox-4x32 bijection with
multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key increments 0x9E3779B9 / 0xBB67AE85
and 10 rounds).

This module is an input generator only: it holds none of the matrix-element
arithmetic.  Every random draw is a pure function of (key, counter), so the
synthetic momenta of event i do not depend on how a batch is split.
"""
from __future__ import annotations

import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint32(0x9E3779B9)
_W1 = np.uint32(0xBB67AE85)
_MASK32 = np.uint64(0xFFFFFFFF)
_SHIFT32 = np.uint64(32)


def philox4x32(counter, key, rounds: int = 10):
    """Apply Philox4x32-``rounds`` to broadcastable uint32 arrays.

    counter: tuple of four uint32 arrays (c0, c1, c2, c3)
    key:     tuple of two uint32 arrays (k0, k1)
    returns: tuple of four uint32 arrays
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint32) for c in counter)
    k0, k1 = (np.asarray(k, dtype=np.uint32) for k in key)
    c0, c1, c2, c3, k0, k1 = np.broadcast_arrays(c0, c1, c2, c3, k0, k1)
    c0, c1, c2, c3 = (c.astype(np.uint32, copy=True) for c in (c0, c1, c2, c3))
    k0 = k0.astype(np.uint32, copy=True)
    k1 = k1.astype(np.uint32, copy=True)
    with np.errstate(over="ignore"):
        for r in range(rounds):
            p0 = _M0 * c0.astype(np.uint64)
            p1 = _M1 * c2.astype(np.uint64)
            hi0 = (p0 >> _SHIFT32).astype(np.uint32)
            lo0 = (p0 & _MASK32).astype(np.uint32)
            hi1 = (p1 >> _SHIFT32).astype(np.uint32)
            lo1 = (p1 & _MASK32).astype(np.uint32)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
            if r != rounds - 1:
                k0 = k0 + _W0
                k1 = k1 + _W1
    return c0, c1, c2, c3


def uniform_pairs(words):
    """Turn four uint32 words into two doubles in the open interval (0, 1).

    Each double takes 53 random bits (27 from one word, 26 from the next) and is
    offset by half an ulp so that neither 0 nor 1 can occur.
    """
    w0, w1, w2, w3 = words
    a = (w0 >> np.uint32(5)).astype(np.float64)
    b = (w1 >> np.uint32(6)).astype(np.float64)
    c = (w2 >> np.uint32(5)).astype(np.float64)
    d = (w3 >> np.uint32(6)).astype(np.float64)
    scale = 1.0 / 9007199254740992.0  # 2**-53
    u0 = (a * 67108864.0 + b + 0.5) * scale
    u1 = (c * 67108864.0 + d + 0.5) * scale
    return u0, u1
