"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11), vectorised in numpy.

Written from the published definition: a 4-word counter and a 2-word key; each of the
ten rounds multiplies counter words 0 and 2 by two fixed odd constants, takes the high
and low halves of the 64-bit products, and xors the high halves with the other two
counter words and the round key; the key is bumped by two Weyl constants between
rounds. Nothing here knows about vehicles: it only turns (key, counter) into words.
"""
from __future__ import annotations

import numpy as np

_MASK = np.uint64(0xFFFFFFFF)
_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = np.uint64(0x9E3779B9)
_W1 = np.uint64(0xBB67AE85)


def philox4x32(ctr, key, rounds: int = 10) -> np.ndarray:
    """Return uint32 words [..., 4] for counters ``ctr`` [..., 4] and keys ``key`` [..., 2].

    ``ctr`` and ``key`` broadcast against each other; both are taken modulo 2**32.
    """
    ctr = np.asarray(ctr, dtype=np.uint64) & _MASK
    key = np.asarray(key, dtype=np.uint64) & _MASK
    shape = np.broadcast_shapes(ctr.shape[:-1], key.shape[:-1])
    c0 = np.broadcast_to(ctr[..., 0], shape).copy()
    c1 = np.broadcast_to(ctr[..., 1], shape).copy()
    c2 = np.broadcast_to(ctr[..., 2], shape).copy()
    c3 = np.broadcast_to(ctr[..., 3], shape).copy()
    k0 = np.broadcast_to(key[..., 0], shape).copy()
    k1 = np.broadcast_to(key[..., 1], shape).copy()
    for r in range(rounds):
        if r:
            k0 = (k0 + _W0) & _MASK
            k1 = (k1 + _W1) & _MASK
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def u24(words: np.ndarray) -> np.ndarray:
    """Uniform on [0, 1) from the top 24 bits of each word (exact in float32)."""
    return (words.astype(np.uint64) >> np.uint64(8)).astype(np.float64) * 2.0 ** -24


def u53(w_hi: np.ndarray, w_lo: np.ndarray) -> np.ndarray:
    """Uniform on [0, 1) with 53 random bits taken from two words."""
    a = (w_hi.astype(np.uint64) >> np.uint64(5)).astype(np.float64)
    b = (w_lo.astype(np.uint64) >> np.uint64(6)).astype(np.float64)
    return (a * 67108864.0 + b) * 2.0 ** -53


def action_value(words: np.ndarray) -> np.ndarray:
    """Action in [-1, 1) from a word: ((w >> 8) - 2**23) * 2**-23, exact in float32."""
    j = (words.astype(np.int64) >> 8) - (1 << 23)
    return (j.astype(np.float64) * 2.0 ** -23).astype(np.float32)
