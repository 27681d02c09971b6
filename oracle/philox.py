"""Philox4x64-10 counter-based generator (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11), written from that definition.

Test infrastructure: part of the FP64 oracle.

A block maps a 256-bit counter (four 64-bit words) and a 128-bit key (two
words) to four 64-bit outputs by ten rounds of

    (hi0, lo0) = mulhilo(M0, x0);  (hi1, lo1) = mulhilo(M1, x2)
    x = (hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0)

with the key bumped by the Weyl constants (W0, W1) between rounds.

The estimator consumes it as follows (the same convention on every side):
key = (seed, chain); counter = (step, index, purpose, 0); a 64-bit word u
becomes the double (u >> 11) * 2^-53 in [0, 1).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

# purposes of the counter's third word
PURPOSE_MOVE, PURPOSE_ACCEPT, PURPOSE_TAU = 0, 1, 2


def _mulhilo(a: np.ndarray, b: np.uint64):
    """128-bit product of uint64 arrays split into (hi, lo) words."""
    a = np.asarray(a, dtype=np.uint64)
    with np.errstate(over="ignore"):
        a_lo, a_hi = a & _MASK32, a >> _S32
        b_lo, b_hi = b & _MASK32, b >> _S32
        ll = a_lo * b_lo
        hl = a_hi * b_lo
        lh = a_lo * b_hi
        hh = a_hi * b_hi
        cross = (ll >> _S32) + (hl & _MASK32) + lh
        hi = hh + (hl >> _S32) + (cross >> _S32)
        lo = a * b
    return hi, lo


def philox4x64(counter, key, rounds: int = 10) -> np.ndarray:
    """Philox4x64 block function.

    counter : array [..., 4] of uint64; key : array [..., 2] (broadcastable).
    Returns array [..., 4] of uint64.
    """
    x = np.array(counter, dtype=np.uint64, copy=True)
    k = np.array(key, dtype=np.uint64, copy=True)
    x0, x1, x2, x3 = (x[..., i] for i in range(4))
    k0 = np.broadcast_to(k[..., 0], x0.shape).copy()
    k1 = np.broadcast_to(k[..., 1], x0.shape).copy()
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r > 0:
                k0 = k0 + W0
                k1 = k1 + W1
            hi0, lo0 = _mulhilo(x0, M0)
            hi1, lo1 = _mulhilo(x2, M1)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return np.stack([x0, x1, x2, x3], axis=-1)


def to_unit(u: np.ndarray) -> np.ndarray:
    """53-bit uniform double in [0, 1) from a 64-bit word."""
    return (np.asarray(u, dtype=np.uint64) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def draw(key, step: int, index, purpose: int) -> np.ndarray:
    """Four uniforms [..., 4] for counter (step, index, purpose, 0)."""
    index = np.asarray(index, dtype=np.uint64)
    ctr = np.zeros(index.shape + (4,), dtype=np.uint64)
    ctr[..., 0] = np.uint64(step)
    ctr[..., 1] = index
    ctr[..., 2] = np.uint64(purpose)
    return to_unit(philox4x64(ctr, np.asarray(key, dtype=np.uint64)))
