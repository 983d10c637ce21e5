"""Philox4x32-10 counter-based generator and the value maps built on it (NumPy side).

This module holds none of the contraction method's arithmetic: it only turns
(seed, tensor id, element index) into a reproducible floating-point value, so
that the CPU oracle and the GPU library can be fed bit-identical inputs without
ever copying data from one to the other.  The GPU twin of every function here
lives in ``synth/csrc/synth_gen.hip``; a GPU test checks the two bit for bit.

Philox4x32 follows Salmon, Moraes, Dror and Shaw, "Parallel random numbers:
as easy as 1, 2, 3" (SC'11): per round the two multipliers act on counter
words 0 and 2, the high halves are xor-ed with the other two words and the key,
and the key is bumped by the two Weyl constants between rounds.  Ten rounds.

Value maps (element e of a tensor, key = (seed, tensor_id)):

* ``uniform`` in [-1, 1): one block at counter (e_lo, e_hi, 0, 0); the 53 high
  bits of (w1:w0) give k, and x = k * 2^-52 - 1, exact in binary64.
* ``normal`` (mean 0, variance 1): the Irwin-Hall sum of twelve U(0,1) draws
  minus 6.  Three blocks at counters (e_lo, e_hi, d, 0), d = 0, 1, 2, give
  twelve 32-bit words w_i; x = (sum w_i) * 2^-32 - 6, computed from the exact
  integer sum, so it is exact in binary64 and independent of summation order.

An optional scale is applied as one correctly rounded binary64 multiply.
"""
from __future__ import annotations

import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
_MASK32 = np.uint64(0xFFFFFFFF)

DIST_UNIFORM = 0
DIST_NORMAL = 1


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox4x32 rounds over arrays of counters; returns four uint32 arrays.

    Arguments are array-likes of unsigned 32-bit values (broadcast together);
    the arithmetic runs in uint64 so that 32x32->64 products are exact.
    """
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & _MASK32 for x in (c0, c1, c2, c3))
    k0 = np.uint64(int(k0) & 0xFFFFFFFF)
    k1 = np.uint64(int(k1) & 0xFFFFFFFF)
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    for r in range(10):
        if r > 0:
            k0 = np.uint64((int(k0) + PHILOX_W0) & 0xFFFFFFFF)
            k1 = np.uint64((int(k1) + PHILOX_W1) & 0xFFFFFFFF)
        p0 = m0 * c0
        p1 = m1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def values_at(e, seed: int, tensor_id: int, dist: int, scale: float = 1.0) -> np.ndarray:
    """Binary64 values of elements ``e`` (int64 array of linear indices)."""
    e = np.asarray(e, dtype=np.uint64)
    elo = e & _MASK32
    ehi = e >> np.uint64(32)
    zero = np.zeros_like(elo)
    if dist == DIST_UNIFORM:
        w0, w1, _, _ = philox4x32_10(elo, ehi, zero, zero, seed, tensor_id)
        k = ((w1.astype(np.uint64) << np.uint64(32)) | w0.astype(np.uint64)) >> np.uint64(11)
        x = k.astype(np.float64) * 2.0 ** -52 - 1.0
    elif dist == DIST_NORMAL:
        s = np.zeros(e.shape, dtype=np.uint64)
        for d in range(3):
            ws = philox4x32_10(elo, ehi, zero + np.uint64(d), zero, seed, tensor_id)
            for w in ws:
                s += w.astype(np.uint64)
        x = s.astype(np.float64) * 2.0 ** -32 - 6.0
    else:
        raise ValueError(f"unknown distribution {dist}")
    if scale != 1.0:
        x = x * np.float64(scale)
    return x


def fill(shape, seed: int, tensor_id: int, dist: int, scale: float = 1.0,
         chunk: int = 1 << 22) -> np.ndarray:
    """A whole C-ordered array whose element with linear index e is values_at(e)."""
    shape = tuple(int(s) for s in shape)
    n = int(np.prod(shape, dtype=np.int64)) if shape else 1
    out = np.empty(n, dtype=np.float64)
    for lo in range(0, n, chunk):
        hi = min(n, lo + chunk)
        out[lo:hi] = values_at(np.arange(lo, hi, dtype=np.int64), seed, tensor_id, dist, scale)
    return out.reshape(shape)
