"""Philox4x64-10 counter-based generator, written from its published definition.

Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11.  A block maps a 4x64-bit counter and a 2x64-bit key through 10 rounds;
each round multiplies counter words 0 and 2 by two fixed odd constants,
swaps/xors the high halves with the other words and the key, and the key is
bumped by two Weyl constants between rounds.

The paper draws its projection matrix Theta and the GCN weights W at random
(Sec. III-A Eq. 5; Sec. III-B).  Both sides of the parity check draw those
numbers from this generator, addressed by (key, counter), so that the draws do
not depend on thread order.

Pinned against ``numpy.random.Philox`` (a library implementation of the same
generator) in ``tests/test_oracle_random.py``.
"""
import numpy as np

MASK32 = np.uint64(0xFFFFFFFF)
M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
ROUNDS = 10

# stream ids (key word 1) used by the method
STREAM_THETA = 0x10          # projection matrix Theta (R)
STREAM_W_BASE = 0x10         # GCN layer k (1-based) uses 0x10 + k
STREAM_RACE = 0x20           # k-means++ exponential race


def _mulhilo(a, b):
    """Full 64x64 -> 128 bit product of uint64 arrays; returns (hi, lo)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a0, a1 = a & MASK32, a >> np.uint64(32)
    b0, b1 = b & MASK32, b >> np.uint64(32)
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> np.uint64(32)) + (p01 & MASK32) + (p10 & MASK32)
    hi = p11 + (p01 >> np.uint64(32)) + (p10 >> np.uint64(32)) + (mid >> np.uint64(32))
    with np.errstate(over="ignore"):
        lo = a * b
    return hi, lo


def philox4x64(ctr, key):
    """One Philox4x64-10 block.

    ctr: uint64 array of shape (..., 4); key: uint64 array of shape (..., 2)
    (broadcastable).  Returns a uint64 array of shape (..., 4).
    """
    ctr = np.asarray(ctr, dtype=np.uint64)
    key = np.asarray(key, dtype=np.uint64)
    x0, x1, x2, x3 = (ctr[..., i].copy() for i in range(4))
    k0 = np.broadcast_to(key[..., 0], x0.shape).copy()
    k1 = np.broadcast_to(key[..., 1], x0.shape).copy()
    with np.errstate(over="ignore"):
        for r in range(ROUNDS):
            if r > 0:
                k0 = k0 + W0
                k1 = k1 + W1
            hi0, lo0 = _mulhilo(M0, x0)
            hi1, lo1 = _mulhilo(M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return np.stack([x0, x1, x2, x3], axis=-1)


def block_grid(seed, stream, rows, col_blocks):
    """Philox blocks for counters (row, col_block, 0, 0), key (seed, stream).

    Returns uint64 array [rows, col_blocks, 4].  This is the layout used for
    every random matrix of the method: row r, columns 4*cb .. 4*cb+3.
    """
    r = np.arange(rows, dtype=np.uint64)[:, None]
    c = np.arange(col_blocks, dtype=np.uint64)[None, :]
    ctr = np.zeros((rows, col_blocks, 4), dtype=np.uint64)
    ctr[..., 0] = r
    ctr[..., 1] = c
    key = np.array([seed, stream], dtype=np.uint64)
    return philox4x64(ctr, key)
