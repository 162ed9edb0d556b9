"""Philox4x32-10, written from its definition in Salmon, Moraes, Dror and
Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11).

The paper's own generators are per-thread STL engines (section "Pseudo-random
number generation"), whose streams depend on the thread count; it names the
Random123 family as the direction it would take.  A counter-based generator
makes every random quantity a pure function of (seed, index), which is what
lets the device path and this oracle agree bit for bit.

Definition used here (N = 4 words of 32 bits, R = 10 rounds):

* state  X = (x0, x1, x2, x3), key K = (k0, k1);
* one round multiplies x0 by M0 = 0xD2511F53 and x2 by M1 = 0xCD9E8D57 as
  64-bit products and returns
  (hi(M1*x2) ^ x1 ^ k0,  lo(M1*x2),  hi(M0*x0) ^ x3 ^ k1,  lo(M0*x0));
* between rounds the key advances by the Weyl constants
  (k0 += 0x9E3779B9, k1 += 0xBB67AE85) modulo 2^32; the first round uses the
  key as given.

Vectorised over many counters with NumPy uint64 arithmetic.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)
SH32 = np.uint64(32)


def philox4x32(ctr, key, rounds=10):
    """Apply Philox4x32-``rounds`` to counters.

    ctr : array (..., 4) of unsigned 32-bit words.
    key : array (..., 2) (broadcast against ``ctr``'s leading shape) or a pair.
    Returns an array (..., 4) of uint32.
    """
    c = np.asarray(ctr, dtype=np.uint64)
    k = np.asarray(key, dtype=np.uint64)
    x0, x1, x2, x3 = (c[..., 0].copy(), c[..., 1].copy(),
                      c[..., 2].copy(), c[..., 3].copy())
    k0 = np.broadcast_to(k[..., 0], x0.shape).astype(np.uint64)
    k1 = np.broadcast_to(k[..., 1], x0.shape).astype(np.uint64)
    for rnd in range(rounds):
        if rnd:
            k0 = (k0 + np.uint64(W0)) & MASK32
            k1 = (k1 + np.uint64(W1)) & MASK32
        p0 = M0 * x0          # < 2^64, exact in uint64
        p1 = M1 * x2
        n0 = ((p1 >> SH32) ^ x1 ^ k0) & MASK32
        n1 = p1 & MASK32
        n2 = ((p0 >> SH32) ^ x3 ^ k1) & MASK32
        n3 = p0 & MASK32
        x0, x1, x2, x3 = n0, n1, n2, n3
    return np.stack([x0, x1, x2, x3], axis=-1).astype(np.uint32)


def seed_key(seed):
    """Key words of a 64-bit seed: (low 32 bits, high 32 bits)."""
    s = int(seed) & 0xFFFFFFFFFFFFFFFF
    return np.array([s & 0xFFFFFFFF, s >> 32], dtype=np.uint64)
