"""Philox4x32-10 and the Uniform(l-u, u-l) start points of Algorithm 2 --
oracle, test infrastructure only.

Philox4x32-10 is the counter-based generator of Salmon, Moraes, Dror and
Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of
  (c0, c1, c2, c3) <- (hi(M1 c2) ^ c1 ^ k0, lo(M1 c2), hi(M0 c0) ^ c3 ^ k1, lo(M0 c0))
with M0 = 0xD2511F53, M1 = 0xCD9E8D57 and the key bumped by
(0x9E3779B9, 0xBB67AE85) between rounds.

Start points (Algorithm 2, lines drawing g and projecting it): for start s
and coordinate j, counter = (j // 2, s mod 2^32, s div 2^32, 0) and
key = (seed mod 2^32, seed div 2^32).  Output words (w0, w1) serve even j and
(w2, w3) odd j; a 53-bit integer (wa >> 5) * 2^26 + (wb >> 6) scaled by
2^-53 gives U in [0, 1), and g_j = (l_j - u_j) + U * (2 (u_j - l_j)).
The coordinates are z_j = sum_i P_ji g_i (ascending i, from 0.0).
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Vectorised Philox4x32-10.  ctr: 4 arrays of uint32-valued integers,
    key: 2 arrays/ints.  Returns 4 uint64 arrays holding 32-bit words."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & MASK for c in ctr)
    k0 = np.asarray(key[0], dtype=np.uint64) & MASK
    k1 = np.asarray(key[1], dtype=np.uint64) & MASK
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + np.uint64(W0)) & MASK
            k1 = (k1 + np.uint64(W1)) & MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ k0), lo1, (hi0 ^ c3 ^ k1), lo0
    return c0, c1, c2, c3


def uniform01(n_starts: int, n: int, seed: int, first_start: int = 0) -> np.ndarray:
    """U[s, j] in [0, 1) for starts first_start .. first_start+n_starts-1."""
    s = np.arange(first_start, first_start + n_starts, dtype=np.uint64)[:, None]
    j = np.arange(n, dtype=np.uint64)[None, :]
    pair = j // np.uint64(2)
    shape = (n_starts, n)
    ctr = (np.broadcast_to(pair, shape), np.broadcast_to(s & MASK, shape),
           np.broadcast_to(s >> np.uint64(32), shape), np.zeros(shape, np.uint64))
    key = (np.uint64(seed & 0xFFFFFFFF), np.uint64((seed >> 32) & 0xFFFFFFFF))
    w0, w1, w2, w3 = philox4x32_10(ctr, key)
    odd = (j % np.uint64(2)) == np.uint64(1)
    wa = np.where(odd, w2, w0)
    wb = np.where(odd, w3, w1)
    a = (wa >> np.uint64(5)).astype(np.float64)
    b = (wb >> np.uint64(6)).astype(np.float64)
    return (a * 67108864.0 + b) * (1.0 / 9007199254740992.0)


def box_starts(P: np.ndarray, l, u, n_starts: int, seed: int, first_start: int = 0):
    """(g, z0): g ~ Uniform(l-u, u-l) componentwise and z0 = P g (Algorithm 2)."""
    lo = (np.asarray(l) - np.asarray(u)).astype(np.float64)
    width = (2 * (np.asarray(u) - np.asarray(l))).astype(np.float64)
    U = uniform01(n_starts, lo.shape[0], seed, first_start)
    g = lo[None, :] + U * width[None, :]
    d, n = P.shape
    z = np.zeros((n_starts, d))
    for i in range(n):
        z = z + P[:, i][None, :] * g[:, i][:, None]
    return g, z
