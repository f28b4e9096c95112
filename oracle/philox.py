"""Philox-4x32-10 counter-based generator and the white-noise field.

Test infrastructure only.  The paper draws its white noise with N-GenIC's
generator (Sec. "Miscellaneous features"), which is not reproduced; the build
uses Philox-4x32-10 as published by Salmon, Moraes, Dror & Shaw, "Parallel
random numbers: as easy as 1, 2, 3" (SC'11), re-implemented here
independently of the HIP path.

Mapping of the stream to the white-noise field w (unit-variance Gaussian in
real space on the particle lattice, Sec. "Correctness of the adjoint method"):
  counter = (i mod 2^32, i div 2^32, 0, 0) with i the row-major lattice index,
  key     = (seed mod 2^32, seed div 2^32),
  u1 = (((x0 << 32 | x1) >> 11) + 1/2) 2^-53 in (0, 1),
  u2 =  ((x2 << 32 | x3) >> 11) 2^-53 in [0, 1),
  w_i = sqrt(-2 ln u1) cos(2 pi u2) in FP64, rounded once to FP32.
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: 4 arrays of uint32 values, key: 2 arrays/scalars; returns 4 uint64
    arrays holding the 32-bit outputs."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) for c in ctr)
    k0 = np.asarray(key[0], dtype=np.uint64)
    k1 = np.asarray(key[1], dtype=np.uint64)
    m0, m1 = np.uint64(M0), np.uint64(M1)
    for _ in range(10):
        p0 = m0 * c0          # 32x32 -> 64-bit products are exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + np.uint64(W0)) & MASK
        k1 = (k1 + np.uint64(W1)) & MASK
    return c0, c1, c2, c3


def raw_stream(seed, n_total):
    i = np.arange(n_total, dtype=np.uint64)
    seed = int(seed)
    return philox4x32_10((i & MASK, i >> np.uint64(32), np.zeros_like(i), np.zeros_like(i)),
                         (seed & 0xFFFFFFFF, seed >> 32))


def white_noise(seed, n):
    """w on the n^3 particle lattice, FP32, shape (n, n, n) (z fastest)."""
    x0, x1, x2, x3 = raw_stream(seed, n ** 3)
    s11 = np.uint64(11)
    h1 = ((x0 << np.uint64(32)) | x1) >> s11
    h2 = ((x2 << np.uint64(32)) | x3) >> s11
    u1 = (h1.astype(np.float64) + 0.5) * 2.0 ** -53
    u2 = h2.astype(np.float64) * 2.0 ** -53
    w = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    return w.astype(np.float32).reshape(n, n, n)
