"""Philox4x32-10 and Box-Muller Gaussians, in NumPy (test infrastructure only).

Philox4x32-10 follows its published definition: J. K. Salmon, M. A. Moraes,
R. O. Dror, D. E. Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11,
Sec. 4 (the Philox S-box built from two 32x32->64 multiplications, ten rounds,
Weyl key schedule).  Pinned by the known-answer vectors in
tests/golden/philox4x32_10_kat.txt.

Gaussian layout (the contract the library's seeded draw also states in
include/powerlu.h): a rows x cols row-major matrix; element e = i*cols + j
belongs to Philox block g = e // 4, output word t = e % 4.  Block g uses
counter (g mod 2^32, g div 2^32, 0, 0) and key (seed mod 2^32, seed div 2^32).
Words are mapped to (0, 1] by u = ((x >> 8) + 1) * 2^-24, and the pairs
(w0, w1), (w2, w3) become Gaussians by the Box-Muller transform:
z_even = sqrt(-2 ln u_a) cos(2 pi u_b), z_odd = sqrt(-2 ln u_a) sin(2 pi u_b).
"""

from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """ctr: (N, 4) uint32-valued, key: (N, 2) or (2,) uint32-valued.
    Returns (N, 4) uint32 outputs after 10 rounds."""
    c = np.asarray(ctr, dtype=np.uint64).reshape(-1, 4).copy()
    k = np.broadcast_to(np.asarray(key, dtype=np.uint64), (c.shape[0], 2)).copy()
    for rnd in range(10):
        if rnd > 0:
            k[:, 0] = (k[:, 0] + W0) & MASK
            k[:, 1] = (k[:, 1] + W1) & MASK
        p0 = M0 * c[:, 0]          # < 2^64, exact in uint64
        p1 = M1 * c[:, 2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = np.stack([hi1 ^ c[:, 1] ^ k[:, 0], lo1,
                      hi0 ^ c[:, 3] ^ k[:, 1], lo0], axis=1)
    return c.astype(np.uint32)


def gaussian_words(rows: int, cols: int, seed: int) -> np.ndarray:
    """The raw Philox words behind a rows x cols Gaussian draw (row-major,
    flattened, length rows*cols)."""
    total = rows * cols
    nblk = (total + 3) // 4
    g = np.arange(nblk, dtype=np.uint64)
    ctr = np.stack([g & MASK, g >> np.uint64(32),
                    np.zeros_like(g), np.zeros_like(g)], axis=1)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)
    return philox4x32_10(ctr, key).reshape(-1)[:total]


def gaussian(rows: int, cols: int, seed: int) -> np.ndarray:
    """rows x cols standard Gaussian matrix (float64) from the layout above."""
    total = rows * cols
    nblk = (total + 3) // 4
    g = np.arange(nblk, dtype=np.uint64)
    ctr = np.stack([g & MASK, g >> np.uint64(32),
                    np.zeros_like(g), np.zeros_like(g)], axis=1)
    key = np.array([seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF], dtype=np.uint64)
    x = philox4x32_10(ctr, key).astype(np.float64)
    u = (np.floor(x / 256.0) + 1.0) * 2.0 ** -24          # (0, 1]
    r0 = np.sqrt(-2.0 * np.log(u[:, 0]))
    r1 = np.sqrt(-2.0 * np.log(u[:, 2]))
    t0 = 2.0 * np.pi * u[:, 1]
    t1 = 2.0 * np.pi * u[:, 3]
    z = np.stack([r0 * np.cos(t0), r0 * np.sin(t0),
                  r1 * np.cos(t1), r1 * np.sin(t1)], axis=1).reshape(-1)
    return z[:total].reshape(rows, cols)
