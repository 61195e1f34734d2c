"""Philox4x32-10 counter-based random numbers and Box-Muller normals (oracle
side; test infrastructure only).

The paper draws its Gaussian noise with R's generator and does not specify
it.  Both this oracle and the HIP library instead use one published
counter-based generator, each implemented independently from its definition:
Philox4x32 with 10 rounds (Salmon, Moraes, Dror and Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11).  One round maps the counter
(c0, c1, c2, c3) under key (k0, k1) to

    (hi(B * c2) ^ c1 ^ k0,  lo(B * c2),  hi(A * c0) ^ c3 ^ k1,  lo(A * c0)),

with multipliers A = 0xD2511F53, B = 0xCD9E8D57 and the key advanced by the
Weyl constants (0x9E3779B9, 0xBB67AE85) between rounds.

Stream layout shared with the HIP path:
  key     = (seed mod 2^32, seed >> 32)
  counter = (block, realization, event, stream)
  stream 0: torus noise of the circulant-embedding draw; element
            q = j * T1 + i of the T2 x T1 torus uses block q // 4, word q % 4.
  stream 1: the off-grid nugget noise xi of observation i (block i // 4,
            word i % 4).
  stream 2: noise used to draw synthetic observed values for test fixtures.
Uniforms are u = (x + 1/2) 2^-32 (exact in FP64, never 0 or 1); normals come
from Box-Muller on the word pairs (0, 1) and (2, 3) of a block:
  z0 = sqrt(-2 ln u0) cos(2 pi u1),  z1 = sqrt(-2 ln u0) sin(2 pi u1).
The realization index is absolute, so a field never depends on how a run was
batched.

Pins (tests/test_oracle_philox.py): scalar pure-integer implementation versus
this vectorised one, uniformity and normal moments, independence across
counters; the HIP path must reproduce these words bit for bit.
"""

import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF

STREAM_TORUS = 0
STREAM_OFFGRID = 1
STREAM_FIXTURE = 2


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  Counters are uint32 arrays (broadcast
    together), the key two Python ints.  Returns four uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint64)
    c1 = np.asarray(c1, dtype=np.uint64)
    c2 = np.asarray(c2, dtype=np.uint64)
    c3 = np.asarray(c3, dtype=np.uint64)
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = int(k0) & MASK32
    k1 = int(k1) & MASK32
    m = np.uint64(MASK32)
    for rnd in range(10):
        if rnd:
            k0 = (k0 + PHILOX_W0) & MASK32
            k1 = (k1 + PHILOX_W1) & MASK32
        p0 = np.uint64(PHILOX_M0) * c0          # < 2^64, no overflow
        p1 = np.uint64(PHILOX_M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & m
        hi1, lo1 = p1 >> np.uint64(32), p1 & m
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
    return tuple(x.astype(np.uint32) for x in (c0, c1, c2, c3))


def seed_key(seed):
    seed = int(seed) & ((1 << 64) - 1)
    return seed & MASK32, seed >> 32


def raw_words(seed, blocks, real, event, stream):
    """The four 32-bit words of each block in ``blocks`` (array of block
    indices) for one (realization, event, stream): shape (len(blocks), 4)."""
    k0, k1 = seed_key(seed)
    blocks = np.asarray(blocks, dtype=np.uint64)
    w = philox4x32_10(blocks, np.uint64(real), np.uint64(event),
                      np.uint64(stream), k0, k1)
    return np.stack(w, axis=-1)


def uniforms(words):
    """u = (x + 1/2) / 2^32 in FP64."""
    return (words.astype(np.float64) + 0.5) * (2.0 ** -32)


def box_muller(u):
    """Normals from uniforms of shape (..., 4): pairs (0,1) and (2,3)."""
    z = np.empty_like(u)
    for a, b in ((0, 1), (2, 3)):
        rad = np.sqrt(-2.0 * np.log(u[..., a]))
        ang = 2.0 * np.pi * u[..., b]
        z[..., a] = rad * np.cos(ang)
        z[..., b] = rad * np.sin(ang)
    return z


def normals(seed, count, real, event=0, stream=STREAM_TORUS):
    """The first ``count`` normals of one (seed, realization, event, stream):
    element q comes from block q // 4, word q % 4."""
    nblk = (count + 3) // 4
    u = uniforms(raw_words(seed, np.arange(nblk), real, event, stream))
    return box_muller(u).reshape(-1)[:count]


def torus_noise(seed, t1, t2, reals, event=0):
    """Stream-0 noise fields epsilon_r of shape (len(reals), t2, t1)."""
    return np.stack([normals(seed, t1 * t2, r, event, STREAM_TORUS)
                     .reshape(t2, t1) for r in reals])


def offgrid_noise(seed, n, reals, event=0):
    """Stream-1 nugget noise xi_r of shape (len(reals), n)."""
    return np.stack([normals(seed, n, r, event, STREAM_OFFGRID)
                     for r in reals])
