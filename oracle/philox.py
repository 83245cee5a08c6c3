"""Philox4x32-10 counter-based generator and the sampler's stream layout, oracle side.

Test infrastructure only (see the package docstring).

Philox4x32-10 follows its published definition (Salmon, Moraes, Dror & Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11): a 4 x 32-bit counter and a 2 x 32-bit key;
each of ten rounds multiplies counter words 0 and 2 by the constants 0xD2511F53 and
0xCD9E8D57 (full 64-bit products split into hi/lo halves), and produces
(hi2 ^ c1 ^ k0, lo2, hi0 ^ c3 ^ k1, lo0); between rounds the key is advanced by the
Weyl constants (0x9E3779B9, 0xBB67AE85).

Stream layout of the sampler (one reading, shared with the HIP side by specification,
not by code): key = (seed mod 2^32, seed >> 32); counter = (particle i, block b,
sweep s, (t << 4) | tag), t = 0 for the burn-in sweeps and t >= 1 for the scale index.
  tag 0: proposal normals; block b yields markers 4b..4b+3 by Box-Muller on the word
         pairs (w0, w1) and (w2, w3): r = sqrt(-2 ln((w_even + 1) 2^-32)),
         theta = 2 pi w_odd 2^-32, normals (r cos theta, r sin theta);
  tag 1: MH uniform u = (w0 + 1/2) 2^-32, block 0;
  tag 2: systematic-resampling offset U = w0 2^-32 at counter (0, 0, 0, (t << 4) | 2);
  tag 3: single-site moves: counter (particle i, coordinate j, cycle s, (t << 4) | 3)
         gives the proposal normal r cos theta from (w0, w1) as above and the MH
         uniform u = (w2 + 1/2) 2^-32.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)

TAG_NORMAL = 0
TAG_UNIFORM = 1
TAG_RESAMPLE = 2
TAG_SINGLE = 3


def philox4x32_10(ctr, key):
    """ctr: (..., 4) uint32-valued array; key: (k0, k1).  Returns (..., 4) uint32."""
    c = np.asarray(ctr, dtype=np.uint64) & MASK32
    c0, c1, c2, c3 = c[..., 0], c[..., 1], c[..., 2], c[..., 3]
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for r in range(10):
        if r:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK32
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK32
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1, hi0 ^ c3 ^ np.uint64(k1), lo0)
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def key_of(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & 0xFFFFFFFF, seed >> 32)


def word3(t: int, tag: int) -> int:
    return ((int(t) << 4) | int(tag)) & 0xFFFFFFFF


def proposal_normals(seed: int, N: int, p: int, sweep: int, t: int):
    """(N, p) standard normals for one sweep (tag 0)."""
    nb = (p + 3) // 4
    ctr = np.zeros((N, nb, 4), dtype=np.uint64)
    ctr[..., 0] = np.arange(N, dtype=np.uint64)[:, None]
    ctr[..., 1] = np.arange(nb, dtype=np.uint64)[None, :]
    ctr[..., 2] = np.uint64(sweep)
    ctr[..., 3] = np.uint64(word3(t, TAG_NORMAL))
    w = philox4x32_10(ctr, key_of(seed)).astype(np.float64)
    two32 = 2.0 ** -32
    r01 = np.sqrt(-2.0 * np.log((w[..., 0] + 1.0) * two32))
    th01 = 2.0 * np.pi * (w[..., 1] * two32)
    r23 = np.sqrt(-2.0 * np.log((w[..., 2] + 1.0) * two32))
    th23 = 2.0 * np.pi * (w[..., 3] * two32)
    z = np.stack([r01 * np.cos(th01), r01 * np.sin(th01),
                  r23 * np.cos(th23), r23 * np.sin(th23)], axis=-1)
    return z.reshape(N, nb * 4)[:, :p]


def mh_uniforms(seed: int, N: int, sweep: int, t: int):
    """(N,) uniforms in (0, 1) for the Metropolis-Hastings decisions (tag 1)."""
    ctr = np.zeros((N, 4), dtype=np.uint64)
    ctr[:, 0] = np.arange(N, dtype=np.uint64)
    ctr[:, 2] = np.uint64(sweep)
    ctr[:, 3] = np.uint64(word3(t, TAG_UNIFORM))
    w = philox4x32_10(ctr, key_of(seed))
    return (w[:, 0].astype(np.float64) + 0.5) * 2.0 ** -32


def resample_u32(seed: int, t: int) -> int:
    """The 32-bit word from which the systematic-resampling offset of scale t is made."""
    ctr = np.array([0, 0, 0, word3(t, TAG_RESAMPLE)], dtype=np.uint64)
    return int(philox4x32_10(ctr, key_of(seed))[0])


def single_site_draws(seed: int, N: int, p: int, cycle: int, t: int):
    """(N, p) proposal normals and (N, p) MH uniforms of one single-site cycle (tag 3)."""
    ctr = np.zeros((N, p, 4), dtype=np.uint64)
    ctr[..., 0] = np.arange(N, dtype=np.uint64)[:, None]
    ctr[..., 1] = np.arange(p, dtype=np.uint64)[None, :]
    ctr[..., 2] = np.uint64(cycle)
    ctr[..., 3] = np.uint64(word3(t, TAG_SINGLE))
    w = philox4x32_10(ctr, key_of(seed)).astype(np.float64)
    two32 = 2.0 ** -32
    z = np.sqrt(-2.0 * np.log((w[..., 0] + 1.0) * two32)) * np.cos(2.0 * np.pi * (w[..., 1] * two32))
    u = (w[..., 2] + 0.5) * two32
    return z, u
