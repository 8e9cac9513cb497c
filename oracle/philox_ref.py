"""Reference counter-based normals for the sampler's eta and delta.

Test infrastructure only: see the package docstring.

The paper draws eta ~ N(0, I_n) and delta ~ N(0, I_p) (Prop 2.1) and does not
say how.  The library draws them from a counter-based generator so that every
draw is a pure function of (seed, chain, draw index); this module restates
that convention from the generator's published definition:

* Philox4x64-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC'11): a 4-word counter and a 2-word key of 64-bit
  words; each of the 10 rounds multiplies words 0 and 2 by two constants,
  takes the 128-bit products' high and low halves and mixes them with words
  1 and 3 and the round key; the key is bumped by two Weyl constants between
  rounds.
* counter = (block i, stream, chain, draw index); stream 0 is eta (length n),
  stream 1 is delta (length p); key = (seed, 0).
* A block's four words (w0, w1, w2, w3) give the normals of elements
  4i .. 4i+3 by the Box-Muller transform in FP64 on the uniforms
  ua = ((w >> 12) + 1/2) 2^-52 in (0, 1) from w0, w2 and ub = (w >> 11) 2^-53
  in [0, 1) from w1, w3:  (sqrt(-2 ln ua) cos 2 pi ub, sqrt(-2 ln ua) sin 2 pi ub).
"""
from __future__ import annotations

import numpy as np

MASK64 = (1 << 64) - 1
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15  # golden ratio
PHILOX_W1 = 0xBB67AE8584CAA73B  # sqrt(3) - 1
ROUNDS = 10

STREAM_ETA = 0
STREAM_DELTA = 1


def philox4x64_scalar(ctr, key, rounds=ROUNDS):
    """Philox4x64 on one counter with Python integers (exact 128-bit products)."""
    x0, x1, x2, x3 = (int(c) & MASK64 for c in ctr)
    k0, k1 = (int(k) & MASK64 for k in key)
    for r in range(rounds):
        if r:
            k0 = (k0 + PHILOX_W0) & MASK64
            k1 = (k1 + PHILOX_W1) & MASK64
        p0 = PHILOX_M0 * x0
        p1 = PHILOX_M1 * x2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return (x0, x1, x2, x3)


def _mulhilo64(a, b):
    """High and low 64-bit halves of a*b for uint64 arrays a and scalar b,
    by schoolbook multiplication on 32-bit halves."""
    m32 = np.uint64(0xFFFFFFFF)
    s32 = np.uint64(32)
    b_lo = np.uint64(b & 0xFFFFFFFF)
    b_hi = np.uint64(b >> 32)
    a_lo = a & m32
    a_hi = a >> s32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> s32) + (lh & m32) + (hl & m32)
    lo = (ll & m32) | (mid << s32)
    hi = hh + (lh >> s32) + (hl >> s32) + (mid >> s32)
    return hi, lo


def philox4x64(ctr, key, rounds=ROUNDS):
    """Vectorised Philox4x64: ``ctr`` is a uint64 array [..., 4], ``key`` a pair."""
    ctr = np.asarray(ctr, dtype=np.uint64)
    x0, x1, x2, x3 = (ctr[..., i].copy() for i in range(4))
    k0, k1 = int(key[0]) & MASK64, int(key[1]) & MASK64
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r:
                k0 = (k0 + PHILOX_W0) & MASK64
                k1 = (k1 + PHILOX_W1) & MASK64
            hi0, lo0 = _mulhilo64(x0, PHILOX_M0)
            hi1, lo1 = _mulhilo64(x2, PHILOX_M1)
            x0, x1, x2, x3 = (hi1 ^ x1 ^ np.uint64(k0), lo1,
                              hi0 ^ x3 ^ np.uint64(k1), lo0)
    return np.stack([x0, x1, x2, x3], axis=-1)


def block_counters(nblocks, stream, chain, draw):
    c = np.zeros((nblocks, 4), dtype=np.uint64)
    c[:, 0] = np.arange(nblocks, dtype=np.uint64)
    c[:, 1] = np.uint64(stream)
    c[:, 2] = np.uint64(chain)
    c[:, 3] = np.uint64(draw)
    return c


def uniforms_from_words(w):
    """(ua, ub) from a [nblocks, 4] word array: ua from words 0 and 2 in (0, 1),
    ub from words 1 and 3 in [0, 1); both exact in FP64."""
    wa = w[:, 0::2]
    wb = w[:, 1::2]
    ua = ((wa >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0 ** -52
    ub = (wb >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return ua, ub


def normals(seed, stream, chain, draw, count):
    """``count`` standard normals of one stream, in FP64 (element order 0..count-1)."""
    if count == 0:
        return np.zeros(0)
    nb = (count + 3) // 4
    w = philox4x64(block_counters(nb, stream, chain, draw), (seed, 0))
    ua, ub = uniforms_from_words(w)
    rad = np.sqrt(-2.0 * np.log(ua))
    ang = (2.0 * np.pi) * ub
    g = np.empty((nb, 4))
    g[:, 0] = rad[:, 0] * np.cos(ang[:, 0])
    g[:, 1] = rad[:, 0] * np.sin(ang[:, 0])
    g[:, 2] = rad[:, 1] * np.cos(ang[:, 1])
    g[:, 3] = rad[:, 1] * np.sin(ang[:, 1])
    return g.reshape(-1)[:count]


def normals_many(seed, stream, chain, draws, count):
    """Normals of one stream for several draw indices at once: [len(draws), count]."""
    draws = np.asarray(draws, dtype=np.uint64)
    nb = (count + 3) // 4
    c = np.zeros((draws.size, nb, 4), dtype=np.uint64)
    c[:, :, 0] = np.arange(nb, dtype=np.uint64)[None, :]
    c[:, :, 1] = np.uint64(stream)
    c[:, :, 2] = np.uint64(chain)
    c[:, :, 3] = draws[:, None]
    w = philox4x64(c.reshape(-1, 4), (seed, 0))
    ua, ub = uniforms_from_words(w)
    rad = np.sqrt(-2.0 * np.log(ua))
    ang = (2.0 * np.pi) * ub
    g = np.empty((w.shape[0], 4))
    g[:, 0] = rad[:, 0] * np.cos(ang[:, 0])
    g[:, 1] = rad[:, 0] * np.sin(ang[:, 0])
    g[:, 2] = rad[:, 1] * np.cos(ang[:, 1])
    g[:, 3] = rad[:, 1] * np.sin(ang[:, 1])
    return g.reshape(draws.size, nb * 4)[:, :count]


def eta_delta(seed, chain, draw, n, p):
    """(eta, delta) for one draw: eta ~ N(0, I_n), delta ~ N(0, I_p) (Prop 2.1)."""
    return (normals(seed, STREAM_ETA, chain, draw, n),
            normals(seed, STREAM_DELTA, chain, draw, p))
