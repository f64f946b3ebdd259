"""Philox4x32-10 counter-based generator (Salmon, Moraes, Dror, Shaw, SC'11).

Written from the published definition: a 128-bit counter (c0..c3) and a
64-bit key (k0, k1); each of the 10 rounds replaces the counter by
    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))
with M0 = 0xD2511F53, M1 = 0xCD9E8D57, and the key is advanced by the Weyl
constants (0x9E3779B9, 0xBB67AE85) before every round after the first.

Conversions used by the path sampler:
  uniform52(a, b) = ((a >> 6) * 2^26 + (b >> 6) + 1/2) * 2^-52, in (0, 1), exact in FP64;
  Box-Muller: (u1, u2) -> sqrt(-2 ln u1) * (cos 2 pi u2, sin 2 pi u2).

Stream layout of the sampler (key = (seed mod 2^32, seed >> 32)), for sweep s:
  level/offset   counter (0, 0, s, 1)          -> words w0, w1
  accept uniform counter (f, 0, s, 2)          -> uniform52(w0, w1) for fragment f
  trial normal   counter (p mod 2^32, p >> 32, s, 3) for pair p = e >> 1 of the flat
                 element index e = n * n_dof + k; element e takes the cos (e even)
                 or the sin (e odd) output.
and of the integrator's regeneration after shifting event v:
  regrowth normal  counter (p mod 2^32, p >> 32, v, 4), p and e as for trial normals
                   (e indexes the shifted path);
and of the gradient-informed (Langevin) path move number t:
  proposal normal  counter (p mod 2^32, p >> 32, t, 5), p and e as for trial normals
  accept uniform   counter (0, 0, t, 6) -> uniform52(w0, w1).
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK = 0xFFFFFFFF

PURPOSE_LEVEL = 1
PURPOSE_ACCEPT = 2
PURPOSE_TRIAL = 3
PURPOSE_REGROW = 4
PURPOSE_LANGEVIN = 5
PURPOSE_LANGEVIN_ACCEPT = 6


def philox4x32_10(ctr, key):
    """Vectorised Philox4x32-10.  ctr: 4 arrays (or ints) of uint32; key: 2 values."""
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & MASK for c in ctr)
    k0 = np.uint64(int(key[0]) & MASK)
    k1 = np.uint64(int(key[1]) & MASK)
    m0 = np.uint64(M0)
    m1 = np.uint64(M1)
    mask = np.uint64(MASK)
    for rnd in range(10):
        if rnd > 0:
            k0 = np.uint64((int(k0) + W0) & MASK)
            k1 = np.uint64((int(k1) + W1) & MASK)
        p0 = m0 * c0                     # < 2^64: exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & mask
        hi1, lo1 = p1 >> np.uint64(32), p1 & mask
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniform52(a, b):
    """Exact double strictly inside (0, 1) from two 32-bit words (26 + 26 bits, centred)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    k = (a >> np.uint64(6)).astype(np.float64) * 67108864.0 + (b >> np.uint64(6)).astype(np.float64)
    return (k + 0.5) * (1.0 / 4503599627370496.0)


def seed_key(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return (seed & MASK, seed >> 32)


def level_and_offset(seed: int, sweep: int, l_min: int, l_max: int):
    """Level l uniform in [l_min, l_max] and offset u uniform in [1, 2^l] (Sec. III)."""
    w = philox4x32_10((0, 0, sweep, PURPOSE_LEVEL), seed_key(seed))
    l = l_min + int(w[0]) % (l_max - l_min + 1)
    u = 1 + int(w[1]) % (1 << l)
    return l, u


def accept_uniforms(seed: int, sweep: int, n_fragments: int):
    f = np.arange(n_fragments, dtype=np.uint64)
    z = np.zeros_like(f)
    w = philox4x32_10((f, z, np.full_like(f, sweep), np.full_like(f, PURPOSE_ACCEPT)),
                      seed_key(seed))
    return uniform52(w[0], w[1])


def trial_normals(seed: int, sweep: int, n_elements: int, first: int = 0,
                  purpose: int = PURPOSE_TRIAL):
    """Standard normals for flat element indices first .. first + n_elements - 1."""
    e = np.arange(first, first + n_elements, dtype=np.uint64)
    p = e >> np.uint64(1)
    w = philox4x32_10((p & np.uint64(MASK), p >> np.uint64(32), np.full_like(p, sweep),
                       np.full_like(p, purpose)), seed_key(seed))
    u1 = uniform52(w[0], w[1])
    u2 = uniform52(w[2], w[3])
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return np.where((e & np.uint64(1)) == 0, rad * np.cos(ang), rad * np.sin(ang))


def regrow_normals(seed: int, event: int, n_elements: int, first: int = 0):
    """Standard normals of the regrowth after shifting event `event`."""
    return trial_normals(seed, event, n_elements, first, PURPOSE_REGROW)


def langevin_normals(seed: int, move: int, n_elements: int, first: int = 0):
    """Standard normals of the proposal of Langevin path move `move`."""
    return trial_normals(seed, move, n_elements, first, PURPOSE_LANGEVIN)


def langevin_uniform(seed: int, move: int) -> float:
    w = philox4x32_10((0, 0, move, PURPOSE_LANGEVIN_ACCEPT), seed_key(seed))
    return float(uniform52(w[0], w[1]))
