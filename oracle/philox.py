"""Counter-based draws of pair elements given implicitly (test infrastructure).

When a workload's M_{u u'}(G') array would not fit in memory (core-level
problems: N_k(N_k+1)/2 pairs x N_c^2 x N_G complex values), the inputs give
only a key and an envelope, and every value is drawn where it is needed:

  M[p, u, u', G] = env[G] * (x + i y) / sqrt(2)

with (x, y) two standard normals from Box-Muller on two uniforms taken from
one Philox4x32-10 block at counter (p, u, u', G) under the 64-bit key
(low word, high word).  Philox4x32-10 is the generator of Salmon, Moraes, Dror
and Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of
two 32x32->64-bit products with the multipliers 0xD2511F53 and 0xCD9E8D57,
the key bumped by the Weyl increments 0x9E3779B9 and 0xBB67AE85 between
rounds.  Uniforms: u1 = (k1 + 1) 2^-53 in (0, 1] from the top 53 bits k1 of
(w1:w0), u2 = k2 2^-53 in [0, 1) from the top 53 bits of (w3:w2); then
x = sqrt(-2 ln u1) cos(2 pi u2), y = sqrt(-2 ln u1) sin(2 pi u2).

Written from those definitions, with NumPy integer arithmetic, for the oracle
only; the GPU library has its own implementation.
"""
from __future__ import annotations

import numpy as np

_M0, _M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
_W0, _W1 = 0x9E3779B9, 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds.  ctr: four arrays (or ints) of 32-bit words,
    broadcast together; key: two 32-bit words.  Returns four uint32 arrays."""
    x0, x1, x2, x3 = np.broadcast_arrays(*[np.asarray(c, dtype=np.uint64) & _MASK for c in ctr])
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for _ in range(10):
        p0 = x0 * _M0
        p1 = x2 * _M1
        x0, x1, x2, x3 = ((p1 >> np.uint64(32)) ^ x1 ^ np.uint64(k0), p1 & _MASK,
                          (p0 >> np.uint64(32)) ^ x3 ^ np.uint64(k1), p0 & _MASK)
        k0 = (k0 + _W0) & 0xFFFFFFFF
        k1 = (k1 + _W1) & 0xFFFFFFFF
    return tuple(v.astype(np.uint32) for v in (x0, x1, x2, x3))


def complex_normal(ctr, key) -> np.ndarray:
    """(x + i y) / sqrt(2) from one Philox block per counter (E|z|^2 = 1)."""
    w0, w1, w2, w3 = (v.astype(np.uint64) for v in philox4x32_10(ctr, key))
    k1 = ((w1 << np.uint64(32)) | w0) >> np.uint64(11)
    k2 = ((w3 << np.uint64(32)) | w2) >> np.uint64(11)
    u1 = (k1.astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = k2.astype(np.float64) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    t = 2.0 * np.pi * u2
    return (r * np.cos(t) + 1j * (r * np.sin(t))) / np.sqrt(2.0)


def split_key(key64: int) -> tuple[int, int]:
    return key64 & 0xFFFFFFFF, (key64 >> 32) & 0xFFFFFFFF


def mcc_pairs(key64: int, env: np.ndarray, ps, nc: int) -> np.ndarray:
    """M[p, u, u', G] for the pairs ps: array [len(ps), nc, nc, ng]."""
    ps = np.asarray(ps, dtype=np.int64)
    ng = len(env)
    p = ps[:, None, None, None]
    u = np.arange(nc)[None, :, None, None]
    u2 = np.arange(nc)[None, None, :, None]
    g = np.arange(ng)[None, None, None, :]
    z = complex_normal((p, u, u2, g), split_key(key64))
    return z * env[None, None, None, :]
