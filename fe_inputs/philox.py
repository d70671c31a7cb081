"""Counter-based element matrices: Philox4x32-10 and exact-arithmetic recipes.

Philox4x32-10 is the counter-based generator of Salmon, Moraes, Dror and
Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11): ten rounds of
two 32x32->64-bit multiplications (multipliers 0xD2511F53, 0xCD9E8D57)
with a Weyl key schedule (0x9E3779B9, 0xBB67AE85).  This numpy version is
written from that definition; the device library has its own.  Both feed the
same recipes, whose arithmetic is exact or a fixed sequence of correctly
rounded IEEE operations, so both produce the same bits.

Entry i = r*n + s of element e takes 32-bit word i mod 4 of Philox(counter
(i div 4, (e+e0) mod 2^32, (e+e0) div 2^32, recipe), key (seed mod 2^32,
seed div 2^32)); u = word * 2^-32.

* laplacian (recipe 0): K_rs = 2u - 1 for r < s, mirrored;
  K_rr = -sum_{s != r} K_rs in increasing s.
* spd (recipe 1): B_rs = (u - 1/2) * sqrt(12) (unit variance);
  K_rs = (sum_t B_rt B_st, t increasing, products then sums, no fused
  multiply-add) / n, plus 1 on the diagonal.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
SQRT3 = 1.7320508075688772
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10; all arguments uint32 arrays (or scalars)."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint32) for x in (c0, c1, c2, c3))
    k0 = np.uint32(k0)
    k1 = np.uint32(k1)
    with np.errstate(over="ignore"):
        for r in range(10):
            if r:
                k0 = np.uint32(k0 + W0)
                k1 = np.uint32(k1 + W1)
            p0 = M0 * c0.astype(np.uint64)
            p1 = M1 * c2.astype(np.uint64)
            hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
            lo0 = (p0 & MASK).astype(np.uint32)
            hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
            lo1 = (p1 & MASK).astype(np.uint32)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


SQRT12 = 3.4641016151377544


def _uniforms(E, n, e0, recipe, seed):
    """[E, n*n] uniforms u in [0, 1): word i mod 4 of the call for i div 4."""
    k0, k1 = seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF
    calls = (n * n + 3) // 4
    e = np.arange(E, dtype=np.uint64) + np.uint64(e0)
    c0 = np.broadcast_to(np.arange(calls, dtype=np.uint32)[None, :], (E, calls))
    c1 = np.broadcast_to((e & MASK).astype(np.uint32)[:, None], (E, calls))
    c2 = np.broadcast_to((e >> np.uint64(32)).astype(np.uint32)[:, None], (E, calls))
    c3 = np.full((E, calls), recipe, dtype=np.uint32)
    w = np.stack(philox4x32_10(c0, c1, c2, c3, k0, k1), axis=-1).reshape(E, 4 * calls)
    return w[:, : n * n].astype(np.float64) * 2.0 ** -32


def ke_laplacian(E, n, seed, e0=0):
    u = _uniforms(E, n, e0, 0, seed)
    V = (2.0 * u - 1.0).reshape(E, n, n)
    K = np.zeros((E, n, n))
    iu = np.triu_indices(n, 1)
    K[:, iu[0], iu[1]] = V[:, iu[0], iu[1]]
    K[:, iu[1], iu[0]] = V[:, iu[0], iu[1]]
    for r in range(n):
        acc = np.zeros(E)
        for s in range(n):
            if s != r:
                acc = acc + K[:, r, s]
        K[:, r, r] = -acc
    return K


def ke_spd(E, n, seed, e0=0):
    u = _uniforms(E, n, e0, 1, seed)
    B = ((u - 0.5) * SQRT12).reshape(E, n, n)
    acc = np.zeros((E, n, n))
    for t in range(n):
        acc = acc + B[:, :, None, t] * B[:, None, :, t]
    K = acc / float(n)
    K[:, np.arange(n), np.arange(n)] += 1.0
    return K
