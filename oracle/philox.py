"""Philox4x64-10 counter-based generator -- oracle side, TEST INFRASTRUCTURE ONLY.

Written from its published definition (Salmon, Moraes, Dror & Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11): ten rounds of two 64x64->128-bit products with the
multipliers 0xD2E7470EE14C6C93 and 0xCA5A826395121157, the round mixing

    (c0, c1, c2, c3) -> (hi(M1 c2) ^ c1 ^ k0,  lo(M1 c2),  hi(M0 c0) ^ c3 ^ k1,  lo(M0 c0))

and the Weyl key schedule k0 += 0x9E3779B97F4A7C15, k1 += 0xBB67AE8584CAA73B between
rounds.  The Monte Carlo step draws its random numbers from this generator keyed by
(seed, 0) at counter (walker, step, call, 0); the HIP library implements the same
generator separately.

Mapping of the 64-bit outputs:
* integer in [0, m):  floor(r * m / 2^64)            (``below``)
* uniform in (0, 1):  ((r >> 12) + 1/2) * 2^-52, exact in fp64 (``uniform``)
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_LO = np.uint64(0xFFFFFFFF)
_32 = np.uint64(32)


def mulhilo(a, b):
    """128-bit product of uint64 arrays, returned as (hi, lo); schoolbook on 32-bit halves."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    al, ah = a & _LO, a >> _32
    bl, bh = b & _LO, b >> _32
    ll = al * bl
    lh = al * bh
    hl = ah * bl
    hh = ah * bh
    mid = (ll >> _32) + (lh & _LO) + (hl & _LO)
    lo = (ll & _LO) | ((mid & _LO) << _32)
    hi = hh + (lh >> _32) + (hl >> _32) + (mid >> _32)
    return hi, lo


def philox4x64(ctr, key, rounds: int = 10):
    """ctr: (..., 4) uint64, key: (..., 2) uint64 -> (..., 4) uint64."""
    c = np.array(ctr, dtype=np.uint64, copy=True)
    key = np.asarray(key, dtype=np.uint64)
    k0 = np.broadcast_to(key[..., 0], c.shape[:-1]).copy()
    k1 = np.broadcast_to(key[..., 1], c.shape[:-1]).copy()
    with np.errstate(over="ignore"):
        for r in range(rounds):
            hi0, lo0 = mulhilo(M0, c[..., 0])
            hi1, lo1 = mulhilo(M1, c[..., 2])
            c = np.stack([hi1 ^ c[..., 1] ^ k0, lo1, hi0 ^ c[..., 3] ^ k1, lo0], axis=-1)
            if r + 1 < rounds:
                k0 = k0 + W0
                k1 = k1 + W1
    return c


def mc_draws(seed: int, walkers, step: int, call: int):
    """The four 64-bit draws of ``call`` for each walker index in ``walkers``."""
    w = np.asarray(walkers, dtype=np.uint64)
    ctr = np.stack([w, np.full_like(w, step), np.full_like(w, call), np.zeros_like(w)], axis=-1)
    key = np.array([seed, 0], dtype=np.uint64)
    return philox4x64(ctr, key)


def below(r, m):
    """floor(r * m / 2^64) for uint64 r and integer m >= 1."""
    hi, _ = mulhilo(r, np.uint64(m))
    return hi.astype(np.int64)


def uniform(r):
    """((r >> 12) + 1/2) 2^-52: 52 random bits, exactly representable, in (0, 1)."""
    return ((np.asarray(r, dtype=np.uint64) >> np.uint64(12)).astype(np.float64) + 0.5) * 2.0 ** -52
