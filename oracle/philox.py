"""Philox4x64-10 counter-based generator (Salmon, Moraes, Dror & Shaw, SC'11).

The round function multiplies counter words 0 and 2 by the Philox multipliers,
taking the 128-bit products' high and low halves; the high halves are xored with the
other two counter words and the round key, and the four words are permuted. The key
is bumped by the Weyl constants between the ten rounds.

Sampling convention (shared by every sampler in this project): for shot number
``shot`` of batch instance ``inst`` with user seed ``seed``, key = (seed, inst) and
counter = (shot, site // 4, 0, 0); the uniform for site ``i`` is output word ``i % 4``
as u = (word >> 11) * 2^-53; the site takes bit 0 iff u < p(bit 0 | prefix).
"""
from __future__ import annotations

_M = (1 << 64) - 1
PHILOX_M0 = 0xD2E7470EE14C6C93
PHILOX_M1 = 0xCA5A826395121157
PHILOX_W0 = 0x9E3779B97F4A7C15
PHILOX_W1 = 0xBB67AE8584CAA73B


def philox4x64_10(ctr, key):
    """Ten rounds of Philox4x64 on a 4-word counter and a 2-word key (python ints)."""
    c0, c1, c2, c3 = (int(v) & _M for v in ctr)
    k0, k1 = (int(v) & _M for v in key)
    for _ in range(10):
        p0 = PHILOX_M0 * c0
        p1 = PHILOX_M1 * c2
        hi0, lo0 = p0 >> 64, p0 & _M
        hi1, lo1 = p1 >> 64, p1 & _M
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + PHILOX_W0) & _M
        k1 = (k1 + PHILOX_W1) & _M
    return c0, c1, c2, c3


def uniform(seed: int, inst: int, shot: int, site: int) -> float:
    """The 53-bit uniform in [0, 1) drawn for (instance, shot, site)."""
    w = philox4x64_10((shot, site // 4, 0, 0), (seed, inst))[site % 4]
    return (w >> 11) * (1.0 / 9007199254740992.0)
