"""Exact perfect sampling of G^k|s> from closed-form marginals (Eqs. (1), (5), (6)).

|<x|psi>|^2 is a_m^2 on the marked set W and a_u^2 elsewhere (Eq. (5)), so the weight of
any bit prefix is a_m^2 * (#W with that prefix) + a_u^2 * (#other completions). Sampling
site by site with the shared Philox stream (see :mod:`oracle.philox`) gives the exact
draw any correct site-by-site sampler must reproduce, at any n.
"""
from __future__ import annotations

import numpy as np

from . import closed_form, philox


def prefix_weight(n: int, marked, k: int, prefix: int, length: int) -> float:
    am, au = closed_form.amplitudes_wr(n, len(marked), k)
    shift = n - length
    hits = sum(1 for x in marked if (int(x) >> shift) == prefix)
    return am * am * hits + au * au * ((1 << shift) - hits)


def sample(n: int, marked, k: int, shots: int, seed: int, inst: int = 0):
    """Returns (bits, p0 at each decision, u at each decision)."""
    bits = np.zeros(shots, dtype=np.uint64)
    p0s = np.zeros((shots, n))
    us = np.zeros((shots, n))
    for sh in range(shots):
        x = 0
        w = 1.0
        for i in range(n):
            w0 = prefix_weight(n, marked, k, x << 1, i + 1)
            p0 = w0 / w
            u = philox.uniform(seed, inst, sh, i)
            p0s[sh, i] = p0
            us[sh, i] = u
            if u < p0:
                x = x << 1
                w = w0
            else:
                x = (x << 1) | 1
                w = w - w0
        bits[sh] = x
    return bits, p0s, us


def sample_from_statevector(psi: np.ndarray, n: int, shots: int, seed: int, inst: int = 0):
    """The same site-by-site rule driven by an explicit statevector (n <= ~24)."""
    prob = np.abs(psi) ** 2
    prob = prob / prob.sum()
    bits = np.zeros(shots, dtype=np.uint64)
    for sh in range(shots):
        lo, hi = 0, 1 << n
        for i in range(n):
            mid = (lo + hi) // 2
            w = prob[lo:hi].sum()
            p0 = prob[lo:mid].sum() / w
            if philox.uniform(seed, inst, sh, i) < p0:
                hi = mid
            else:
                lo = mid
        bits[sh] = lo
    return bits
