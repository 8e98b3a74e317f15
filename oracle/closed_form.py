"""Closed forms of Grover search (Section II of the paper).

With N = 2^n and M marked items, sin(theta) = sqrt(M/N) (Eq. (2)). After k iterations
G^k|s> = sin((2k+1)theta)|w> + cos((2k+1)theta)|r> (Eq. (5)), with |w>, |r> the
normalised uniform superpositions over marked / unmarked indices (Eq. (1)), so
P(k) = sin^2((2k+1)theta) (Eq. (6)) and every amplitude is known.
"""
from __future__ import annotations

import math

import numpy as np


def theta(n: int, M: int) -> float:
    """theta = asin(sqrt(M/N)) exactly (Eq. (2)); not the small-angle form."""
    return math.asin(math.sqrt(M / float(2 ** n)))


def p_marked(n: int, M: int, k: int) -> float:
    """Success probability after k iterations, sin^2((2k+1) theta) (Eq. (6))."""
    return math.sin((2 * k + 1) * theta(n, M)) ** 2


def amplitudes_wr(n: int, M: int, k: int):
    """(a_marked, a_unmarked): every marked amplitude is sin(phi)/sqrt(M), every other one
    cos(phi)/sqrt(N-M), phi = (2k+1)theta (Eqs. (1) and (5)); real and positive-phase under
    the sign convention O = I - 2 sum_x |x><x|, D = 2|s><s| - I (Eq. (4))."""
    phi = (2 * k + 1) * theta(n, M)
    N = float(2 ** n)
    return math.sin(phi) / math.sqrt(M), math.cos(phi) / math.sqrt(N - M)


def amplitude(n: int, marked, k: int, x: int) -> float:
    """<x|G^k|s> from Eq. (5)."""
    am, au = amplitudes_wr(n, len(marked), k)
    return am if int(x) in set(int(v) for v in marked) else au


def statevector(n: int, marked, k: int) -> np.ndarray:
    """All 2^n amplitudes of G^k|s> from Eq. (5) (n <= ~26 on a host)."""
    am, au = amplitudes_wr(n, len(marked), k)
    psi = np.full(1 << n, au, dtype=np.float64)
    psi[np.asarray(marked, dtype=np.int64)] = am
    return psi
