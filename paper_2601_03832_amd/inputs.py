"""Seeded synthetic workload generators shared by the HIP path's callers and the oracle.

This module only draws inputs (qubit counts, marked sets, iteration counts, seeds);
it holds none of the simulation's arithmetic.

* Marked sets are drawn with SplitMix64 (Steele, Lea & Flood, OOPSLA 2014), using
  rejection so the M marked indices of one instance are distinct. The paper does
  not say how its marked item is chosen (Section II fixes M = 1 only).
* The iteration count follows Eq. (8), k = round(pi/4 * sqrt(N)), generalised to
  k = round(pi/4 * sqrt(N/M)) for M marked items (the small-angle form of Eq. (7)).
* Bit convention: site i of the chain carries bit (n-1-i) of a basis index x
  (most significant bit first); marked indices and sampled bitstrings share it.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List

import numpy as np

_MASK64 = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 stream generator (Steele, Lea & Flood 2014)."""

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK64
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK64
        return z ^ (z >> 31)

    def below(self, m: int) -> int:
        """Uniform integer in [0, m) by multiply-shift of the top 32 bits (m < 2^32)."""
        return ((self.next() >> 32) * m) >> 32


def k_rule(n: int, M: int) -> int:
    """Iteration count round(pi/4 * sqrt(2^n / M)) (Eq. (8), extended to M marked items).

    pi/4*sqrt(N/M) is irrational for every (n, M) used here, so no .5 tie occurs.
    """
    return int(round(math.pi / 4.0 * math.sqrt(float(2 ** n) / M)))


def draw_marked(n: int, M: int, rng: SplitMix64) -> np.ndarray:
    """M distinct indices in [0, 2^n): the top n bits of successive SplitMix64 words."""
    if not (1 <= n <= 63):
        raise ValueError("n must be in [1, 63]")
    if not (1 <= M < (1 << n)):
        raise ValueError("M must be in [1, 2^n - 1]")
    seen = set()
    out: List[int] = []
    while len(out) < M:
        x = rng.next() >> (64 - n)
        if x not in seen:
            seen.add(x)
            out.append(x)
    return np.array(out, dtype=np.uint64)


@dataclass
class Instance:
    """One independent Grover search: n qubits, marked set W, k iterations, bond cap."""

    n: int
    marked: np.ndarray
    k: int
    chi_cap: int

    @property
    def M(self) -> int:
        return int(len(self.marked))


@dataclass
class Workload:
    name: str
    instances: List[Instance]
    precision: str  # "fp64" or "mixed"
    shots: List[int] = field(default_factory=list)
    shot_seed: int = 0
    description: str = ""


def _single(name, n, M, cap, seed, precision, shots, shot_seed, desc, k=None):
    rng = SplitMix64(seed)
    W = draw_marked(n, M, rng)
    return Workload(name, [Instance(n, W, k_rule(n, M) if k is None else k, cap)],
                    precision, shots, shot_seed, desc)


def config_c1() -> Workload:
    """n=10, one marked state, k=25, FP64, chi cap 4 (small case checked against the full statevector)."""
    return _single("c1_n10_k25_fp64", 10, 1, 4, 1001, "fp64", [], 2001,
                   "n=10, M=1, k=25, complex128, chi cap 4")


def config_c2() -> Workload:
    """n=20, one marked state, k=804, FP64, chi cap 4, 4096 perfect-sampling shots."""
    return _single("c2_n20_k804_fp64", 20, 1, 4, 1002, "fp64", [4096], 2002,
                   "n=20, M=1, k=804, complex128, chi cap 4, 4096 shots")


def config_c3(precision: str = "fp64") -> Workload:
    """n=29, one marked state, k=18198, chi cap 4 (precision study: fp64 vs mixed)."""
    return _single("c3_n29_k18198_" + precision, 29, 1, 4, 1003, precision, [], 2003,
                   "n=29, M=1, k=18198, chi cap 4")


def config_c4(count: int = 4096, seed: int = 1004) -> Workload:
    """Batched mixed precision: n uniform in [12, 28], M uniform in {1, 2, 4}, cap M+2, own k."""
    rng = SplitMix64(seed)
    insts = []
    for _ in range(count):
        n = 12 + rng.below(17)
        M = (1, 2, 4)[rng.below(3)]
        W = draw_marked(n, M, rng)
        insts.append(Instance(n, W, k_rule(n, M), M + 2))
    return Workload("c4_batch%d_n12-28_M124_mixed" % count, insts, "mixed", [4096], 2004,
                    "%d instances, n~U[12,28], M~U{1,2,4}, own k, cap M+2, complex64 bulk + FP64 "
                    "recompression" % count)


def config_c5(count: int = 256, seed: int = 1005, k: int | None = None) -> Workload:
    """256 instances at n=40 with 16 marked states each, cap 32, shots 1/8/4096."""
    rng = SplitMix64(seed)
    insts = []
    for _ in range(count):
        W = draw_marked(40, 16, rng)
        insts.append(Instance(40, W, k_rule(40, 16) if k is None else k, 32))
    return Workload("c5_batch%d_n40_M16_mixed" % count, insts, "mixed", [1, 8, 4096], 2005,
                    "%d instances, n=40, M=16, cap 32" % count)


def random_batch(count: int, n_lo: int, n_hi: int, Ms, seed: int, cap_extra: int = 1,
                 k_scale: float = 1.0) -> List[Instance]:
    """Small mixed batches for tests: n uniform in [n_lo, n_hi], M from Ms, k scaled down."""
    rng = SplitMix64(seed)
    out = []
    for _ in range(count):
        n = n_lo + rng.below(n_hi - n_lo + 1)
        M = Ms[rng.below(len(Ms))]
        M = min(M, (1 << n) - 1)
        W = draw_marked(n, M, rng)
        k = max(1, int(round(k_rule(n, M) * k_scale)))
        out.append(Instance(n, W, k, M + cap_extra))
    return out
