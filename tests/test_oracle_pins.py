"""Pins of the CPU oracle to facts other than itself: textbook special cases, closed forms
derived independently in the test, brute force, numpy's own Philox, and invariants.
None of these tests touch the GPU library."""
import math

import numpy as np
import pytest

from oracle import closed_form as cf
from oracle import mps, philox, sampling
from oracle import statevector as sv
from paper_2601_03832_amd import inputs


# ---------------------------------------------------------------- closed form (Eqs. 2, 5, 6)
def test_two_qubit_search_is_certain_after_one_iteration():
    # Textbook: N=4, M=1 gives theta = 30 degrees, so one iteration lands on |x>.
    for x in range(4):
        assert cf.p_marked(2, 1, 1) == pytest.approx(1.0, abs=1e-15)
        psi = sv.grover_sv(2, [x], 1)
        expect = np.zeros(4)
        expect[x] = 1.0
        assert np.allclose(psi, expect, atol=1e-15)


def test_quarter_marked_is_certain_after_one_iteration():
    # M = N/4 gives sin(theta) = 1/2 for any n.
    for n in (3, 4, 6):
        W = list(range(0, 1 << n, 4))
        assert cf.p_marked(n, len(W), 1) == pytest.approx(1.0, abs=1e-14)
        assert sv.grover_sv(n, W, 1)[W].sum() ** 2 / len(W) == pytest.approx(1.0, abs=1e-13)


def test_zero_iterations_is_uniform():
    for n, M in ((5, 1), (9, 3), (30, 7)):
        assert cf.p_marked(n, M, 0) == pytest.approx(M / 2.0 ** n, rel=1e-14)


def test_amplitudes_are_normalised():
    for n, M, k in ((10, 1, 25), (20, 1, 804), (40, 16, 205887), (17, 4, 123)):
        am, au = cf.amplitudes_wr(n, M, k)
        assert M * am * am + (2 ** n - M) * au * au == pytest.approx(1.0, abs=1e-13)


def test_closed_form_matches_plain_iteration():
    # Two independent routes: the rotation formula vs k explicit reflections.
    rng = inputs.SplitMix64(7)
    for n in (3, 5, 8, 11):
        for M in (1, 2, 3):
            W = inputs.draw_marked(n, M, rng)
            for k in (0, 1, 2, 5, inputs.k_rule(n, M)):
                psi = sv.grover_sv(n, W, k)
                assert np.allclose(psi, cf.statevector(n, W, k), atol=1e-13)


def test_k_rule_values():
    # Eq. (8) for M = 1; the M > 1 extension uses sqrt(N/M). The rule is not round(k_opt):
    # at n = 9 the rule gives 18 while pi/(4 theta) - 1/2 = 17.27.
    assert [inputs.k_rule(n, 1) for n in (10, 20, 29)] == [25, 804, 18198]
    assert inputs.k_rule(40, 16) == 205887
    assert inputs.k_rule(9, 1) == 18
    assert math.pi / (4 * cf.theta(9, 1)) - 0.5 == pytest.approx(17.27, abs=0.01)


def test_optimal_k_is_near_peak():
    for n in (10, 20, 29):
        k = inputs.k_rule(n, 1)
        assert cf.p_marked(n, 1, k) > 0.999
        assert cf.p_marked(n, 1, k) >= cf.p_marked(n, 1, k + 3)


# ---------------------------------------------------------------- gate decomposition (Eq. 4, Fig. 1A)
@pytest.mark.parametrize("n,W", [(2, [1]), (3, [5]), (4, [0, 9]), (6, [63, 17, 2]), (8, [200])])
def test_dense_circuit_is_minus_G(n, W):
    N = 1 << n
    U = sv.dense_grover_unitary(n, W)
    assert np.allclose(U @ U.T, np.eye(N), atol=1e-12)          # unitary (real orthogonal)
    s = np.full(N, 1 / math.sqrt(N))
    # brute-force G from its action on every basis vector through the plain definition
    G = np.stack([sv.grover_sv(n, W, 1, psi=np.eye(N)[:, j].copy()) for j in range(N)], axis=1)
    assert np.allclose(U, -G, atol=1e-12)
    # diffusion part: H^n (2|0><0| - I) H^n = 2|s><s| - I (Eq. 4)
    assert np.allclose(G @ s, sv.grover_sv(n, W, 1), atol=1e-13)


def test_gate_level_circuit_matches_iteration_up_to_sign():
    for n, W, k in ((5, [3], 4), (7, [100, 5], 3), (9, [0], 6)):
        assert np.allclose(sv.grover_gates(n, W, k), (-1) ** k * sv.grover_sv(n, W, k), atol=1e-12)


# ---------------------------------------------------------------- Philox (Salmon et al. SC'11)
def test_philox_matches_numpy():
    # numpy's Philox is Philox4x64-10 and bumps the counter before each block.
    for key, ctr in (([0, 0], [0, 0, 0, 0]), ([5, 7], [3, 0, 0, 0]),
                     ([2 ** 64 - 1, 12345], [2 ** 63 + 9, 4, 2 ** 64 - 2, 1])):
        bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                             counter=np.array(ctr, dtype=np.uint64))
        got = [int(v) for v in bg.random_raw(8)]
        c = list(ctr)
        exp = []
        for _ in range(2):
            c[0] = (c[0] + 1) % 2 ** 64
            if c[0] == 0:
                c[1] = (c[1] + 1) % 2 ** 64
            exp += list(philox.philox4x64_10(c, key))
        assert got == exp


def test_uniform_range():
    us = [philox.uniform(11, 3, s, i) for s in range(50) for i in range(9)]
    assert min(us) >= 0.0 and max(us) < 1.0
    assert abs(np.mean(us) - 0.5) < 0.05


# ---------------------------------------------------------------- MPS oracle vs the plain definition
@pytest.mark.parametrize("n,M,k", [(1, 1, 1), (2, 1, 1), (3, 2, 2), (6, 1, 6), (8, 3, 4), (10, 1, 25),
                                   (11, 4, 7), (12, 2, 9)])
def test_mps_matches_statevector(n, M, k):
    W = inputs.draw_marked(n, M, inputs.SplitMix64(100 + n * 7 + M))
    m = mps.run(n, W, k, chi_cap=M + 1)
    psi = sv.grover_sv(n, W, k)
    assert np.allclose(m.statevector(), psi, atol=1e-13)
    assert m.marked_prob() == pytest.approx(cf.p_marked(n, M, k), abs=1e-12)
    assert m.norm2() == pytest.approx(1.0, abs=1e-13)


def test_mps_bond_dims_follow_exact_rank():
    # Schmidt rank of any state a*sum_W|x> + b*sum_{not W}|x> is <= M+1 at every cut.
    n, M = 12, 3
    W = inputs.draw_marked(n, M, inputs.SplitMix64(5))
    m = mps.run(n, W, 5, chi_cap=8)
    dims = m.bond_dims()
    for l in range(1, n):
        assert dims[l] <= min(2 ** l, 2 ** (n - l), M + 1)
    # a generic draw reaches the bound away from the edges
    assert max(dims) == M + 1


def _schmidt_m1(n, x, k, cut):
    """Independent closed form of the two Schmidt values of a|x> + b*sum_{y!=x}|y> at a cut:
    psi = (a-b)|xL>|xR> + b*2^{n/2}|sL>|sR>, orthogonalised by hand into a 2x2 core."""
    am, au = cf.amplitudes_wr(n, 1, k)
    L, R = 2 ** cut, 2 ** (n - cut)
    # basis on the left: e1 = |sL>, e2 = (|xL> - <sL|xL>|sL>)/norm ; same on the right
    cl = 1 / math.sqrt(L)
    cr = 1 / math.sqrt(R)
    nl = math.sqrt(1 - cl * cl)
    nr = math.sqrt(1 - cr * cr)
    d = am - au
    core = np.array([[d * cl * cr + au * math.sqrt(L * R), d * cl * nr],
                     [d * nl * cr, d * nl * nr]])
    return np.sort(np.linalg.svd(core, compute_uv=False))[::-1]


def test_mps_schmidt_values_match_closed_form():
    n, k = 10, 25
    W = inputs.config_c1().instances[0].marked
    m = mps.run(n, W, k, chi_cap=4)
    for cut in (1, 3, 5, 9):
        assert np.allclose(m.schmidt_values(cut), _schmidt_m1(n, int(W[0]), k, cut), atol=1e-12)
    # values quoted in the build survey, computed from the same 2x2 core
    assert np.allclose(_schmidt_m1(n, int(W[0]), k, 1), [0.99986527, 0.0164144], atol=1e-7)
    assert np.allclose(_schmidt_m1(n, int(W[0]), k, 5), [0.99974656, 0.02251271], atol=1e-7)


def test_mps_truncation_below_rank_loses_weight():
    n, M = 9, 3
    W = inputs.draw_marked(n, M, inputs.SplitMix64(77))
    exact = mps.run(n, W, 3, chi_cap=M + 1)
    cut = mps.run(n, W, 3, chi_cap=2)
    assert exact.discarded < 1e-20
    assert cut.discarded > 1e-8
    assert abs(cut.marked_prob() - cf.p_marked(n, M, 3)) > 1e-6


def test_mps_mid_run_against_closed_form_n20():
    inst = inputs.config_c2().instances[0]
    m = mps.GroverMPS(inst.n, inst.marked, inst.chi_cap)
    for j in (10, 20):
        m.iterate(10)
        assert m.marked_prob() == pytest.approx(cf.p_marked(20, 1, j), abs=1e-12)


def test_mps_amplitude_at_marked_and_unmarked():
    n, M, k = 14, 2, 11
    W = inputs.draw_marked(n, M, inputs.SplitMix64(3))
    m = mps.run(n, W, k, chi_cap=3)
    am, au = cf.amplitudes_wr(n, M, k)
    for x in W:
        assert m.amplitude(int(x)).real == pytest.approx(am, abs=1e-13)
    for x in (0, 1, 12345, (1 << n) - 1):
        if x not in set(int(v) for v in W):
            assert m.amplitude(x).real == pytest.approx(au, abs=1e-13)


# ---------------------------------------------------------------- sampling
def test_samplers_agree_exactly():
    n, M, k = 9, 2, 5
    W = inputs.draw_marked(n, M, inputs.SplitMix64(12))
    psi = sv.grover_sv(n, W, k)
    b_cf, p0s, us = sampling.sample(n, W, k, 200, seed=99, inst=4)
    b_sv = sampling.sample_from_statevector(psi, n, 200, seed=99, inst=4)
    m = mps.run(n, W, k, chi_cap=M + 1)
    b_mps, p0m, _ = m.sample(200, seed=99, inst=4)
    near = np.abs(us - p0s).min(axis=1) < 1e-9
    assert np.array_equal(b_cf[~near], b_sv[~near])
    assert np.array_equal(b_cf[~near], b_mps[~near])


def test_sampling_histogram_chi_square():
    # Near P = 1/2 the marked fraction is a fair binomial check; n=10, k=12 gives P = 0.49598.
    n, k = 10, 12
    W = [333]
    p = cf.p_marked(n, 1, k)
    assert p == pytest.approx(0.49598, abs=1e-5)
    bits, _, _ = sampling.sample(n, W, k, 2000, seed=5)
    hits = int(np.sum(bits == 333))
    sd = math.sqrt(2000 * p * (1 - p))
    assert abs(hits - 2000 * p) < 4.5 * sd
    # unmarked outcomes spread evenly over the other 1023 values (chi-square on 8 bins)
    other = bits[bits != 333].astype(np.int64) >> 7
    counts = np.bincount(other, minlength=8)
    exp = len(other) / 8.0
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    assert chi2 < 24.3   # 7 dof, p = 0.001
