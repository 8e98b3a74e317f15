"""The all-FP32 path (GMPS_FP32, lane-group kernel) against the FP64 oracle.

Every step runs in FP32 with round-to-nearest, so the result is the oracle's up to an
accumulated rounding error, not to a fixed tolerance. Each of the R = k (M + 1) reflections
rebuilds the chain through n QR steps and n SVD steps, whose inner products have at most
D = 12 terms. Each step perturbs the state by at most about c D u relative, with u = 2^-24.
Round-to-nearest errors can add up coherently over the reflections, so the state error is
bounded by R n c D u (taken with c = 2: one rounding in the product, one in the
factorisation). The amplitude bound below is that figure. The bound on P is twice it,
since |P - P'| <= 2 |psi - psi'| for unit states. A dropped term, a wrong sign or a
transposed operand gives an O(1) error and fails the bound.
"""
import sys

import numpy as np
import pytest

from oracle import closed_form as cf
from oracle import sampling as osamp
from oracle import statevector as sv
from paper_2601_03832_amd import gmps, inputs

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def amp_bound(n, M, k):
    return max(k, 1) * (M + 1) * n * 2 * 12 * U32


def run(instances, **kw):
    b = gmps.Batch(instances, "fp32", **kw)
    b.init_uniform()
    b.iterate([i.k for i in instances])
    return b


def test_fp32_c1_full_statevector(gpu):
    say("case: fp32 C1 n=10 k=25")
    inst = inputs.config_c1().instances[0]
    b = run([inst])
    bound = amp_bound(10, 1, 25)
    p = b.marked_prob()[0]
    assert abs(p - cf.p_marked(10, 1, 25)) < 2 * bound
    psi = sv.grover_sv(10, inst.marked, 25)
    amps = b.amplitudes(0, np.arange(1024, dtype=np.uint64))
    err = np.max(np.abs(amps - psi))
    say("  max |d amp| = %.2e (bound %.2e), |dP| = %.2e" % (err, bound, abs(p - cf.p_marked(10, 1, 25))))
    assert err < bound
    d = b.diagnostics()
    assert d["k_done"][0] == 25 and d["status"][0] == 0
    # FP32 work is counted as such
    assert d["flops32"][0] > 0 and d["flops64"][0] == 0
    b.close()


def test_fp32_ragged_batch(gpu):
    say("case: fp32 ragged batch n in [2,14], M in {1..4}")
    insts = inputs.random_batch(37, 2, 14, (1, 2, 3, 4), seed=31, cap_extra=1)
    b = run(insts)
    p = b.marked_prob()
    for i, inst in enumerate(insts):
        bound = amp_bound(inst.n, inst.M, inst.k)
        assert abs(p[i] - cf.p_marked(inst.n, inst.M, inst.k)) < 2 * bound, (i, inst.n, inst.M, inst.k)
    for i in (0, 5, 17, 36):
        inst = insts[i]
        psi = sv.grover_sv(inst.n, inst.marked, inst.k)
        amps = b.amplitudes(i, np.arange(1 << inst.n, dtype=np.uint64))
        assert np.max(np.abs(amps - psi)) < amp_bound(inst.n, inst.M, inst.k)
    d = b.diagnostics()
    for i, inst in enumerate(insts):
        prof = d["bond_dims"][i]
        for l in range(1, inst.n):
            assert prof[l] <= min(2 ** l, 2 ** (inst.n - l), inst.M + 1)
    b.close()


def test_fp32_edge_cases(gpu):
    say("case: fp32 edge cases n=1, n=2, M=N-1, k=0")
    insts = [inputs.Instance(1, np.array([1], np.uint64), 1, 2),
             inputs.Instance(2, np.array([2], np.uint64), 1, 2),
             inputs.Instance(3, np.arange(5, dtype=np.uint64), 3, 6),
             inputs.Instance(6, np.array([0, 63], np.uint64), 0, 3)]
    b = run(insts)
    p = b.marked_prob()
    for i, inst in enumerate(insts):
        exp = cf.p_marked(inst.n, inst.M, inst.k)
        assert abs(p[i] - exp) < 2 * amp_bound(inst.n, inst.M, inst.k), (i, p[i], exp)
    assert b.diagnostics()["k_done"].tolist() == [1, 1, 3, 0]
    b.close()


def test_fp32_needs_the_lane_group_kernel(gpu):
    say("case: fp32 rejects the team kernel and bond caps above 6")
    inst = inputs.Instance(10, np.array([3], np.uint64), 2, 2)
    with pytest.raises(gmps.GmpsError) as e:
        gmps.Batch([inst], "fp32", kernel="team")
    assert e.value.code == gmps.GMPS_E_UNSUPPORTED
    rng = inputs.SplitMix64(9)
    wide = inputs.Instance(14, inputs.draw_marked(14, 8, rng), 2, 9)
    with pytest.raises(gmps.GmpsError) as e:
        gmps.Batch([wide], "fp32")
    assert e.value.code == gmps.GMPS_E_UNSUPPORTED


def test_fp32_full_k_within_bound(gpu):
    """M = 1 at n = 16 and 20 for the full k (hundreds of iterations): the FP32 error stays
    within the accumulated-rounding bound, the mixed path on the same kernel within 1e-6, and
    both results are valid probabilities."""
    say("case: fp32 vs mixed, M=1, n=16 and 20 at the full k")
    rng = inputs.SplitMix64(77)
    insts = [inputs.Instance(n, inputs.draw_marked(n, 1, rng), inputs.k_rule(n, 1), 2) for n in (16, 20)]
    errs = {}
    for prec in ("fp32", "mixed"):
        b = gmps.Batch(insts, prec, kernel="group")
        b.init_uniform()
        b.iterate([i.k for i in insts])
        p = b.marked_prob(allow_numeric=True)
        b.close()
        errs[prec] = [abs(p[i] - cf.p_marked(x.n, 1, x.k)) for i, x in enumerate(insts)]
        assert all(0.0 <= q <= 1.0 + 1e-6 for q in p)
        say("  %s |dP| = %s" % (prec, ", ".join("%.2e" % e for e in errs[prec])))
    for i, x in enumerate(insts):
        assert errs["fp32"][i] < 2 * amp_bound(x.n, 1, x.k)
        assert errs["mixed"][i] < 1e-6


def test_fp32_sampling_matches_oracle(gpu):
    """Perfect sampling from FP32 states replays the oracle's exact site-by-site draw with the
    same Philox uniforms; a shot may differ only where its uniform lies within the marginal's
    error (twice the amplitude bound) of the decision threshold."""
    say("case: fp32 sampling replay, 12 instances x 64 shots")
    insts = inputs.random_batch(12, 5, 12, (1, 2, 4), seed=99)
    b = run(insts)
    bits, hits = b.sample(64, 4242)
    nbad = 0
    for i, inst in enumerate(insts):
        tie = 2 * amp_bound(inst.n, inst.M, inst.k)
        exp, p0s, us = osamp.sample(inst.n, inst.marked, inst.k, 64, 4242, i)
        for sh in np.nonzero(bits[i] != exp)[0]:
            x, y = int(bits[i][sh]), int(exp[sh])
            first = next(t for t in range(inst.n) if ((x ^ y) >> (inst.n - 1 - t)) & 1)
            assert abs(us[sh, first] - p0s[sh, first]) < tie, (i, sh, first)
            nbad += 1
        assert hits[i] == sum(1 for x in bits[i] if int(x) in set(int(v) for v in inst.marked))
    say("  %d of %d shots differ at near-ties" % (nbad, 64 * len(insts)))
    b.close()


def test_fp32_no_underflow_in_the_qr(gpu):
    """Regression: in FP32 the squared norm of a QR column entry near 1e-20 is a denormal, which
    v_rsq_f32 flushes (an infinite estimate, NaN after the Newton step); it hit M = 2 instances
    of the 4096-instance workload with n >= 25 in their first iteration. The QR treats squared
    norms below 1e-30 as zero on the FP32 path."""
    say("case: fp32, every M=2, n>=25 instance of the 4096-instance workload, 2 iterations")
    insts = [inputs.Instance(i.n, i.marked, 2, i.chi_cap) for i in inputs.config_c4().instances
             if i.M == 2 and i.n >= 25]
    b = run(insts)
    p = b.marked_prob()
    d = b.diagnostics()
    assert np.all(np.isfinite(p)) and not np.any(d["status"] & gmps.ST_NAN)
    for i, inst in enumerate(insts):
        assert abs(p[i] - cf.p_marked(inst.n, 2, 2)) < 2 * amp_bound(inst.n, 2, 2), (i, inst.n)
    say("  %d instances finite" % len(insts))
    b.close()


def _angle(b, idx, inst):
    """Rotation angle phi~ = atan2(<w|psi>, <r|psi>) of the state (Eq. (5)): <w|psi> from the
    marked amplitudes, <r|psi> from them and the overlap with |s>."""
    import math
    n, M = inst.n, inst.M
    a = b.amplitudes(idx, np.asarray(inst.marked, dtype=np.uint64)).real
    s = b.overlap_uniform(idx).real
    N = float(2 ** n)
    w = float(np.sum(a)) / math.sqrt(M)
    r = (math.sqrt(N) * s - math.sqrt(M) * w) / math.sqrt(N - M)
    return math.atan2(w, r)


# The paper's FP32 MPS runs (Section IV, Fig. 3) lose P at the optimal k: 0.997 at n = 18 and
# 0.877 at n = 28. At the peak P = cos^2(delta) for an angle error delta, so the smaller of the
# two is an angle error of acos(sqrt(0.997)) = 0.055 rad. The gate is a tenth of that, fixed
# from the paper's figure, not from this path's errors: a degradation of the paper's kind fails
# it at every n from 16 to 28, half way (where P moves at first order) and at the full k.
PAPER_FP32_DELTA = 0.055
FP32_ANGLE_GATE = PAPER_FP32_DELTA / 10


def test_fp32_precision_study_angle(gpu):
    """M = 1 at n = 16, 18, ..., 28 (one instance of each stratum of the 4096-instance
    workload) in FP32 on the lane-group kernel: the rotation angle half way and at the full k,
    and P at both points, within the gate above."""
    import math
    c4 = inputs.config_c4().instances
    insts = [[i for i in c4 if i.n == n and i.M == 1][0] for n in range(16, 29, 2)]
    say("case: fp32 precision study, M=1, n=16..28, half and full k")
    b = gmps.Batch(insts, "fp32")
    b.init_uniform()
    half = [i.k // 2 for i in insts]
    for stage, ks, step in (("half k", half, half), ("full k", [i.k for i in insts], [i.k - h for i, h in zip(insts, half)])):
        b.iterate(step)
        p = b.marked_prob(allow_numeric=True)
        for j, inst in enumerate(insts):
            phi = (2 * ks[j] + 1) * cf.theta(inst.n, 1)
            dphi = _angle(b, j, inst) - phi
            dp = p[j] - cf.p_marked(inst.n, 1, ks[j])
            say("  %s n=%d k=%d: dP %.2e, angle error %.2e" % (stage, inst.n, ks[j], dp, dphi))
            assert abs(dphi) <= FP32_ANGLE_GATE, (stage, inst.n, dphi)
            assert abs(dp) <= math.sin(FP32_ANGLE_GATE) ** 2 + abs(math.sin(2 * phi)) * FP32_ANGLE_GATE, (stage, inst.n, dp)
    b.close()
