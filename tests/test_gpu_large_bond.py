"""Parity of the team kernel on bond caps the lane-group kernel does not hold (CM 8, 17, 32).

Small n: every amplitude against the statevector, P against the closed form of Eq. (6).
n = 40, M = 16 (the 256-instance workload's shape, exact bond 17): a prefix of k iterations
against the closed form, gated on the rotation angle (from P, Eq. (6), and from the mean marked
amplitude, Eq. (5)) since P itself is tiny early in the run, the oracle MPS's exact bond profile
and amplitudes on one instance, and a sampling replay against the oracle's closed-form sampler.
Tolerances as in the other parity tests."""
import sys

import numpy as np
import pytest

from oracle import closed_form as cf
from oracle import mps as omps
from oracle import sampling as osamp
from oracle import statevector as sv
from paper_2601_03832_amd import gmps, inputs

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-6}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def bound_ok(prof, n, M):
    return all(prof[l] <= min(2 ** l, 2 ** (n - l), M + 1) for l in range(1, n))


@pytest.mark.parametrize("precision,pc", [("fp64", False), ("fp64", True), ("mixed", False)],
                         ids=["fp64-mpo", "fp64-precontract", "mixed-mpo"])
def test_large_cap_small_n_statevector(gpu, precision, pc):
    say("case: large caps at small n, %s, precontract=%s" % (precision, pc))
    rng = inputs.SplitMix64(4711)
    insts = []
    for n, M, extra in ((9, 7, 1), (10, 9, 2), (10, 16, 1), (11, 13, 4), (12, 24, 3), (12, 31, 1), (6, 5, 30)):
        W = inputs.draw_marked(n, M, rng)
        if pc and M + 1 > 17:
            continue  # pre-contraction is built for bond caps up to 17 (see the tests below)
        insts.append(inputs.Instance(n, W, inputs.k_rule(n, M), M + extra))
    b = gmps.Batch(insts, precision, kernel="team", precontract=pc)
    b.init_uniform()
    b.iterate([i.k for i in insts])
    p = b.marked_prob()
    d = b.diagnostics()
    for i, inst in enumerate(insts):
        assert abs(p[i] - cf.p_marked(inst.n, inst.M, inst.k)) < TOL[precision], (i, inst.n, inst.M)
        psi = sv.grover_sv(inst.n, inst.marked, inst.k)
        amps = b.amplitudes(i, np.arange(1 << inst.n, dtype=np.uint64))
        assert np.max(np.abs(amps - psi)) < (1e-11 if precision == "fp64" else 2e-6), (i, inst.n, inst.M)
        # the Schmidt rank at a cut depends on how the marked states share prefixes: the
        # oracle's MPS (exact arithmetic up to rounding) gives the profile. complex64 storage
        # can leave a noise direction just above the mixed path's cut (5e-7 relative); it
        # carries no weight at the 1e-6 level (checked above), so there the profile may
        # exceed the exact one, never the rank bound
        ref = omps.run(inst.n, inst.marked, inst.k, inst.chi_cap).bond_dims()
        if precision == "fp64":
            assert d["bond_dims"][i] == ref, i
        else:
            assert all(a >= r for a, r in zip(d["bond_dims"][i], ref)), (i, d["bond_dims"][i], ref)
        assert bound_ok(d["bond_dims"][i], inst.n, inst.M)
        assert d["status"][i] == 0


def test_precontract_refusals(gpu):
    """The pre-contracted variant is not built for the bond-32 class, and it runs on FP64 only
    (on complex64 storage its rotation angle drifts, in both sweep orders): gmps_create refuses
    both rather than running something else under the flag."""
    W = inputs.draw_marked(12, 24, inputs.SplitMix64(4712))
    inst = inputs.Instance(12, W, inputs.k_rule(12, 24), 27)
    for precision in ("fp64", "mixed"):
        with pytest.raises(gmps.GmpsError) as e:
            gmps.Batch([inst], precision, kernel="team", precontract=True)
        assert e.value.code == gmps.GMPS_E_UNSUPPORTED
    small = inputs.Instance(12, W[:4], inputs.k_rule(12, 4), 6)   # bond-5 class (pipelined)
    mid = inputs.Instance(12, W[:12], inputs.k_rule(12, 12), 13)  # bond-17 class
    lossy = inputs.Instance(12, W[:4], inputs.k_rule(12, 4), 4)   # cap below the exact rank 5
    for bad in (small, mid, lossy):
        for pipe in (True, False):
            with pytest.raises(gmps.GmpsError) as e:
                gmps.Batch([bad], "mixed", kernel="team", precontract=True, pipeline=pipe)
            assert e.value.code == gmps.GMPS_E_UNSUPPORTED
    for ok in (small, mid, lossy):
        gmps.Batch([ok], "fp64", kernel="team", precontract=True).close()


@pytest.mark.skip(reason="the pre-contracted kernel of the bond-32 class (CM = 32, 256-thread teams) is not "
                         "built: an FP64 build returned NaN with every bond 1 at M = 24 and 31, and a later "
                         "build faulted with a memory aperture violation; no cause has been found in the "
                         "code, so the case stays off the GPU until one is")
def test_precontract_bond32_class_matches_statevector(gpu):
    rng = inputs.SplitMix64(4713)
    insts = []
    for n, M in ((12, 24), (12, 31)):
        W = inputs.draw_marked(n, M, rng)
        insts.append(inputs.Instance(n, W, inputs.k_rule(n, M), M + 1))
    b = gmps.Batch(insts, "fp64", kernel="team", precontract=True)
    b.init_uniform()
    b.iterate([i.k for i in insts])
    p = b.marked_prob()
    for i, inst in enumerate(insts):
        assert abs(p[i] - cf.p_marked(inst.n, inst.M, inst.k)) < TOL["fp64"]
        psi = sv.grover_sv(inst.n, inst.marked, inst.k)
        amps = b.amplitudes(i, np.arange(1 << inst.n, dtype=np.uint64))
        assert np.max(np.abs(amps - psi)) < 1e-11


# The angle gate: an error dphi of the rotation angle phi = (2k+1) theta moves P by
# sin(2 phi) dphi, at most dphi, and the run passes the point where P is steepest; the
# tolerance on P (1e-10 on FP64) therefore bounds the angle by 1e-10 rad. Early in an n = 40 run
# P itself is tiny (2e-4 after 2000 iterations), so an absolute P gate cannot fail there; the
# angle gate can. The angle is read two ways: from P = sin^2(phi) (Eq. (6)) and from the state's
# components along the normalised marked and unmarked superpositions (Eq. (5)).
# n = 40 runs need FP64: with complex64 storage the angle drifts by about 2e-9 (bond-2 MPO
# reflections) and 3e-10 (pre-contracted) per iteration, which the full k = 205887 turns into
# P errors far above 1e-6, so the mixed path makes no accuracy claim there.
PHI_TOL = {"fp64": 1e-10}


@pytest.mark.parametrize("pc,k", [(False, 300), (True, 2000)], ids=["mpo", "precontract"])
@pytest.mark.parametrize("precision", ["fp64"])
def test_n40_m16_prefix(gpu, precision, pc, k):
    say("case: n=40 M=16 cap 32, 2 instances, k=%d, %s, precontract=%s" % (k, precision, pc))
    w = inputs.config_c5(count=2, k=k)
    insts = w.instances
    b = gmps.Batch(insts, precision, precontract=pc)
    b.init_uniform()
    b.iterate(k)
    p = b.marked_prob()
    d = b.diagnostics()
    phi = (2 * k + 1) * cf.theta(40, 16)
    am, au = cf.amplitudes_wr(40, 16, k)
    for i, inst in enumerate(insts):
        dphi_p = np.arcsin(np.sqrt(p[i])) - phi
        say("  inst %d: P %.6e exact %.6e, angle error from P %.2e" % (i, p[i], cf.p_marked(40, 16, k), dphi_p))
        assert abs(dphi_p) <= PHI_TOL[precision], (i, dphi_p)
        assert abs(p[i] - cf.p_marked(40, 16, k)) < TOL[precision], (i, p[i])
        assert bound_ok(d["bond_dims"][i], 40, 16), d["bond_dims"][i]
        assert d["status"][i] == 0
        marked = np.asarray(inst.marked, dtype=np.uint64)
        a_m = b.amplitudes(i, marked)
        # the rotation angle from <w|psi> and <r|psi> (Eq. (5); <s|psi> from the overlap read-out)
        N = 2.0 ** 40
        wc = float(np.sum(a_m.real)) / 4.0
        rc = (np.sqrt(N) * b.overlap_uniform(i).real - 4.0 * wc) / np.sqrt(N - 16)
        dphi_a = np.arctan2(wc, rc) - phi
        say("  inst %d: angle error from <w|psi>, <r|psi> %.2e, marked spread %.2e"
            % (i, dphi_a, float(np.max(np.abs(a_m - np.mean(a_m))))))
        assert abs(dphi_a) <= PHI_TOL[precision], (i, dphi_a)
        # single marked amplitudes may drift apart along directions orthogonal to |w>, which
        # move P only at second order: the spread whose squared norm is the P tolerance
        assert np.max(np.abs(a_m - np.mean(a_m))) <= np.sqrt(TOL[precision] / 16), i


def test_n40_m16_oracle_and_sampling(gpu):
    k = 2
    say("case: n=40 M=16 fp64, k=%d against the oracle MPS, 64-shot replay" % k)
    w = inputs.config_c5(count=2, k=k)
    inst = w.instances[0]
    b = gmps.Batch(w.instances, "fp64")
    b.init_uniform()
    b.iterate(k)
    ref = omps.run(40, inst.marked, k, inst.chi_cap)
    assert b.diagnostics()["bond_dims"][0] == ref.bond_dims()
    assert abs(b.marked_prob()[0] - ref.marked_prob()) < 1e-10
    xs = np.concatenate([np.asarray(inst.marked, dtype=np.uint64), np.array([0, 12345, (1 << 40) - 1], np.uint64)])
    ga = b.amplitudes(0, xs)
    ra = np.array([ref.amplitude(int(x)) for x in xs])
    assert np.max(np.abs(ga - ra)) < 1e-12
    bits, hits = b.sample(64, 777)
    exp, p0s, us = osamp.sample(40, inst.marked, k, 64, 777, 0)
    bad = np.nonzero(bits[0] != exp)[0]
    for sh in bad:
        x, y = int(bits[0][sh]), int(exp[sh])
        first = next(i for i in range(40) if ((x ^ y) >> (39 - i)) & 1)
        assert abs(us[sh, first] - p0s[sh, first]) < 1e-9
    assert hits[0] == sum(1 for x in bits[0] if int(x) in set(int(v) for v in inst.marked))
