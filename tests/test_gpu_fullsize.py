"""Parity at the full workload sizes, in the launch configuration bench.py times.

Every gate below follows from the two accuracy requirements alone, |P - P_exact| <= 1e-10 on
the FP64 path and <= 1e-6 on the mixed path (P from Eq. (6), P_exact = sin^2((2k+1) theta)),
and none is taken from a measured error:

* P itself, at the final k and mid-run. At the final k P sits at its peak, where it moves only
  at second order with an error of the rotation angle phi = (2k+1) theta; half way P ~ 1/2 and it
  moves at first order, sin(2 phi) dphi.
* The angle itself, at every checkpoint. By Eq. (5) the state is cos(phi) |r> + sin(phi) |w>,
  |w> and |r> the normalised uniform superpositions over the marked and the unmarked indices.
  Its components along them follow from the marked amplitudes and the overlap with
  |s> = |+>^n: <w|psi> = sum_W a_x / sqrt(M), <r|psi> = (sqrt(N) <s|psi> - sqrt(M) <w|psi>) /
  sqrt(N-M), and phi~ = atan2(<w|psi>, <r|psi>). The gate is the P the angle implies,
  |sin^2(phi~) - sin^2(phi)| <= tol: P itself gathers the angle error and the weight outside the
  span of |w> and |r>, and the angle alone cannot hide behind the second. Half way that is
  |dphi| <= tol; at the peak P is flat in phi, and the checkpoints before it see any angle error
  the state carries there, since G rotates the plane rigidly.
* The spread of the single marked amplitudes around their mean: G maps the marked directions
  orthogonal to |w> to themselves, so errors there move P only through their squared norm; the
  spread whose squared norm (over M amplitudes) equals tol is sqrt(tol / M).

Single unmarked amplitudes carry errors outside the span of |s> and the marked states, which P
sees only at second order; they are checked element by element against the statevector oracle
in the smaller parity tests.

Cases: the 4096-instance mixed batch (n 12..28, M 1/2/4, own k) at half and full k on the
pipelined and sequential sweeps, with 4096 shots per instance against the binomial law, and the
same batch in FP64 through the pre-contracted reflections, pipelined and sequential; the longest
chain of that batch (n=28, M=4) every 500 iterations (FP64 and mixed, both sweep orders, and
FP64 pre-contracted); n=29, k=18198 (the precision study) every 1000 iterations, FP64 and
mixed.
"""
import math
import sys

import numpy as np
import pytest

from oracle import closed_form as cf
from paper_2601_03832_amd import gmps, inputs

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-10, "mixed": 1e-6}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def angle_of(b, idx, inst):
    """(phi~, spread): the state's rotation angle from <w|psi> and <r|psi> (module docstring),
    and the largest deviation of a marked amplitude from their mean (normalised state)."""
    n, M = inst.n, inst.M
    a = b.amplitudes(idx, np.asarray(inst.marked, dtype=np.uint64)).real
    s = b.overlap_uniform(idx).real
    N = float(2 ** n)
    w = float(np.sum(a)) / math.sqrt(M)
    r = (math.sqrt(N) * s - math.sqrt(M) * w) / math.sqrt(N - M)
    return math.atan2(w, r), float(np.max(np.abs(a - np.mean(a))))


def check_angle(b, idx, inst, k, precision, label=""):
    tol = TOL[precision]
    phi, spread = angle_of(b, idx, inst)
    ex = (2 * k + 1) * cf.theta(inst.n, inst.M)
    dphi = phi - ex
    assert abs(math.sin(phi) ** 2 - math.sin(ex) ** 2) <= tol, (label, idx, dphi)
    assert spread <= math.sqrt(tol / inst.M), (label, idx, spread)
    return dphi, spread


@pytest.mark.parametrize("pc,pipe", [(False, True), (False, False)], ids=["mpo", "mpo-seq"])
def test_batched_mixed_full_size(gpu, pc, pipe):
    say("case: 4096-instance mixed batch, half and full k, precontract=%s pipeline=%s" % (pc, pipe))
    w = inputs.config_c4()
    ks = np.array([i.k for i in w.instances])
    half = ks // 2
    b = gmps.Batch(w.instances, "mixed", precontract=pc, pipeline=pipe)
    b.init_uniform()
    for stage, kk, step in (("half k", half, half), ("full k", ks, ks - half)):
        b.iterate(step)
        p = b.marked_prob(allow_numeric=True)
        exp = np.array([cf.p_marked(i.n, i.M, int(kk[j])) for j, i in enumerate(w.instances)])
        err = np.abs(p - exp)
        say("  %s: max |dP| = %.3g" % (stage, err.max()))
        assert err.max() <= TOL["mixed"], (stage, int(np.argmax(err)))
        # one instance per stratum: the marked set against Eq. (5)
        seen = set()
        worst = 0.0
        for idx, inst in enumerate(w.instances):
            key = (inst.n, inst.M)
            if key in seen:
                continue
            seen.add(key)
            dm, _ = check_angle(b, idx, inst, int(kk[idx]), "mixed", stage)
            worst = max(worst, abs(dm))
        say("  %s: strata %d, largest angle error %.3g" % (stage, len(seen), worst))
    d = b.diagnostics()
    assert not np.any(d["status"] & gmps.ST_NAN)
    assert list(d["k_done"]) == list(ks)
    # sampling: hits per instance against the binomial law of P
    exp = np.array([cf.p_marked(i.n, i.M, i.k) for i in w.instances])
    _, hits = b.sample(4096, w.shot_seed)
    for i, inst in enumerate(w.instances):
        q = exp[i]
        sd = math.sqrt(4096 * q * (1 - q)) + 1.0
        assert abs(hits[i] - 4096 * q) <= 6 * sd, (i, hits[i], q)
    say("sampling ok")


@pytest.mark.parametrize("pipe", [True, False], ids=["pipelined", "sequential"])
def test_batched_fp64_precontracted_full_size(gpu, pipe):
    """The 4096-instance workload in FP64 through the pre-contracted reflections (the fastest
    path), pipelined and sequential sweeps: P of every instance at half and full k, and
    4096-shot hit counts."""
    say("case: 4096-instance batch, fp64, pre-contracted reflections, pipeline=%s, half and full k" % pipe)
    w = inputs.config_c4()
    ks = np.array([i.k for i in w.instances])
    half = ks // 2
    b = gmps.Batch(w.instances, "fp64", precontract=True, pipeline=pipe)
    b.init_uniform()
    for stage, kk, step in (("half k", half, half), ("full k", ks, ks - half)):
        b.iterate(step)
        p = b.marked_prob()
        exp = np.array([cf.p_marked(i.n, i.M, int(kk[j])) for j, i in enumerate(w.instances)])
        err = np.abs(p - exp)
        say("  %s: max |dP| = %.3g" % (stage, err.max()))
        assert err.max() <= TOL["fp64"], (stage, int(np.argmax(err)))
    exp = np.array([cf.p_marked(i.n, i.M, i.k) for i in w.instances])
    _, hits = b.sample(4096, w.shot_seed)
    for i in range(len(w.instances)):
        q = exp[i]
        sd = math.sqrt(4096 * q * (1 - q)) + 1.0
        assert abs(hits[i] - 4096 * q) <= 6 * sd, (i, hits[i], q)
    b.close()


@pytest.mark.parametrize("precision,pipe,pc", [("fp64", True, False), ("fp64", False, False), ("mixed", True, False),
                                               ("mixed", False, False), ("fp64", True, True)],
                         ids=["fp64-pipelined", "fp64-sequential", "mixed-pipelined", "mixed-sequential", "fp64-pc"])
def test_longest_chain_every_500(gpu, precision, pipe, pc):
    """The workload's longest chain, n=28, M=4, k=6434, checked every 500 iterations."""
    w = inputs.config_c4()
    inst = next(i for i in w.instances if i.n == 28 and i.M == 4)
    say("case: n=28 M=4 k=%d %s pipeline=%s precontract=%s, every 500 iterations" % (inst.k, precision, pipe, pc))
    b = gmps.Batch([inst], precision, pipeline=pipe, precontract=pc)
    b.init_uniform()
    done = 0
    worst = 0.0
    while done < inst.k:
        step = min(500, inst.k - done)
        b.iterate(step)
        done += step
        dp = b.marked_prob(allow_numeric=True)[0] - cf.p_marked(28, 4, done)
        dm, spread = check_angle(b, 0, inst, done, precision, "k=%d" % done)
        say("  k=%5d  dP %.3e  angle %.3e  spread %.3e" % (done, dp, dm, spread))
        worst = max(worst, abs(dp))
        assert abs(dp) <= TOL[precision], (done, dp)
    say("  max |dP| %.3e" % worst)


def test_n29_precision_study(gpu):
    """n=29, k=18198 (one marked state): P and the marked amplitude against the closed form
    every 1000 iterations and at the end, FP64 and mixed side by side."""
    say("case: n=29 precision study, mixed vs fp64, every 1000 iterations")
    inst = inputs.config_c3("mixed").instances[0]
    bm = gmps.Batch([inst], "mixed")
    bd = gmps.Batch([inst], "fp64")
    bm.init_uniform()
    bd.init_uniform()
    done = 0
    log = []
    while done < inst.k:
        step = min(1000, inst.k - done)
        bm.iterate(step)
        bd.iterate(step)
        done += step
        ex = cf.p_marked(29, 1, done)
        em = bm.marked_prob(allow_numeric=True)[0] - ex
        ed = bd.marked_prob()[0] - ex
        am, _ = check_angle(bm, 0, inst, done, "mixed", "k=%d mixed" % done)
        ad, _ = check_angle(bd, 0, inst, done, "fp64", "k=%d fp64" % done)
        log.append((done, em, ed, am, ad))
        say("  k=%5d  dP mixed %.3e  fp64 %.3e   angle mixed %.3e  fp64 %.3e" % (done, em, ed, am, ad))
        assert abs(ed) <= TOL["fp64"], (done, ed)
        assert abs(em) <= TOL["mixed"], (done, em)
    assert log[-1][0] == inst.k


def test_n29_fp64_full_k(gpu):
    say("case: n=29 k=18198 fp64")
    inst = inputs.config_c3("fp64").instances[0]
    b = gmps.Batch([inst], "fp64")
    b.init_uniform()
    b.iterate(inst.k)
    p = b.marked_prob()[0]
    assert abs(p - cf.p_marked(29, 1, inst.k)) <= 1e-10
    am, au = cf.amplitudes_wr(29, 1, inst.k)
    a = b.amplitudes(0, np.array([int(inst.marked[0]), 7], dtype=np.uint64))
    assert abs(a[0] - am) <= 1e-10 and abs(a[1] - au) <= 1e-15
