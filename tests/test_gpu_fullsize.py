"""Parity at the full workload sizes, in the launch configuration bench.py times.

* 4096-instance mixed batch (n 12..28, M 1/2/4, own k): every instance's P against the
  closed form (<= 1e-6), sampled amplitudes of every stratum against Eq. (5), and 4096
  shots per instance whose hit counts must match the closed-form probability
  (binomial bound) -- the oracle evaluates all of these one by one.
* n=29, k=18198, one marked state: FP64 P within 1e-10; the mixed path is logged every
  1000 iterations (the precision study) and must stay within 1e-6 at the end.
"""
import math
import sys

import numpy as np
import pytest

from oracle import closed_form as cf
from paper_2601_03832_amd import gmps, inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("pc,pipe", [(False, True), (False, False), (True, True)], ids=["mpo", "mpo-seq", "precontract"])
def test_batched_mixed_full_size(gpu, pc, pipe):
    say("case: 4096-instance mixed batch at full k, precontract=%s pipeline=%s" % (pc, pipe))
    w = inputs.config_c4()
    b = gmps.Batch(w.instances, "mixed", precontract=pc, pipeline=pipe)
    b.init_uniform()
    b.iterate([i.k for i in w.instances])
    p = b.marked_prob(allow_numeric=True)
    exp = np.array([cf.p_marked(i.n, i.M, i.k) for i in w.instances])
    err = np.abs(p - exp)
    say("max |dP| = %.3g" % err.max())
    assert err.max() <= 1e-6
    d = b.diagnostics()
    assert not np.any(d["status"] & gmps.ST_NAN)
    assert list(d["k_done"]) == [i.k for i in w.instances]
    # one instance per stratum: marked and unmarked amplitudes vs Eq. (5)
    seen = set()
    for idx, inst in enumerate(w.instances):
        key = (inst.n, inst.M)
        if key in seen:
            continue
        seen.add(key)
        am, au = cf.amplitudes_wr(inst.n, inst.M, inst.k)
        probe = [int(x) for x in inst.marked] + [0, (1 << inst.n) - 1, 12345 % (1 << inst.n)]
        probe = [x for x in dict.fromkeys(probe)]
        amps = b.amplitudes(idx, np.array(probe, dtype=np.uint64))
        marked = set(int(x) for x in inst.marked)
        # An error d shared by all M marked amplitudes moves P by 2*M*|am|*d, one shared by all
        # N-M unmarked amplitudes by 2*(N-M)*|au|*d: the bounds below are the amplitude errors
        # that would move P by the 1e-6 mixed-path tolerance.
        # The gate of the mixed path is on P. Single marked amplitudes drift apart in ways that
        # leave P unchanged to first order (G maps the marked directions orthogonal to |w> to
        # themselves, so rounding errors there random-walk): each reflection stores ~2n site
        # tensors in complex64 (unit roundoff 2^-24), so after k(M+1) reflections the relative
        # drift has scale sqrt(2 n k (M+1)) 2^-24 (8e-5 at n=28, M=4). Each amplitude is held to
        # four times that, and the marked weight read from the amplitudes must reproduce P.
        # Unmarked amplitudes are tiny near the optimum; an error d shared by all N-M of them
        # moves P by 2*(N-M)*|au|*d, so they are held to ten times the d that moves P by 1e-6.
        N = float(2 ** inst.n)
        tol_u = 10 * 1e-6 / (2 * (N - inst.M) * max(abs(au), 1e-300))
        for x, a in zip(probe, amps):
            walk = 4.0 * math.sqrt(2.0 * inst.n * inst.k * (inst.M + 1)) * 2.0 ** -24
            ref, tol = (am, walk * abs(am)) if x in marked else (au, tol_u)
            # the global phase is fixed by the sign convention, so compare signed values
            assert abs(a - ref) <= tol, (idx, x, a, ref, tol)
        wsum = float(np.sum(np.abs(amps[:inst.M]) ** 2))
        assert abs(wsum - p[idx]) <= 1e-6, (idx, wsum, p[idx])
    # sampling: hits per instance against the binomial law of P
    _, hits = b.sample(4096, w.shot_seed)
    for i, inst in enumerate(w.instances):
        q = exp[i]
        sd = math.sqrt(4096 * q * (1 - q)) + 1.0
        assert abs(hits[i] - 4096 * q) <= 6 * sd, (i, hits[i], q)
    say("sampling ok; strata checked: %d" % len(seen))


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


def test_n29_precision_study(gpu):
    say("case: n=29 precision study, mixed vs fp64, logged every 1000 iterations")
    inst = inputs.config_c3("mixed").instances[0]
    log = []
    bm = gmps.Batch([inst], "mixed")
    bd = gmps.Batch([inst], "fp64")
    bm.init_uniform()
    bd.init_uniform()
    done = 0
    while done < inst.k:
        step = min(1000, inst.k - done)
        bm.iterate(step)
        bd.iterate(step)
        done += step
        ex = cf.p_marked(29, 1, done)
        em = abs(bm.marked_prob(allow_numeric=True)[0] - ex)
        ed = abs(bd.marked_prob()[0] - ex)
        log.append((done, em, ed))
        say("  k=%5d  |dP| mixed %.3e  fp64 %.3e" % (done, em, ed))
    assert log[-1][2] <= 1e-10
    assert log[-1][1] <= 1e-6
