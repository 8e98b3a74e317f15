"""The Common method (Section III-A, Fig. 1(B)): the k-layer gate-level circuit of Fig. 1(A),
built once (gmps_circuit_build) and simulated gate by gate (grover_circuit_run), against the
gate-level statevector oracle (oracle.statevector.grover_gates, which applies the same gate
list to a dense vector) element by element, and against the iterative path: as gates a layer
is -G (the gate-level diffusion is I - 2|s><s|), so k layers give (-1)^k G^k |s>."""
import sys

import numpy as np
import pytest

from oracle import closed_form as cf
from oracle import statevector as sv
from paper_2601_03832_amd import gmps, inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_common(insts, k=None):
    b = gmps.Batch(insts, "fp64", kernel="team")
    b.init_uniform()
    b.build_circuit([i.k for i in insts] if k is None else k)
    b.run_circuit()
    return b


def full_state(b, idx, n):
    return b.amplitudes(idx, np.arange(1 << n, dtype=np.uint64))


def test_c1_common_matches_the_gate_oracle(gpu):
    say("case: C1 (n=10, M=1, k=25) through the gate-level circuit")
    w = inputs.config_c1()
    inst = w.instances[0]
    b = run_common([inst])
    psi = full_state(b, 0, inst.n)
    ref = sv.grover_gates(inst.n, inst.marked, inst.k)
    assert np.max(np.abs(psi - ref)) < 1e-12
    assert abs(b.marked_prob()[0] - cf.p_marked(inst.n, 1, inst.k)) < 1e-10
    d = b.diagnostics()
    assert d["k_done"][0] == inst.k and d["status"][0] == 0
    b.close()


def ragged():
    """Classes of bond 2 to 17 (n 3..12, M up to 12, lossless caps), and 12 instances of
    (n = 8, M = 1) that share a bundle of four 16-lane teams with gate streams of different
    lengths (their marked indices have different numbers of zeros)."""
    out = inputs.random_batch(30, 3, 12, (1, 2, 3, 4, 6, 12), seed=808, cap_extra=1, k_scale=0.4)
    rng = inputs.SplitMix64(809)
    out += [inputs.Instance(8, inputs.draw_marked(8, 1, rng), 5, 2) for _ in range(12)]
    return out


def test_ragged_common_matches_the_gate_oracle(gpu):
    insts = ragged()
    say("case: %d instances through the gate-level circuit, element by element" % len(insts))
    b = run_common(insts)
    for idx, inst in enumerate(insts):
        psi = full_state(b, idx, inst.n)
        ref = sv.grover_gates(inst.n, inst.marked, inst.k)
        assert np.max(np.abs(psi - ref)) < 1e-11, (idx, inst.n, inst.M, inst.k)
    b.close()


def test_common_equals_iterative_up_to_the_sign(gpu):
    insts = ragged()
    say("case: Common vs Iterative on the same %d instances" % len(insts))
    bc = run_common(insts)
    bi = gmps.Batch(insts, "fp64", kernel="team")
    bi.init_uniform()
    bi.iterate([i.k for i in insts])
    for idx, inst in enumerate(insts):
        a = full_state(bc, idx, inst.n)
        c = full_state(bi, idx, inst.n)
        assert np.max(np.abs(a - (-1) ** inst.k * c)) < 1e-11, idx
    assert np.max(np.abs(bc.marked_prob() - bi.marked_prob())) < 1e-12
    bc.close()
    bi.close()


def test_c2_common(gpu):
    say("case: C2 (n=20, k=804) through the gate-level circuit")
    inst = inputs.config_c2().instances[0]
    b = run_common([inst])
    assert abs(b.marked_prob()[0] - cf.p_marked(inst.n, 1, inst.k)) < 1e-10
    am, au = cf.amplitudes_wr(inst.n, 1, inst.k)
    a = b.amplitudes(0, np.array([int(inst.marked[0]), (int(inst.marked[0]) + 1) % (1 << inst.n)], dtype=np.uint64))
    sign = (-1) ** inst.k
    assert abs(a[0] - sign * am) < 1e-10 and abs(a[1] - sign * au) < 1e-12
    b.close()


def test_common_edge_cases_and_refusals(gpu):
    say("case: Common method edge cases and refusals")
    rng = inputs.SplitMix64(810)
    # k = 0: an empty circuit leaves |s>
    inst = inputs.Instance(7, inputs.draw_marked(7, 2, rng), 0, 3)
    b = run_common([inst])
    assert np.max(np.abs(full_state(b, 0, 7) - 2 ** -3.5)) < 1e-14
    b.close()
    # no circuit built
    b = gmps.Batch([inputs.Instance(6, [3], 2, 2)], "fp64", kernel="team")
    b.init_uniform()
    with pytest.raises(gmps.GmpsError) as e:
        b.run_circuit()
    assert e.value.code == gmps.GMPS_E_ARG
    b.close()
    # complex64 storage, one site, the bond-32 class
    for insts, prec in (([inputs.Instance(6, [3], 2, 2)], "mixed"), ([inputs.Instance(1, [1], 1, 2)], "fp64"),
                        ([inputs.Instance(12, inputs.draw_marked(12, 24, rng), 1, 25)], "fp64")):
        b = gmps.Batch(insts, prec, kernel="team")
        b.init_uniform()
        with pytest.raises(gmps.GmpsError) as e:
            b.build_circuit([1])
        assert e.value.code == gmps.GMPS_E_UNSUPPORTED
        b.close()
