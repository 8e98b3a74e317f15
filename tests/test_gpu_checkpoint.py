"""Checkpoint and resume (gmps_state_export / gmps_state_import): a batch exported after k1
iterations and imported into a fresh handle over the same instances continues exactly as the
original does (same kernels on the same stored state: bit-identical amplitudes, P and
counters), on both precisions; a checkpoint of another batch is refused before any device
memory is written."""
import sys

import numpy as np
import pytest

from paper_2601_03832_amd import gmps, inputs

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_resume_continues_bit_identically(gpu, precision):
    say("case: checkpoint after k1, resume, k2 more, %s" % precision)
    insts = inputs.random_batch(20, 6, 16, (1, 2, 4), seed=1212, cap_extra=1)
    k1 = [max(1, i.k // 3) for i in insts]
    k2 = [i.k - a for i, a in zip(insts, k1)]
    a = gmps.Batch(insts, precision)
    a.init_uniform()
    a.iterate(k1)
    state = a.export_state()
    b = gmps.Batch(insts, precision)
    b.import_state(state)
    a.iterate(k2)
    b.iterate(k2)
    for idx, inst in enumerate(insts):
        xs = np.arange(1 << inst.n, dtype=np.uint64) if inst.n <= 12 else np.asarray(inst.marked, dtype=np.uint64)
        assert np.array_equal(a.amplitudes(idx, xs), b.amplitudes(idx, xs)), idx
    assert np.array_equal(a.marked_prob(allow_numeric=True), b.marked_prob(allow_numeric=True))
    da, db = a.diagnostics(), b.diagnostics()
    assert list(da["k_done"]) == list(db["k_done"]) == [i.k for i in insts]
    assert da["bond_dims"] == db["bond_dims"]
    a.close()
    b.close()


def test_import_refuses_another_batch(gpu):
    insts = inputs.random_batch(4, 6, 10, (1, 2), seed=1213, cap_extra=1)
    a = gmps.Batch(insts, "fp64")
    a.init_uniform()
    state = a.export_state()
    bigger = [inputs.Instance(insts[0].n + 1, insts[0].marked, insts[0].k, insts[0].chi_cap)] + insts[1:]
    for other, prec in ((insts[:3], "fp64"), (insts, "mixed"), (bigger, "fp64")):
        b = gmps.Batch(other, prec)
        b.init_uniform()
        with pytest.raises(gmps.GmpsError) as e:
            b.import_state(state)
        assert e.value.code == gmps.GMPS_E_ARG
        b.close()
    with pytest.raises(gmps.GmpsError):
        a.import_state(state[:100])
    a.close()
