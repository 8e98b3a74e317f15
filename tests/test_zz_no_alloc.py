"""sample_shots_noalloc (static device scratch) against sample_shots (workspace staging).

Both run the same sampling kernel on the same chain with the same Philox stream, so the
bitstrings and hit counts must agree bit for bit. Two calls in a row, the second on a smaller
batch with fewer shots, check that the static array's leftover contents (counters, offsets,
bits of the first call) do not leak into the second. A request beyond the array is refused
before anything runs.
"""
import sys

import numpy as np
import pytest

from paper_2601_03832_amd import gmps, inputs

pytestmark = pytest.mark.gpu

SCRATCH = 16 << 20  # GMPS_NOALLOC_SCRATCH_BYTES


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _batch(instances, precision):
    b = gmps.Batch(instances, precision)
    b.init_uniform()
    b.iterate(np.array([i.k for i in instances], dtype=np.int64))
    return b


def _same(b, shots, seed):
    bits_a, hits_a = b.sample(shots, seed)
    bits_b, hits_b = b.sample(shots, seed, noalloc=True)
    assert list(hits_a) == list(hits_b)
    for i in range(b.B):
        assert np.array_equal(bits_a[i], bits_b[i]), i
    return hits_b


def test_noalloc_sampling_matches_sample_shots(gpu):
    big = inputs.random_batch(40, 8, 20, (1, 2, 4), seed=71, k_scale=0.6)
    small = inputs.random_batch(5, 6, 14, (1, 3), seed=72, k_scale=1.0)
    say("case: sample_shots_noalloc, 40 mixed instances x 3000 shots, then 5 fp64 instances")
    b1 = _batch(big, "mixed")
    h1 = _same(b1, 3000, 101)
    assert h1.sum() > 0
    b2 = _batch(small, "fp64")
    shots = np.array([700, 0, 13, 250, 1], dtype=np.int64)
    _same(b2, shots, 102)
    # the first batch again, fewer shots, after the smaller call left its contents behind
    _same(b1, 64, 103)
    b1.close()
    b2.close()


def test_noalloc_refuses_requests_beyond_its_array(gpu):
    inst = inputs.random_batch(2, 8, 8, (1,), seed=73)
    say("case: sample_shots_noalloc beyond the static array")
    b = _batch(inst, "fp64")
    too_many = SCRATCH // 8  # one instance's bits alone exceed the array
    with pytest.raises(gmps.GmpsError) as e:
        b.sample(np.array([10, too_many], dtype=np.int64), 5, noalloc=True)
    assert e.value.code == gmps.GMPS_E_WORKSPACE
    # the same handle still samples afterwards
    _same(b, 100, 6)
    b.close()
