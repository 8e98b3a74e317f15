"""The benchmark's algorithmic flop model (the roofline's numerator), pinned by hand and by the
per-iterate totals the workload's specification prints for the single-instance cases."""
import bench
from paper_2601_03832_amd import inputs


def test_two_site_reflection_by_hand():
    # n = 2, M = 1: bonds [1, 2, 1]; MPO-doubled middle bond 4.
    # QR sweep: R*A 8*1*1*2*4 = 64; QR of the 2 x 4 tile 8*(2*4*2^2 - 2*2^3/3) = 213.33;
    # last site R*A 8*2*4*2 = 128. Truncation: Jacobi of 2 x 2, 6 sweeps * 1 rotation * 56*2
    # = 672; (U S)*A 8*2*1*2*2 = 64.
    prof = bench.exact_rank_profile(2, 1, 4)
    assert prof == [1, 2, 1]
    expect = 64 + 8 * (32 - 16 / 3) + 128 + 672 + 64
    assert abs(bench.reflection_flops(prof) - expect) < 1e-9


def test_exact_rank_profile():
    assert bench.exact_rank_profile(10, 1, 4) == [1] + [2] * 9 + [1]
    assert bench.exact_rank_profile(6, 4, 6) == [1, 2, 4, 5, 4, 2, 1]
    assert bench.exact_rank_profile(6, 16, 3) == [1, 2, 3, 3, 3, 2, 1]


def test_single_instance_totals_per_iterate():
    # printed per-iterate model totals of the three single-instance cases: 1.7e5, 3.9e5, 6.0e5
    for w, printed in ((inputs.config_c1(), 1.7e5), (inputs.config_c2(), 3.9e5), (inputs.config_c3(), 6.0e5)):
        i = w.instances[0]
        per_it = (i.M + 1) * bench.reflection_flops(bench.exact_rank_profile(i.n, i.M, i.chi_cap))
        assert abs(per_it - printed) <= 0.05e5, (w.name, per_it)


def test_batched_totals():
    w = inputs.config_c4()
    tot = bench.model_flops(w.instances, [i.k for i in w.instances])
    assert 4.4e13 <= tot <= 4.7e13  # printed: about 4.5e13 for the whole batch
    i = inputs.config_c5(count=1).instances[0]
    per_it = (i.M + 1) * bench.reflection_flops(bench.exact_rank_profile(i.n, i.M, i.chi_cap))
    assert abs(per_it - 4.5e9) <= 0.05e9  # printed: 4.5e9 per iterate
