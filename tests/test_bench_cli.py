"""bench.py's contract checks that need no GPU: a multi-GPU request exits with a message
before any device is touched, the accuracy gate's closed form agrees with the oracle's, and
the counter record is tied to the device sources."""
import json
import os
import subprocess
import sys

import pytest

from oracle import closed_form as cf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and "--gpus 2" in r.stderr
    assert r.stdout.strip() == ""


@pytest.mark.parametrize("n,M,k", [(10, 1, 25), (20, 1, 804), (28, 4, 6434), (40, 16, 205887), (3, 2, 1)])
def test_accuracy_gate_matches_the_oracle_closed_form(n, M, k):
    assert abs(bench.exact_p(n, M, k) - cf.p_marked(n, M, k)) < 1e-15


def test_traffic_record_is_tied_to_the_device_sources():
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic_grover_kernel.json")))
    for key in ("kernel_hash", "bytes_per_launch", "fetch_factor", "write_factor", "source"):
        assert key in rec
    assert os.path.exists(os.path.join(ROOT, rec["source"]))
    # the record is used only while it matches the sources it was measured on
    got = bench.traffic_record()
    assert (got is not None) == (rec["kernel_hash"] == bench.kernel_hash())
