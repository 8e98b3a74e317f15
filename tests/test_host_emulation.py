"""The iterate kernel bodies run on the CPU under sanitizers, lanes emulated as threads.

tests/host_emu/emu_kernel.cpp calls run_team, run_team_pc, run_team_circ or run_pipe (the device code of
csrc/, unchanged except that `extern __shared__` reads `extern` in the copies compiled here)
with every lane of the workgroup an OS thread. Cross-lane operations (DPP, swizzle,
bpermute, ballot) and barriers synchronise exactly the lanes they involve, and a lane group
that does not arrive complete is reported as divergent; every buffer is its own heap block of
the size the library gives it, so AddressSanitizer sees any access outside a per-lane array,
the LDS block or a global buffer, and ThreadSanitizer sees any LDS or global access between
lanes that no barrier or wave fence orders. Each run is then compared with the statevector
oracle.

Cases: the gate-level circuit kernel of the Common method; the pipelined pre-contracted reflections (one reflection for the whole oracle, and one
per marked index where M exceeds the class bond); the bond-32 class (CM = 32, 256-thread teams, four waves) with bond-2 MPO and with
pre-contracted reflections at n = 12, M = 24 and 31 (the cases whose GPU build of the
pre-contracted variant failed; the variant stays off on the GPU); the pipelined two-wave
kernel of the bond-5 class (the headline launch's longest chains), mixed under
ThreadSanitizer and FP64 under AddressSanitizer; under ThreadSanitizer also the pipelined
bond-2 class (four 16-lane teams per wave) and the sequential team kernel of the bond-5 class.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from oracle import statevector as sv
from paper_2601_03832_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "host_emu")
CSRC = os.path.join(ROOT, "paper_2601_03832_amd", "csrc")
HEADERS = ("gmps_pipe.h", "gmps_team.h", "gmps_device.h", "gmps_internal.h")


@pytest.fixture(scope="module")
def tree(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("emu")
    os.makedirs(d / "pkg" / "csrc")
    os.makedirs(d / "include")
    for h in HEADERS:
        with open(os.path.join(CSRC, h)) as f:
            (d / "pkg" / "csrc" / h).write_text(f.read().replace("extern __shared__", "extern"))
    shutil.copy(os.path.join(ROOT, "include", "gmps.h"), d / "include" / "gmps.h")
    return d


def build(tree, kind, w, s, sanitize):
    exe = tree / ("emu_%d_%d_%s_%s" % (kind, w, s, sanitize.replace(",", "_")))
    if not exe.exists():
        cmd = ["g++", "-std=c++20", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread", "-fsanitize=" + sanitize,
               "-DEMU_KIND=%d" % kind, "-DEMU_W=%d" % w, "-DEMU_S=%s" % s, "-I" + EMU,
               "-I" + str(tree / "pkg" / "csrc"), os.path.join(EMU, "emu_kernel.cpp"), "-o", str(exe)]
        if "undefined" in sanitize:
            cmd.insert(6, "-fno-sanitize-recover=undefined")
        subprocess.run(cmd, check=True, timeout=600)
    return exe


def run(exe, n, M, cap, k, W):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", TSAN_OPTIONS="halt_on_error=1:exitcode=66")
    stdin = "%d %d %d %d\n%s\n" % (n, M, cap, k, " ".join(str(int(x)) for x in W))
    r = subprocess.run([str(exe)], input=stdin, capture_output=True, text=True, timeout=900, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    for bad in ("runtime error", "ThreadSanitizer", "AddressSanitizer", "divergent"):
        assert bad not in r.stderr, r.stderr[-4000:]
    lines = r.stdout.strip().split("\n")
    st, drift, tw, kd = lines[0].split()
    bonds = [int(x) for x in lines[1].split()]
    amps = np.array([complex(float(a), float(b)) for a, b in (l.split() for l in lines[2:])])
    return int(st), float(drift), int(kd), bonds, amps


def large_cap_instances():
    """The (n, M, cap) of the large-cap GPU test, drawn in its order from its seed."""
    rng = inputs.SplitMix64(4711)
    out = {}
    for n, M, extra in ((9, 7, 1), (10, 9, 2), (10, 16, 1), (11, 13, 4), (12, 24, 3), (12, 31, 1), (6, 5, 30)):
        out[(n, M)] = (inputs.draw_marked(n, M, rng), M + extra)
    return out


@pytest.mark.parametrize("kind", [0, 1], ids=["mpo", "precontract"])
@pytest.mark.parametrize("M", [24, 31])
def test_bond32_class_under_address_sanitizer(tree, kind, M):
    W, cap = large_cap_instances()[(12, M)]
    exe = build(tree, kind, 5, "double", "address,undefined")
    st, drift, kd, bonds, amps = run(exe, 12, M, cap, 1, W)
    assert st == 0 and kd == 1
    assert np.max(np.abs(amps - sv.grover_sv(12, W, 1))) < 1e-12


@pytest.mark.parametrize("s,sanitize,tol", [("float", "thread", 1e-6), ("double", "address,undefined", 1e-12)],
                         ids=["mixed-tsan", "fp64-asan"])
def test_pipelined_bond5_kernel(tree, s, sanitize, tol):
    W = inputs.draw_marked(10, 4, inputs.SplitMix64(21))
    exe = build(tree, 2, 2, s, sanitize)
    st, drift, kd, bonds, amps = run(exe, 10, 4, 6, 3, W)
    assert st == 0 and kd == 3
    assert np.max(np.abs(amps - sv.grover_sv(10, W, 3))) < tol


@pytest.mark.parametrize("kind,w,M", [(2, 0, 1), (0, 2, 4)], ids=["pipelined-bond2", "sequential-bond5"])
def test_more_classes_under_thread_sanitizer(tree, kind, w, M):
    W = inputs.draw_marked(10, M, inputs.SplitMix64(30 + M))
    exe = build(tree, kind, w, "float", "thread")
    st, drift, kd, bonds, amps = run(exe, 10, M, M + 1, 2, W)
    assert st == 0 and kd == 2
    assert np.max(np.abs(amps - sv.grover_sv(10, W, 2))) < 1e-6


@pytest.mark.parametrize("w,n,M,k,sanitize", [(2, 10, 4, 3, "thread"), (0, 9, 1, 4, "thread"),
                                              (2, 5, 8, 2, "address,undefined")],
                         ids=["bond5-whole-oracle-tsan", "bond2-tsan", "bond5-per-index-asan"])
def test_pipelined_precontracted(tree, w, n, M, k, sanitize):
    W = inputs.draw_marked(n, M, inputs.SplitMix64(40 + n))
    exe = build(tree, 3, w, "double", sanitize)
    st, drift, kd, bonds, amps = run(exe, n, M, M + 1, k, W)
    assert st == 0 and kd == k
    assert max(bonds) > 1
    assert np.max(np.abs(amps - sv.grover_sv(n, W, k))) < 1e-12


@pytest.mark.parametrize("w,n,M,k,sanitize", [(0, 9, 1, 3, "thread"), (2, 10, 4, 2, "address,undefined")],
                         ids=["bond2-tsan", "bond5-asan"])
def test_gate_level_circuit(tree, w, n, M, k, sanitize):
    """run_team_circ (the Common method) on the k-layer gate list of Fig. 1(A), against the
    gate-level statevector oracle."""
    W = inputs.draw_marked(n, M, inputs.SplitMix64(60 + n))
    exe = build(tree, 4, w, "double", sanitize)
    st, drift, kd, bonds, amps = run(exe, n, M, M + 1, k, W)
    assert st == 0 and kd == k
    assert max(bonds) > 1
    assert np.max(np.abs(amps - sv.grover_gates(n, W, k))) < 1e-12
