"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every function
include/gmps.h declares, sizes workspaces and rejects bad arguments before any device call."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2601_03832_amd import gmps, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gmps.h")
SV_HEADER = os.path.join(ROOT, "include", "gsv.h")


def _declared(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\**\s+\**(\w+)\s*\(", text, flags=re.M)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(gmps.LIB_PATH):
        pytest.fail("libgmps.so is not built; run python -m paper_2601_03832_amd.build")
    return gmps.load()


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for must in ("mps_init_uniform", "grover_iterate", "marked_prob", "sample_shots", "gmps_create",
                 "gmps_destroy", "gmps_workspace_bytes", "gmps_strerror"):
        assert must in names


def test_library_exports_every_declared_symbol(lib):
    declared = _declared() + _declared(SV_HEADER)
    for name in declared:
        assert hasattr(lib, name), name
    assert set(gmps.EXPORTED) <= set(declared)


def test_statevector_workspace_and_argument_checks(lib):
    lib.gsv_workspace_bytes.restype = ctypes.c_size_t
    b64 = lib.gsv_workspace_bytes(20, 1, gmps.GMPS_FP64)
    b32 = lib.gsv_workspace_bytes(20, 1, gmps.GMPS_MIXED)
    assert b64 >= 8 << 20 and b32 >= 4 << 20 and b64 > b32 and b64 % 256 == 0
    assert lib.gsv_workspace_bytes(34, 1, gmps.GMPS_FP64) >= 8 << 34
    for n, M in ((0, 1), (35, 1), (3, 8), (3, 0)):
        assert lib.gsv_workspace_bytes(n, M, gmps.GMPS_FP64) == 0
    h = ctypes.c_void_p()
    P64 = ctypes.POINTER(ctypes.c_uint64)
    dup = np.array([3, 3], dtype=np.uint64)
    big = np.array([1 << 10], dtype=np.uint64)
    ok = np.array([3], dtype=np.uint64)
    assert lib.gsv_create(ctypes.byref(h), 10, dup.ctypes.data_as(P64), 2, gmps.GMPS_FP64, ctypes.c_void_p(256),
                          1 << 30, None) == gmps.GMPS_E_ARG
    assert lib.gsv_create(ctypes.byref(h), 10, big.ctypes.data_as(P64), 1, gmps.GMPS_FP64, ctypes.c_void_p(256),
                          1 << 30, None) == gmps.GMPS_E_ARG
    assert lib.gsv_create(ctypes.byref(h), 10, ok.ctypes.data_as(P64), 1, gmps.GMPS_FP64, ctypes.c_void_p(0),
                          1 << 30, None) == gmps.GMPS_E_WORKSPACE
    assert lib.gsv_create(ctypes.byref(h), 10, ok.ctypes.data_as(P64), 1, gmps.GMPS_FP64, ctypes.c_void_p(256),
                          16, None) == gmps.GMPS_E_WORKSPACE
    for fn in ("gsv_init_uniform", "gsv_destroy"):
        getattr(lib, fn).argtypes = [ctypes.c_void_p]
    assert lib.gsv_init_uniform(None) == gmps.GMPS_E_ARG
    assert lib.gsv_destroy(None) == gmps.GMPS_OK


def test_strerror_names_every_code(lib):
    for code in (0, -1, -2, -3, -4, -5):
        s = gmps.strerror(code)
        assert s and s != "unknown status"
    assert gmps.strerror(-99) == "unknown status"


def test_workspace_bytes(lib):
    c1 = inputs.config_c1().instances
    arr, _ = gmps.pack_instances(c1)
    b64 = lib.gmps_workspace_bytes(arr, 1, gmps.GMPS_FP64)
    b32 = lib.gmps_workspace_bytes(arr, 1, gmps.GMPS_MIXED)
    assert b64 > b32 > 0 and b64 % 256 == 0
    # invalid: n = 0, M >= 2^n, cap 0, B = 0, bad precision
    for n, M, cap in ((0, 1, 2), (3, 8, 2), (5, 1, 0), (64, 1, 2)):
        bad = (gmps.GmpsInstance * 1)()
        bad[0].n, bad[0].M, bad[0].chi_cap = n, M, cap
        assert lib.gmps_workspace_bytes(bad, 1, gmps.GMPS_FP64) == 0
    assert lib.gmps_workspace_bytes(arr, 0, gmps.GMPS_FP64) == 0
    assert lib.gmps_workspace_bytes(arr, 1, 7) == 0


def test_bond_cap_beyond_tile_classes_is_unsupported(lib):
    big = (gmps.GmpsInstance * 1)()
    big[0].n, big[0].M, big[0].chi_cap = 30, 40, 41   # effective cap min(41, M+1) = 41
    assert lib.gmps_workspace_bytes(big, 1, gmps.GMPS_MIXED) == 0
    h = ctypes.c_void_p()
    marked = np.arange(40, dtype=np.uint64)
    rc = lib.gmps_create(ctypes.byref(h), big, 1, marked.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                         gmps.GMPS_MIXED, None, ctypes.c_void_p(256), 1 << 30, None)
    assert rc == gmps.GMPS_E_UNSUPPORTED


def _create(lib, insts, marked, ws_ptr=256, ws_bytes=1 << 30, prec=gmps.GMPS_FP64):
    h = ctypes.c_void_p()
    return lib.gmps_create(ctypes.byref(h), insts, len(insts),
                           marked.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), prec, None,
                           ctypes.c_void_p(ws_ptr), ws_bytes, None)


def test_create_rejects_bad_marked_sets_before_touching_a_device(lib):
    inst = (gmps.GmpsInstance * 1)()
    inst[0].n, inst[0].M, inst[0].chi_cap, inst[0].marked_off = 4, 2, 3, 0
    assert _create(lib, inst, np.array([3, 3], dtype=np.uint64)) == gmps.GMPS_E_ARG      # duplicate
    assert _create(lib, inst, np.array([3, 16], dtype=np.uint64)) == gmps.GMPS_E_ARG     # out of range
    inst[0].reserved = 1
    assert _create(lib, inst, np.array([3, 4], dtype=np.uint64)) == gmps.GMPS_E_ARG      # reserved != 0


def test_create_checks_the_workspace(lib):
    inst = (gmps.GmpsInstance * 1)()
    inst[0].n, inst[0].M, inst[0].chi_cap = 6, 1, 2
    m = np.array([5], dtype=np.uint64)
    need = lib.gmps_workspace_bytes(inst, 1, gmps.GMPS_FP64)
    assert _create(lib, inst, m, ws_ptr=0) == gmps.GMPS_E_WORKSPACE
    assert _create(lib, inst, m, ws_bytes=need - 1) == gmps.GMPS_E_WORKSPACE
    assert _create(lib, inst, m, ws_ptr=256 + 8) == gmps.GMPS_E_WORKSPACE


def test_calls_on_null_handle_fail_cleanly(lib):
    assert lib.mps_init_uniform(None) == gmps.GMPS_E_ARG
    k = np.array([1], dtype=np.int64)
    assert lib.grover_iterate(None, k.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 1) == gmps.GMPS_E_ARG
    assert lib.marked_prob(None, None) == gmps.GMPS_E_ARG
    assert lib.gmps_destroy(None) == gmps.GMPS_OK


def test_binding_refuses_to_run_without_a_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    with pytest.raises(RuntimeError):
        gmps.Batch(inputs.config_c1().instances)


def test_struct_layouts_match_the_binding(tmp_path):
    """The ctypes mirrors of gmps_options, gmps_instance and gmps_plan have the header's field
    offsets."""
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    src = tmp_path / "layout.c"
    opt_fields = [f for f, _ in gmps.GmpsOptions._fields_]
    inst_fields = [f for f, _ in gmps.GmpsInstance._fields_]
    plan_fields = [f for f, _ in gmps.GmpsPlan._fields_]
    body = ["#include <stdio.h>", "#include <stddef.h>", '#include "gmps.h"', "int main(void) {",
            'printf("%zu\\n", sizeof(gmps_options));', 'printf("%zu\\n", sizeof(gmps_instance));',
            'printf("%zu\\n", sizeof(gmps_plan));']
    body += ['printf("%%zu\\n", offsetof(gmps_options, %s));' % f for f in opt_fields]
    body += ['printf("%%zu\\n", offsetof(gmps_instance, %s));' % f for f in inst_fields]
    body += ['printf("%%zu\\n", offsetof(gmps_plan, %s));' % f for f in plan_fields]
    body += ["return 0; }"]
    src.write_text("\n".join(body) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(gmps.GmpsOptions)
    assert vals[1] == ctypes.sizeof(gmps.GmpsInstance)
    assert vals[2] == ctypes.sizeof(gmps.GmpsPlan)
    offs = vals[3:]
    got = [getattr(gmps.GmpsOptions, f).offset for f in opt_fields] + [getattr(gmps.GmpsInstance, f).offset for f in inst_fields] + \
        [getattr(gmps.GmpsPlan, f).offset for f in plan_fields]
    assert offs == got


def test_precision_codes_match_the_header():
    text = open(HEADER).read()
    codes = dict((k, int(v)) for k, v in re.findall(r"\b(GMPS_(?:FP64|MIXED|FP32))\s*=\s*(\d+)", text))
    assert codes == {"GMPS_FP64": gmps.GMPS_FP64, "GMPS_MIXED": gmps.GMPS_MIXED, "GMPS_FP32": gmps.GMPS_FP32}


def test_fp32_workspace_and_rejections_before_touching_a_device(lib):
    """GMPS_FP32 stores complex64 sites like the mixed path; it runs on the lane-group kernel
    only, so the team kernel and bond caps above that kernel's classes are refused."""
    c1 = inputs.config_c1().instances
    arr, _ = gmps.pack_instances(c1)
    assert lib.gmps_workspace_bytes(arr, 1, gmps.GMPS_FP32) == lib.gmps_workspace_bytes(arr, 1, gmps.GMPS_MIXED) > 0
    assert lib.gsv_workspace_bytes(10, 1, gmps.GMPS_FP32) == 0
    wide = (gmps.GmpsInstance * 1)()
    wide[0].n, wide[0].M, wide[0].chi_cap = 14, 8, 9    # effective cap 9 > 6
    assert _create(lib, wide, np.arange(8, dtype=np.uint64), prec=gmps.GMPS_FP32) == gmps.GMPS_E_UNSUPPORTED
    narrow = (gmps.GmpsInstance * 1)()
    narrow[0].n, narrow[0].M, narrow[0].chi_cap = 10, 1, 2
    opt = gmps.GmpsOptions()
    opt.kernel = gmps.KERNELS["team"]
    h = ctypes.c_void_p()
    m = np.array([3], dtype=np.uint64)
    rc = lib.gmps_create(ctypes.byref(h), narrow, 1, m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                         gmps.GMPS_FP32, ctypes.byref(opt), ctypes.c_void_p(256), 1 << 30, None)
    assert rc == gmps.GMPS_E_UNSUPPORTED


def test_circuit_bytes_counts_the_gates_of_fig1a(lib):
    """gmps_circuit_bytes: one 32-bit word per gate of k layers of Fig. 1(A). Per marked x: an X
    on each qubit where x has a 0, before and after the n-controlled Z; then the diffusion as
    H and X on every qubit, the n-controlled Z, X and H on every qubit."""
    insts = [inputs.Instance(6, [0b101101, 0], 3, 4), inputs.Instance(9, [511], 2, 2), inputs.Instance(4, [5], 0, 2)]
    arr, marked = gmps.pack_instances(insts)
    ks = np.array([i.k for i in insts], dtype=np.int64)
    got = lib.gmps_circuit_bytes(arr, len(insts), marked.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                 ks.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), len(ks))
    # (6, {101101, 000000}): zeros 2 and 6 -> (2*2+1) + (2*6+1) + (4*6+1) = 43 gates per layer
    # (9, {111111111}): 1 + 37 = 38; (4, {0101}): 5 + 17 = 22, but k = 0 -> no gates
    assert got == 4 * (3 * 43 + 2 * 38 + 0)
    one = np.array([1], dtype=np.int64)
    assert lib.gmps_circuit_bytes(arr, len(insts), marked.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                  one.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 1) == 4 * (43 + 38 + 22)
    bad = np.array([-1], dtype=np.int64)
    assert lib.gmps_circuit_bytes(arr, len(insts), marked.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                  bad.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 1) == 0
    assert lib.grover_circuit_run(None) == gmps.GMPS_E_ARG
    assert lib.gmps_circuit_build(None, one.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), 1, None, 0) == gmps.GMPS_E_ARG


def test_jacobi_probe_library_shapes():
    """The Jacobi test probe (tests/gpu_probes) loads without a GPU and reports each team class's
    Jacobi shape as the team layout defines it: KJ = chi_max + 1 rounded up to even columns, and
    2 chi_max rows (the bond-2 MPO's largest bond) held as PJ lanes per column times RJ rows per
    lane, PJ the largest of 16, 8, 4, 2 with KJ * PJ <= the team width."""
    path = os.path.join(ROOT, "tests", "gpu_probes", "libjacobi_probe.so")
    if not os.path.exists(path):
        pytest.fail("the Jacobi probe is not built; run __graft_entry__.build()")
    probe = ctypes.CDLL(path)
    probe.gmps_probe_jacobi_shape.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    assert hasattr(probe, "gmps_probe_team_jacobi")
    for w, (cap, tw) in enumerate([(2, 16), (3, 32), (5, 64), (8, 64), (17, 192), (32, 256)]):
        kj, rows = ctypes.c_int(), ctypes.c_int()
        assert probe.gmps_probe_jacobi_shape(w, ctypes.byref(kj), ctypes.byref(rows)) == 0
        want_kj = (cap + 2) // 2 * 2
        pj = next(p for p in (16, 8, 4, 2) if want_kj * p <= tw)
        rj = -(-2 * cap // pj)
        assert (kj.value, rows.value) == (want_kj, min(2 * cap, pj * rj)), (w, kj.value, rows.value)
    kj, rows = ctypes.c_int(), ctypes.c_int()
    assert probe.gmps_probe_jacobi_shape(6, ctypes.byref(kj), ctypes.byref(rows)) == -1
