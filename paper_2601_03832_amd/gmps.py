"""ctypes binding of libgmps (include/gmps.h): argument marshalling only.

Every step of the simulation runs in the HIP kernels of ``csrc/``. PyTorch supplies the
device workspace (a uint8 tensor) and the stream. If the shared library is missing, or no
GPU is visible, constructing a :class:`Batch` raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgmps.so")

GMPS_FP64 = 0
GMPS_MIXED = 1
GMPS_FP32 = 2
GMPS_OK = 0
GMPS_E_ARG = -1
GMPS_E_WORKSPACE = -2
GMPS_E_HIP = -3
GMPS_E_UNSUPPORTED = -4
GMPS_E_NUMERIC = -5
ST_NAN, ST_DRIFT, ST_TRUNC = 1, 2, 4
BOND_STRIDE = 64
KERNELS = {"auto": 0, "group": 1, "team": 2}

EXPORTED = ("gmps_workspace_bytes", "gmps_create", "mps_init_uniform", "grover_iterate", "grover_iterate_sample", "marked_prob",
            "sample_shots", "sample_shots_noalloc", "gmps_amplitudes", "gmps_overlap_uniform", "gmps_autotune", "gmps_diagnostics", "gmps_last_iterate_ms", "gmps_destroy",
            "gmps_circuit_bytes", "gmps_circuit_build", "grover_circuit_run",
            "gmps_state_bytes", "gmps_state_export", "gmps_state_import",
            "gmps_strerror", "gsv_workspace_bytes", "gsv_create", "gsv_init_uniform", "gsv_iterate",
            "gsv_marked_prob", "gsv_amplitudes", "gsv_last_iterate_ms", "gsv_destroy")


class GmpsInstance(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("M", ctypes.c_int32), ("chi_cap", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("marked_off", ctypes.c_int64)]


class GmpsOptions(ctypes.Structure):
    _fields_ = [("trunc_tol", ctypes.c_double), ("max_sweeps", ctypes.c_int32),
                ("waves_per_cu", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("round_mode", ctypes.c_int32), ("jacobi_warm", ctypes.c_int32),
                ("kernel", ctypes.c_int32), ("precontract", ctypes.c_int32),
                ("pipeline", ctypes.c_int32)]


class GmpsPlan(ctypes.Structure):
    _fields_ = [("pipeline", ctypes.c_int32), ("precontract", ctypes.c_int32), ("waves_per_cu", ctypes.c_int32),
                ("cached", ctypes.c_int32), ("candidates", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("ms", ctypes.c_double)]


class GmpsError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__("%s failed: %s (%d)" % (what, strerror(code), code))
        self.code = code


_lib = None


def load(path: Optional[str] = None):
    """Loads libgmps.so (built in-tree by ``paper_2601_03832_amd.build``); raises if absent."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError("libgmps.so not built (%s); run python -m paper_2601_03832_amd.build" % path)
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    i32, i64, u64, dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double
    lib.gmps_workspace_bytes.restype = ctypes.c_size_t
    lib.gmps_workspace_bytes.argtypes = [ctypes.POINTER(GmpsInstance), i32, ctypes.c_int]
    lib.gmps_create.restype = ctypes.c_int
    lib.gmps_create.argtypes = [ctypes.POINTER(P), ctypes.POINTER(GmpsInstance), i32, ctypes.POINTER(u64),
                                ctypes.c_int, ctypes.POINTER(GmpsOptions), P, ctypes.c_size_t, P]
    lib.mps_init_uniform.restype = ctypes.c_int
    lib.mps_init_uniform.argtypes = [P]
    lib.grover_iterate.restype = ctypes.c_int
    lib.grover_iterate.argtypes = [P, ctypes.POINTER(i64), i32]
    lib.grover_iterate_sample.restype = ctypes.c_int
    lib.grover_iterate_sample.argtypes = [P, ctypes.POINTER(i64), i32, ctypes.POINTER(i64), i32, u64,
                                          ctypes.POINTER(i64)]
    lib.marked_prob.restype = ctypes.c_int
    lib.marked_prob.argtypes = [P, ctypes.POINTER(dbl)]
    lib.sample_shots.restype = ctypes.c_int
    lib.sample_shots.argtypes = [P, ctypes.POINTER(i64), i32, u64, ctypes.POINTER(u64), ctypes.POINTER(i64)]
    lib.sample_shots_noalloc.restype = ctypes.c_int
    lib.sample_shots_noalloc.argtypes = [P, ctypes.POINTER(i64), i32, u64, ctypes.POINTER(u64), ctypes.POINTER(i64)]
    lib.gmps_amplitudes.restype = ctypes.c_int
    lib.gmps_amplitudes.argtypes = [P, i32, ctypes.POINTER(u64), i64, ctypes.POINTER(dbl)]
    lib.gmps_overlap_uniform.restype = ctypes.c_int
    lib.gmps_overlap_uniform.argtypes = [P, i32, ctypes.POINTER(dbl)]
    lib.gmps_autotune.restype = ctypes.c_int
    lib.gmps_autotune.argtypes = [P, ctypes.POINTER(i64), i32, i32, ctypes.c_char_p, ctypes.POINTER(GmpsPlan)]
    lib.gmps_circuit_bytes.restype = ctypes.c_size_t
    lib.gmps_circuit_bytes.argtypes = [ctypes.POINTER(GmpsInstance), i32, ctypes.POINTER(u64), ctypes.POINTER(i64), i32]
    lib.gmps_circuit_build.restype = ctypes.c_int
    lib.gmps_circuit_build.argtypes = [P, ctypes.POINTER(i64), i32, P, ctypes.c_size_t]
    lib.grover_circuit_run.restype = ctypes.c_int
    lib.grover_circuit_run.argtypes = [P]
    lib.gmps_state_bytes.restype = ctypes.c_size_t
    lib.gmps_state_bytes.argtypes = [P]
    lib.gmps_state_export.restype = ctypes.c_int
    lib.gmps_state_export.argtypes = [P, P, ctypes.c_size_t]
    lib.gmps_state_import.restype = ctypes.c_int
    lib.gmps_state_import.argtypes = [P, P, ctypes.c_size_t]
    lib.gmps_diagnostics.restype = ctypes.c_int
    lib.gmps_diagnostics.argtypes = [P, ctypes.POINTER(dbl), ctypes.POINTER(dbl), ctypes.POINTER(i32),
                                     ctypes.POINTER(i32), ctypes.POINTER(i64), ctypes.POINTER(dbl)]
    lib.gmps_last_iterate_ms.restype = ctypes.c_int
    lib.gmps_last_iterate_ms.argtypes = [P, ctypes.POINTER(dbl)]
    lib.gmps_destroy.restype = ctypes.c_int
    lib.gmps_destroy.argtypes = [P]
    lib.gmps_strerror.restype = ctypes.c_char_p
    lib.gmps_strerror.argtypes = [ctypes.c_int]
    lib.gsv_workspace_bytes.restype = ctypes.c_size_t
    lib.gsv_workspace_bytes.argtypes = [i32, i32, ctypes.c_int]
    lib.gsv_create.restype = ctypes.c_int
    lib.gsv_create.argtypes = [ctypes.POINTER(P), i32, ctypes.POINTER(u64), i32, ctypes.c_int, P, ctypes.c_size_t, P]
    for name in ("gsv_init_uniform", "gsv_destroy"):
        getattr(lib, name).restype = ctypes.c_int
        getattr(lib, name).argtypes = [P]
    lib.gsv_iterate.restype = ctypes.c_int
    lib.gsv_iterate.argtypes = [P, i64]
    lib.gsv_marked_prob.restype = ctypes.c_int
    lib.gsv_marked_prob.argtypes = [P, ctypes.POINTER(dbl)]
    lib.gsv_amplitudes.restype = ctypes.c_int
    lib.gsv_amplitudes.argtypes = [P, ctypes.POINTER(u64), i64, ctypes.POINTER(dbl)]
    lib.gsv_last_iterate_ms.restype = ctypes.c_int
    lib.gsv_last_iterate_ms.argtypes = [P, ctypes.POINTER(dbl)]
    _lib = lib
    return lib


def strerror(code: int) -> str:
    return load().gmps_strerror(int(code)).decode()


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def pack_instances(instances):
    """(ctypes array of GmpsInstance, packed uint64 marked array) from inputs.Instance objects."""
    arr = (GmpsInstance * len(instances))()
    marked = []
    off = 0
    for i, inst in enumerate(instances):
        W = np.asarray(inst.marked, dtype=np.uint64)
        arr[i].n = int(inst.n)
        arr[i].M = int(len(W))
        arr[i].chi_cap = int(inst.chi_cap)
        arr[i].reserved = 0
        arr[i].marked_off = off
        marked.append(W)
        off += len(W)
    return arr, np.ascontiguousarray(np.concatenate(marked) if marked else np.zeros(1, np.uint64))


def workspace_bytes(instances, precision: str) -> int:
    arr, _ = pack_instances(instances)
    return int(load().gmps_workspace_bytes(arr, len(instances), _prec(precision)))


def _prec(precision: str) -> int:
    if precision in ("fp64", GMPS_FP64):
        return GMPS_FP64
    if precision in ("mixed", GMPS_MIXED):
        return GMPS_MIXED
    if precision in ("fp32", GMPS_FP32):
        return GMPS_FP32
    raise ValueError("precision must be 'fp64', 'mixed' or 'fp32'")


class Batch:
    """A batch of independent Grover instances resident on the current GPU.

    The device workspace is a torch uint8 tensor owned by this object; all work is
    enqueued on ``stream`` (default: torch's current stream)."""

    def __init__(self, instances: Sequence, precision: str = "fp64", trunc_tol: float = 0.0,
                 max_sweeps: int = 0, waves_per_cu: int = 0, use_graph: bool = True, stream=None,
                 device=None, stochastic_rounding: Optional[bool] = None, jacobi_warm: Optional[bool] = None,
                 kernel: str = "auto", precontract: bool = False, pipeline: bool = True):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libgmps needs a ROCm GPU; none is visible")
        self.lib = load()
        self.instances = list(instances)
        self.B = len(self.instances)
        self.precision = precision
        self.n = np.array([i.n for i in self.instances], dtype=np.int64)
        self._arr, self._marked = pack_instances(self.instances)
        prec = _prec(precision)
        nbytes = int(self.lib.gmps_workspace_bytes(self._arr, self.B, prec))
        if nbytes == 0:
            raise GmpsError(GMPS_E_ARG, "gmps_workspace_bytes")
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        opt = GmpsOptions()
        opt.trunc_tol = float(trunc_tol)
        opt.max_sweeps = int(max_sweeps)
        opt.waves_per_cu = int(waves_per_cu)
        opt.use_graph = 1 if use_graph else -1
        opt.round_mode = 0 if stochastic_rounding is None else (1 if stochastic_rounding else -1)
        opt.jacobi_warm = 0 if jacobi_warm is None else (1 if jacobi_warm else -1)
        opt.kernel = KERNELS[kernel]
        opt.precontract = 1 if precontract else -1
        opt.pipeline = 1 if pipeline else -1
        self._opt = opt
        h = ctypes.c_void_p()
        rc = self.lib.gmps_create(ctypes.byref(h), self._arr, self.B, _ptr(self._marked, ctypes.c_uint64), prec,
                                  ctypes.byref(opt), ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                  ctypes.c_void_p(self.stream.cuda_stream))
        if rc != GMPS_OK:
            raise GmpsError(rc, "gmps_create")
        self.handle = h

    # -- lifecycle ---------------------------------------------------------------------
    def close(self):
        if getattr(self, "handle", None):
            self.lib.gmps_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what, allow_numeric=False):
        if rc == GMPS_OK or (allow_numeric and rc == GMPS_E_NUMERIC):
            return rc
        raise GmpsError(rc, what)

    # -- the four hot-path calls ----------------------------------------------------------
    def init_uniform(self):
        self._check(self.lib.mps_init_uniform(self.handle), "mps_init_uniform")

    def iterate(self, k):
        ks = np.ascontiguousarray(np.atleast_1d(np.asarray(k, dtype=np.int64)))
        self._check(self.lib.grover_iterate(self.handle, _ptr(ks, ctypes.c_int64), len(ks)), "grover_iterate")

    def autotune(self, k, probe_iters: int = 64, cache_path: Optional[str] = None) -> dict:
        """gmps_autotune: time the launch plans this batch allows on a probe scaled from the
        iteration counts k, switch to the fastest, leave every instance at |s>."""
        ks = np.ascontiguousarray(np.atleast_1d(np.asarray(k, dtype=np.int64)))
        plan = GmpsPlan()
        path = cache_path.encode() if cache_path else None
        self._check(self.lib.gmps_autotune(self.handle, _ptr(ks, ctypes.c_int64), len(ks), int(probe_iters), path,
                                           ctypes.byref(plan)), "gmps_autotune")
        return {"pipeline": plan.pipeline > 0, "precontract": plan.precontract > 0, "waves_per_cu": plan.waves_per_cu,
                "cached": bool(plan.cached), "candidates": plan.candidates, "probe_ms": plan.ms}

    def iterate_sample(self, k, shots, seed: int) -> np.ndarray:
        """grover_iterate_sample: iterate, then sample every final state in the same graph
        launch; returns the per-instance hit counts."""
        ks = np.ascontiguousarray(np.atleast_1d(np.asarray(k, dtype=np.int64)))
        sh = np.ascontiguousarray(np.atleast_1d(np.asarray(shots, dtype=np.int64)))
        hits = np.zeros(self.B, dtype=np.int64)
        self._check(self.lib.grover_iterate_sample(self.handle, _ptr(ks, ctypes.c_int64), len(ks),
                                                   _ptr(sh, ctypes.c_int64), len(sh), ctypes.c_uint64(seed),
                                                   _ptr(hits, ctypes.c_int64)), "grover_iterate_sample")
        return hits

    # -- the Common method: the k-layer gate-level circuit --------------------------------
    def build_circuit(self, k) -> int:
        """gmps_circuit_build: every instance's k-layer gate list (Fig. 1(A) gates), in a device
        buffer owned by this object; returns its size in bytes."""
        import torch
        ks = np.ascontiguousarray(np.atleast_1d(np.asarray(k, dtype=np.int64)))
        nbytes = int(self.lib.gmps_circuit_bytes(self._arr, self.B, _ptr(self._marked, ctypes.c_uint64),
                                                 _ptr(ks, ctypes.c_int64), len(ks)))
        self.circuit_buffer = torch.empty(max(nbytes, 4), dtype=torch.uint8, device=self.workspace.device)
        self._check(self.lib.gmps_circuit_build(self.handle, _ptr(ks, ctypes.c_int64), len(ks),
                                                ctypes.c_void_p(self.circuit_buffer.data_ptr()), nbytes),
                    "gmps_circuit_build")
        return nbytes

    def run_circuit(self):
        """grover_circuit_run: simulate the built circuits gate by gate."""
        self._check(self.lib.grover_circuit_run(self.handle), "grover_circuit_run")

    # -- checkpoint and resume ---------------------------------------------------------------
    def export_state(self) -> np.ndarray:
        """gmps_state_export: the batch's whole state as a host byte array."""
        buf = np.zeros(int(self.lib.gmps_state_bytes(self.handle)), dtype=np.uint8)
        self._check(self.lib.gmps_state_export(self.handle, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes),
                    "gmps_state_export")
        return buf

    def import_state(self, buf: np.ndarray):
        """gmps_state_import: continue from a checkpoint of a batch over the same instances."""
        buf = np.ascontiguousarray(buf, dtype=np.uint8)
        self._check(self.lib.gmps_state_import(self.handle, buf.ctypes.data_as(ctypes.c_void_p), buf.nbytes),
                    "gmps_state_import")

    def marked_prob(self, allow_numeric: bool = False) -> np.ndarray:
        out = np.zeros(self.B, dtype=np.float64)
        self.last_status = self._check(self.lib.marked_prob(self.handle, _ptr(out, ctypes.c_double)),
                                       "marked_prob", allow_numeric)
        return out

    def sample(self, shots, seed: int, noalloc: bool = False):
        """Shots per instance (one value or B values) -> (bitstrings per instance, hits).
        noalloc: use sample_shots_noalloc (static device array) instead of sample_shots."""
        sh = np.ascontiguousarray(np.atleast_1d(np.asarray(shots, dtype=np.int64)))
        per = sh if len(sh) == self.B else np.full(self.B, sh[0], dtype=np.int64)
        bits = np.zeros(max(int(per.sum()), 1), dtype=np.uint64)
        hits = np.zeros(self.B, dtype=np.int64)
        fn = self.lib.sample_shots_noalloc if noalloc else self.lib.sample_shots
        self._check(fn(self.handle, _ptr(sh, ctypes.c_int64), len(sh), ctypes.c_uint64(seed),
                       _ptr(bits, ctypes.c_uint64), _ptr(hits, ctypes.c_int64)),
                    "sample_shots_noalloc" if noalloc else "sample_shots")
        offs = np.concatenate([[0], np.cumsum(per)])
        return [bits[offs[i]:offs[i + 1]] for i in range(self.B)], hits

    # -- read-out -----------------------------------------------------------------------------
    def amplitudes(self, inst: int, xs) -> np.ndarray:
        xs = np.ascontiguousarray(np.asarray(xs, dtype=np.uint64))
        out = np.zeros(2 * len(xs), dtype=np.float64)
        self._check(self.lib.gmps_amplitudes(self.handle, int(inst), _ptr(xs, ctypes.c_uint64), len(xs),
                                             _ptr(out, ctypes.c_double)), "gmps_amplitudes")
        return out[0::2] + 1j * out[1::2]

    def overlap_uniform(self, inst: int) -> complex:
        """<s|psi> / ||psi|| for instance inst (|s> = |+>^n)."""
        out = np.zeros(2, dtype=np.float64)
        self._check(self.lib.gmps_overlap_uniform(self.handle, int(inst), _ptr(out, ctypes.c_double)),
                    "gmps_overlap_uniform")
        return complex(out[0], out[1])

    def diagnostics(self) -> dict:
        B = self.B
        drift = np.zeros(B)
        trunc = np.zeros(B)
        bonds = np.zeros(B * BOND_STRIDE, dtype=np.int32)
        status = np.zeros(B, dtype=np.int32)
        kd = np.zeros(B, dtype=np.int64)
        flops = np.zeros(2 * B)
        self._check(self.lib.gmps_diagnostics(self.handle, _ptr(drift, ctypes.c_double), _ptr(trunc, ctypes.c_double),
                                              _ptr(bonds, ctypes.c_int32), _ptr(status, ctypes.c_int32),
                                              _ptr(kd, ctypes.c_int64), _ptr(flops, ctypes.c_double)),
                    "gmps_diagnostics")
        bonds = bonds.reshape(B, BOND_STRIDE)
        return {"norm_drift": drift, "trunc_weight": trunc, "status": status, "k_done": kd,
                "bond_dims": [bonds[i, :self.instances[i].n + 1].tolist() for i in range(B)],
                "flops64": flops[0::2], "flops32": flops[1::2]}

    def last_iterate_ms(self) -> float:
        v = ctypes.c_double()
        self._check(self.lib.gmps_last_iterate_ms(self.handle, ctypes.byref(v)), "gmps_last_iterate_ms")
        return v.value


class StateVector:
    """Dense-statevector iterative Grover (include/gsv.h) for one instance on the current GPU:
    the paper's comparison backend. precision 'fp64' (FP64 vector) or 'mixed' (FP32 vector,
    FP64 sums)."""

    def __init__(self, n: int, marked, precision: str = "fp64", stream=None, device=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("libgmps needs a ROCm GPU; none is visible")
        self.lib = load()
        self.n = int(n)
        self.marked = np.ascontiguousarray(np.asarray(marked, dtype=np.uint64))
        prec = _prec(precision)
        nbytes = int(self.lib.gsv_workspace_bytes(self.n, len(self.marked), prec))
        if nbytes == 0:
            raise GmpsError(GMPS_E_ARG, "gsv_workspace_bytes")
        dev = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=dev)
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        h = ctypes.c_void_p()
        rc = self.lib.gsv_create(ctypes.byref(h), self.n, _ptr(self.marked, ctypes.c_uint64), len(self.marked), prec,
                                 ctypes.c_void_p(self.workspace.data_ptr()), nbytes,
                                 ctypes.c_void_p(self.stream.cuda_stream))
        if rc != GMPS_OK:
            raise GmpsError(rc, "gsv_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            self.lib.gsv_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != GMPS_OK:
            raise GmpsError(rc, what)

    def init_uniform(self):
        self._check(self.lib.gsv_init_uniform(self.handle), "gsv_init_uniform")

    def iterate(self, k: int):
        self._check(self.lib.gsv_iterate(self.handle, int(k)), "gsv_iterate")

    def marked_prob(self) -> float:
        v = ctypes.c_double()
        self._check(self.lib.gsv_marked_prob(self.handle, ctypes.byref(v)), "gsv_marked_prob")
        return v.value

    def amplitudes(self, xs) -> np.ndarray:
        xs = np.ascontiguousarray(np.asarray(xs, dtype=np.uint64))
        out = np.zeros(len(xs), dtype=np.float64)
        self._check(self.lib.gsv_amplitudes(self.handle, _ptr(xs, ctypes.c_uint64), len(xs),
                                            _ptr(out, ctypes.c_double)), "gsv_amplitudes")
        return out

    def last_iterate_ms(self) -> float:
        v = ctypes.c_double()
        self._check(self.lib.gsv_last_iterate_ms(self.handle, ctypes.byref(v)), "gsv_last_iterate_ms")
        return v.value
