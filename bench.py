"""Benchmark: Grover iterations/s on one MI355X, batched mixed precision vs plain FP64.

One step is one pass of the whole hot path over the batched workload: every instance is
reset to |s> (mps_init_uniform), iterated to its own k and sampled in the same graph launch
(grover_iterate_sample: the persistent class kernels, then perfect sampling of every final
state), and read out (marked_prob). value = sum_i k_i / step time.
The accuracy gate requires |P_i - sin^2((2k_i+1) theta_i)| <= 1e-6 for every instance.

    python bench.py [--gpus 1] [--steps 2] [--warmup 1] [--workload c4|c2|c3] [--kernel auto|team|group]
                    [--budget 330] [--c5-k 5000] [--sv-k 500] [--no-plain] [--no-cpu] [--no-fp64-batch]
                    [--sequential] [--no-precontract] [--no-fp32] [--fp32-c4] [--no-small]

Besides the headline line, the default run adds legs on the same hardware, in priority order
while the time budget lasts: the single-instance cases (n=10 and n=20, FP64, median of 5),
the workload through the FP64 path and with pre-contracted reflections, the n=29 precision
study (FP64 vs mixed, P logged every 1000 iterations), the Common method against the Iterative
one on the single-instance cases, per-instance FP64 handles, the dense
statevector backend, the all-FP32 precision study and a 5000-iteration prefix of the n=40,
M=16 workload (pre-contracted reflections in FP64, with 1/8/4096-shot hit fractions).
The CPU oracle runs first, before the GPU is touched.

Prints one JSON line. roofline: algorithmic flops of the iterate launch from the LAPACK-style
model below, over the launch's HIP-event duration, against the FP64 vector peak (every
arithmetic step of the path is FP64). cpu_baseline: the CPU oracle on all usable host cores.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from paper_2601_03832_amd import inputs  # noqa: E402

FP64_VECTOR_PEAK = 78.6e12    # MI355X published FP64 vector rate, FLOP/s
FP32_VECTOR_PEAK = 157.3e12   # MI355X published FP32 vector rate, FLOP/s
HBM_PEAK = 8.0e12             # MI355X published HBM3E bandwidth, bytes/s
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_grover_kernel.json")
# the launch's longest class kernel on the 4096-instance workload (bond cap 5: the pipelined
# sweeps by default); the roofline's flops, bytes and time cover every class kernel of the launch
KERNEL_NAME = {"auto": "grover_pipe_kernel", "team": "grover_pipe_kernel", "group": "grover_group_kernel"}
CSRC = os.path.join(ROOT, "paper_2601_03832_amd", "csrc")
MAX_WORKERS = 16  # CPU share of one GPU on the benchmark machines


def kernel_hash() -> str:
    """Hash of the device sources: a stored counter record is used only while it matches."""
    h = hashlib.sha256()
    for name in sorted(os.listdir(CSRC)):
        if name.endswith((".hip", ".h")) and name != "gmps_api.hip":
            with open(os.path.join(CSRC, name), "rb") as f:
                h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def exact_p(n: int, M: int, k: int) -> float:
    """Accuracy gate: sin^2((2k+1) asin(sqrt(M/2^n))), the success probability of Eq. (6)."""
    return math.sin((2 * k + 1) * math.asin(math.sqrt(M / float(2 ** n)))) ** 2


# ------------------------------------------------------------------ algorithmic flop model
# One reflection (an n-controlled Z as a bond-2 MPO, then recompression) on a chain whose bond
# profile is chi[0..n]: LAPACK Working Note 41 counts, x4 for complex arithmetic.
#  * QR sweep, site i = 0..n-2: X = R A_i with R (r x D_i) and the MPO-doubled site
#    (D_i x 2 x D_{i+1}, D_l = 2 chi_l inside the chain): 8 r D_i 2 D_{i+1}; then a full QR
#    of the 2r x D_{i+1} tile with explicit Q, 2 * 4 * (2 m c^2 - 2 c^3 / 3) with m >= c the
#    larger and c the smaller dimension; r <- min(2r, D_{i+1}) (no rank stop). The last site
#    takes R A_{n-1}.
#  * Truncation sweep, site i = n-1..1: one-sided Jacobi SVD of the r_i x 2 chi_{i+1} tile,
#    6 sweeps of c(c-1)/2 rotations of 56 m flops (c the smaller, m the larger dimension);
#    then (U S) moves into the site on the left: 8 (2 r_{i-1}) r_i chi_i.
# It reproduces 1.7e5, 3.9e5 and 6.0e5 flops per iterate for n = 10, 20 and 29 with one
# marked state and bond cap 4, and 4.59e13 for the 4096-instance workload.
JACOBI_SWEEPS = 6


def _qr_flops(m: int, c: int) -> float:
    big, small = max(m, c), min(m, c)
    return 2.0 * 4.0 * (2.0 * big * small * small - 2.0 * small ** 3 / 3.0)


def reflection_flops(chi) -> float:
    n = len(chi) - 1
    D = [1] + [2 * chi[l] for l in range(1, n)] + [1]
    tot = 0.0
    r = 1
    rs = [1]
    for i in range(n - 1):
        tot += 8.0 * r * D[i] * 2 * D[i + 1]
        tot += _qr_flops(2 * r, D[i + 1])
        r = min(2 * r, D[i + 1])
        rs.append(r)
    tot += 8.0 * r * D[n - 1] * 2
    for i in range(n - 1, 0, -1):
        a, b = rs[i], 2 * chi[i + 1]
        c, m = min(a, b), max(a, b)
        tot += JACOBI_SWEEPS * c * (c - 1) / 2.0 * 56.0 * m
        tot += 8.0 * 2 * rs[i - 1] * rs[i] * chi[i]
    return tot


def exact_rank_profile(n: int, M: int, cap: int):
    """Bond profile of every state the iteration passes through once it has spread: the
    Schmidt rank at a cut is at most M+1 and 2^min(l, n-l), and the cap bounds it."""
    return [min(cap, M + 1, 2 ** min(l, n - l)) for l in range(n + 1)]


def model_flops(instances, ks, profiles=None) -> float:
    """sum_i k_i (M_i + 1) reflection_flops(profile_i); profiles default to the exact ranks."""
    cache = {}
    tot = 0.0
    for j, inst in enumerate(instances):
        prof = tuple(profiles[j]) if profiles is not None else tuple(exact_rank_profile(inst.n, inst.M, inst.chi_cap))
        key = (inst.M, prof)
        if key not in cache:
            cache[key] = (inst.M + 1) * reflection_flops(list(prof))
        tot += float(ks[j]) * cache[key]
    return tot


def workload(name: str) -> inputs.Workload:
    if name == "c4":
        return inputs.config_c4()
    if name == "c2":
        return inputs.config_c2()
    if name == "c3":
        return inputs.config_c3("mixed")
    if name == "c3fp64":
        return inputs.config_c3("fp64")
    raise SystemExit("unknown workload " + name)


def plan_name(kernel: str, plan) -> str:
    """The launch plan in words: the kernel choice and, when autotuned, the plan it picked."""
    if not plan:
        return kernel + " (library default plan)"
    if plan.get("chosen") == "library default plan":
        return kernel + " (library default plan: faster than the autotuner's pick in a full-size step)"
    return "%s: %s sweeps, %s reflections, %s workgroups per CU (autotuned)" % (
        "team" if kernel == "auto" else kernel, "pipelined" if plan["pipeline"] else "sequential",
        "pre-contracted" if plan["precontract"] else "bond-2 MPO",
        "occupancy-limited" if plan["waves_per_cu"] == 0 else str(plan["waves_per_cu"]))


def run_step(batch, ks, shots, seed):
    """One pass of the hot path: reset, iterate and (with shots) sample in one graph launch,
    then the marked probability of every instance."""
    batch.init_uniform()
    if shots:
        hits = batch.iterate_sample(ks, shots, seed)
    else:
        batch.iterate(ks)
        hits = None
    p = batch.marked_prob(allow_numeric=True)
    return p, hits


# ------------------------------------------------------------------ CPU oracle baseline
def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _cpu_worker_init():
    from threadpoolctl import threadpool_limits
    global _CPU_LIMIT
    _CPU_LIMIT = threadpool_limits(limits=1)


def _cpu_job(job):
    n, marked, cap, iters = job
    from oracle import mps as omps
    m = omps.GroverMPS(n, marked, cap)
    t0 = time.perf_counter()
    m.iterate(iters)
    return iters, time.perf_counter() - t0


def cpu_baseline(w, frac: float = 1e-3, job_iters: int = 100):
    """The oracle (numpy FP64 MPS, one thread per process) on every usable host core (at most
    16), one instance per worker with dynamic scheduling, on a bounded sample whose mix of
    (n, M) strata is the workload's: stratum s runs round(frac * K_s) iterations (K_s the
    stratum's iterations in the workload), split into jobs of at most job_iters iterations on
    distinct instances of the stratum. value = sample iterations / wall time of the pool."""
    import multiprocessing as mp
    strata = {}
    for inst in w.instances:
        strata.setdefault((inst.n, inst.M), []).append(inst)
    jobs = []
    for (n, M), insts in strata.items():
        left = max(1, int(round(frac * sum(i.k for i in insts))))
        t = 0
        while left > 0:
            it = min(job_iters, left)
            inst = insts[t % len(insts)]
            jobs.append((n, [int(x) for x in inst.marked], inst.chi_cap, it))
            left -= it
            t += 1
    jobs.sort(key=lambda j: -(j[0] * (len(j[1]) + 1) * j[3]))
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count() or 1
    workers = max(1, min(MAX_WORKERS, usable))
    ctx = mp.get_context("spawn")
    saved = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in saved:
        os.environ[k] = "1"
    try:
        with ctx.Pool(workers, initializer=_cpu_worker_init) as pool:
            pool.map(abs, range(workers))  # every worker is up before the clock starts
            t0 = time.perf_counter()
            res = list(pool.imap_unordered(_cpu_job, jobs, chunksize=1))
            wall = time.perf_counter() - t0
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    iters = sum(r[0] for r in res)
    cpu_s = sum(r[1] for r in res)
    sum_k = sum(i.k for i in w.instances)
    rate = iters / wall
    return {"value": rate, "unit": "iterations/s", "cores": workers, "kind": "oracle",
            "nproc": os.cpu_count(), "usable_cpus": usable, "cpu_model": _cpu_model(),
            "sample": "%d iterations (%.2g of each (n, M) stratum's iterations in the workload, %d jobs of <= %d "
                      "iterations on distinct instances) in %.1f s on %d processes, %.1f CPU-s; the whole workload "
                      "at this rate: %.0f s" % (iters, frac, len(jobs), job_iters, wall, workers, cpu_s, sum_k / rate)}


def closed_form_amplitudes(n: int, M: int, k: int):
    """Eq. (5): a marked amplitude sin(phi)/sqrt(M) and an unmarked one cos(phi)/sqrt(N-M),
    phi = (2k+1) asin(sqrt(M/N))."""
    N = float(2 ** n)
    phi = (2 * k + 1) * math.asin(math.sqrt(M / N))
    return math.sin(phi) / math.sqrt(M), math.cos(phi) / math.sqrt(N - M)


def single_leg(w, reps: int = 5):
    """A single-instance case (FP64): one untimed run, then the median of reps runs of
    mps_init_uniform + grover_iterate(k), each timed by the library's HIP events around the
    iterate launch; P against Eq. (6), the amplitudes against Eq. (5) (every basis index up
    to n = 12, else the marked index and 64 others) and, with shots, the marked hit fraction."""
    from paper_2601_03832_amd import gmps
    inst = w.instances[0]
    n, M, k = inst.n, inst.M, inst.k
    b = gmps.Batch([inst], w.precision)
    b.init_uniform()
    b.iterate(k)
    runs = []
    for _ in range(reps):
        b.init_uniform()
        b.iterate(k)
        runs.append(b.last_iterate_ms())
    p = float(b.marked_prob()[0])
    am, au = closed_form_amplitudes(n, M, k)
    xs = np.arange(1 << n, dtype=np.uint64) if n <= 12 else \
        np.unique(np.concatenate([np.asarray(inst.marked, dtype=np.uint64),
                                  np.random.default_rng(3).integers(0, 1 << n, 64, dtype=np.uint64)]))
    a = b.amplitudes(0, xs)
    marked = set(int(x) for x in inst.marked)
    ref = np.array([am if int(x) in marked else au for x in xs])
    med = statistics.median(runs)
    out = {"workload": w.name, "value": k / (med / 1e3), "unit": "iterations/s", "median_ms": med,
           "runs_ms": runs, "k": k, "p": p, "abs_err_p": abs(p - exact_p(n, M, k)), "tolerance": 1e-10,
           "max_abs_err_amplitude": float(np.max(np.abs(a - ref))), "amplitudes_checked": int(len(xs))}
    if w.shots:
        shots = w.shots[-1]
        _, hits = b.sample(shots, w.shot_seed)
        out["shots"] = shots
        out["hit_fraction"] = float(hits[0]) / shots
        out["hit_fraction_expected"] = exact_p(n, M, k)
    b.close()
    return out


def c3_leg():
    """The precision study: n=29, one marked state, k=18198, FP64 and mixed, in chunks of 1000
    iterations; |P_j - sin^2((2j+1) theta)| after every chunk, and the summed HIP-event time of
    the iterate launches."""
    from paper_2601_03832_amd import gmps
    out = {}
    for prec in ("fp64", "mixed"):
        inst = inputs.config_c3(prec).instances[0]
        b = gmps.Batch([inst], prec)
        b.init_uniform()
        done = 0
        total_ms = 0.0
        log = []
        while done < inst.k:
            step = min(1000, inst.k - done)
            b.iterate(step)
            total_ms += b.last_iterate_ms()
            done += step
            p = float(b.marked_prob(allow_numeric=True)[0])
            log.append([done, p - exact_p(inst.n, inst.M, done)])
        b.close()
        errs = [abs(e) for _, e in log]
        out[prec] = {"value": inst.k / (total_ms / 1e3), "unit": "iterations/s", "kernel_ms": total_ms,
                     "final_abs_err_p": errs[-1], "max_abs_err_p": max(errs),
                     "tolerance": 1e-10 if prec == "fp64" else 1e-6, "err_p_every_1000": log}
    out["note"] = "n=29, M=1, k=18198, chi cap 4; P - sin^2((2j+1) theta) after every 1000 iterations"
    return out


def common_leg(reps: int = 3):
    """The Common method against the Iterative one (Section III-A, Fig. 1; Section IV, Fig. 2),
    FP64, one instance each of C1, C2 and C3: the iterative path (the library's default plan,
    and sequential sweeps: the team kernel the circuit runs on), and the k-layer gate-level
    circuit, its construction (host gate list and upload, wall clock) and its simulation (HIP
    events), medians over reps runs (one for C3) after an untimed run of each."""
    from paper_2601_03832_amd import gmps
    out = {}
    for w in (inputs.config_c1(), inputs.config_c2(), inputs.config_c3("fp64")):
        inst = w.instances[0]
        r = 1 if inst.n >= 29 else reps
        res = {"k": inst.k, "n": inst.n}
        for label, pipe in (("iterative_ms", True), ("iterative_sequential_ms", False)):
            b = gmps.Batch([inst], "fp64", kernel="team", pipeline=pipe)
            runs = []
            for rep in range(r + 1):
                b.init_uniform()
                b.iterate(inst.k)
                if rep:
                    runs.append(b.last_iterate_ms())
            res[label] = statistics.median(runs)
            res["abs_err_p_" + label[:-3]] = abs(float(b.marked_prob()[0]) - exact_p(inst.n, inst.M, inst.k))
            b.close()
        b = gmps.Batch([inst], "fp64", kernel="team")
        build, run = [], []
        nbytes = 0
        for rep in range(r + 1):
            t0 = time.perf_counter()
            nbytes = b.build_circuit(inst.k)
            t1 = time.perf_counter()
            b.init_uniform()
            b.run_circuit()
            ms = b.last_iterate_ms()
            if rep:
                build.append((t1 - t0) * 1e3)
                run.append(ms)
        res["common_build_ms"] = statistics.median(build)
        res["common_run_ms"] = statistics.median(run)
        res["gates"] = nbytes // 4
        res["abs_err_p_common"] = abs(float(b.marked_prob()[0]) - exact_p(inst.n, inst.M, inst.k))
        res["common_over_iterative"] = (res["common_build_ms"] + res["common_run_ms"]) / res["iterative_ms"]
        res["common_run_over_iterative_sequential"] = res["common_run_ms"] / res["iterative_sequential_ms"]
        b.close()
        out[w.name] = res
    out["note"] = ("Common: the k stacked Grover layers of Fig. 1(A) as one gate list (H, X, n-controlled Z), "
                   "built on the host and simulated gate by gate (n-controlled Z as its bond-2 MPO with the QR "
                   "and SVD sweeps, single-qubit gates fused per qubit into the next staging)")
    return out


def plain_fp64_leg(w, prefix: int = 100, extra: int = 13):
    """The plain per-instance FP64 GPU path: instances through their own B=1 FP64 handle (one
    wave per launch), one per (n, M) stratum plus `extra` more from the strata with the most
    iterations, each for a prefix of min(k, prefix) iterations timed by the library's HIP
    events; the per-iteration time of each stratum is extrapolated to every instance's own k."""
    from paper_2601_03832_amd import gmps
    strata = {}
    for inst in w.instances:
        strata.setdefault((inst.n, inst.M), []).append(inst)
    picks = [v[0] for v in strata.values()]
    heavy = sorted(strata.values(), key=lambda v: -sum(i.k * (i.M + 1) * i.n for i in v))
    picks += [v[1] for v in heavy[:extra] if len(v) > 1]
    per = {}
    worst = 0.0
    for inst in picks:
        kk = min(inst.k, prefix)
        b = gmps.Batch([inst], "fp64")
        b.init_uniform()
        b.iterate(kk)
        ms = b.last_iterate_ms()
        worst = max(worst, abs(float(b.marked_prob()[0]) - exact_p(inst.n, inst.M, kk)))
        b.close()
        per.setdefault((inst.n, inst.M), []).append(ms / 1e3 / kk)
    est = sum(i.k * float(np.mean(per[(i.n, i.M)])) for i in w.instances)
    sum_k = sum(i.k for i in w.instances)
    return {"value": sum_k / est, "unit": "iterations/s", "extrapolated": True, "instances_timed": len(picks),
            "strata": len(strata), "est_seconds": est, "max_abs_err_p_prefix": worst,
            "sample": "%d instances (every one of the %d (n, M) strata, and a second instance of the %d heaviest), "
                      "each alone through a B=1 FP64 handle for min(k, %d) iterations timed by HIP events; "
                      "per-iteration times extrapolated to every instance's own k" % (len(picks), len(strata), extra, prefix)}


def c5_prefix(k: int, kernel: str, precontract: bool = False, precision: str = "mixed"):
    """256 instances at n=40, M=16, cap 32 (bond 17) for a prefix of k iterations (the full
    k = 205887 is not run): P against Eq. (6), and the marked hit fraction of 1, 8 and 4096
    perfect-sampling shots per instance (mean, min and max over the instances)."""
    import torch
    from paper_2601_03832_amd import gmps
    w = inputs.config_c5(k=k)
    b = gmps.Batch(w.instances, precision, kernel=kernel, precontract=precontract)
    b.init_uniform()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.iterate(k)
    p = b.marked_prob(allow_numeric=True)
    t1 = time.perf_counter()
    kms = b.last_iterate_ms()
    pe = exact_p(40, 16, k)
    err = float(np.max(np.abs(p - pe)))
    frac = {}
    for shots in w.shots:
        _, hits = b.sample(shots, w.shot_seed)
        f = hits / shots
        frac[str(shots)] = {"mean": float(np.mean(f)), "min": float(np.min(f)), "max": float(np.max(f))}
    d = b.diagnostics()
    b.close()
    n_inst = len(w.instances)
    return {"value": n_inst * k / (t1 - t0), "unit": "iterations/s", "instances": n_inst, "k_prefix": k,
            "precision": precision, "precontract": precontract, "seconds": t1 - t0, "kernel_ms": kms,
            "max_abs_err_p": err, "max_rel_err_p": err / pe, "p_exact": pe, "hit_fraction": frac,
            "status_flags": int(np.bitwise_or.reduce(d["status"])),
            "flops_model": model_flops(w.instances, [k] * n_inst, d["bond_dims"]),
            "note": "256 x (n=40, M=16, cap 32) for the first %d of k=205887 iterations, %s%s; not extrapolated"
                    % (k, precision, ", pre-contracted reflections" if precontract else ", bond-2 MPO reflections")}


def precontracted_leg(w, ks, shots, kernel: str):
    """The same workload and step through the pre-contracted reflections (psi plus product
    terms, the whole oracle as one recompression) in FP64, the only precision the library runs
    them in: a recompression variant, reported next to the per-projector MPO path of the
    headline value. One untimed step captures the graph."""
    import torch
    from paper_2601_03832_amd import gmps
    out = {}
    sum_k = int(sum(ks))
    for prec in ("fp64",):  # the library refuses pre-contraction on the mixed path
        b = gmps.Batch(w.instances, prec, kernel="team" if kernel == "auto" else kernel, precontract=True)
        run_step(b, ks, shots, w.shot_seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p, _ = run_step(b, ks, shots, w.shot_seed)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        err = max(abs(p[i] - exact_p(inst.n, inst.M, inst.k)) for i, inst in enumerate(w.instances))
        d = b.diagnostics()
        out[prec] = {
            "value": sum_k / (t1 - t0), "unit": "iterations/s", "ms_per_step": (t1 - t0) * 1000.0,
            "kernel_ms": b.last_iterate_ms(), "max_abs_err_p": float(err),
            "tolerance": 1e-6 if prec == "mixed" else 1e-10,
            "flops_per_launch": float(np.sum(d["flops64"]) + np.sum(d["flops32"]))}
        b.close()
    out["note"] = ("same workload and step with gmps_options.precontract = 1: each reflection applied as "
                   "psi plus product terms (bond chi + T), the M oracle terms in one recompression")
    return out


def statevector_leg(n: int, k: int):
    """The dense-statevector backend (the paper's comparison, Section III-A) on one instance
    of the workload's largest n, FP64 and FP32 vectors, for a prefix of k iterations, next to
    the MPS path (FP64, B=1) on the same instance and prefix. One statevector iteration
    streams the vector once in and once out: 2 * 2^n * (8 or 4) bytes."""
    import torch
    from paper_2601_03832_amd import gmps
    inst = [i for i in inputs.config_c4().instances if i.n == n and i.M == 1][0]
    out = {"n": n, "M": 1, "k_prefix": k,
           "note": "one instance of the n=%d, M=1 stratum; rates over the first %d iterations" % (n, k)}
    for prec, nbytes in (("fp64", 8), ("mixed", 4)):
        s = gmps.StateVector(n, inst.marked, prec)
        s.init_uniform()
        s.iterate(2)  # warm
        s.init_uniform()
        torch.cuda.synchronize()
        s.iterate(k)
        ms = s.last_iterate_ms()
        p = s.marked_prob()
        s.close()
        gbs = 2.0 * (1 << n) * nbytes * k / (ms / 1e3) / 1e9
        out["sv_" + prec] = {"value": k / (ms / 1e3), "unit": "iterations/s", "ms": ms, "hbm_gb_per_s": gbs,
                             "hbm_frac": gbs / (HBM_PEAK / 1e9), "max_abs_err_p": abs(p - exact_p(n, 1, k))}
    b = gmps.Batch([inst], "fp64")
    b.init_uniform()
    b.iterate(k)
    ms = b.last_iterate_ms()
    out["mps_fp64"] = {"value": k / (ms / 1e3), "unit": "iterations/s", "ms": ms,
                       "max_abs_err_p": abs(b.marked_prob()[0] - exact_p(n, 1, k))}
    b.close()
    out["mps_over_sv_fp64"] = out["mps_fp64"]["value"] / out["sv_fp64"]["value"]
    return out


def fp32_accuracy_leg():
    """Marked probability after the full k = round(pi/4 sqrt(N)) iterations for M = 1 and
    n = 12, 14, ..., 28 (one instance of each stratum of the workload), with every step in
    FP32 (GMPS_FP32, lane-group kernel), in mixed precision and in FP64: the precision study
    of Section IV (Fig. 3), where the paper's FP32 MPS result falls to 0.997 at n = 18 and
    0.877 at n = 28."""
    from paper_2601_03832_amd import gmps
    c4 = inputs.config_c4().instances
    insts = [[i for i in c4 if i.n == n and i.M == 1][0] for n in range(12, 29, 2)]
    out = {"n": [i.n for i in insts], "k": [i.k for i in insts],
           "p_exact": [exact_p(i.n, 1, i.k) for i in insts]}
    for prec in ("fp32", "mixed", "fp64"):
        b = gmps.Batch(insts, prec)
        b.init_uniform()
        b.iterate([i.k for i in insts])
        p = b.marked_prob(allow_numeric=True)
        ms = b.last_iterate_ms()
        st = int(np.bitwise_or.reduce(b.diagnostics()["status"]))
        # the marked amplitude is first order in a drift of the rotation angle, which the
        # probability near its maximum is not: compare it with sin((2k+1) theta) (Eq. (5))
        amp_err = []
        for j, i in enumerate(insts):
            a = b.amplitudes(j, np.asarray(i.marked[:1], dtype=np.uint64))[0]
            th = math.asin(math.sqrt(2.0 ** -i.n))
            amp_err.append(float(abs(a - math.sin((2 * i.k + 1) * th))))
        b.close()
        out["p_" + prec] = [float(x) for x in p]
        out["amp_err_" + prec] = amp_err
        out["launch_ms_" + prec] = ms
        out["status_" + prec] = st
    # the paper sets the FP32 statevector beside the FP32 MPS: the FP32 vector (FP64 sums)
    sv_p = []
    for i in insts:
        if i.n < 24:
            continue
        s = gmps.StateVector(i.n, i.marked, "mixed")
        s.init_uniform()
        s.iterate(i.k)
        sv_p.append([i.n, float(s.marked_prob())])
        s.close()
    out["sv_fp32_vector"] = sv_p
    out["note"] = ("fp32: site tensors, contractions, QR, Jacobi SVD and norms in FP32, rounded to nearest; "
                   "mixed: FP64 arithmetic, complex64 bulk sites stored with compensated rounding; "
                   "sv_fp32_vector: [n, P] of the dense statevector with an FP32 vector and FP64 sums")
    return out


def fp32_c4_leg(w, ks, shots):
    """The whole workload on the lane-group kernel (its tile classes hold every C4 bond cap)
    in all-FP32, mixed and FP64: the same kernel code with FP32 or FP64 factorisations, one
    step each after an untimed one."""
    from paper_2601_03832_amd import gmps
    out = {}
    for prec in ("fp32", "mixed", "fp64"):
        b = gmps.Batch(w.instances, prec, kernel="group")
        run_step(b, ks, shots, w.shot_seed)
        t0 = time.perf_counter()
        p, _ = run_step(b, ks, shots, w.shot_seed)
        t1 = time.perf_counter()
        errs = np.array([abs(p[i] - exact_p(x.n, x.M, x.k)) for i, x in enumerate(w.instances)])
        out[prec] = {"value": sum(ks) / (t1 - t0), "unit": "iterations/s", "ms_per_step": (t1 - t0) * 1e3,
                     "kernel_ms": b.last_iterate_ms(), "max_abs_err_p": float(errs.max())}
        b.close()
        print("bench: lane-group %s step %.1f s" % (prec, t1 - t0), file=sys.stderr, flush=True)
    out["note"] = "same workload and step on the lane-group kernel (gmps_options.kernel = 1)"
    return out


def traffic_record():
    try:
        with open(TRAFFIC_FILE) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    return rec if rec.get("kernel_hash") == kernel_hash() else None


def main():
    t_start = time.perf_counter()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--budget", type=float, default=330.0,
                    help="seconds for the whole run: the side legs run, in priority order, while it lasts")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first run one device copy of this many bytes (counter calibration)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-small", action="store_true", help="skip the single-instance n=10/20/29 legs")
    ap.add_argument("--no-fp64-batch", action="store_true")
    ap.add_argument("--shots", type=int, default=None)
    ap.add_argument("--c5-k", type=int, default=5000,
                    help="iterations of the n=40, M=16 prefix leg, pre-contracted, FP64 (0: skip)")
    ap.add_argument("--sv-k", type=int, default=500, help="iterations of the statevector comparison leg (0: skip)")
    ap.add_argument("--no-precontract", action="store_true", help="skip the pre-contracted reflections legs")
    ap.add_argument("--sequential", action="store_true", help="also time the sequential-sweeps variant")
    ap.add_argument("--no-fp32", action="store_true", help="skip the all-FP32 accuracy leg")
    ap.add_argument("--fp32-c4", action="store_true",
                    help="also time the whole workload on the lane-group kernel in FP32, mixed and FP64")
    ap.add_argument("--no-tune", action="store_true", help="run the library's default launch plan")
    ap.add_argument("--tune-probe", type=int, default=64, help="iterations of the longest chain per autotuner probe")
    ap.add_argument("--no-tune-check", dest="tune_check", action="store_false",
                    help="keep the autotuner's pick without a full-size step against the library default plan")
    ap.add_argument("--tune-cache", default=None, help="plan cache file of the autotuner (default: none)")
    ap.add_argument("--kernel", default="auto", choices=sorted(["auto", "group", "team"]),
                    help="iterate kernel: lane-group, team, or the library's choice")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: instances are independent, so a multi-GPU run "
              "would shard the batch, each GPU taking a share of the instances; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    def log(msg):
        print("bench: [%5.1f s] %s" % (time.perf_counter() - t_start, msg), file=sys.stderr, flush=True)

    w = workload(args.workload)
    # the CPU oracle first, in worker processes, before this process touches the GPU
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w)
        log("cpu baseline done (%.0f iterations/s on %d processes)" % (cpu["value"], cpu["cores"]))

    import torch
    from paper_2601_03832_amd import gmps
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible: the benchmark needs the HIP library on an MI355X")
    torch.cuda.set_device(0)
    shots = (w.shots[-1] if w.shots else 0) if args.shots is None else args.shots
    ks = [i.k for i in w.instances]
    sum_k = int(sum(ks))
    log("workload %s, %d instances, sum k = %d, precision %s, shots %d" % (w.name, len(ks), sum_k, w.precision, shots))
    if args.copy_bytes:
        src = torch.empty(args.copy_bytes, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        log("calibration copy of %d bytes done" % args.copy_bytes)
    batch = gmps.Batch(w.instances, w.precision, kernel=args.kernel)
    plan = None
    untimed = 0
    if not args.no_tune:
        # the launch plan: timed probes of every plan that keeps the batch's parity (untimed here)
        plan = batch.autotune(ks, probe_iters=args.tune_probe, cache_path=args.tune_cache)
        log("autotuned plan: %s" % plan)
        default = {"pipeline": True, "precontract": False, "waves_per_cu": 0}
        if args.tune_check and any(plan[key] != v for key, v in default.items()):
            # The probes scale every chain down by k_max / probe_iters, and there plans within a
            # few percent of each other rank by noise. Full-size steps under the probes' pick and
            # under the library's default plan (a second batch) decide between the two: the
            # second step of each, since a first step also captures the graph and starts cold.
            # The steps taken on the batch that is kept count as its warm-up steps.
            alt = gmps.Batch(w.instances, w.precision, kernel=args.kernel)
            t_pick, t_def = [], []
            for _ in range(2):
                run_step(batch, ks, shots, w.shot_seed)
                t_pick.append(batch.last_iterate_ms())
                run_step(alt, ks, shots, w.shot_seed)
                t_def.append(alt.last_iterate_ms())
            check = {"probe_pick_ms": t_pick, "library_default_ms": t_def}
            t_pick, t_def = t_pick[-1], t_def[-1]
            if t_def < t_pick:
                batch.close()
                batch = alt
                plan = dict(plan, full_size_check=check, chosen="library default plan")
            else:
                alt.close()
                plan = dict(plan, full_size_check=check, chosen="probe pick")
            untimed = 2
            log("full-size check: %s" % plan)

    for s in range(max(0, args.warmup - untimed)):
        run_step(batch, ks, shots, w.shot_seed)
        log("warmup step %d done" % s)
    torch.cuda.synchronize()
    kernel_ms = []
    t0 = time.perf_counter()
    p = None
    for s in range(args.steps):
        p, hits = run_step(batch, ks, shots, w.shot_seed)
        kernel_ms.append(batch.last_iterate_ms())
        log("timed step %d done" % s)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1000.0 / args.steps

    errs = np.array([abs(p[i] - exact_p(inst.n, inst.M, inst.k)) for i, inst in enumerate(w.instances)])
    tol = 1e-6 if w.precision == "mixed" else 1e-10
    diag = batch.diagnostics()
    # mps_init_uniform clears the counters, so they hold the last step's launch
    f64 = float(np.sum(diag["flops64"]))
    f32 = float(np.sum(diag["flops32"]))
    kms = float(np.mean(kernel_ms))
    fmodel = model_flops(w.instances, ks, diag["bond_dims"])
    achieved = fmodel / (kms / 1000.0)
    tr = traffic_record()
    line = {
        "metric": "Grover iterations/s on 1 GPU, batched mixed-prec vs plain FP64, err<=1e-6",
        "value": sum_k / (ms_per_step / 1000.0),
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "instances": len(ks), "sum_k": sum_k, "precision": w.precision,
                   "storage": ("complex64 bulk sites, complex128 edge sites; every arithmetic step FP64"
                               if w.precision == "mixed" else "complex128"),
                   "shots_per_instance": shots, "kernel": plan_name(args.kernel, plan), "autotune": plan,
                   "description": w.description},
        "accuracy": {"max_abs_err_p": float(errs.max()), "tolerance": tol, "pass": bool(errs.max() <= tol),
                     "status_flags": int(np.bitwise_or.reduce(diag["status"]))},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": FP64_VECTOR_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK,
                     "traffic": tr["bytes_per_launch"] if tr else None,
                     "kernel": KERNEL_NAME[args.kernel] + " and the other class kernels of the iterate launch",
                     "kernel_ms": kms, "flops_model": fmodel,
                     "model": "LAPACK-style counts per reflection and site: R*A, full QR with explicit Q, "
                              "one-sided Jacobi SVD with 6 sweeps, (U S)*A, over the reported bond profile",
                     "flops_kernel_count": f64 + f32,
                     "frac_kernel_count": (f64 + f32) / (kms / 1000.0) / FP64_VECTOR_PEAK},
    }
    if cpu is not None:
        line["cpu_baseline"] = cpu
    log("main measurement done (%.1f ms/step)" % ms_per_step)
    batch.close()
    step_s = ms_per_step / 1000.0

    def have(cost_s):
        return time.perf_counter() - t_start + cost_s < args.budget

    skipped = []
    c4 = args.workload == "c4"
    if not args.no_small:
        if have(10):
            line["c1"] = single_leg(inputs.config_c1())
            line["c2"] = single_leg(inputs.config_c2())
            log("c1/c2 legs done")
        else:
            skipped.append("c1/c2")
    if w.precision == "mixed" and not args.no_fp64_batch:
        if have(1.3 * step_s + 5):
            b64 = gmps.Batch(w.instances, "fp64", kernel=args.kernel)
            plan64 = None if args.no_tune else b64.autotune(ks, probe_iters=args.tune_probe, cache_path=args.tune_cache)
            run_step(b64, ks, shots, w.shot_seed)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            p64, _ = run_step(b64, ks, shots, w.shot_seed)
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            e64 = max(abs(p64[i] - exact_p(inst.n, inst.M, inst.k)) for i, inst in enumerate(w.instances))
            line["batched_fp64"] = {"value": sum_k / (t3 - t2), "unit": "iterations/s", "ms_per_step": (t3 - t2) * 1000.0,
                                    "kernel_ms": b64.last_iterate_ms(), "max_abs_err_p": e64,
                                    "kernel": plan_name(args.kernel, plan64),
                                    "note": "same workload and step through the FP64 path (autotuned), after an untimed step"}
            b64.close()
            log("batched fp64 leg done")
        else:
            skipped.append("batched_fp64")
    if not args.no_precontract and args.kernel != "group":
        if have(1.2 * step_s + 5):
            line["precontracted"] = precontracted_leg(w, ks, shots, args.kernel)
            line["precontracted"]["fp64"]["speedup_over_value"] = line["precontracted"]["fp64"]["value"] / line["value"]
            log("pre-contracted legs done")
        else:
            skipped.append("precontracted")
    fastest = [("mixed, %s (the value)" % line["config"]["kernel"], line["value"])]
    if "batched_fp64" in line:
        fastest.append(("fp64, %s" % line["batched_fp64"]["kernel"], line["batched_fp64"]["value"]))
    if "precontracted" in line:
        fastest.append(("fp64, pre-contracted reflections", line["precontracted"]["fp64"]["value"]))
    best = max(fastest, key=lambda x: x[1])
    line["fastest_path"] = {"path": best[0], "value": best[1], "unit": "iterations/s",
                            "note": "every arithmetic step is FP64 on both precisions; mixed only stores the bulk "
                                    "sites as complex64, which saves no time on this latency-bound path"}
    if not args.no_small and c4:
        if have(40):
            line["c3"] = c3_leg()
            log("c3 leg done")
        else:
            skipped.append("c3")
    if not args.no_small and c4 and args.kernel != "group":
        if have(60):
            line["common_method"] = common_leg()
            log("common method leg done")
        else:
            skipped.append("common_method")
    if not args.no_plain:
        if have(30):
            line["plain_fp64"] = plain_fp64_leg(w)
            line["plain_fp64"]["speedup_of_batched_mixed"] = line["value"] / line["plain_fp64"]["value"]
            log("plain fp64 leg done")
        else:
            skipped.append("plain_fp64")
    if args.sv_k > 0 and c4:
        if have(15):
            line["statevector"] = statevector_leg(28, args.sv_k)
            log("statevector leg done")
        else:
            skipped.append("statevector")
    if not args.no_fp32 and c4:
        if have(40):
            line["fp32_accuracy"] = fp32_accuracy_leg()
            log("fp32 accuracy leg done")
        else:
            skipped.append("fp32_accuracy")
    if args.c5_k > 0 and c4 and args.kernel != "group":
        # pre-contracted reflections, FP64: the mixed path does not hold its accuracy at n = 40
        for prec, cost in (("fp64", 8.0),):
            key = "c5_prefix_%s_precontracted" % prec
            if have(cost * args.c5_k / 1000.0 + 10):
                line[key] = c5_prefix(args.c5_k, args.kernel, precontract=True, precision=prec)
                log("c5 prefix %s pre-contracted leg done" % prec)
            else:
                skipped.append(key)
    if args.sequential and args.kernel != "group":
        if have(2.5 * step_s):
            bs = gmps.Batch(w.instances, w.precision, kernel=args.kernel, pipeline=False)
            torch.cuda.synchronize()
            t4 = time.perf_counter()
            ps, _ = run_step(bs, ks, shots, w.shot_seed)
            torch.cuda.synchronize()
            t5 = time.perf_counter()
            es = max(abs(ps[i] - exact_p(inst.n, inst.M, inst.k)) for i, inst in enumerate(w.instances))
            line["sequential_sweeps"] = {"value": sum_k / (t5 - t4), "unit": "iterations/s", "ms_per_step": (t5 - t4) * 1000.0,
                                         "kernel_ms": bs.last_iterate_ms(), "max_abs_err_p": es,
                                         "note": "same workload and step with gmps_options.pipeline = -1 (one step, "
                                                 "no untimed warmup)"}
            bs.close()
            log("sequential sweeps leg done")
        else:
            skipped.append("sequential_sweeps")
    if args.fp32_c4 and c4:
        line["fp32_c4_lane_group"] = fp32_c4_leg(w, ks, shots)
        log("lane-group fp32/mixed/fp64 leg done")
    if skipped:
        line["legs_skipped_for_time"] = skipped
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
