"""Benchmark: Grover iterations/s on one MI355X, batched mixed precision vs plain FP64.

One step is one pass of the whole hot path over the batched workload: every instance is
reset to |s> (mps_init_uniform), iterated to its own k (grover_iterate, one persistent
launch), read out (marked_prob) and sampled (sample_shots). value = sum_i k_i / step time.
The accuracy gate requires |P_i - sin^2((2k_i+1) theta_i)| <= 1e-6 for every instance.

    python bench.py [--gpus 1] [--steps 2] [--warmup 1] [--workload c4|c2|c3] [--kernel auto|team|group]
                    [--c5-k 48] [--sv-k 500] [--no-plain] [--no-cpu] [--no-fp64-batch]
                    [--no-sequential] [--no-precontract] [--no-fp32] [--fp32-c4]

Besides the headline line, the default run adds legs on the same hardware: the workload
through the FP64 path, with sequential sweeps and with pre-contracted reflections; a prefix of
the n=40, M=16 workload; the dense statevector backend; the all-FP32 precision study (M=1,
n=12..28); B=1 FP64 handles; and the CPU oracle. --fp32-c4 also times the whole workload on
the lane-group kernel in FP32, mixed and FP64.

Prints one JSON line. roofline: the iterate kernel's algorithmic flops per launch (FP32
flops weighted by the FP64/FP32 peak ratio) over its HIP-event duration, against the FP64
vector peak. cpu_baseline: the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
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
# the iterate kernel each --kernel choice runs (the library's choice is the team kernel)
# the launch's longest class kernel on the 4096-instance workload (bond cap 5: the pipelined
# sweeps by default); the roofline's flops, bytes and time cover every class kernel of the launch
KERNEL_NAME = {"auto": "grover_pipe_kernel", "team": "grover_pipe_kernel", "group": "grover_group_kernel"}
CSRC = os.path.join(ROOT, "paper_2601_03832_amd", "csrc")


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


def run_step(batch, ks, shots, seed):
    batch.init_uniform()
    batch.iterate(ks)
    p = batch.marked_prob(allow_numeric=True)
    _, hits = batch.sample(shots, seed) if shots else (None, None)
    return p, hits


def plain_fp64_rate(w, budget_s: float):
    """The same instances through one B=1 FP64 handle each (one wave per launch), on a
    stratified subset: one instance per (n, M) stratum, in increasing k, until the time
    budget is spent."""
    import torch
    from paper_2601_03832_amd import gmps
    seen = {}
    for inst in w.instances:
        seen.setdefault((inst.n, inst.M), inst)
    picks = sorted(seen.values(), key=lambda i: (i.k * (i.M + 1) * (i.n - 1), i.n, i.M))
    tot_k = 0
    tot_s = 0.0
    worst = 0.0
    used = []
    for inst in picks:
        if tot_s > budget_s:
            break
        b = gmps.Batch([inst], "fp64")
        b.init_uniform()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        b.iterate(inst.k)
        p = b.marked_prob()[0]
        t1 = time.perf_counter()
        worst = max(worst, abs(p - exact_p(inst.n, inst.M, inst.k)))
        tot_k += inst.k
        tot_s += t1 - t0
        used.append((inst.n, inst.M))
        b.close()
    return {"value": tot_k / tot_s, "unit": "iterations/s", "instances": len(used),
            "sum_k": tot_k, "seconds": tot_s, "max_abs_err": worst,
            "sample": "one instance per (n, M) stratum of the same workload, cheapest strata first "
                      "(%d of %d strata within a %.0f s budget), each alone through its own B=1 FP64 "
                      "handle" % (len(used), len(picks), budget_s)}


def cpu_baseline(w, iters_per_stratum: int = 100):
    """The oracle (numpy FP64 MPS, one thread) on a bounded sample: a few iterations of one
    instance per (n, M) stratum; the per-iteration time of each stratum is extrapolated to
    every instance's own k."""
    try:
        from threadpoolctl import threadpool_limits
    except Exception:  # pragma: no cover
        threadpool_limits = None
    from oracle import mps as omps
    strata = {}
    for inst in w.instances:
        strata.setdefault((inst.n, inst.M), inst)
    per_iter = {}
    ctx = threadpool_limits(limits=1) if threadpool_limits else None
    t_all = time.perf_counter()
    try:
        if ctx:
            ctx.__enter__()
        for key, inst in strata.items():
            m = omps.GroverMPS(inst.n, inst.marked, inst.chi_cap)
            m.iterate(1)  # warm
            t0 = time.perf_counter()
            m.iterate(iters_per_stratum)
            per_iter[key] = (time.perf_counter() - t0) / iters_per_stratum
    finally:
        if ctx:
            ctx.__exit__(None, None, None)
    wall = time.perf_counter() - t_all
    est = sum(inst.k * per_iter[(inst.n, inst.M)] for inst in w.instances)
    tot_k = sum(inst.k for inst in w.instances)
    return {"value": tot_k / est, "unit": "iterations/s", "cores": 1, "kind": "oracle",
            "sample": "%d iterations of one instance per (n,M) stratum (%d strata, %.1f s of CPU), "
                      "extrapolated to every instance's k (est. %.0f s for the whole workload)"
                      % (iters_per_stratum, len(strata), wall, est)}


def c5_prefix(k: int, kernel: str, precontract: bool = False):
    """256 instances at n=40, M=16, cap 32 (bond 17), mixed, for a prefix of k iterations:
    the full k=205887 takes hours, so the rate and the accuracy are reported on the prefix."""
    import torch
    from paper_2601_03832_amd import gmps
    w = inputs.config_c5(k=k)
    b = gmps.Batch(w.instances, w.precision, kernel=kernel, precontract=precontract)
    b.init_uniform()
    b.iterate(k)  # warm (graph capture)
    torch.cuda.synchronize()
    b.init_uniform()
    t0 = time.perf_counter()
    b.iterate(k)
    p = b.marked_prob(allow_numeric=True)
    t1 = time.perf_counter()
    err = float(np.max(np.abs(p - exact_p(40, 16, k))))
    frac = {}
    for shots in w.shots:
        _, hits = b.sample(shots, w.shot_seed)
        frac[str(shots)] = float(np.mean(hits / shots))
    kms = b.last_iterate_ms()
    d = b.diagnostics()
    b.close()
    n_inst = len(w.instances)
    return {"value": n_inst * k / (t1 - t0), "unit": "iterations/s", "instances": n_inst, "k_prefix": k,
            "seconds": t1 - t0, "kernel_ms": kms, "max_abs_err_p": err, "p_exact": exact_p(40, 16, k),
            "mean_hit_fraction": frac, "flops_per_launch": float(np.sum(d["flops64"]) + np.sum(d["flops32"])),
            "note": "256 x (n=40, M=16, cap 32) for the first %d of k=205887 iterations, mixed%s; not extrapolated"
                    % (k, ", pre-contracted reflections" if precontract else "")}


def precontracted_leg(w, ks, shots, kernel: str):
    """The same workload and step through the pre-contracted reflections (psi plus product
    terms, the whole oracle as one recompression): a recompression variant, reported next to
    the per-projector MPO path of the headline value. One untimed step captures the graph."""
    import torch
    from paper_2601_03832_amd import gmps
    out = {}
    sum_k = int(sum(ks))
    for prec in ("mixed", "fp64"):
        b = gmps.Batch(w.instances, prec, kernel="team" if kernel == "auto" else kernel, precontract=True)
        run_step(b, ks, shots, w.shot_seed)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p, _ = run_step(b, ks, shots, w.shot_seed)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        err = max(abs(p[i] - exact_p(inst.n, inst.M, inst.k)) for i, inst in enumerate(w.instances))
        d = b.diagnostics()
        out["mixed" if prec == "mixed" else "fp64"] = {
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
                   "mixed: complex64 sites, FP64 factorisations, stochastic rounding; sv_fp32_vector: [n, P] "
                   "of the dense statevector with an FP32 vector and FP64 sums")
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
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4")
    ap.add_argument("--plain-budget", type=float, default=20.0)
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="first run one device copy of this many bytes (counter calibration)")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64-batch", action="store_true")
    ap.add_argument("--shots", type=int, default=None)
    ap.add_argument("--c5-k", type=int, default=48, help="iterations of the n=40, M=16 prefix leg (0: skip)")
    ap.add_argument("--sv-k", type=int, default=500, help="iterations of the statevector comparison leg (0: skip)")
    ap.add_argument("--no-precontract", action="store_true", help="skip the pre-contracted reflections legs")
    ap.add_argument("--no-sequential", action="store_true", help="skip the sequential-sweeps leg")
    ap.add_argument("--no-fp32", action="store_true", help="skip the all-FP32 accuracy leg")
    ap.add_argument("--fp32-c4", action="store_true",
                    help="also time the whole workload on the lane-group kernel in FP32, mixed and FP64")
    ap.add_argument("--kernel", default="auto", choices=sorted(["auto", "group", "team"]),
                    help="iterate kernel: lane-group, team, or the library's choice")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: instances are independent, so a multi-GPU run "
              "would shard the batch, each GPU taking a share of the instances; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2601_03832_amd import gmps
    if not torch.cuda.is_available():
        raise SystemExit("no GPU visible: the benchmark needs the HIP library on an MI355X")
    torch.cuda.set_device(0)
    w = workload(args.workload)
    shots = (w.shots[-1] if w.shots else 0) if args.shots is None else args.shots
    ks = [i.k for i in w.instances]
    sum_k = int(sum(ks))
    print("bench: workload %s, %d instances, sum k = %d, precision %s, shots %d"
          % (w.name, len(ks), sum_k, w.precision, shots), file=sys.stderr, flush=True)
    if args.copy_bytes:
        src = torch.empty(args.copy_bytes, dtype=torch.uint8, device="cuda").fill_(1)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
        print("bench: calibration copy of %d bytes done" % args.copy_bytes, file=sys.stderr, flush=True)
    batch = gmps.Batch(w.instances, w.precision, kernel=args.kernel)

    for s in range(args.warmup):
        run_step(batch, ks, shots, w.shot_seed)
        print("bench: warmup step %d done" % s, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    kernel_ms = []
    t0 = time.perf_counter()
    p = None
    for s in range(args.steps):
        p, hits = run_step(batch, ks, shots, w.shot_seed)
        kernel_ms.append(batch.last_iterate_ms())
        print("bench: timed step %d done" % s, file=sys.stderr, flush=True)
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
    # FP64-equivalent work: FP32 flops count at the FP64/FP32 peak ratio
    achieved = (f64 + f32 * FP64_VECTOR_PEAK / FP32_VECTOR_PEAK) / (kms / 1000.0)
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
        "dtype": "c64/f64" if w.precision == "mixed" else "f64",
        "data": "synthetic",
        "config": {"workload": w.name, "instances": len(ks), "sum_k": sum_k, "precision": w.precision,
                   "shots_per_instance": shots, "kernel": args.kernel, "description": w.description},
        "accuracy": {"max_abs_err_p": float(errs.max()), "tolerance": tol, "pass": bool(errs.max() <= tol),
                     "status_flags": int(np.bitwise_or.reduce(diag["status"]))},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": FP64_VECTOR_PEAK / 1e12,
                     "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK,
                     "traffic": tr["bytes_per_launch"] if tr else None,
                     "kernel": KERNEL_NAME[args.kernel], "kernel_ms": kms,
                     "flops64_per_launch": f64, "flops32_per_launch": f32},
    }
    print("bench: main measurement done (%.1f ms/step)" % ms_per_step, file=sys.stderr, flush=True)
    batch.close()
    if w.precision == "mixed" and not args.no_fp64_batch:
        b64 = gmps.Batch(w.instances, "fp64", kernel=args.kernel)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        p64, _ = run_step(b64, ks, shots, w.shot_seed)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        e64 = max(abs(p64[i] - exact_p(inst.n, inst.M, inst.k)) for i, inst in enumerate(w.instances))
        line["batched_fp64"] = {"value": sum_k / (t3 - t2), "unit": "iterations/s", "ms_per_step": (t3 - t2) * 1000.0,
                                "kernel_ms": b64.last_iterate_ms(), "max_abs_err_p": e64,
                                "note": "same workload and step through the FP64 path (one untimed-warmup-free step)"}
        b64.close()
        print("bench: batched fp64 leg done", file=sys.stderr, flush=True)
    if not args.no_sequential and args.kernel != "group":
        bs = gmps.Batch(w.instances, w.precision, kernel=args.kernel, pipeline=False)
        torch.cuda.synchronize()
        t4 = time.perf_counter()
        ps, _ = run_step(bs, ks, shots, w.shot_seed)
        torch.cuda.synchronize()
        t5 = time.perf_counter()
        es = max(abs(ps[i] - exact_p(inst.n, inst.M, inst.k)) for i, inst in enumerate(w.instances))
        line["sequential_sweeps"] = {"value": sum_k / (t5 - t4), "unit": "iterations/s", "ms_per_step": (t5 - t4) * 1000.0,
                                     "kernel_ms": bs.last_iterate_ms(), "max_abs_err_p": es,
                                     "note": "same workload and step with gmps_options.pipeline = -1: each reflection's "
                                             "canonicalisation and truncation sweeps in turn on one wave per instance "
                                             "(one step, no untimed warmup)"}
        bs.close()
        print("bench: sequential sweeps leg done", file=sys.stderr, flush=True)
    if not args.no_precontract and args.kernel != "group":
        line["precontracted"] = precontracted_leg(w, ks, shots, args.kernel)
        line["precontracted"]["mixed"]["speedup_over_value"] = line["precontracted"]["mixed"]["value"] / line["value"]
        print("bench: pre-contracted legs done", file=sys.stderr, flush=True)
    if args.c5_k > 0 and args.workload == "c4":
        line["c5_prefix"] = c5_prefix(args.c5_k, args.kernel)
        print("bench: c5 prefix leg done", file=sys.stderr, flush=True)
        if not args.no_precontract and args.kernel != "group":
            line["c5_prefix_precontracted"] = c5_prefix(args.c5_k, args.kernel, precontract=True)
            print("bench: c5 prefix pre-contracted leg done", file=sys.stderr, flush=True)
    if args.sv_k > 0 and args.workload == "c4":
        line["statevector"] = statevector_leg(28, args.sv_k)
        print("bench: statevector leg done", file=sys.stderr, flush=True)
    if not args.no_fp32 and args.workload == "c4":
        line["fp32_accuracy"] = fp32_accuracy_leg()
        print("bench: fp32 accuracy leg done", file=sys.stderr, flush=True)
    if args.fp32_c4 and args.workload == "c4":
        line["fp32_c4_lane_group"] = fp32_c4_leg(w, ks, shots)
        print("bench: lane-group fp32/mixed/fp64 leg done", file=sys.stderr, flush=True)
    if not args.no_plain:
        line["plain_fp64"] = plain_fp64_rate(w, args.plain_budget)
        line["plain_fp64"]["speedup_of_batched_mixed"] = line["value"] / line["plain_fp64"]["value"]
        print("bench: plain fp64 leg done", file=sys.stderr, flush=True)
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(w)
        print("bench: cpu baseline leg done", file=sys.stderr, flush=True)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
