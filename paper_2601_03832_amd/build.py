"""Builds libgmps.so (HIP, gfx950) in-tree with hipcc.

    python -m paper_2601_03832_amd.build
"""
from __future__ import annotations

import hashlib
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libgmps.so")
SOURCES = ["gmps_group.hip", "gmps_team.hip", "gmps_team_cm2.hip", "gmps_team_cm3.hip", "gmps_team_cm5.hip",
           "gmps_team_cm8.hip", "gmps_team_cm17.hip", "gmps_team_cm32.hip", "gmps_pipe_cm2.hip", "gmps_pipe_cm3.hip",
           "gmps_pipe_cm5.hip", "gmps_pipe_cm8.hip",
           "gmps_readout.hip", "gmps_api.hip", "gsv.hip"]
ARCH = os.environ.get("GMPS_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build libgmps)")


def source_hash() -> str:
    """Hash of the device sources and the public headers; it keys the autotuner's plan cache."""
    h = hashlib.sha256()
    for d in (CSRC, os.path.join(ROOT, "include")):
        for name in sorted(os.listdir(d)):
            if name.endswith((".hip", ".h")):
                with open(os.path.join(d, name), "rb") as f:
                    h.update(name.encode() + f.read())
    return h.hexdigest()[:16]


def flags(extra=()):
    return ["-O3", "-std=c++17", "-fPIC", "--offload-arch=" + ARCH, '-DGMPS_SOURCE_HASH="%s"' % source_hash(),
            # packed FP32 instructions are kept out of every kernel
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include"), *extra]


def _stale(src: str, obj: str) -> bool:
    if not os.path.exists(obj):
        return True
    deps = [src] + [os.path.join(CSRC, h) for h in os.listdir(CSRC) if h.endswith(".h")] + \
           [os.path.join(ROOT, "include", h) for h in os.listdir(os.path.join(ROOT, "include"))]
    return max(os.path.getmtime(d) for d in deps) > os.path.getmtime(obj)


def build(verbose: bool = False, save_temps: str | None = None, incremental: bool = False) -> str:
    cc = hipcc()
    tmp = os.path.join(HERE, "_build")
    os.makedirs(tmp, exist_ok=True)
    cmds = []
    objs = []
    for src in SOURCES:
        obj = os.path.join(tmp, src.replace(".hip", ".o"))
        extra = []
        if save_temps:
            extra = ["-save-temps=obj", "-Rpass-analysis=kernel-resource-usage"]
        objs.append(obj)
        if incremental and not _stale(os.path.join(CSRC, src), obj):
            continue
        cmds.append([cc, *flags(extra), "-c", os.path.join(CSRC, src), "-o", obj])
    # the translation units are independent: compile them side by side
    procs = []
    for cmd in cmds:
        if verbose:
            print(" ".join(cmd), flush=True)
        procs.append(subprocess.Popen(cmd))
    bad = [c for c, p in zip(cmds, procs) if p.wait() != 0]
    if bad:
        raise subprocess.CalledProcessError(1, bad[0])
    out_tmp = LIB + ".tmp"
    cmd = [cc, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", out_tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out_tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="--incremental" in sys.argv))
