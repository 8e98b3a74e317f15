"""Builds the test probes of this folder (HIP, gfx950) next to their sources, with the library's
compile flags and device headers. __graft_entry__.build() runs it after building the library."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)
PROBES = {"jacobi_probe.hip": "libjacobi_probe.so"}


def build(verbose: bool = False) -> list[str]:
    from paper_2601_03832_amd import build as pkg
    out = []
    for src, lib in PROBES.items():
        target = os.path.join(HERE, lib)
        cmd = [pkg.hipcc(), *pkg.flags(["-I" + pkg.CSRC]), "-shared", "-o", target + ".tmp", os.path.join(HERE, src)]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        os.replace(target + ".tmp", target)
        out.append(target)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
