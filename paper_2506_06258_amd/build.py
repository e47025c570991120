"""Build ``libpdhcg.so`` (HIP, gfx950) in-tree with hipcc.

Usage: ``python -m paper_2506_06258_amd.build`` or ``build()`` from Python.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpdhcg.so")
SOURCES = ["pdhcg_kernels.hip", "pdhcg_api.hip", "pdhcg_batch.hip", "pdhcg_adjoint.hip", "pdhcg_long.hip",
           "pdhcg_pdhg.hip", "pdhcg_ksec.hip", "pdhcg_team.hip"]
ARCH = os.environ.get("PDHCG_OFFLOAD_ARCH", "gfx950")


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc"):
        if cand and os.path.exists(cand):
            return cand
    return "hipcc"


def flags() -> list[str]:
    return [
        f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        # no packed fp32 instructions in device code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-Wall", "-Wno-unused-function",
    ]


def build(verbose: bool = False) -> str:
    """Compile every HIP source into libpdhcg.so (always recompiles)."""
    objs = []
    jobs = []
    for s in SOURCES:
        obj = os.path.join(CSRC, s.replace(".hip", ".o"))
        cmd = [hipcc(), *flags(), "-c", "-o", obj, os.path.join(CSRC, s)]
        cmd.remove("-shared")
        jobs.append((cmd, s))
        objs.append(obj)
    procs = [(subprocess.Popen(c, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), s)
             for c, s in jobs]
    for p, s in procs:
        out, _ = p.communicate()
        if verbose or p.returncode:
            sys.stderr.write(out.decode(errors="replace"))
        if p.returncode:
            raise RuntimeError(f"hipcc failed on {s}")
    tmp = LIB + ".tmp"
    link = [hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs]
    subprocess.check_call(link)
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
