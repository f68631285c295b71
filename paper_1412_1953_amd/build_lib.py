"""Build ``libmgcccs.so`` for gfx950 in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = [os.path.join(HERE, "csrc", f) for f in ("kernels.hip", "noalloc.hip", "api.cpp", "setup.cpp")]
OUT = os.path.join(HERE, "libmgcccs.so")
FLAGS = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
         # no implicit contraction: a multiply feeds an add through an explicit
         # fma only, so that the same expression gives the same bits in every
         # kernel that evaluates it (the launch schedules rely on that)
         "-ffp-contract=off",
         # packed FP32 instructions are disabled on purpose: the compiler must
         # not emit v_pk_* FP32 arithmetic for any kernel in this library
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def build(verbose: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    tmp = OUT + ".tmp"
    cmd = [hipcc, *FLAGS, *SRC, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(res.stderr)
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
