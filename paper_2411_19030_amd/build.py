"""Build libpt.so (HIP, gfx950) in-tree with hipcc.

Usage: python -m paper_2411_19030_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libpt.so")
ARCH = os.environ.get("PT_OFFLOAD_ARCH", "gfx950")

SOURCES = [os.path.join(CSRC, "pt_host.hip"), os.path.join(CSRC, "pt_filter.hip"),
           os.path.join(CSRC, "pt_cmesh.hip")]
DEPS = [os.path.join(CSRC, f) for f in os.listdir(CSRC)] + [os.path.join(ROOT, "include", "pt.h")]


def hipcc_command(out: str = LIB, extra=()) -> list[str]:
    return [
        "hipcc", f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        # packed FP32 instructions stay off in all HIP code of this library
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I", os.path.join(ROOT, "include"),
        *extra, *SOURCES, "-o", out,
    ]


def build(verbose: bool = True) -> str:
    tmp = LIB + ".tmp"
    cmd = hipcc_command(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed")
    warn = "\n".join(l for l in res.stderr.splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    if warn and verbose:
        print(warn)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
