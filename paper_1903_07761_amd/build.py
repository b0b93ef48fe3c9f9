"""Build the HIP library libcz.so in-tree (hipcc, gfx950)."""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libcz.so")
SOURCES = ["cz_kernels.hip", "cz_api.hip", "cz_server.hip", "cz_precond.hip", "cz_roi.hip", "cz_huff.hip"]
HEADERS = ["cz_kernels.h", "cz_lines.h", "cz_lookback.h", "cz_host.h", os.path.join("..", "..", "include", "cz.h")]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
# Arithmetic exactly as written: no contraction into FMA, IEEE denormals.
# Packed FP32 instructions are disabled (the compiler otherwise forms
# v_pk_* ops from scalar or float2 code).
FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-fno-gpu-flush-denormals-to-zero", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def build(verbose: bool = False) -> str:
    objs = []
    for src in SOURCES:
        obj = os.path.join(CSRC, src.replace(".hip", ".o"))
        cmd = [HIPCC, *FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        noise = [ln for ln in r.stderr.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if r.returncode != 0:
            sys.stderr.write("\n".join(noise) + "\n")
            raise RuntimeError(f"hipcc failed on {src}")
        if noise and verbose:
            print("\n".join(noise))
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stderr)
        raise RuntimeError("link of libcz.so failed")
    os.replace(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
