"""Build libngdbf.so (the HIP kernels and the C ABI of include/ngdbf.h) for gfx950.

Flags that the decoder's bit-exact contract depends on:
  -ffp-contract=off          no fusion of a*b+c beyond the explicit fmaf calls
  -fno-gpu-flush-denormals-to-zero, no fast-math: IEEE binary32 semantics,
                             correctly rounded division and square root
  -target-feature -packed-fp32-ops: keep the compiler from forming packed
                             fp32 instructions
"""
from __future__ import annotations

import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libngdbf.so")
# (source, extra flags, object name): the extended decoder families are one
# source compiled once per family, so that their kernel sets build in parallel
UNITS = [("decode.hip", [], "decode"),
         *[("decode_ext.hip", [f"-DNGDBF_EXT_FAMILY={k}"], f"decode_ext{k}") for k in range(4)],
         ("channel.hip", [], "channel"), ("probe.hip", [], "probe"), ("server.cpp", [], "server")]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = os.environ.get("NGDBF_ARCH", "gfx950")

FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
    "-ffp-contract=off", "-fno-fast-math", "-fno-gpu-flush-denormals-to-zero",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-result",
    f"-I{os.path.join(ROOT, 'include')}",
]


def build(verbose: bool = False) -> str:
    """Compile every source to an object (in parallel), then link the library."""
    with tempfile.TemporaryDirectory(prefix="ngdbf_build_") as tmpdir:
        procs, objs = [], []
        for src, extra, name in UNITS:
            obj = os.path.join(tmpdir, name + ".o")
            cmd = [HIPCC, *FLAGS, *extra, "-c", os.path.join(HERE, "csrc", src), "-o", obj]
            if verbose:
                print(" ".join(cmd), flush=True)
            procs.append((subprocess.Popen(cmd), cmd))
            objs.append(obj)
        failed = [cmd for p, cmd in procs if p.wait() != 0]
        if failed:
            raise subprocess.CalledProcessError(1, failed[0])
        tmp = LIB + ".tmp"
        cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
