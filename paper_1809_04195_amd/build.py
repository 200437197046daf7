"""Build the gfx950 shared library ``libt2s.so`` in-tree with hipcc."""

from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libt2s.so")
ARCH = os.environ.get("T2S_OFFLOAD_ARCH", "gfx950")

HIP_FLAGS = [
    f"--offload-arch={ARCH}",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Wall",
    "-Wno-unused-function",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    objs, procs = [], []
    # the three translation units compile concurrently
    for src, lang in (("kernels.hip", "hip"), ("unet.hip", "hip"), ("api.cpp", "c++")):
        obj = os.path.join(objdir, src + ".o")
        cmd = [hipcc, *HIP_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]
        if lang == "c++":
            cmd = [hipcc, f"--offload-arch={ARCH}", "-O2", "-std=c++17", "-fPIC", "-Wall", "-c",
                   os.path.join(CSRC, src), "-o", obj]
        print("+", " ".join(cmd), flush=True)
        procs.append((cmd, subprocess.Popen(cmd)))
        objs.append(obj)
    for cmd, pr in procs:
        if pr.wait() != 0:
            raise subprocess.CalledProcessError(pr.returncode, cmd)
    tmp = LIB + ".tmp"
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


def build_sanitized(verbose: bool = True) -> str:
    """A copy of the library whose host code in api.cpp (plan tables, validation, the
    ADMM / stream schedulers) is built with AddressSanitizer and UBSan, linked with the
    objects of the last build(): ``_build/libt2s_asan.so``.  Load it with the clang ASan
    runtime preloaded (the CPU tests do).  Device code is unaffected."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    objdir = os.path.join(HERE, "_build")
    objs = [os.path.join(objdir, "kernels.hip.o"), os.path.join(objdir, "unet.hip.o")]
    for o in objs:
        if not os.path.exists(o):
            raise FileNotFoundError(f"{o} is missing: run build() first")
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
    api = os.path.join(objdir, "api.asan.o")
    _run([hipcc, f"--offload-arch={ARCH}", "-O1", "-g", "-std=c++17", "-fPIC", "-Wall", "-fno-omit-frame-pointer",
          *san, "-c", os.path.join(CSRC, "api.cpp"), "-o", api])
    out = os.path.join(objdir, "libt2s_asan.so")
    _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-shared-libasan", *san, "-o", out, *objs, api])
    return out


if __name__ == "__main__":
    build()
    sys.exit(0)
