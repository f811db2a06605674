"""Build the gfx950 HIP library ``_build/libbmq.so`` in-tree with hipcc.

Flags that matter for the result:
* ``-ffp-contract=off``: the codec's float32 steps must round exactly as
  written (its own log2/exp2 use explicit fused multiply-adds), so the
  compiler may not contract other multiply-adds.
* ``-Xclang -target-feature -Xclang -packed-fp32-ops``: no packed FP32 math.
* ``-fno-gpu-flush-denormals-to-zero``: IEEE float32 denormals on the device.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
SO = os.path.join(BUILD, "libbmq.so")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc" if os.path.exists("/opt/rocm/bin/hipcc") else "hipcc")
ARCH = "gfx950"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-ffp-contract=off", "-I", os.path.join(ROOT, "include")]
DEVICE = [f"--offload-arch={ARCH}", "-fno-gpu-flush-denormals-to-zero",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(" ".join(cmd) + "\n" + r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed ({r.returncode})")
    return r


# host-code sanitizers (AddressSanitizer + UndefinedBehaviorSanitizer) for the
# runtime; device code is never built with them
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
SO_SANITIZED = os.path.join(BUILD, "libbmq_sanitized.so")


def build(verbose: bool = False, sanitize: bool = False) -> str:
    """Build _build/libbmq.so; with sanitize, _build/libbmq_sanitized.so whose
    host runtime is instrumented (load it with BMQ_SO=<path> and the clang
    ASan runtime preloaded, e.g. for the CPU test suite)."""
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    k_obj = os.path.join(BUILD, "bmq_kernels.o")
    _run([HIPCC] + COMMON + DEVICE + ["-c", os.path.join(CSRC, "bmq_kernels.hip"), "-o", k_obj])
    objs.append(k_obj)
    m_obj = os.path.join(BUILD, "bmq_mlp.o")
    _run([HIPCC] + COMMON + DEVICE + ["-c", os.path.join(CSRC, "bmq_mlp.hip"), "-o", m_obj])
    objs.append(m_obj)
    r_obj = os.path.join(BUILD, "bmq_runtime_sanitized.o" if sanitize else "bmq_runtime.o")
    extra = SANITIZE + ["-g", "-fno-omit-frame-pointer"] if sanitize else []
    _run([HIPCC] + COMMON + extra + ["-Wall", "-c", os.path.join(CSRC, "bmq_runtime.cpp"), "-o", r_obj])
    objs.append(r_obj)
    out = SO_SANITIZED if sanitize else SO
    tmp = out + ".tmp"
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC"] + (SANITIZE if sanitize else []) + ["-o", tmp] + objs)
    os.replace(tmp, out)
    if verbose:
        print("built", out)
    return out


if __name__ == "__main__":
    build(verbose=True, sanitize="--sanitize" in sys.argv)
