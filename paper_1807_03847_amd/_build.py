"""Build step: compiles the HIP sources under ``csrc/`` into ``libkatz.so`` for
gfx950 with hipcc.  Run ``python -m paper_1807_03847_amd._build``."""
from __future__ import annotations

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libkatz.so")
SOURCES = ["katz_kernels.hip", "katz_select_wg.hip", "katz_criteria.hip", "katz_linear.hip", "katz_dynamic.hip", "katz_transpose.hip", "katz_batch.hip", "katz_api.hip", "katz_server.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "-O3", "-std=c++17", "--offload-arch=gfx950", "-fPIC", "-shared",
    # No fused multiply-add contraction: every bound is evaluated with the
    # operations as written, the same as the plain FP64 method.
    "-ffp-contract=off",
    "-fvisibility=hidden",
    # Packed FP32 instructions are disabled for all device code.
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
]


def build() -> str:
    srcs = [os.path.join(HERE, "csrc", s) for s in SOURCES]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, *FLAGS, "-I", os.path.join(ROOT, "include"), *srcs, "-o", tmp]
    proc = subprocess.run(cmd, capture_output=True, text=True)
    if proc.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + proc.stdout + proc.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build())
