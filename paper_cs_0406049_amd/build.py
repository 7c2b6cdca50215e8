"""Build libmi355_sincos.so in-tree with hipcc for gfx950.

    python -m paper_cs_0406049_amd.build          # rebuild
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libmi355_sincos.so")

SOURCES = ["plain.hip", "forms.hip", "ablation.hip", "probes.hip", "capi.cpp", "serve.cpp", "tuning.cpp"]
HEADERS = ["internal.hpp", "sincos_core.hpp", "stream.hpp", "serve.hpp", "sqrt_rn.hpp", "rcp_rn.hpp"]

# -ffp-contract=off: the SPLIT arithmetic must not be fused (FUSED uses
# explicit fma builtins, CONTRACT re-enables contraction with a pragma).
# -packed-fp32-ops: no v_pk_*_f32 packed FP32 instructions.
HIPFLAGS = [
    "--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC", "-shared",
    "-ffp-contract=off", "-fno-fast-math", "-fvisibility=hidden",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def build(verbose: bool = False) -> str:
    """Compile every source into the shared library (always recompiles)."""
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc(), *HIPFLAGS, "-I", os.path.join(ROOT, "include"), *sources(), "-o", tmp,
           "-lpthread"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


# GPU test helpers built beside the tests (not part of the library).
TEST_HELPERS = [("tests/native/sqrt_rn_check.hip", "tests/native/libsqrt_rn_check.so"),
                ("tests/native/rcp_rn_check.hip", "tests/native/librcp_rn_check.so"),
                ("tests/native/lockstep_check.hip", "tests/native/liblockstep_check.so")]


def build_test_helpers(verbose: bool = False) -> None:
    """Compile the GPU tests' helper libraries with the library's flags."""
    for src, out in TEST_HELPERS:
        out = os.path.join(ROOT, out)
        tmp = out + ".tmp%d" % os.getpid()
        cmd = [hipcc(), *HIPFLAGS, os.path.join(ROOT, src), "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.check_call(cmd)
        os.replace(tmp, out)


def is_built() -> bool:
    return os.path.exists(LIB)


if __name__ == "__main__":
    build(verbose=True)
    print(LIB)
    sys.exit(0)
