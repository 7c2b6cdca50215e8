"""The C ABI from plain C (no Python, no torch): tests/native/abi_example.c
compiles against include/sincos.h and links the library; on a GPU it runs the
plain, ragged-plan, interleaved and server paths and checks them."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "native", "abi_example.c")
EXE = os.path.join(ROOT, "tests", "native", "abi_example")
LIBDIR = os.path.join(ROOT, "paper_cs_0406049_amd")


def build_example(out=EXE):
    from paper_cs_0406049_amd import build as hipbuild
    if not hipbuild.is_built():
        hipbuild.build()
    subprocess.check_call([
        "gcc", "-std=c11", "-O2", "-Wall", "-Wextra", SRC, "-o", out,
        "-I", "/opt/rocm/include", "-L", LIBDIR, "-lmi355_sincos",
        "-L", "/opt/rocm/lib", "-lamdhip64", "-lm",
        "-Wl,-rpath," + LIBDIR, "-Wl,-rpath,/opt/rocm/lib"])
    return out


def test_example_compiles_and_links(tmp_path):
    build_example(str(tmp_path / "abi_example"))


@pytest.mark.gpu
def test_example_runs_on_the_gpu(tmp_path):
    exe = build_example(str(tmp_path / "abi_example"))   # never a build from an older header
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "abi_example: ok" in r.stdout, (r.stdout, r.stderr[-2000:])
