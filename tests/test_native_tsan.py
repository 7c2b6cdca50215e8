"""Race detection for the host side of the library: the request server's
scheduler, driven by several threads with the simulated executor, built with
ThreadSanitizer on the host code (device code is built normally) and run on
the CPU."""
import os
import shutil
import subprocess

import pytest

from paper_cs_0406049_amd import build as hipbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.slow
def test_server_under_thread_sanitizer(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "serve_stress"
    cmd = [hipcc, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-ffp-contract=off",
           "-Xarch_host", "-fsanitize=thread",
           "-I", os.path.join(ROOT, "include"),
           *hipbuild.sources(), os.path.join(ROOT, "tests", "native", "serve_stress.cpp"),
           "-o", str(exe), "-lpthread"]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 second_deadlock_stack=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert "ThreadSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0 and "serve_stress: ok" in r.stdout, (r.returncode, r.stderr[-2000:])
