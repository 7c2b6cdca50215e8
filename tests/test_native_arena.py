"""The request server's output arena (first fit, coalescing) against a plain
model over random allocation and release sequences, built with the host
compiler under AddressSanitizer and UndefinedBehaviorSanitizer
(tests/native/arena_model.cpp)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_arena_matches_its_model(tmp_path):
    gxx = shutil.which("g++")
    if not gxx:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "arena_model"
    src = os.path.join(ROOT, "tests", "native", "arena_model.cpp")
    subprocess.check_call([gxx, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", src, "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0 and "arena_model: ok" in r.stdout, r.stderr[-3000:]
    assert "Sanitizer" not in r.stderr, r.stderr[-3000:]
