"""Host-side checks of the library under sanitizers, on the CPU: the request
server's scheduler driven by several threads with the simulated executor
(tests/native/serve_stress.cpp), and the GPU-free paths of the C ABI -- the
tuning parser on truncated and random text, buffer sizes, argument checks
(tests/native/host_paths.cpp).  Host code is built with ThreadSanitizer, or
with AddressSanitizer + UndefinedBehaviorSanitizer; device code is built
normally and never runs."""
import os
import shutil
import subprocess

import pytest

from paper_cs_0406049_amd import build as hipbuild

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SANITIZERS = {
    "thread": (["-Xarch_host", "-fsanitize=thread"],
               {"TSAN_OPTIONS": "halt_on_error=1 second_deadlock_stack=1"}, "ThreadSanitizer"),
    "address+undefined": (["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                           "-Xarch_host", "-fno-omit-frame-pointer",
                           "-Xarch_host", "-fno-sanitize-recover=undefined"],
                          {"ASAN_OPTIONS": "detect_leaks=1",
                           "UBSAN_OPTIONS": "print_stacktrace=1 halt_on_error=1"},
                          "Sanitizer"),
}
PROGRAMS = {"serve_stress": "serve_stress: ok", "host_paths": "host_paths: ok"}


DEVICE_SOURCES = ("plain.hip", "forms.hip", "ablation.hip")   # kernels: built once, no sanitizer


def _hipcc():
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    return hipcc


@pytest.fixture(scope="module")
def device_objects(tmp_path_factory):
    """The sources that hold kernels, compiled once (their host side is
    only launch stubs); the host-side sources are rebuilt per sanitizer."""
    out = tmp_path_factory.mktemp("devobj")
    objs = []
    for src in DEVICE_SOURCES:
        obj = out / (src + ".o")
        subprocess.check_call([_hipcc(), "--offload-arch=gfx950", "-O1", "-std=c++17",
                               "-ffp-contract=off", "-Xclang", "-target-feature", "-Xclang",
                               "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-c",
                               os.path.join(hipbuild.CSRC, src), "-o", str(obj)],
                              stderr=subprocess.DEVNULL)
        objs.append(str(obj))
    return objs


@pytest.mark.slow
@pytest.mark.parametrize("program", sorted(PROGRAMS))
@pytest.mark.parametrize("sanitizer", sorted(SANITIZERS))
def test_host_code_under_sanitizer(tmp_path, device_objects, sanitizer, program):
    flags, env_add, marker = SANITIZERS[sanitizer]
    exe = tmp_path / program
    host_sources = [s for s in hipbuild.sources() if os.path.basename(s) not in DEVICE_SOURCES]
    cmd = [_hipcc(), "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-ffp-contract=off",
           *flags, "-I", os.path.join(ROOT, "include"), *host_sources,
           os.path.join(ROOT, "tests", "native", program + ".cpp"), "-x", "none", *device_objects,
           "-o", str(exe), "-lpthread"]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    env = dict(os.environ, **env_add)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert marker not in r.stderr, r.stderr[-4000:]
    assert r.returncode == 0 and PROGRAMS[program] in r.stdout, (r.returncode, r.stderr[-2000:])
