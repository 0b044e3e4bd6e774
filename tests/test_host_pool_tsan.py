"""The host service pool under ThreadSanitizer and AddressSanitizer +
UndefinedBehaviorSanitizer (CPU only, host code only).

tests/pool_tsan_driver.cpp drives the pool through the GPU's slot protocol
from host threads while other threads change the fd and buffer tables the
pollers read without locks.  Built with g++ -fsanitize=thread together with
capi.cpp and host_pool.cpp, any data race ends the run with exit code 66;
built with -fsanitize=address,undefined, any invalid access or undefined
operation does.  A last phase runs with the doorbell on, so that pollers
block and wake while callers keep arriving.  The driver also checks every
result against the file's bytes and the ledger's exactly-once property."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1705_06965_amd", "csrc")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


@pytest.mark.parametrize("sanitizer", ["thread", "address,undefined"])
def test_pool_under_sanitizer(tmp_path, tmpdata, sanitizer):
    gxx = shutil.which("g++")
    if not gxx or not os.path.exists(os.path.join(ROCM, "include", "hip", "hip_runtime.h")):
        pytest.skip("g++ or the HIP headers are missing")
    exe = str(tmp_path / "pool_sanitized_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fsanitize=" + sanitizer,
           "-fno-sanitize-recover=all", "-D__HIP_PLATFORM_AMD__",
           "-I" + os.path.join(ROCM, "include"), "-I" + os.path.join(ROOT, "include"),
           "-I" + CSRC, "-I" + os.path.join(ROOT, "tests", "native"),
           os.path.join(ROOT, "tests", "pool_tsan_driver.cpp"),
           os.path.join(ROOT, "tests", "native", "gsys_test_hooks.cpp"),
           os.path.join(CSRC, "capi.cpp"), os.path.join(CSRC, "host_pool.cpp"), "-o", exe,
           "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-lhsa-runtime64", "-pthread",
           "-Wl,-rpath," + os.path.join(ROCM, "lib")]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    if b.returncode != 0 and ("tsan" in b.stderr or "asan" in b.stderr or "ubsan" in b.stderr):
        pytest.skip("no sanitizer runtime: " + b.stderr[-300:])
    assert b.returncode == 0, b.stderr[-3000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66",
               ASAN_OPTIONS="detect_leaks=0 exitcode=66", UBSAN_OPTIONS="exitcode=66")
    r = subprocess.run([exe, tmpdata], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert r.stdout.count(" ok: ") == 7, r.stdout
