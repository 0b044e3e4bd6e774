"""Build libgsys.so in-tree for gfx950 (hipcc for the HIP sources, g++ for
the plain C++ host pool), the demo user program's library beside it, and the
test-hook library under tests/native."""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "libgsys.so")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
HIPCC = os.path.join(ROCM, "bin", "hipcc")
ARCH = os.environ.get("GSYS_OFFLOAD_ARCH", "gfx950")

HIP_SOURCES = ["k_fnv.hip", "k_wordscan.hip", "k_kv.hip", "k_serve.hip", "k_canary.hip",
               "k_permute.hip", "k_fileio.hip", "k_launch.hip"]
# a user program of the library, built against include/ only
DEMO_SRC = os.path.join(HERE, "demo", "pread_fnv.hip")
DEMO_LIB = os.path.join(HERE, "libgsys_demo.so")
# the test-only hook library (tests load it; the product never does)
HOOKS_DIR = os.path.join(ROOT, "tests", "native")
HOOKS_SRC = os.path.join(HOOKS_DIR, "gsys_test_hooks.cpp")
HOOKS_LIB = os.path.join(HOOKS_DIR, "libgsys_testing.so")
HOST_HIP_SOURCES = ["capi.cpp"]      # host code that calls the HIP runtime
HOST_SOURCES = ["host_pool.cpp", "kv_loadgen.cpp", "pread_probe.cpp"]     # plain C++17 + POSIX

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
# packed fp32 instructions are disabled for all device code
DEVICE = ["--offload-arch=" + ARCH, "-Xclang", "-target-feature", "-Xclang",
          "-packed-fp32-ops", "-munsafe-fp-atomics"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n%s\n%s%s" % (" ".join(cmd), r.stdout, r.stderr))
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    for s in HIP_SOURCES:
        src = os.path.join(CSRC, s)
        if not os.path.exists(src):
            continue
        jobs.append([HIPCC, "-x", "hip", "-c", src, "-o", os.path.join(BUILD, s + ".o")]
                    + COMMON + DEVICE)
    for s in HOST_HIP_SOURCES:
        jobs.append([HIPCC, "-c", os.path.join(CSRC, s), "-o", os.path.join(BUILD, s + ".o"),
                     "-D__HIP_PLATFORM_AMD__"] + COMMON + DEVICE
                    + ["-Wno-unused-value", "-Wno-unused-result"])
    for s in HOST_SOURCES:
        jobs.append(["g++", "-c", os.path.join(CSRC, s), "-o", os.path.join(BUILD, s + ".o"),
                     "-pthread"] + COMMON)
    with cf.ThreadPoolExecutor(max_workers=min(8, len(jobs))) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                sys.stderr.write(r.stdout + r.stderr)
    objs = [j[j.index("-o") + 1] for j in jobs]
    tmp = LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "-shared", "-fPIC", "--offload-arch=" + ARCH, "-Wl,-soname,libgsys.so", "-o", tmp] + objs
         + ["-pthread", "-Wl,--no-undefined", "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-lhsa-runtime64"])
    os.replace(tmp, LIB)
    # the demo program links against the library it was built with
    tmp = DEMO_LIB + ".tmp%d" % os.getpid()
    _run([HIPCC, "-x", "hip", DEMO_SRC, "-shared", "-fPIC", "-O3", "-std=c++17", "-Wall",
          "-I" + os.path.join(ROOT, "include"), "-o", tmp] + DEVICE
         + ["-L" + HERE, "-lgsys", "-Wl,-rpath,$ORIGIN", "-Wl,--no-undefined",
            "-L" + os.path.join(ROCM, "lib"), "-lamdhip64"])
    os.replace(tmp, DEMO_LIB)
    if os.path.exists(HOOKS_SRC):
        tmp = HOOKS_LIB + ".tmp%d" % os.getpid()
        _run(["g++", "-shared", "-fPIC", "-O2", "-std=c++17", "-Wall", "-pthread",
              "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-I" + HOOKS_DIR,
              HOOKS_SRC, "-o", tmp, "-L" + HERE, "-lgsys",
              "-Wl,-rpath,$ORIGIN/../../paper_1705_06965_amd", "-Wl,--no-undefined"])
        os.replace(tmp, HOOKS_LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
