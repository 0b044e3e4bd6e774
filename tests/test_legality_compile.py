"""Legality of granularity x ordering (section 4.1): work-item calls are
implicitly strong and kernel calls are relaxed only.  The two illegal cells
must not compile; the six other (G, O) instantiations must."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = "/opt/rocm/bin/hipcc"

SRC = """
#include "gsys_device.hpp"
__global__ void k() { (void)gsys::Legal<gsys::G::%s, gsys::O::%s>::ok; }
"""


def _compile(g, o, tmp_path):
    src = tmp_path / ("legal_%s_%s.hip" % (g, o))
    src.write_text(SRC % (g, o))
    r = subprocess.run([HIPCC, "-x", "hip", "-std=c++17", "--offload-arch=gfx950",
                        "-fsyntax-only", "-I" + os.path.join(ROOT, "include"),
                        "-I" + os.path.join(ROOT, "paper_1705_06965_amd", "csrc"), str(src)],
                       capture_output=True, text=True)
    return r.returncode, r.stderr


pytestmark = pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")


@pytest.mark.parametrize("g,o", [("WorkItem", "Relaxed"), ("Kernel", "Strong")])
def test_illegal_cells_fail_to_compile(g, o, tmp_path):
    rc, err = _compile(g, o, tmp_path)
    assert rc != 0
    assert "static assertion failed" in err or "static_assert" in err


@pytest.mark.parametrize("g,o", [("WorkItem", "Strong"), ("WorkGroup", "Strong"),
                                 ("WorkGroup", "Relaxed"), ("Kernel", "Relaxed")])
def test_legal_cells_compile(g, o, tmp_path):
    rc, err = _compile(g, o, tmp_path)
    assert rc == 0, err


API_SRC = """
#include "gsys_device.hpp"
__global__ void k(gsys_dev_ctx c) {
  (void)gsys::gsys_call<gsys::G::%s, gsys::O::%s, gsys::B::Blocking>(c, GSYS_NR_PREAD64, 0, 0, 0, 0);
  (void)gsys::pwrite<gsys::G::%s, gsys::O::%s>(c, 3, 0, 64, 0);
}
"""


def _compile_api(g, o, tmp_path):
    src = tmp_path / ("api_%s_%s.hip" % (g, o))
    src.write_text(API_SRC % (g, o, g, o))
    r = subprocess.run([HIPCC, "-x", "hip", "-std=c++17", "--offload-arch=gfx950",
                        "-fsyntax-only", "-I" + os.path.join(ROOT, "include"), str(src)],
                       capture_output=True, text=True)
    return r.returncode, r.stderr


@pytest.mark.parametrize("g,o", [("WorkItem", "Relaxed"), ("Kernel", "Strong")])
def test_public_api_rejects_illegal_cells(g, o, tmp_path):
    """The public calls (gsys_call and the typed wrappers), compiled against
    include/ alone, refuse the two illegal cells."""
    rc, err = _compile_api(g, o, tmp_path)
    assert rc != 0
    assert "static assertion failed" in err or "static_assert" in err


@pytest.mark.parametrize("g,o", [("WorkItem", "Strong"), ("WorkGroup", "Strong"),
                                 ("WorkGroup", "Relaxed"), ("Kernel", "Relaxed")])
def test_public_api_compiles_legal_cells(g, o, tmp_path):
    rc, err = _compile_api(g, o, tmp_path)
    assert rc == 0, err
