"""The boundary as a user program sees it: paper_1705_06965_amd/demo/pread_fnv.hip,
built against include/gsys.h and include/gsys_device.hpp only, preads items
of a file with gsys::pread at work-item, work-group (non-blocking, then
gsys_wait) and kernel granularity (section 4.1; also two kernel calls at
two call sites, and a refused call at a site past the last) and hashes them; it is
started through gsys_launch in the plain, persistent and graph modes.
Every launch's per-item FNV-1a-64 and byte counts equal the oracle's, also
when one argument array is reused with new buffers, offsets and item counts
between graph replays, with eager launches in between."""
import ctypes as C
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

ITEM = 512
FILE_BYTES = 8 << 20


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def env(tmpdata):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    os.environ.setdefault("GSYS_DATA_DIR", tmpdata)
    import paper_1705_06965_amd as g
    path = synth.random_file(7, FILE_BYTES, name="launch_8m.bin")
    demo = C.CDLL(os.path.join(os.path.dirname(g.LIB_PATH), "libgsys_demo.so"))
    demo.gsys_demo_pread_fnv.restype = C.c_int
    demo.gsys_demo_pread_fnv.argtypes = [C.c_void_p, C.c_uint32, C.c_uint32, C.c_uint32,
                                         C.c_uint32, C.c_int, C.c_uint64, C.c_uint64, C.c_uint64,
                                         C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64, C.c_void_p]
    ctx = g.Context(ring_slots=4096, device_timeout_ns=20_000_000_000)
    fd = os.open(path, os.O_RDONLY)
    ctx.allow_fd(fd, g.FD_READ)
    staging = ctx.host_alloc(4096 * ITEM)
    yield g, ctx, demo, path, fd, staging, torch
    ctx.allow_fd(fd, 0)
    os.close(fd)
    assert ctx.shutdown() == 0


def launch(env, gran, mode, n, seed):
    """One launch on fresh output tensors; returns (fnv, ret, offsets)."""
    g, ctx, demo, path, fd, staging, torch = env
    rng = np.random.default_rng(seed)
    if gran == g.GRAN_WI:
        offs = (rng.integers(0, FILE_BYTES // ITEM, n) * ITEM).astype(np.uint64)
        off0 = 0
    else:
        off0 = int(rng.integers(0, (FILE_BYTES - n * ITEM) // 16)) * 16
        offs = (off0 + ITEM * np.arange(n)).astype(np.uint64)
    offs_d = torch.from_numpy(offs.view(np.int64)).cuda()
    out_fnv = torch.zeros(n, dtype=torch.int64, device="cuda")
    out_ret = torch.full((n,), -999, dtype=torch.int64, device="cuda")
    block = 256
    grid = {g.PLAIN: (n + block - 1) // block if gran not in (g.GRAN_KERNEL, GRAN_SITES)
            else 16}.get(mode, 100000)
    rc = demo.gsys_demo_pread_fnv(ctx.h, gran, mode, grid, block, fd, staging.dev,
                                  offs_d.data_ptr(), off0, n, ITEM, out_fnv.data_ptr(),
                                  out_ret.data_ptr(), None)
    assert rc == 0, g.lib.gsys_strerror(rc)
    torch.cuda.synchronize()
    assert ctx.wait(20_000_000_000) == 0
    return out_fnv.cpu().numpy().view(np.uint64), out_ret.cpu().numpy(), offs


def check(env, got_fnv, got_ret, offs, label):
    _, _, _, path, _, _, _ = env
    want_fnv, want_ret = oracle.pread_fnv(path, offs, ITEM)
    assert (got_ret == want_ret).all(), label
    assert (got_fnv == want_fnv).all(), label


GRANS = ["WI", "WG", "K", "K2"]
GRAN_SITES = 3       # the demo's two kernel-granularity calls at call sites 1 and 2


@pytest.mark.parametrize("gname", GRANS)
@pytest.mark.parametrize("mname", ["PLAIN", "PERSISTENT", "GRAPH"])
def test_user_kernel_matches_oracle(env, gname, mname):
    g = env[0]
    gran = {"WI": g.GRAN_WI, "WG": g.GRAN_WG, "K": g.GRAN_KERNEL, "K2": GRAN_SITES}[gname]
    mode = getattr(g, mname)
    # new offsets, outputs and item counts on every launch through the same
    # argument array; a ragged last work-group in each
    for k, n in enumerate((3001, 1777, 4096, 1)):
        say("launch", gname, mname, n)
        f, r, offs = launch(env, gran, mode, n, seed=100 * k + gran)
        check(env, f, r, offs, (gname, mname, n))
        if mode == g.GRAPH:
            # eager work between replays
            f2, r2, offs2 = launch(env, gran, g.PLAIN, 999, seed=7 + k)
            check(env, f2, r2, offs2, (gname, "eager", k))


def test_launch_refusals(env):
    g, ctx, demo, *_ = env
    import errno
    d = g.gsys_launch_desc()
    assert g.lib.gsys_launch(ctx.h, C.byref(d), None) == -errno.EINVAL           # no kernel
    assert demo.gsys_demo_pread_fnv(ctx.h, 4, g.PLAIN, 1, 64, 0, 0, 0, 0, 1, ITEM, 1, 1,
                                    None) == -errno.EINVAL                       # bad granularity


@pytest.mark.parametrize("flood", [0, 256, 60000, 65536 + 256])
def test_late_wait_of_a_non_blocking_call(env, flood):
    """A non-blocking call's result is waited for two launches after it was
    issued, with `flood` other calls in between.  Until C newer tickets
    are claimed (C = 65,536 completion records for this ring of 4,096
    slots) the wait returns the call's own result, the bytes it read; after
    that its record may hold a later call's result, and the wait reports
    -EOVERFLOW instead of that value (without the check it would return
    the 0 of a later 0-byte pread)."""
    import errno
    g, ctx, demo, path, fd, staging, torch = env
    demo.gsys_demo_late_wait.restype = C.c_int
    demo.gsys_demo_late_wait.argtypes = [C.c_void_p, C.c_int, C.c_uint64, C.c_uint32, C.c_uint64,
                                         C.c_uint64, C.c_uint64, C.c_uint64, C.c_void_p]
    keep = torch.zeros(2, dtype=torch.int64, device="cuda")
    out_ret = torch.full((max(1, flood),), -999, dtype=torch.int64, device="cuda")
    out_wait = torch.full((1,), -999, dtype=torch.int64, device="cuda")
    say("late wait, flood", flood)
    rc = demo.gsys_demo_late_wait(ctx.h, fd, staging.dev, ITEM, flood, keep.data_ptr(),
                                  out_ret.data_ptr(), out_wait.data_ptr(), None)
    assert rc == 0, g.lib.gsys_strerror(rc)
    torch.cuda.synchronize()
    assert ctx.wait(20_000_000_000) == 0
    if flood:
        assert (out_ret.cpu().numpy() == 0).all()
    got = int(out_wait.cpu().item())
    if flood < 65536:
        assert got == ITEM
    else:
        assert got == -errno.EOVERFLOW
