"""GPU-issued calls with the doorbell on (GSYS_CFG_DOORBELL): the host
pollers block while the GPU is quiet, and the kernels' calls must wake them
through the HSA interrupt signal.  Every cell and form must still give the
oracle's vector bit for bit, the pollers must really have blocked, and no
call may wait for the backstop (raised to 20 s here, so that a lost wake-up
shows as a slow run instead of being hidden by a short one)."""
import os
import sys
import time

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

BACKSTOP_US = 20_000_000


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_06965_amd as g
    os.environ["GSYS_DOORBELL_BACKSTOP_US"] = str(BACKSTOP_US)
    try:
        ctx = g.Context(ring_slots=1 << 16, device_timeout_ns=60_000_000_000,
                        flags=g.CFG_DOORBELL, doorbell_idle_us=100)
    finally:
        del os.environ["GSYS_DOORBELL_BACKSTOP_US"]
    yield g, ctx
    assert ctx.shutdown() == 0


def _quiet():
    time.sleep(0.005)  # far beyond the 100 us idle threshold: every poller blocks


def test_tiny_calls_after_pauses(gs):
    g, ctx = gs
    from paper_1705_06965_amd.fnv import FnvRunner
    p = synth.random_file(1, 262144, name="c1_256k.bin")
    offs = synth.tiny_offsets(64)
    want_fnv, want_ret = oracle.pread_fnv(p, offs, 4096)
    r = FnvRunner(ctx, p, offs, 4096, wg_size=64)
    s0 = ctx.stats()["doorbell_sleeps"]
    worst = 0.0
    for rep in range(20):
        _quiet()
        say("tiny rep", rep)
        t0 = time.perf_counter()
        f, ret = r.run("WI", "strong", "block")
        worst = max(worst, time.perf_counter() - t0)
        assert (ret == want_ret).all()
        assert (f == want_fnv).all()
    say("worst run %.3f ms" % (worst * 1e3))
    assert worst < 2.0
    assert ctx.stats()["doorbell_sleeps"] - s0 >= 20
    r.close()


@pytest.fixture(scope="module")
def mid(gs):
    g, ctx = gs
    from paper_1705_06965_amd.fnv import FnvRunner
    size = 16 << 20
    p = synth.random_file(3, size, name="c3_16m.bin")
    n = 4 * 256 + 37
    offs = synth.sweep_offsets(n, size // 4096, config=3)
    want = oracle.pread_fnv(p, offs, 4096, threads=8)
    r = FnvRunner(ctx, p, offs, 4096, wg_size=256)
    yield r, want
    r.close()


@pytest.mark.parametrize("cell", [("WI", "strong", "block"), ("WI", "strong", "nonblock"),
                                  ("WG", "strong", "block"), ("WG", "strong", "nonblock"),
                                  ("WG", "relaxed", "block"), ("WG", "relaxed", "nonblock"),
                                  ("K", "relaxed", "block"), ("K", "relaxed", "nonblock")])
def test_all_cells_after_a_pause(gs, mid, cell):
    g, ctx = gs
    r, (want_fnv, want_ret) = mid
    s0 = ctx.stats()["doorbell_sleeps"]
    _quiet()
    say("cell", cell)
    t0 = time.perf_counter()
    f, ret = r.run(*cell)
    dt = time.perf_counter() - t0
    assert (ret == want_ret).all()
    assert (f == want_fnv).all()
    assert dt < 5.0, dt
    assert ctx.stats()["doorbell_sleeps"] > s0


@pytest.mark.parametrize("form", ["persistent", "graph"])
def test_forms_after_a_pause(gs, mid, form):
    g, ctx = gs
    r, (want_fnv, want_ret) = mid
    fm = g.PERSISTENT if form == "persistent" else g.GRAPH
    for rep in range(2):
        _quiet()
        say("form", form, "rep", rep)
        t0 = time.perf_counter()
        f, ret = r.run(form=fm)
        assert time.perf_counter() - t0 < 5.0
        assert (ret == want_ret).all()
        assert (f == want_fnv).all()
