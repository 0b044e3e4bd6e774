"""Visibility canary for producer calls on the GPU: every work-item's stamp
written before a pwrite at its granularity must reach the file (section 4.1:
producers need all stores of their group done before the call)."""
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

CELLS = [("WI", "strong", "block"), ("WI", "strong", "nonblock"),
         ("WG", "strong", "block"), ("WG", "strong", "nonblock"),
         ("WG", "relaxed", "block"), ("WG", "relaxed", "nonblock"),
         ("K", "relaxed", "block"), ("K", "relaxed", "nonblock")]


def stamps(seed: int, n: int) -> np.ndarray:
    i = np.arange(n, dtype=np.uint64)[:, None]
    k = np.arange(8, dtype=np.uint64)[None, :]
    with np.errstate(over="ignore"):
        a = np.uint64(seed) * np.uint64(0x9E3779B97F4A7C15)
        b = (i * np.uint64(8) + k + np.uint64(1)) * np.uint64(0xD1B54A32D192ED03)
    return (a ^ b).astype("<u8").view(np.uint8).reshape(n * 64)


@pytest.fixture(scope="module")
def gs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_06965_amd as g
    ctx = g.Context(ring_slots=1 << 14, device_timeout_ns=30_000_000_000, flags=g.CFG_LEDGER)
    yield g, ctx
    assert ctx.shutdown() == 0


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("n,wg", [(3001, 256), (2048, 1024)])
def test_canary(gs, tmpdata, cell, n, wg):
    import torch
    g, ctx = gs
    path = os.path.join(tmpdata, "canary_%s_%s_%s_%d.bin" % (cell + (n,)))
    fd = os.open(path, os.O_RDWR | os.O_CREAT | os.O_TRUNC, 0o600)
    ctx.allow_fd(fd, g.FD_WRITE)
    buf = ctx.host_alloc(n * 64)
    buf.array[:] = 0
    out = torch.full((max(1, (n + wg - 1) // wg, n),), -12345, dtype=torch.int64, device="cuda")
    seed = 1000 + n + CELLS.index(cell)
    ctx.ledger(reset=True)
    print("canary", cell, n, wg, flush=True)
    g.check(g.lib.gsys_canary(ctx.h, fd, buf.dev, n, seed, out.data_ptr(), g.cell_code(*cell),
                              wg, 0), "gsys_canary")
    torch.cuda.synchronize()
    assert ctx.wait(30_000_000_000) == 0
    want = stamps(seed, n)
    got = np.fromfile(path, dtype=np.uint8)
    assert len(got) == n * 64
    bad = np.nonzero(got != want)[0]
    assert len(bad) == 0, "first stale byte at %d" % bad[0]
    r = out.cpu().numpy()
    led = ctx.ledger(reset=True)
    if cell[0] == "WI":
        assert (r[:n] == 64).all()
        assert len(led) == n
    elif cell[0] == "WG":
        groups = (n + wg - 1) // wg
        sizes = np.minimum(wg, n - wg * np.arange(groups)) * 64
        assert (r[:groups] == sizes).all()
        assert len(led) == groups
    else:
        assert r[0] == n * 64
        assert len(led) == 1
    os.close(fd)
    buf.free()
