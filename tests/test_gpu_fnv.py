"""GPU parity of the per-item pread + FNV-1a workload against the oracle.

Every cell of the granularity x ordering x blocking grid (8 legal cells,
section 4.1) and the persistent / graph forms must give the oracle's vector
bit for bit.  Calls go through the C ABI (gsys_fnv4k)."""
import errno
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_06965_amd as g
    ctx = g.Context(ring_slots=1 << 16, device_timeout_ns=60_000_000_000, flags=g.CFG_LEDGER,
                    ledger_capacity=1 << 22)
    yield g, ctx
    assert ctx.shutdown() == 0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_tiny_plain_wi_strong_blocking(gs):
    """1 work-group of 64 work-items, pread 4 KiB at 4096*i of a 256 KiB file."""
    g, ctx = gs
    from paper_1705_06965_amd.fnv import FnvRunner
    p = synth.random_file(1, 262144, name="c1_256k.bin")
    offs = synth.tiny_offsets(64)
    want_fnv, want_ret = oracle.pread_fnv(p, offs, 4096)
    r = FnvRunner(ctx, p, offs, 4096, wg_size=64)
    say("tiny WI/strong/block")
    f, ret = r.run("WI", "strong", "block")
    assert (ret == 4096).all()
    assert (f == want_fnv).all()
    led = ctx.ledger(reset=True)
    assert len(led) == 64 and len(set(led[:, 0].tolist())) == 64
    r.close()


@pytest.fixture(scope="module")
def mid(gs):
    g, ctx = gs
    from paper_1705_06965_amd.fnv import FnvRunner
    size = 64 << 20
    p = synth.random_file(2, size, name="c2_64m.bin")
    n = 16 * 256 + 37          # 16 full work-groups and a ragged tail
    offs = synth.sweep_offsets(n, size // 4096)
    want = oracle.pread_fnv(p, offs, 4096, threads=8)
    r = FnvRunner(ctx, p, offs, 4096, wg_size=256)
    yield r, want
    r.close()


def assert_quiescent(ctx):
    """Every claimed ticket has retired after the drain: each slot it used is
    FREE for its next lap (freed by the GPU waiter of a blocking call, by the
    host for a non-blocking one).  The retire scan may be running on a
    poller when the drain asks for it, so this looks a few times."""
    import time
    st = {}
    for _ in range(200):
        assert ctx.wait(5_000_000_000) == 0
        st = ctx.stats()
        if st["retired_lo"] == st["claimed"]:
            return
        time.sleep(0.01)
    raise AssertionError("ring not quiescent: %d of %d tickets retired"
                         % (st["retired_lo"], st["claimed"]))


@pytest.mark.parametrize("cell", [("WI", "strong", "block"), ("WI", "strong", "nonblock"),
                                  ("WG", "strong", "block"), ("WG", "strong", "nonblock"),
                                  ("WG", "relaxed", "block"), ("WG", "relaxed", "nonblock"),
                                  ("K", "relaxed", "block"), ("K", "relaxed", "nonblock")])
def test_all_legal_cells_match_oracle(gs, mid, cell):
    g, ctx = gs
    r, (want_fnv, want_ret) = mid
    ctx.ledger(reset=True)
    say("cell", cell, "n", r.n)
    f, ret = r.run(*cell)
    assert (ret == want_ret).all()
    assert (f == want_fnv).all()
    # exactly once: one ledger record per ring request of the cell (one per
    # work-item, per work-group or per launch), each ticket once, and each
    # request's result the bytes its items read
    led = ctx.ledger(reset=True)
    per = {"WI": 1, "WG": 256, "K": r.n}[cell[0]]
    want_requests = (r.n + per - 1) // per
    assert len(led) == want_requests
    assert len(np.unique(led[:, 0])) == want_requests
    assert (led[:, 1] == g.NR_PREAD64).all()
    got_bytes = np.sort(led[:, 2].astype(np.int64))
    sizes = [min(per, r.n - k * per) * 4096 for k in range(want_requests)]
    assert (got_bytes == np.sort(np.array(sizes, dtype=np.int64))).all()
    assert_quiescent(ctx)


@pytest.mark.parametrize("form", ["persistent", "graph"])
def test_persistent_and_graph_forms(gs, mid, form):
    g, ctx = gs
    r, (want_fnv, want_ret) = mid
    fm = g.PERSISTENT if form == "persistent" else g.GRAPH
    for rep in range(2 if form == "graph" else 1):
        say("form", form, "rep", rep)
        f, ret = r.run(form=fm)
        assert (ret == want_ret).all()
        assert (f == want_fnv).all()
        assert_quiescent(ctx)


def test_smallest_ring(gs, mid):
    """A ring of 64 slots, the smallest the library takes (one wavefront's
    claim): nearly every claim waits for its slot to be freed for its lap
    (back-pressure, section 5), in all 8 cells, both forms, with 64- and
    256-wide work-groups.  Results equal the oracle's and the ring is
    quiescent after each drain."""
    g, _ = gs
    from paper_1705_06965_amd.fnv import FnvRunner
    r0, (want_fnv, want_ret) = mid
    offs = r0.offsets.cpu().numpy().view(np.uint64)
    ctx = g.Context(ring_slots=64, device_timeout_ns=60_000_000_000)
    try:
        for wg in (64, 256):
            r = FnvRunner(ctx, r0.path, offs, 4096, wg_size=wg)
            for cell in [("WI", "strong", "block"), ("WI", "strong", "nonblock"),
                         ("WG", "strong", "block"), ("WG", "strong", "nonblock"),
                         ("WG", "relaxed", "block"), ("WG", "relaxed", "nonblock"),
                         ("K", "relaxed", "block"), ("K", "relaxed", "nonblock"), None, "graph"]:
                say("ring 64, wg", wg, cell)
                if cell is None:
                    f, ret = r.run(form=g.PERSISTENT)
                elif cell == "graph":
                    f, ret = r.run(form=g.GRAPH)
                else:
                    f, ret = r.run(*cell)
                assert (ret == want_ret).all(), (wg, cell)
                assert (f == want_fnv).all(), (wg, cell)
                assert_quiescent(ctx)
            st = ctx.stats()
            assert st["claimed"] > 64 * 20          # many laps of the ring
            r.close()
    finally:
        assert ctx.shutdown() == 0


@pytest.mark.parametrize("ring_batches", [4, 6])
def test_persistent_staging_ring(gs, mid, ring_batches):
    """A staging ring smaller than the data: each resident work-group reuses
    two batch buffers, so batches share memory across iterations."""
    g, ctx = gs
    from paper_1705_06965_amd.fnv import FnvRunner
    r0, (want_fnv, want_ret) = mid
    offs = r0.offsets.cpu().numpy().view(np.uint64)
    r = FnvRunner(ctx, r0.path, offs, 4096, wg_size=256,
                  staging_bytes=ring_batches * 256 * 4096)
    for fm in (g.PERSISTENT, g.GRAPH, g.GRAPH):
        say("staging ring", ring_batches, fm)
        f, ret = r.run(form=fm)
        assert (ret == want_ret).all()
        assert (f == want_fnv).all()
    with pytest.raises(g.GsysError):
        r.launch(g.cell_code("WI", "strong", "block"), g.PLAIN)  # plain needs every item
    r.close()


def test_illegal_cells_rejected(gs, mid):
    g, ctx = gs
    r, _ = mid
    with pytest.raises(g.GsysError):
        r.launch(g.cell(g.GRAN_WI, False, True))       # work-item relaxed
    with pytest.raises(g.GsysError):
        r.launch(g.cell(g.GRAN_KERNEL, True, True))    # kernel strong


def test_short_reads_and_small_items(gs, tmpdata):
    """Reads that cross EOF return short counts; checksums cover what was read."""
    g, ctx = gs
    from paper_1705_06965_amd.fnv import FnvRunner
    p = os.path.join(tmpdata, "eof.bin")
    data = np.random.default_rng(11).integers(0, 256, 100_000, dtype=np.uint8)
    data.tofile(p)
    offs = np.array([0, 99_990, 100_000, 200_000, 50_001, 96_000, 7, 99_999] * 40,
                    dtype=np.uint64)
    for item in (64, 4096):
        want_fnv, want_ret = oracle.pread_fnv(p, offs, item)
        r = FnvRunner(ctx, p, offs, item, wg_size=64)
        for cell in (("WI", "strong", "block"), ("WG", "relaxed", "block"),
                     ("K", "relaxed", "nonblock")):
            say("eof", item, cell)
            f, ret = r.run(*cell)
            assert (ret == want_ret).all()
            assert (f == want_fnv).all()
        r.close()


def test_largest_items(gs):
    """Items of 1 MiB, the largest the entry point takes: two work-groups of
    64 (the second ragged), reads that cross or start past the end of the
    file, in a work-item, a work-group and a kernel cell and the persistent
    form."""
    g, ctx = gs
    from paper_1705_06965_amd.fnv import FnvRunner
    p = synth.random_file(2, 64 << 20, name="c2_64m.bin")
    item = 1 << 20
    rng = np.random.default_rng([170506965, 77])
    offs = (rng.integers(0, (64 << 20) // 256, 100) * 256).astype(np.uint64)
    offs[[3, 70]] = (64 << 20) - 1000            # 1,000 bytes before EOF
    offs[[5, 99]] = (64 << 20) + 4096            # past EOF
    offs[64] = (64 << 20) - item                 # ends exactly at EOF
    want_fnv, want_ret = oracle.pread_fnv(p, offs, item, threads=8)
    assert {0, 1000, item} <= set(want_ret.tolist())
    r = FnvRunner(ctx, p, offs, item, wg_size=64)
    for cell in (("WI", "strong", "block"), ("WG", "relaxed", "nonblock"),
                 ("K", "relaxed", "block"), None):
        say("1 MiB items", cell)
        f, ret = r.run(*cell) if cell else r.run(form=g.PERSISTENT)
        assert (ret == want_ret).all(), cell
        assert (f == want_fnv).all(), cell
    r.close()


def test_single_item_and_revoked_fd(gs):
    g, ctx = gs
    from paper_1705_06965_amd.fnv import FnvRunner
    p = synth.random_file(1, 262144, name="c1_256k.bin")
    offs = np.array([4096 * 5], dtype=np.uint64)
    want_fnv, want_ret = oracle.pread_fnv(p, offs, 4096)
    r = FnvRunner(ctx, p, offs, 4096, wg_size=64)
    f, ret = r.run("WG", "strong", "block")
    assert ret[0] == 4096 and f[0] == want_fnv[0]
    # revoked fd: every call completes with -EBADF, the checksum covers no bytes
    ctx.allow_fd(r.fd, 0)
    f, ret = r.run("WI", "strong", "block")
    assert ret[0] == -9 and f[0] == 0xcbf29ce484222325
    ctx.allow_fd(r.fd, g.FD_READ)
    r.close()


@pytest.fixture(scope="module")
def full(gs):
    """The microbenchmark sweep at its full size: 262,144 preads of 4 KiB at
    uniform random 4 KiB-aligned offsets of a 1 GiB file, 1,024 work-groups
    of 256; the oracle's whole vector."""
    g, ctx = gs
    from paper_1705_06965_amd.fnv import FnvRunner
    size = 1 << 30
    p = synth.random_file(2, size, name="c2_1g.bin")
    n = 1024 * 256
    offs = synth.sweep_offsets(n, size // 4096)
    want = oracle.pread_fnv(p, offs, 4096, threads=8)
    r = FnvRunner(ctx, p, offs, 4096, wg_size=256)
    yield r, offs, want
    r.close()


@pytest.mark.parametrize("cell", [("WI", "strong", "block"), ("WI", "strong", "nonblock"),
                                  ("WG", "strong", "block"), ("WG", "strong", "nonblock"),
                                  ("WG", "relaxed", "block"), ("WG", "relaxed", "nonblock"),
                                  ("K", "relaxed", "block"), ("K", "relaxed", "nonblock"),
                                  "persistent", "graph"])
def test_full_sweep_every_cell(gs, full, cell):
    """Every legal cell and both batching forms (the graph form in the
    benchmark's launch configuration) give the oracle's whole vector."""
    g, ctx = gs
    r, offs, (want_fnv, want_ret) = full
    say("full sweep", cell)
    if cell == "persistent":
        f, ret = r.run(form=g.PERSISTENT)
    elif cell == "graph":
        f, ret = r.run(form=g.GRAPH)
        f, ret = r.run(form=g.GRAPH)  # a replay
    else:
        f, ret = r.run(*cell)
    assert (ret == want_ret).all() and (ret == 4096).all()
    assert (f == want_fnv).all()
    # equal offsets give equal checksums
    _, first, inv = np.unique(offs, return_index=True, return_inverse=True)
    assert (f == f[first][inv]).all()


@pytest.mark.parametrize("wg", [512, 1024])
def test_wide_work_groups_match_oracle(gs, mid, wg):
    """The call path with 512- and 1,024-wide work-groups (section 6, Fig. 5
    right: work-group size): every legal cell and the persistent form, on
    4,133 items (a ragged last work-group)."""
    g, ctx = gs
    from paper_1705_06965_amd.fnv import FnvRunner
    r0, (want_fnv, want_ret) = mid
    offs = r0.offsets.cpu().numpy().view(np.uint64)
    r = FnvRunner(ctx, r0.path, offs, 4096, wg_size=wg)
    for cell in [("WI", "strong", "block"), ("WI", "strong", "nonblock"),
                 ("WG", "strong", "block"), ("WG", "strong", "nonblock"),
                 ("WG", "relaxed", "block"), ("WG", "relaxed", "nonblock"),
                 ("K", "relaxed", "block"), ("K", "relaxed", "nonblock"), None]:
        say("wg", wg, cell)
        f, ret = r.run(*cell) if cell else r.run(form=g.PERSISTENT)
        assert (ret == want_ret).all(), (wg, cell)
        assert (f == want_fnv).all(), (wg, cell)
    r.close()


@pytest.mark.parametrize("piece", [64, 256, 4096, 65536])
def test_coalesced_work_item_calls(gs, tmpdata, piece):
    """Coalescing (section 4.2, Fig. 7): work-item preads of consecutive
    pieces through a pool that bundles up to K = 8 ready requests for up to
    T = 10 us and merges contiguous ones into one pread; every item's bytes
    and checksum equal the oracle's, and small pieces were merged."""
    g, _ = gs
    from paper_1705_06965_amd.fnv import FnvRunner
    p = synth.random_file(2, 64 << 20, name="c2_64m.bin")
    n = min(4096, (64 << 20) // piece)
    offs = (np.arange(n, dtype=np.uint64) * np.uint64(piece))
    want_fnv, want_ret = oracle.pread_fnv(p, offs, piece, threads=8)
    ctx = g.Context(ring_slots=1 << 14, device_timeout_ns=60_000_000_000, coalesce_max=8,
                    coalesce_window_ns=10_000)
    try:
        r = FnvRunner(ctx, p, offs, piece, wg_size=256)
        for cell in (("WI", "strong", "block"), ("WI", "strong", "nonblock")):
            ctx.stats(reset=True)
            say("coalesced", piece, cell)
            f, ret = r.run(*cell)
            assert (ret == want_ret).all()
            assert (f == want_fnv).all()
            st = ctx.stats()
            assert st["requests"] == n
            if piece <= 256:
                assert st["merged"] > 0 and st["host_calls"] < n
        r.close()
    finally:
        assert ctx.shutdown() == 0


def test_injected_errno_seen_by_the_gpu(gs):
    """The host answers 7 of the 64 work-item preads with -EIO (fault
    injection): exactly 7 items report -EIO on the GPU, the other 57 read
    their bytes and hash to the oracle's values."""
    import errno
    g, ctx = gs
    from paper_1705_06965_amd.fnv import FnvRunner
    p = synth.random_file(1, 262144, name="c1_256k.bin")
    offs = synth.tiny_offsets(64)
    want_fnv, want_ret = oracle.pread_fnv(p, offs, 4096)
    r = FnvRunner(ctx, p, offs, 4096, wg_size=64)
    import gsys_hooks as hooks
    assert hooks.lib.gsys_test_inject(ctx.h, g.NR_PREAD64, errno.EIO, 7) == 0
    say("tiny with 7 injected -EIO")
    f, ret = r.run("WI", "strong", "block")
    bad = ret == -errno.EIO
    assert bad.sum() == 7
    assert (ret[~bad] == want_ret[~bad]).all() and (f[~bad] == want_fnv[~bad]).all()
    r.close()


@pytest.mark.parametrize("wg", [64, 256, 1024])
def test_direct_descriptor_lists_match_oracle(gs, mid, wg, monkeypatch):
    """Strong work-group cells with every work-item writing its own
    descriptor straight into the host-visible list (GSYS_LDS_LISTS=0, the
    alternative to aggregating the list in LDS): the oracle's vector."""
    g, ctx = gs
    from paper_1705_06965_amd.fnv import FnvRunner
    r0, (want_fnv, want_ret) = mid
    offs = r0.offsets.cpu().numpy().view(np.uint64)
    r = FnvRunner(ctx, r0.path, offs, 4096, wg_size=wg)
    monkeypatch.setenv("GSYS_LDS_LISTS", "0")
    for cell in [("WG", "strong", "block"), ("WG", "strong", "nonblock")]:
        say("direct lists", wg, cell)
        f, ret = r.run(*cell)
        assert (ret == want_ret).all(), (wg, cell)
        assert (f == want_fnv).all(), (wg, cell)
    r.close()


def test_failed_item_does_not_mark_its_group(gs, mid):
    """Items whose pread fails (offsets past 2^63: -EINVAL from the host)
    inside a work-group's or the kernel's descriptor list: those items
    report -EINVAL and hash nothing, and every other item of the same list
    keeps its own bytes and checksum, as the oracle's one-call-per-item
    reads give (a list call's result is the bytes it moved; each descriptor
    carries its own result)."""
    g, ctx = gs
    from paper_1705_06965_amd.fnv import FnvRunner
    r0, _ = mid
    offs = r0.offsets.cpu().numpy().view(np.uint64).copy()
    bad = [5, 300, 301, len(offs) - 1]
    offs[bad[0]] = np.uint64(1 << 63)
    offs[bad[1]] = np.uint64(1 << 63)
    offs[bad[2]] = np.uint64((1 << 63) + 4096)   # adjacent to the one before: one merged pread
    offs[bad[3]] = np.uint64((1 << 64) - 4096)
    want_fnv, want_ret = oracle.pread_fnv(r0.path, offs, 4096)
    assert (want_ret[bad] == -errno.EINVAL).all() and (np.delete(want_ret, bad) == 4096).all()
    r = FnvRunner(ctx, r0.path, offs, 4096, wg_size=256)
    for cell in [("WI", "strong", "block"), ("WG", "strong", "block"), ("WG", "strong", "nonblock"),
                 ("WG", "relaxed", "block"), ("WG", "relaxed", "nonblock"),
                 ("K", "relaxed", "block"), ("K", "relaxed", "nonblock"), None]:
        say("failed items", cell)
        f, ret = r.run(*cell) if cell else r.run(form=g.PERSISTENT)
        assert (ret == want_ret).all(), (cell, np.nonzero(ret != want_ret)[0][:8])
        assert (f == want_fnv).all(), cell
    r.close()
