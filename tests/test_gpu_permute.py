"""GPU parity of the block-permutation + pwrite workload (the ordering /
blocking microbenchmark of section 6, Fig. 6) against the oracle.

All four work-group cells (strong / relaxed x blocking / non-blocking) must
write the oracle's file byte for byte; every block is written by exactly one
pwrite (the ledger), and the host-side argument checks reject what the
kernel cannot take.  Calls go through the C ABI (gsys_permute)."""
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
    ctx = g.Context(ring_slots=1 << 14, device_timeout_ns=60_000_000_000, flags=g.CFG_LEDGER,
                    ledger_capacity=1 << 16)
    yield g, ctx
    assert ctx.shutdown() == 0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_file(tmpdata, name, data, sigma, tau, iters, threads=8):
    p = os.path.join(tmpdata, name)
    fd = os.open(p, os.O_RDWR | os.O_CREAT | os.O_TRUNC, 0o600)
    try:
        ret = oracle.permute(fd, data, sigma, tau, iters, threads=threads)
    finally:
        os.close(fd)
    assert (ret == 8192).all()
    return np.fromfile(p, dtype=np.uint8)


def check_ledger(g, ctx, n):
    led = ctx.ledger(reset=True)
    assert len(led) == n
    assert len(set(led[:, 0].tolist())) == n          # one call per block, once
    assert (led[:, 1] == g.NR_PWRITE64).all()
    assert (led[:, 2].view(np.int64) == 8192).all()


@pytest.fixture(scope="module")
def small():
    return synth.permute_set(n_blocks=37)


CELLS = [("WG", "strong", "block"), ("WG", "strong", "nonblock"),
         ("WG", "relaxed", "block"), ("WG", "relaxed", "nonblock")]


@pytest.mark.parametrize("cell", CELLS)
@pytest.mark.parametrize("iters", [0, 1, 5])
def test_permute_cells(gs, tmpdata, small, cell, iters):
    g, ctx = gs
    from paper_1705_06965_amd.permute import PermuteRunner
    want = oracle_file(tmpdata, "perm_oracle_%d.bin" % iters, small.data, small.sigma,
                       small.tau, iters)
    path = os.path.join(tmpdata, "perm_gpu_%s_%s_%d.bin" % (cell[1], cell[2], iters))
    r = PermuteRunner(ctx, path, small.data, small.sigma, small.tau)
    ctx.ledger(reset=True)
    say("permute", cell, iters)
    ret = r.run(iters, *cell)
    if cell[2] == "block":
        assert (ret == 8192).all()
    else:
        assert (ret == g.NOT_WAITED).all()
    got = r.file_bytes()
    assert len(got) == len(want)
    bad = np.nonzero(got != want)[0]
    assert len(bad) == 0, "first differing byte %d (block %d)" % (bad[0], bad[0] // 8192)
    check_ledger(g, ctx, 37)
    r.close()


def test_permute_one_block_and_file_offset(gs, tmpdata):
    g, ctx = gs
    from paper_1705_06965_amd.permute import PermuteRunner
    ps = synth.permute_set(n_blocks=1)
    want = oracle_file(tmpdata, "perm_one.bin", ps.data, ps.sigma, ps.tau, 9)
    path = os.path.join(tmpdata, "perm_one_gpu.bin")
    with open(path, "wb") as f:
        f.write(b"\xa5" * 12288)
    r = PermuteRunner(ctx, path, ps.data, ps.sigma, ps.tau, file_off=4096)
    ctx.ledger(reset=True)
    say("permute one block, offset 4096")
    assert r.run(9, "WG", "relaxed", "block").tolist() == [8192]
    whole = np.fromfile(path, dtype=np.uint8)
    assert (whole[:4096] == 0xa5).all()
    assert np.array_equal(whole[4096:4096 + 8192], want)
    check_ledger(g, ctx, 1)
    r.close()


@pytest.mark.parametrize("cell", [("WG", "strong", "block"), ("WG", "relaxed", "nonblock")])
def test_permute_full_size_sampled(gs, tmpdata, cell):
    """8,192 blocks (64 MiB) at 16 rounds, the benchmark's launch; 48 sampled
    blocks recomputed by the oracle, and every block written once."""
    g, ctx = gs
    from paper_1705_06965_amd.permute import PermuteRunner
    ps = synth.permute_set(n_blocks=8192)
    path = os.path.join(tmpdata, "perm_full_%s_%s.bin" % (cell[1], cell[2]))
    r = PermuteRunner(ctx, path, ps.data, ps.sigma, ps.tau)
    ctx.ledger(reset=True)
    say("permute full", cell)
    ret = r.run(16, *cell)
    assert (ret == (8192 if cell[2] == "block" else g.NOT_WAITED)).all()
    check_ledger(g, ctx, 8192)
    got = r.file_bytes().reshape(8192, 8192)
    pick = np.unique(np.concatenate([[0, 8191], np.random.default_rng(5).integers(0, 8192, 46)]))
    sub = ps.data.reshape(8192, 1024)[pick].ravel()
    want = oracle_file(tmpdata, "perm_full_oracle.bin", sub, ps.sigma, ps.tau, 16)
    assert np.array_equal(got[pick].ravel(), want)
    r.close()


def test_permute_argument_checks(gs, tmpdata, small):
    import torch
    g, ctx = gs
    from paper_1705_06965_amd.permute import PermuteRunner
    path = os.path.join(tmpdata, "perm_args.bin")
    r = PermuteRunner(ctx, path, small.data, small.sigma, small.tau)
    call = lambda sig, tau, n, staging, cell: g.lib.gsys_permute(
        ctx.h, r.fd, r.data.data_ptr(), sig.ctypes.data, tau.ctypes.data, n, 1, staging, 0,
        r.out_ret.data_ptr(), cell, 0)
    wg = g.cell_code("WG", "strong", "block")
    dup = small.sigma.copy()
    dup[7] = dup[8]
    assert call(dup, small.tau, 37, r.staging.dev, wg) == -errno.EINVAL
    big = small.tau.copy()
    big[0] = 64
    assert call(small.sigma, big, 37, r.staging.dev, wg) == -errno.EINVAL
    for c in (g.cell_code("WI", "strong", "block"), g.cell_code("K", "relaxed", "block")):
        assert call(small.sigma, small.tau, 37, r.staging.dev, c) == -errno.EINVAL
    # staging outside every registered buffer, or too short for the blocks
    dev_buf = torch.zeros(37 * 1024, dtype=torch.int64, device="cuda")
    assert call(small.sigma, small.tau, 37, dev_buf.data_ptr(), wg) == -errno.EFAULT
    assert call(small.sigma, small.tau, 38, r.staging.dev, wg) == -errno.EFAULT
    # nothing to do: no launch, no call
    ctx.ledger(reset=True)
    assert call(small.sigma, small.tau, 0, r.staging.dev, wg) == 0
    torch.cuda.synchronize()
    assert ctx.wait(5_000_000_000) == 0
    assert len(ctx.ledger(reset=True)) == 0
    r.close()
