"""GPU parity of the stateful file calls against the oracle, through the C
ABI (gsys_file_roundtrip, gsys_file_kernel_io): read() and write() advance
the file offset, so their results follow the order the calls execute in.

Work-group granularity: every work-group creates its file beneath an allowed
directory with openat, writes it in pieces with write(), closes it, opens it
read-only, reads it back in the same pieces plus one read at the end of the
file, closes it and counts differences.  Every call's result must equal the
oracle's (which issues the same sequence on the CPU), except the descriptor
numbers, which only have to be valid; the files and the bytes read back must
equal the data.  Kernel granularity: consecutive launches append through one
descriptor and then consume the file through another, in launch order."""
import collections
import errno
import os
import sys

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def gs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_06965_amd as g
    ctx = g.Context(ring_slots=1 << 12, device_timeout_ns=20_000_000_000, flags=g.CFG_LEDGER,
                    ledger_capacity=1 << 20)
    yield g, ctx
    assert ctx.shutdown() == 0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("fb,piece,o", [(0, 4096, "strong"), (1, 4096, "relaxed"),
                                        (4097, 4096, "strong"), (100_000, 1000, "relaxed"),
                                        (65_537, 1 << 20, "strong"), (300_000, 65_536, "relaxed")])
def test_roundtrip_matches_oracle(gs, tmpdata, fb, piece, o):
    g, ctx = gs
    from paper_1705_06965_amd.fileio import FileRoundtrip
    names = ["f%02d.bin" % i for i in range(24)]
    data = np.random.default_rng([fb, piece, 5]).integers(0, 256, (len(names), fb),
                                                          dtype=np.uint8)
    d = os.path.join(tmpdata, "gpu_rt_%d_%d_%s" % (fb, piece, o))
    d_cpu = d + "_cpu"
    os.makedirs(d, exist_ok=True)
    os.makedirs(d_cpu, exist_ok=True)
    want, want_back = oracle.file_roundtrip(d_cpu, names, data, piece, threads=8)
    r = FileRoundtrip(ctx, d, names)
    ctx.ledger(reset=True)
    say("roundtrip", fb, piece, o)
    rets, mism, back = r.run(data, piece, o)
    k = (fb + piece - 1) // piece
    fd_cols = [0, k + 2]
    other = [c for c in range(2 * k + 5) if c not in fd_cols]
    assert (rets[:, fd_cols] >= 0).all() and (want[:, fd_cols] >= 0).all()
    assert (rets[:, other] == want[:, other]).all()
    assert not mism.any()
    assert (back == data).all() and (want_back == data).all()
    for f, n in enumerate(names):
        with open(os.path.join(d, n), "rb") as fh:
            assert fh.read() == data[f].tobytes()
    # per file: 2 openat, k writes, k + 1 reads, 2 close, each exactly once
    led = ctx.ledger(reset=True)
    nr = collections.Counter(led[:, 1].tolist())
    nf = len(names)
    assert nr[g.NR_OPENAT] == 2 * nf and nr[g.NR_CLOSE] == 2 * nf
    assert nr[g.NR_WRITE] == k * nf and nr[g.NR_READ] == (k + 1) * nf
    assert len(set(led[:, 0].tolist())) == len(led)
    r.close()


def test_roundtrip_refusals(gs, tmpdata):
    """A name escaping the directory fails its first openat (-EXDEV) and
    nothing else is called for it; with the directory allowed for reading
    only, creating a file is refused (-EPERM)."""
    g, ctx = gs
    from paper_1705_06965_amd.fileio import FileRoundtrip
    d = os.path.join(tmpdata, "gpu_rt_refuse")
    os.makedirs(d, exist_ok=True)
    names = ["ok.bin", "../escape.bin", "sub/missing.bin"]
    data = np.arange(3 * 5000, dtype=np.uint64).astype(np.uint8).reshape(3, 5000)
    r = FileRoundtrip(ctx, d, names)
    say("roundtrip refusals")
    rets, mism, back = r.run(data, 4096, "strong")
    assert rets[0, 0] >= 0 and rets[0, 1:3].tolist() == [4096, 904] and rets[0, 3] == 0
    assert rets[1, 0] == -errno.EXDEV and (rets[1, 1:] == -12345).all()
    assert rets[2, 0] == -errno.ENOENT and (rets[2, 1:] == -12345).all()
    assert not mism.any() and (back[0] == data[0]).all()
    assert not os.path.exists(os.path.join(tmpdata, "escape.bin"))
    ctx.allow_fd(r.dirfd, g.FD_READ | g.FD_DIR)
    say("roundtrip read-only directory")
    rets, mism, _ = r.run(data[:1].repeat(3, axis=0), 4096, "relaxed")
    assert (rets[:, 0] == -errno.EPERM).all() and (rets[:, 1:] == -12345).all()
    r.close()


@pytest.mark.parametrize("grid", [1, 7, 300])
def test_kernel_granularity_append_then_consume(gs, tmpdata, grid):
    g, ctx = gs
    from paper_1705_06965_amd.fileio import kernel_io
    p = os.path.join(tmpdata, "kio_%d.bin" % grid)
    rng = np.random.default_rng(grid)
    parts = [rng.integers(0, 256, n, dtype=np.uint8) for n in (100_000, 1, 3 * 65_536 + 5, 4096)]
    wfd = os.open(p, os.O_WRONLY | os.O_CREAT | os.O_TRUNC, 0o600)
    ctx.allow_fd(wfd, g.FD_WRITE)
    try:
        for i, part in enumerate(parts):
            say("kernel write", grid, i)
            ret, mism = kernel_io(ctx, wfd, g.NR_WRITE, part, grid=grid)
            assert ret == len(part) and mism == 0
    finally:
        ctx.allow_fd(wfd, 0)
        os.close(wfd)
    with open(p, "rb") as fh:
        assert fh.read() == b"".join(x.tobytes() for x in parts)
    rfd = os.open(p, os.O_RDONLY)
    ctx.allow_fd(rfd, g.FD_READ)
    try:
        for i, part in enumerate(parts):
            say("kernel read", grid, i)
            ret, mism = kernel_io(ctx, rfd, g.NR_READ, part, grid=grid)
            assert ret == len(part) and mism == 0
        ret, mism = kernel_io(ctx, rfd, g.NR_READ, np.zeros(16, dtype=np.uint8), grid=grid)
        assert ret == 0 and mism == 0
    finally:
        ctx.allow_fd(rfd, 0)
        os.close(rfd)
