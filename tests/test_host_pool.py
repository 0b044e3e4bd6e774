"""Host service pool on the CPU, driven through the GPU's slot protocol by
host threads (GSYS_CFG_NO_DEVICE contexts).  Results are checked against the
oracle and against the file bytes; the ledger checks exactly-once service."""
import ctypes as C
import errno
import os
import socket

import numpy as np
import pytest

import oracle
import synth
import paper_1705_06965_amd as g
import gsys_hooks as hooks


@pytest.fixture(scope="module")
def datafile(tmpdata):
    os.environ["GSYS_DATA_DIR"] = tmpdata
    p = synth.random_file(2, 4 << 20, name="pool_4m.bin")
    return p


def _ctx(**kw):
    kw.setdefault("flags", 0)
    kw["flags"] |= g.CFG_NO_DEVICE | g.CFG_NO_PIN | g.CFG_LEDGER
    kw.setdefault("service_threads", 4)
    return g.Context(**kw)


def _run(ctx, fd, offs, threads, group, mode, item=4096):
    n = len(offs)
    buf = ctx.host_alloc(n * item)
    lists = ctx.host_alloc(n * 16)
    rets = np.zeros(n, dtype=np.int64)
    offs = np.ascontiguousarray(offs, dtype=np.uint64)
    rc = hooks.lib.gsys_test_emulate(ctx.h, threads, n // threads, group, mode, fd, buf.dev,
                                 lists.dev, item, offs.ctypes.data, rets.ctypes.data,
                                 20_000_000_000)
    assert rc == 0, g.lib.gsys_strerror(rc)
    return buf, rets


@pytest.mark.parametrize("group,mode", [(64, hooks.EMU_BLOCKING), (8, 0), (1, hooks.EMU_BLOCKING),
                                        (64, hooks.EMU_LIST | hooks.EMU_BLOCKING), (16, hooks.EMU_LIST)])
def test_emulated_wavefronts_match_oracle(datafile, group, mode):
    n_blocks = (4 << 20) // 4096
    offs = synth.sweep_offsets(2048, n_blocks)
    want_fnv, want_ret = oracle.pread_fnv(datafile, offs, 4096)
    fd = os.open(datafile, os.O_RDONLY)
    ctx = _ctx(ring_slots=1024)
    try:
        ctx.allow_fd(fd, g.FD_READ)
        buf, rets = _run(ctx, fd, offs, 8, group, mode)
        assert (rets == want_ret).all()
        data = buf.view(np.uint8).reshape(len(offs), 4096)
        got = np.array([oracle.fnv1a64(data[i]) for i in range(len(offs))], dtype=np.uint64)
        assert (got == want_fnv).all()
        assert ctx.wait(5_000_000_000) == 0
        led = ctx.ledger()
        st = ctx.stats()
        claimed = st["claimed"]
        # exactly once: every claimed ticket serviced once, nothing else
        assert len(led) == claimed
        assert (np.sort(led[:, 0]) == np.arange(claimed, dtype=np.uint64)).all()
        if mode & hooks.EMU_LIST:
            assert claimed == len(offs) // group
            assert st["host_calls"] <= len(offs)
        else:
            assert claimed == len(offs)
            assert st["host_calls"] == len(offs)
    finally:
        assert ctx.shutdown() == 0
        os.close(fd)


def test_tiny_ring_back_pressure_and_quiescence(datafile):
    """D = 64 with 8 emulated wavefronts of 64: every claim wraps the ring."""
    offs = synth.sweep_offsets(4096, 1024)
    want_fnv, want_ret = oracle.pread_fnv(datafile, offs, 256)
    fd = os.open(datafile, os.O_RDONLY)
    ctx = _ctx(ring_slots=64, service_threads=3)
    try:
        ctx.allow_fd(fd, g.FD_READ)
        buf, rets = _run(ctx, fd, offs, 8, 64, hooks.EMU_BLOCKING, item=256)
        assert (rets == 256).all()
        data = buf.view(np.uint8).reshape(len(offs), 256)
        for i in range(0, len(offs), 97):
            assert oracle.fnv1a64(data[i]) == want_fnv[i]
        assert ctx.wait(5_000_000_000) == 0
        st = ctx.stats()
        assert st["claimed"] == 4096 and st["retired_lo"] == 4096
        ctl = np.zeros(64, dtype=np.uint64)
        hooks.lib.gsys_test_ring_ctl(ctx.h, ctl.ctypes.data, 64)
        # quiescent: every slot FREE for its next lap
        t = np.arange(64, dtype=np.uint64) + np.uint64(4096)
        assert (ctl == (t << np.uint64(3))).all()
    finally:
        ctx.shutdown()
        os.close(fd)


def test_coalescing_merges_adjacent_reads(datafile):
    offs = np.arange(1024, dtype=np.uint64) * np.uint64(4096)
    fd = os.open(datafile, os.O_RDONLY)
    ctx = _ctx(ring_slots=4096, service_threads=2, coalesce_max=8, coalesce_window_ns=200_000)
    try:
        ctx.allow_fd(fd, g.FD_READ)
        buf, rets = _run(ctx, fd, offs, 1, 64, hooks.EMU_BLOCKING)
        assert (rets == 4096).all()
        assert buf.view(np.uint8)[:4 << 20].tobytes() == open(datafile, "rb").read()
        st = ctx.stats()
        assert st["merged"] > 0
        assert st["host_calls"] < 1024
        assert sum(st["bundle_hist"][1:]) > 0
    finally:
        ctx.shutdown()
        os.close(fd)


def test_short_reads_at_eof(tmpdata):
    p = os.path.join(tmpdata, "short.bin")
    data = np.random.default_rng(5).integers(0, 256, 10000, dtype=np.uint8).tobytes()
    open(p, "wb").write(data)
    offs = np.array([0, 4096, 8192, 9999, 10000, 12288, 5904, 5905], dtype=np.uint64)
    want_fnv, want_ret = oracle.pread_fnv(p, offs, 4096)
    fd = os.open(p, os.O_RDONLY)
    ctx = _ctx()
    try:
        ctx.allow_fd(fd, g.FD_READ)
        for mode in (hooks.EMU_BLOCKING, hooks.EMU_LIST | hooks.EMU_BLOCKING):
            buf, rets = _run(ctx, fd, offs, 1, 8, mode)
            assert rets.tolist() == want_ret.tolist()
            d = buf.view(np.uint8).reshape(8, 4096)
            for i in range(8):
                assert oracle.fnv1a64(d[i, :max(0, rets[i])]) == want_fnv[i]
    finally:
        ctx.shutdown()
        os.close(fd)


def _raw(ctx, nr, args, flags=g.F_BLOCKING):
    a = np.array([int(x) & 0xFFFFFFFFFFFFFFFF for x in args] + [0] * (6 - len(args)),
                 dtype=np.uint64)
    r = np.zeros(1, dtype=np.int64)
    rc = hooks.lib.gsys_test_raw_call(ctx.h, nr, flags, a.ctypes.data, r.ctypes.data, 5_000_000_000)
    assert rc == 0
    return int(r[0])


def test_whitelist_rejects(datafile):
    fd = os.open(datafile, os.O_RDONLY)
    wfd = os.open(os.path.join(os.path.dirname(datafile), "w.bin"), os.O_RDWR | os.O_CREAT, 0o600)
    ctx = _ctx(arena_bytes=8 << 20)
    try:
        buf = ctx.host_alloc(8192)
        # fd not allowed yet
        assert _raw(ctx, g.NR_PREAD64, [fd, buf.dev, 16, 0]) == -errno.EBADF
        ctx.allow_fd(fd, g.FD_READ)
        assert _raw(ctx, g.NR_PREAD64, [fd, buf.dev, 16, 0]) == 16
        # read-only fd used for pwrite
        assert _raw(ctx, g.NR_PWRITE64, [fd, buf.dev, 16, 0]) == -errno.EBADF
        # range outside any registered buffer
        assert _raw(ctx, g.NR_PREAD64, [fd, buf.dev + 8000, 4096, 0]) == -errno.EFAULT
        assert _raw(ctx, g.NR_PREAD64, [fd, 0x1000, 16, 0]) == -errno.EFAULT
        # calls outside the whitelist
        for nr in (2, 57, 59, 62, 85):  # open, fork, execve, kill, creat
            assert _raw(ctx, nr, [0, 0, 0]) == -errno.EPERM
        # close: only descriptors a GPU openat opened (never the caller's)
        assert _raw(ctx, g.NR_CLOSE, [0]) == -errno.EBADF
        assert _raw(ctx, g.NR_CLOSE, [fd]) == -errno.EBADF
        # madvise: only MADV_DONTNEED, only inside the arena
        assert _raw(ctx, g.NR_MADVISE, [buf.dev & ~4095, 4096, 8]) == -errno.EINVAL  # MADV_FREE
        assert _raw(ctx, g.NR_MADVISE, [buf.dev & ~4095, 4096, 4]) == -errno.EFAULT  # not arena
        # revoke
        ctx.allow_fd(fd, 0)
        assert _raw(ctx, g.NR_PREAD64, [fd, buf.dev, 16, 0]) == -errno.EBADF
        ctx.allow_fd(wfd, g.FD_WRITE)
        buf.array[:16] = np.arange(16, dtype=np.uint8)
        assert _raw(ctx, g.NR_PWRITE64, [wfd, buf.dev, 16, 100]) == 16
        assert os.pread(wfd, 16, 100) == bytes(range(16))
        st = ctx.stats()
        assert st["rejected"] == 5
        assert st["errno_hist"][0] == 5 and st["errno_hist"][1] >= 3
    finally:
        ctx.shutdown()
        os.close(fd)
        os.close(wfd)


def test_arena_mmap_madvise_munmap(datafile):
    """mmap inside the arena, fill it with pread, read it back with pwrite,
    madvise(MADV_DONTNEED) -> zero pages (madvise(2)), munmap."""
    fd = os.open(datafile, os.O_RDONLY)
    outp = os.path.join(os.path.dirname(datafile), "arena_out.bin")
    wfd = os.open(outp, os.O_RDWR | os.O_CREAT | os.O_TRUNC, 0o600)
    ctx = _ctx(arena_bytes=16 << 20)
    try:
        ctx.allow_fd(fd, g.FD_READ)
        ctx.allow_fd(wfd, g.FD_WRITE)
        base = _raw(ctx, g.NR_MMAP, [0, 2 << 20, 3, 0x22, -1, 0])  # outside the arena
        assert base == -errno.EFAULT
        arena = ctx.device_ctx().arena
        assert arena == ctx_arena_base(ctx)
        # file-backed or shared mappings are refused
        assert _raw(ctx, g.NR_MMAP, [arena, 2 << 20, 3, 0x01, fd, 0]) == -errno.EINVAL
        addr = _raw(ctx, g.NR_MMAP, [arena, 2 << 20, 3, 0x22 | 0x10, -1, 0])
        assert addr == arena
        assert _raw(ctx, g.NR_PREAD64, [fd, addr, 2 << 20, 0]) == 2 << 20
        assert _raw(ctx, g.NR_PWRITE64, [wfd, addr, 2 << 20, 0]) == 2 << 20
        assert os.pread(wfd, 2 << 20, 0) == open(datafile, "rb").read(2 << 20)
        assert _raw(ctx, g.NR_MADVISE, [addr, 2 << 20, 4], flags=0) == 0
        assert _raw(ctx, g.NR_PWRITE64, [wfd, addr, 2 << 20, 0]) == 2 << 20
        assert os.pread(wfd, 2 << 20, 0) == bytes(2 << 20)
        assert _raw(ctx, g.NR_MUNMAP, [addr, 2 << 20]) == 0
        # after munmap the range is reserved again: reading into it faults
        assert _raw(ctx, g.NR_PREAD64, [fd, addr, 4096, 0]) == -errno.EFAULT
    finally:
        ctx.shutdown()
        os.close(fd)
        os.close(wfd)


def ctx_arena_base(ctx):
    # the arena is the only 2 MiB-aligned PROT_NONE reservation of its size;
    # read it from /proc/self/maps
    want = ctx.cfg.arena_bytes
    for line in open("/proc/self/maps"):
        rng, perms = line.split()[:2]
        lo, hi = (int(x, 16) for x in rng.split("-"))
        if perms.startswith("---p") and hi - lo == want and lo % (2 << 20) == 0:
            return lo
    raise AssertionError("arena not found")


def test_udp_loopback_sendto_recvfrom():
    srv = socket.socket(socket.AF_INET, socket.SOCK_DGRAM)
    srv.bind(("127.0.0.1", 0))
    cli = socket.socket(socket.AF_INET, socket.SOCK_DGRAM)
    cli.bind(("127.0.0.1", 0))
    ctx = _ctx()
    try:
        ctx.allow_fd(srv.fileno(), g.FD_SOCK)
        buf = ctx.host_alloc(4096)
        # empty socket: recvfrom never blocks a poller
        assert _raw(ctx, g.NR_RECVFROM, [srv.fileno(), buf.dev, 2048, 0, buf.dev + 2048, 0]) \
            == -errno.EAGAIN
        cli.sendto(b"hello gpu", srv.getsockname())
        import time
        time.sleep(0.05)
        n = _raw(ctx, g.NR_RECVFROM, [srv.fileno(), buf.dev, 2048, 0, buf.dev + 2048, 0])
        assert n == 9 and buf.array[:9].tobytes() == b"hello gpu"
        # reply to the sender address that recvfrom filled in
        buf.array[:5] = np.frombuffer(b"reply", dtype=np.uint8)
        assert _raw(ctx, g.NR_SENDTO, [srv.fileno(), buf.dev, 5, 0, buf.dev + 2048, 16]) == 5
        assert cli.recvfrom(64)[0] == b"reply"
        # non-loopback destination refused
        sa = buf.view(np.uint8, 16, 2048).copy()
        sa[4:8] = [8, 8, 8, 8]
        buf.array[3072:3088] = sa
        assert _raw(ctx, g.NR_SENDTO, [srv.fileno(), buf.dev, 5, 0, buf.dev + 3072, 16]) \
            == -errno.EINVAL
    finally:
        ctx.shutdown()
        srv.close()
        cli.close()


def test_drain_times_out_on_unpublished_claims():
    ctx = _ctx()
    t = hooks.lib.gsys_test_claim_only(ctx.h, 3)
    assert t == 0
    assert ctx.wait(50_000_000) == -errno.ETIMEDOUT
    assert ctx.shutdown(50_000_000) == -errno.ETIMEDOUT


def test_exported_symbols_exist():
    """libgsys.so exports every function include/ declares and none of the
    test hooks; the hook library exports every hook its header declares."""
    names = g.exported_symbols()
    assert "gsys_init" in names and "gsys_fnv4k" in names and "gsys_serve_run_noalloc" in names
    assert not [n for n in names if n.startswith("gsys_test_")]
    for n in names:
        assert hasattr(g.lib, n), n
    import subprocess
    dyn = subprocess.run(["nm", "-D", "--defined-only", g.LIB_PATH], capture_output=True,
                         text=True).stdout
    assert "gsys_test_" not in dyn
    hook_names = hooks.declared()
    assert "gsys_test_emulate" in hook_names and "gsys_test_inject" in hook_names
    for n in hook_names:
        assert hasattr(hooks.lib, n), n


def test_binding_arity_matches_the_header():
    """Every function include/gsys.h declares is bound with as many argument
    types as its prototype has parameters (the ctypes layer cannot check
    this itself: a missing or extra argument would shift every later one)."""
    import re
    src = open(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                            "include", "gsys.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    protos = re.findall(r"^[A-Za-z_][A-Za-z0-9_ ]*?[\s*]+(gsys_\w+)\s*\(([^;]*?)\)\s*;", src,
                        flags=re.M | re.S)
    assert len(protos) >= 25
    for name, params in protos:
        params = " ".join(params.split())
        n = 0 if params in ("", "void") else params.count(",") + 1
        f = getattr(g.lib, name)
        assert f.argtypes is not None and len(f.argtypes) == n, (name, n, f.argtypes)


def _links_to(path):
    """Open descriptors of this process that refer to `path`."""
    real = os.path.realpath(path)
    n = 0
    for name in os.listdir("/proc/self/fd"):
        try:
            if os.readlink("/proc/self/fd/" + name) == real:
                n += 1
        except OSError:
            pass
    return n


@pytest.mark.parametrize("shared", [False, True])
def test_per_thread_file_copies(datafile, shared):
    """Positional calls on a regular file run through each service thread's
    own open file description (unless GSYS_CFG_SHARED_FDS): the results are
    the same either way, and the copies are closed when the pool stops."""
    offs = synth.sweep_offsets(1024, (4 << 20) // 4096)
    want_fnv, want_ret = oracle.pread_fnv(datafile, offs, 4096)
    fd = os.open(datafile, os.O_RDONLY)
    base = _links_to(datafile)
    ctx = _ctx(ring_slots=1024, flags=g.CFG_SHARED_FDS if shared else 0)
    try:
        ctx.allow_fd(fd, g.FD_READ)
        buf, rets = _run(ctx, fd, offs, 8, 1, hooks.EMU_BLOCKING)
        assert (rets == want_ret).all()
        data = buf.view(np.uint8).reshape(len(offs), 4096)
        got = np.array([oracle.fnv1a64(data[i]) for i in range(len(offs))], dtype=np.uint64)
        assert (got == want_fnv).all()
        copies = _links_to(datafile) - base
        if shared:
            assert copies == 0
        else:
            assert 1 <= copies <= 4          # at most one per service thread
    finally:
        assert ctx.shutdown() == 0
    assert _links_to(datafile) == base
    os.close(fd)


def test_reused_fd_number_reads_the_new_file(tmpdata):
    """A thread's copy belongs to the file the fd number named when it was
    made: after the number is revoked, closed and re-allowed for another
    file, calls read the new file."""
    a = os.path.join(tmpdata, "fd_a.bin")
    b = os.path.join(tmpdata, "fd_b.bin")
    open(a, "wb").write(b"A" * 8192)
    open(b, "wb").write(b"B" * 8192)
    ctx = _ctx(ring_slots=256, service_threads=2)
    fa = os.open(a, os.O_RDONLY)
    try:
        ctx.allow_fd(fa, g.FD_READ)
        offs = np.zeros(64, dtype=np.uint64)
        buf, rets = _run(ctx, fa, offs, 4, 1, hooks.EMU_BLOCKING)
        assert (rets == 4096).all() and (buf.view(np.uint8)[:64 * 4096] == ord("A")).all()
        ctx.allow_fd(fa, 0)
        fb = os.open(b, os.O_RDONLY)
        os.dup2(fb, fa)                       # the same number now names fd_b.bin
        os.close(fb)
        ctx.allow_fd(fa, g.FD_READ)
        buf2, rets2 = _run(ctx, fa, offs, 4, 1, hooks.EMU_BLOCKING)
        assert (rets2 == 4096).all() and (buf2.view(np.uint8)[:64 * 4096] == ord("B")).all()
    finally:
        assert ctx.shutdown() == 0
        os.close(fa)


def test_copies_keep_append_and_write_modes(tmpdata):
    """pwrite through a copy writes the caller's file; a write-only fd's copy
    is write-only (a pread on it is refused by the kernel, as on the
    original)."""
    p = os.path.join(tmpdata, "fd_w.bin")
    fd = os.open(p, os.O_WRONLY | os.O_CREAT | os.O_TRUNC, 0o600)
    ctx = _ctx(ring_slots=256, service_threads=2)
    try:
        ctx.allow_fd(fd, g.FD_READ | g.FD_WRITE)
        src = ctx.host_alloc(4096)
        src.array[:4096] = np.arange(4096, dtype=np.uint64).astype(np.uint8)
        ret = C.c_int64(0)
        args = (C.c_uint64 * 6)(fd, src.dev, 4096, 8192, 0, 0)
        assert hooks.lib.gsys_test_raw_call(ctx.h, g.NR_PWRITE64, g.F_BLOCKING, args, C.byref(ret),
                                        5_000_000_000) == 0
        assert ret.value == 4096
        got = open(p, "rb").read()
        assert len(got) == 12288 and got[8192:] == src.array[:4096].tobytes()
        args = (C.c_uint64 * 6)(fd, src.dev, 4096, 0, 0, 0)
        assert hooks.lib.gsys_test_raw_call(ctx.h, g.NR_PREAD64, g.F_BLOCKING, args, C.byref(ret),
                                        5_000_000_000) == 0
        assert ret.value == -errno.EBADF
    finally:
        assert ctx.shutdown() == 0
        os.close(fd)


def _path(ctx, name: bytes):
    b = ctx.host_alloc(g.PATH_MAX)
    b.array[:g.PATH_MAX] = 0
    b.array[:len(name)] = np.frombuffer(name, dtype=np.uint8)
    return b


def test_openat_read_close_beneath_an_allowed_directory(tmpdata):
    """openat resolves beneath a GSYS_FD_DIR directory, the new fd reads
    sequentially (the file offset advances), close gives it back; escapes,
    unknown flags, writes into a read-only directory and foreign closes are
    refused."""
    d = os.path.join(tmpdata, "opendir")
    os.makedirs(os.path.join(d, "sub"), exist_ok=True)
    body = bytes(range(256)) * 64
    open(os.path.join(d, "sub", "f.bin"), "wb").write(body)
    open(os.path.join(tmpdata, "outside.bin"), "wb").write(b"secret")
    link = os.path.join(d, "escape")
    if not os.path.lexists(link):
        os.symlink(os.path.join(tmpdata, "outside.bin"), link)
    dfd = os.open(d, os.O_RDONLY | os.O_DIRECTORY)
    ctx = _ctx(ring_slots=256, service_threads=2)
    try:
        buf = ctx.host_alloc(1 << 16)
        good = _path(ctx, b"sub/f.bin")
        # the directory must be allowed, and as a directory
        assert _raw(ctx, g.NR_OPENAT, [dfd, good.dev, os.O_RDONLY, 0]) == -errno.EBADF
        ffd = os.open(os.path.join(d, "sub", "f.bin"), os.O_RDONLY)
        with pytest.raises(g.GsysError) as ei:
            ctx.allow_fd(ffd, g.FD_READ | g.FD_DIR)
        assert ei.value.errno == errno.ENOTDIR
        os.close(ffd)
        ctx.allow_fd(dfd, g.FD_READ | g.FD_DIR)
        fd = _raw(ctx, g.NR_OPENAT, [dfd, good.dev, os.O_RDONLY, 0])
        assert fd >= 0
        # read() advances the file offset: two reads return consecutive bytes
        assert _raw(ctx, g.NR_READ, [fd, buf.dev, 4000]) == 4000
        assert _raw(ctx, g.NR_READ, [fd, buf.dev + 4000, 1 << 14]) == len(body) - 4000
        assert _raw(ctx, g.NR_READ, [fd, buf.dev, 16]) == 0          # end of file
        assert buf.array[:len(body)].tobytes() == body
        # a read-only open cannot write
        assert _raw(ctx, g.NR_WRITE, [fd, buf.dev, 16]) == -errno.EBADF
        assert _raw(ctx, g.NR_CLOSE, [fd]) == 0
        assert _raw(ctx, g.NR_CLOSE, [fd]) == -errno.EBADF        # already closed
        assert _raw(ctx, g.NR_READ, [fd, buf.dev, 16]) == -errno.EBADF
        # escapes: absolute path, "..", a symlink out of the directory
        for bad in (b"/etc/hostname", b"../outside.bin", b"sub/../../outside.bin", b"escape"):
            p = _path(ctx, bad)
            r = _raw(ctx, g.NR_OPENAT, [dfd, p.dev, os.O_RDONLY, 0])
            assert r in (-errno.EXDEV, -errno.ELOOP), (bad, r)
        # flags outside the whitelist; writing into a read-only directory
        assert _raw(ctx, g.NR_OPENAT, [dfd, good.dev, os.O_RDONLY | os.O_DIRECTORY, 0]) == -errno.EINVAL
        assert _raw(ctx, g.NR_OPENAT, [dfd, good.dev, os.O_RDONLY | 0o10000000, 0]) == -errno.EINVAL
        assert _raw(ctx, g.NR_OPENAT, [dfd, good.dev, os.O_WRONLY, 0]) == -errno.EPERM
        new = _path(ctx, b"made.bin")
        assert _raw(ctx, g.NR_OPENAT, [dfd, new.dev, os.O_WRONLY | os.O_CREAT, 0o644]) == -errno.EPERM
        # a path without a NUL in GSYS_PATH_MAX bytes, a path outside any buffer
        long = ctx.host_alloc(g.PATH_MAX)
        long.array[:g.PATH_MAX] = ord("a")
        assert _raw(ctx, g.NR_OPENAT, [dfd, long.dev, os.O_RDONLY, 0]) == -errno.ENAMETOOLONG
        assert _raw(ctx, g.NR_OPENAT, [dfd, 0x1000, os.O_RDONLY, 0]) == -errno.EFAULT
        # a writable directory: create, write, read back through the caller
        ctx.allow_fd(dfd, g.FD_READ | g.FD_WRITE | g.FD_DIR)
        wfd = _raw(ctx, g.NR_OPENAT, [dfd, new.dev, os.O_WRONLY | os.O_CREAT | os.O_TRUNC, 0o600])
        assert wfd >= 0
        assert _raw(ctx, g.NR_WRITE, [wfd, buf.dev, 100]) == 100
        assert _raw(ctx, g.NR_WRITE, [wfd, buf.dev + 100, 28]) == 28
        assert _raw(ctx, g.NR_READ, [wfd, buf.dev, 16]) == -errno.EBADF   # write-only
        assert _raw(ctx, g.NR_CLOSE, [wfd]) == 0
        assert open(os.path.join(d, "made.bin"), "rb").read() == body[:128]
        assert (os.stat(os.path.join(d, "made.bin")).st_mode & 0o777) == 0o600
        # an fd left open is closed by the pool at shutdown
        left = _raw(ctx, g.NR_OPENAT, [dfd, good.dev, os.O_RDONLY, 0])
        assert left >= 0 and os.readlink("/proc/self/fd/%d" % left).endswith("sub/f.bin")
    finally:
        assert ctx.shutdown() == 0
        os.close(dfd)
    assert not os.path.exists("/proc/self/fd/%d" % left) or \
        not os.readlink("/proc/self/fd/%d" % left).endswith("sub/f.bin")


NETDESC = np.dtype([("buf_off", "<u4"), ("len_ret", "<i4"), ("addr_len", "<u4"), ("pad", "<u4"),
                    ("addr", "u1", 16)])


def test_socket_lists_keep_per_datagram_semantics():
    """Receive and send lists run as batched kernel calls but keep the
    one-call-per-descriptor results: datagrams in order, truncation to the
    buffer, -EINVAL / -EFAULT for bad descriptors without ending the list,
    -EAGAIN for every receive after the socket is drained, -EINVAL for a
    non-loopback destination, more than one batch per list."""
    import time
    srv = socket.socket(socket.AF_INET, socket.SOCK_DGRAM)
    srv.setsockopt(socket.SOL_SOCKET, socket.SO_RCVBUF, 1 << 22)
    srv.bind(("127.0.0.1", 0))
    cli = socket.socket(socket.AF_INET, socket.SOCK_DGRAM)
    cli.bind(("127.0.0.1", 0))
    ctx = _ctx()
    try:
        ctx.allow_fd(srv.fileno(), g.FD_SOCK)
        n_dgram, n_desc = 150, 200
        payload = [bytes([i % 251]) * (1 + (i * 37) % 300) for i in range(n_dgram)]
        for p in payload:
            cli.sendto(p, srv.getsockname())
        time.sleep(0.1)
        bufs = ctx.host_alloc(n_desc * 512)
        lst = ctx.host_alloc(n_desc * NETDESC.itemsize)
        d = np.zeros(n_desc, dtype=NETDESC)
        d["buf_off"] = np.arange(n_desc) * 512
        d["len_ret"] = 512
        d["len_ret"][10] = -1                       # invalid length
        d["buf_off"][20] = 1 << 30                  # outside any registered buffer
        d["len_ret"][30] = 8                        # shorter than its datagram
        lst.array[:d.nbytes] = d.view(np.uint8)
        r = _raw(ctx, g.NR_RECVFROM, [srv.fileno(), lst.dev, n_desc, bufs.dev, 0],
                 flags=g.F_BLOCKING | g.F_LIST)
        out = lst.array[:d.nbytes].view(NETDESC)
        got = out["len_ret"]
        assert r == int(got[got > 0].sum())         # the list ran: the bytes it moved
        assert got[10] == -errno.EINVAL and got[20] == -errno.EFAULT
        valid = [i for i in range(n_desc) if i not in (10, 20)]
        for k, i in enumerate(valid):
            if k < n_dgram:
                want = min(len(payload[k]), 8 if i == 30 else 512)
                assert got[i] == want, (i, k)
                assert bufs.array[i * 512:i * 512 + want].tobytes() == payload[k][:want]
            else:
                assert got[i] == -errno.EAGAIN, i
        # send back to the recorded senders; one destination is not loopback
        s = np.zeros(n_dgram, dtype=NETDESC)
        s["buf_off"] = np.array(valid[:n_dgram]) * 512
        s["len_ret"] = [min(len(payload[k]), 8 if valid[k] == 30 else 512) for k in range(n_dgram)]
        s["addr_len"] = out["addr_len"][valid[:n_dgram]]
        s["addr"] = out["addr"][valid[:n_dgram]]
        s["addr"][5, 4:8] = [8, 8, 8, 8]
        lst.array[:s.nbytes] = s.view(np.uint8)
        r = _raw(ctx, g.NR_SENDTO, [srv.fileno(), lst.dev, n_dgram, bufs.dev, 0],
                 flags=g.F_BLOCKING | g.F_LIST)
        sent = lst.array[:s.nbytes].view(NETDESC)["len_ret"]
        assert r == int(sent[sent > 0].sum())
        assert sent[5] == -errno.EINVAL
        assert (np.delete(sent, 5) == np.delete(s["len_ret"], 5)).all()
        cli.settimeout(2.0)
        echoed = [cli.recvfrom(1024)[0] for _ in range(n_dgram - 1)]
        want = [payload[k][:s["len_ret"][k]] for k in range(n_dgram) if k != 5]
        assert echoed == want
        st = ctx.stats()
        assert st["merged"] > 0                      # datagrams shared kernel calls
    finally:
        ctx.shutdown()
        srv.close()
        cli.close()


def test_doorbell_wakes_blocked_pollers(datafile, monkeypatch):
    """Idle pollers block on the doorbell; every call after a pause is still
    served, and woken by the doorbell rather than the backstop: the backstop
    is raised to 30 s, so one lost wake-up times the call out (5 s)."""
    import time
    monkeypatch.setenv("GSYS_DOORBELL_BACKSTOP_US", str(30_000_000))
    data = np.fromfile(datafile, dtype=np.uint8)
    fd = os.open(datafile, os.O_RDONLY)
    ctx = _ctx(flags=g.CFG_DOORBELL, doorbell_idle_us=100)
    try:
        ctx.allow_fd(fd, g.FD_READ)
        buf = ctx.host_alloc(4096)
        for i in range(30):
            time.sleep(0.004)  # every poller has time to block
            off = (i * 7919 % 1024) * 4096
            assert _raw(ctx, g.NR_PREAD64, [fd, buf.dev, 4096, off]) == 4096
            assert (buf.view(np.uint8)[:4096] == data[off:off + 4096]).all()
        st = ctx.stats()
        assert st["doorbell_sleeps"] >= 30
        assert st["requests"] == 30
    finally:
        assert ctx.shutdown() == 0
        os.close(fd)


def test_doorbell_races_with_callers(datafile, monkeypatch):
    """Calls arrive at random moments around the pollers' decision to block
    (idle threshold 20 us, gaps of 0-300 us), from wavefront-sized groups
    and single calls; results match the oracle and nothing waits for the
    30 s backstop."""
    import time
    monkeypatch.setenv("GSYS_DOORBELL_BACKSTOP_US", str(30_000_000))
    rng = np.random.default_rng(7)
    n_blocks = (4 << 20) // 4096
    fd = os.open(datafile, os.O_RDONLY)
    ctx = _ctx(flags=g.CFG_DOORBELL, doorbell_idle_us=20, ring_slots=1024)
    try:
        ctx.allow_fd(fd, g.FD_READ)
        for burst in range(12):
            offs = synth.sweep_offsets(256, n_blocks, config=10 + burst)
            want_fnv, want_ret = oracle.pread_fnv(datafile, offs, 4096)
            group, mode = [(64, hooks.EMU_BLOCKING), (1, 0), (16, hooks.EMU_LIST)][burst % 3]
            buf, rets = _run(ctx, fd, offs, 4, group, mode)
            assert (rets == want_ret).all()
            data = buf.view(np.uint8).reshape(len(offs), 4096)
            got = np.array([oracle.fnv1a64(data[i]) for i in range(len(offs))], dtype=np.uint64)
            assert (got == want_fnv).all()
            buf.free()
            time.sleep(float(rng.uniform(0, 300e-6)))
        data = np.fromfile(datafile, dtype=np.uint8)
        one = ctx.host_alloc(4096)
        for i in range(300):
            time.sleep(float(rng.uniform(0, 300e-6)))
            off = int(rng.integers(0, n_blocks)) * 4096
            assert _raw(ctx, g.NR_PREAD64, [fd, one.dev, 4096, off]) == 4096
            assert (one.view(np.uint8)[:4096] == data[off:off + 4096]).all()
        assert ctx.wait(5_000_000_000) == 0
        assert ctx.stats()["doorbell_sleeps"] > 0
    finally:
        assert ctx.shutdown() == 0
        os.close(fd)


def test_no_doorbell_no_sleeps(datafile):
    ctx = _ctx()
    try:
        fd = os.open(datafile, os.O_RDONLY)
        ctx.allow_fd(fd, g.FD_READ)
        buf = ctx.host_alloc(4096)
        assert _raw(ctx, g.NR_PREAD64, [fd, buf.dev, 4096, 0]) == 4096
        assert ctx.stats()["doorbell_sleeps"] == 0
        os.close(fd)
    finally:
        ctx.shutdown()


def test_idle_pollers_take_requests_from_a_busy_stripe(tmpdata):
    """Ticket 0 is a 256 MiB pread that keeps the owner of stripe 0 busy; the
    7 small preads that follow it in the same stripe (tickets 1..7) are
    served by the other, idle pollers long before it ends."""
    import threading
    import time
    p = os.path.join(tmpdata, "big_256m.bin")
    with open(p, "wb") as f:
        f.write(np.random.default_rng(3).integers(0, 256, 256 << 20, dtype=np.uint8).tobytes())
    fd = os.open(p, os.O_RDONLY)
    ctx = _ctx(service_threads=4, ring_slots=64)
    try:
        ctx.allow_fd(fd, g.FD_READ)
        big = ctx.host_alloc(256 << 20)
        small = ctx.host_alloc(7 * 4096)
        t_big = []

        def big_call():
            t0 = time.perf_counter()
            assert _raw(ctx, g.NR_PREAD64, [fd, big.dev, 256 << 20, 0]) == 256 << 20
            t_big.append(time.perf_counter() - t0)

        th = threading.Thread(target=big_call)
        th.start()
        time.sleep(0.002)  # ticket 0 is in service
        t_small = []
        for i in range(7):
            t0 = time.perf_counter()
            assert _raw(ctx, g.NR_PREAD64, [fd, small.dev + 4096 * i, 4096, 4096 * (i + 1)]) == 4096
            t_small.append(time.perf_counter() - t0)
        th.join()
        assert max(t_small) < t_big[0] / 4, (t_small, t_big)
        led = ctx.ledger()
        assert sorted(led[:, 0].tolist()) == list(range(8))
        owner = int(led[led[:, 0] == 0][0, 5]) & 0xff
        thieves = {int(x) & 0xff for x in led[led[:, 0] > 0][:, 5]}
        assert owner not in thieves
        data = np.fromfile(p, dtype=np.uint8, count=8 * 4096)
        assert (small.view(np.uint8)[:7 * 4096] == data[4096:8 * 4096]).all()
    finally:
        assert ctx.shutdown() == 0
        os.close(fd)


def test_injected_errno_reaches_the_caller(datafile):
    """With -EIO injected for the next 5 preads, exactly 5 of a wavefront's
    64 emulated calls return -EIO and the other 59 read their bytes; the
    errno histogram counts the 5 under 'other'."""
    fd = os.open(datafile, os.O_RDONLY)
    ctx = _ctx(ring_slots=256)
    try:
        ctx.allow_fd(fd, g.FD_READ)
        assert hooks.lib.gsys_test_inject(ctx.h, g.NR_PREAD64, errno.EIO, 5) == 0
        offs = synth.sweep_offsets(64, (4 << 20) // 4096)
        buf, rets = _run(ctx, fd, offs, 1, 64, hooks.EMU_BLOCKING)
        assert (rets == -errno.EIO).sum() == 5
        ok = rets != -errno.EIO
        assert (rets[ok] == 4096).all()
        data = np.fromfile(datafile, dtype=np.uint8)
        got = buf.view(np.uint8).reshape(64, 4096)
        for i in np.nonzero(ok)[0]:
            assert (got[i] == data[int(offs[i]):int(offs[i]) + 4096]).all()
        assert ctx.stats()["errno_hist"][7] == 5
        # used up: the next call runs normally
        assert _raw(ctx, g.NR_PREAD64, [fd, buf.dev, 16, 0]) == 16
        assert hooks.lib.gsys_test_inject(ctx.h, g.NR_PREAD64, 0, 1) == -errno.EINVAL
    finally:
        ctx.shutdown()
        os.close(fd)


def test_injected_errno_fails_a_whole_list(datafile):
    """A fault injected for a descriptor-list call fails the whole call
    before anything runs: the call returns -EIO and every descriptor keeps
    what the caller wrote; the next list runs normally."""
    fd = os.open(datafile, os.O_RDONLY)
    ctx = _ctx(ring_slots=256)
    try:
        ctx.allow_fd(fd, g.FD_READ)
        buf = ctx.host_alloc(8 * 4096)
        lst = ctx.host_alloc(8 * 16)
        d = np.zeros(8, dtype=[("off", "<u8"), ("buf_off", "<u4"), ("len_ret", "<i4")])
        d["off"] = np.arange(8) * 8192
        d["buf_off"] = np.arange(8) * 4096
        d["len_ret"] = 4096
        lst.array[:d.nbytes] = d.view(np.uint8)
        assert hooks.lib.gsys_test_inject(ctx.h, g.NR_PREAD64, errno.EIO, 1) == 0
        r = _raw(ctx, g.NR_PREAD64, [fd, lst.dev, 8, buf.dev], flags=g.F_BLOCKING | g.F_LIST)
        assert r == -errno.EIO
        assert (lst.array[:d.nbytes].view(d.dtype)["len_ret"] == 4096).all()
        assert not buf.array.any()
        assert ctx.stats()["errno_hist"][7] == 1
        r = _raw(ctx, g.NR_PREAD64, [fd, lst.dev, 8, buf.dev], flags=g.F_BLOCKING | g.F_LIST)
        assert r == 8 * 4096
        data = np.fromfile(datafile, dtype=np.uint8)
        for i in range(8):
            assert (buf.array[i * 4096:(i + 1) * 4096] == data[i * 8192:i * 8192 + 4096]).all()
    finally:
        ctx.shutdown()
        os.close(fd)


def test_stats_reset_and_ledger_capacity(datafile):
    """Statistics and ledger records are kept per poller and summed when read:
    a reset makes the current sums the new zero, the ledger keeps at most its
    capacity of records between resets (each a distinct serviced ticket), and
    gsys_wait sees every completion."""
    n_blocks = (4 << 20) // 4096
    offs = synth.sweep_offsets(2048, n_blocks)
    fd = os.open(datafile, os.O_RDONLY)
    ctx = _ctx(ring_slots=1024, ledger_capacity=300)
    try:
        ctx.allow_fd(fd, g.FD_READ)
        for run in range(2):
            _, rets = _run(ctx, fd, offs, 8, 8, 0)
            assert (rets == 4096).all()
            assert ctx.wait(5_000_000_000) == 0
            st = ctx.stats(reset=True)
            assert st["requests"] == len(offs) and st["host_calls"] == len(offs)
            assert st["bytes_in"] == 4096 * len(offs)
            assert st["bundles"] >= 1 and sum(st["bundle_hist"]) == st["bundles"]
            after = ctx.stats()
            assert after["requests"] == 0 and after["host_calls"] == 0 and after["bytes_in"] == 0
            led = ctx.ledger(reset=True)
            assert 0 < len(led) <= 300
            tickets = led[:, 0]
            assert len(np.unique(tickets)) == len(tickets)
            assert (np.diff(tickets.astype(np.int64)) > 0).all()       # sorted by ticket
            assert (tickets >= run * len(offs)).all() and (tickets < (run + 1) * len(offs)).all()
            assert (led[:, 2] == 4096).all()
            assert len(ctx.ledger()) == 0
    finally:
        assert ctx.shutdown() == 0
        os.close(fd)
