"""Argument checks of the entry points on the CPU: a CPU-only context
(GSYS_CFG_NO_DEVICE) answers -EINVAL or -EFAULT for a bad call and -ENODEV
once every check passes (the launch itself needs a GPU).  Empty inputs
(no items, no files) return 0 without launching, whatever their output
pointers."""
import errno

import pytest

import paper_1705_06965_amd as g

WG_BLOCK = g.cell(g.GRAN_WG, strong=True, blocking=True)
DEV = 0x10000          # device addresses are not dereferenced before the launch


@pytest.fixture(scope="module")
def ctx():
    c = g.Context(flags=g.CFG_NO_DEVICE | g.CFG_NO_PIN, service_threads=1)
    yield c
    c.shutdown()


def roundtrip(c, nfiles=2, file_bytes=1000, piece=256, staging=None, paths=None,
              rets=DEV, mismatch=DEV, data=DEV, cell=WG_BLOCK, staging_bytes=None):
    area = (max(file_bytes, 16) + 15) // 16 * 16
    if staging_bytes is None:
        staging_bytes = 2 * area * nfiles
    return g.lib.gsys_file_roundtrip(c.h, 3, paths, nfiles, data, file_bytes, piece, staging,
                                     staging_bytes, rets, mismatch, cell, None)


def test_roundtrip_checks(ctx):
    st = ctx.host_alloc(1 << 16)
    pa = ctx.host_alloc(2 * g.PATH_MAX)
    try:
        ok = dict(staging=st.dev, paths=pa.dev)
        assert roundtrip(ctx, **ok) == -errno.ENODEV
        # no files: nothing to do, and the outputs may be null
        assert roundtrip(ctx, nfiles=0, rets=0, mismatch=0, data=0, paths=0, staging=0) == 0
        # the cell is checked first: stateful calls are blocking work-group calls
        for bad in (g.cell(g.GRAN_WI, True, True), g.cell(g.GRAN_WG, True, False),
                    g.cell(g.GRAN_KERNEL, False, True)):
            assert roundtrip(ctx, nfiles=0, cell=bad, **ok) == -errno.EINVAL
            assert roundtrip(ctx, cell=bad, **ok) == -errno.EINVAL
        assert roundtrip(ctx, rets=0, **ok) == -errno.EINVAL
        assert roundtrip(ctx, mismatch=0, **ok) == -errno.EINVAL
        assert roundtrip(ctx, data=0, **ok) == -errno.EINVAL
        assert roundtrip(ctx, data=0, file_bytes=0, **ok) == -errno.ENODEV   # empty files
        assert roundtrip(ctx, piece=0, **ok) == -errno.EINVAL
        assert roundtrip(ctx, file_bytes=(1 << 31) + 1, **ok) == -errno.EINVAL
        assert roundtrip(ctx, file_bytes=(1 << 20) + 1, piece=1, **ok) == -errno.EINVAL
        assert roundtrip(ctx, staging_bytes=2 * 1008 * 2 - 1, **ok) == -errno.EINVAL
        assert roundtrip(ctx, staging=DEV, paths=pa.dev) == -errno.EFAULT
        assert roundtrip(ctx, staging=st.dev, paths=DEV) == -errno.EFAULT
    finally:
        st.free()
        pa.free()


def test_kernel_io_checks(ctx):
    st = ctx.host_alloc(1 << 16)
    try:
        def kio(nr=g.NR_WRITE, data=DEV, nbytes=4096, staging=st.dev, ret=DEV, mismatch=DEV,
                grid=4):
            return g.lib.gsys_file_kernel_io(ctx.h, 3, nr, data, nbytes, staging, ret, mismatch,
                                             grid, None)
        assert kio() == -errno.ENODEV
        assert kio(nr=g.NR_READ) == -errno.ENODEV
        assert kio(nr=g.NR_PREAD64) == -errno.EINVAL
        for k in ("data", "nbytes", "ret", "mismatch", "grid"):
            assert kio(**{k: 0}) == -errno.EINVAL, k
        assert kio(grid=65536) == -errno.EINVAL
        assert kio(nbytes=(1 << 16) + 1) == -errno.EFAULT     # past the registered range
        assert kio(staging=DEV) == -errno.EFAULT
    finally:
        st.free()


def test_empty_inputs_launch_nothing(ctx):
    # checksums: no items
    assert g.lib.gsys_fnv4k(ctx.h, 3, 0, 0, 4096, 0, 0, 0, 0, 0, g.cell(g.GRAN_WI, True, True),
                            g.PLAIN, 256, None) == 0
    assert g.lib.gsys_fnv4k_consume(ctx.h, 0, 0, 0, 4096, 0, 256, 0, None) == 0
    # the open / read / close search: no files, once its shapes pass
    def wo(nfiles, nq=2, chunk=4096):
        return g.lib.gsys_wordcount_open(ctx.h, 3, 0, nfiles, 0, 0, nq, 0, 0, chunk, 0, 0, 0, 0,
                                         None)
    assert wo(0) == 0
    assert wo(0, nq=0) == -errno.EINVAL
    assert wo(0, nq=65) == -errno.EINVAL
    assert wo(0, chunk=100) == -errno.EINVAL
    assert wo(1) == -errno.EINVAL          # a file but null outputs


def test_consume_checks(ctx):
    def cs(staging=DEV, rets=DEV, n=100, item=4096, out=DEV, wg=256, grid=0):
        return g.lib.gsys_fnv4k_consume(ctx.h, staging, rets, n, item, out, wg, grid, None)
    for k in ("staging", "rets", "out"):
        assert cs(**{k: 0}) == -errno.EINVAL, k
    for item in (0, 100, (1 << 20) + 64):
        assert cs(item=item) == -errno.EINVAL
    for wg in (0, 32, 96, 2048):
        assert cs(wg=wg) == -errno.EINVAL


def test_checksum_shape_checks(ctx):
    n = 200
    st = ctx.host_alloc(n * 4096)
    li = ctx.host_alloc(n * 16)
    try:
        def fv(n=n, item=4096, wg=64, offsets=DEV, staging=st.dev, staging_bytes=n * 4096,
               lists=li.dev, out_fnv=DEV, out_ret=DEV, form=g.PLAIN):
            return g.lib.gsys_fnv4k(ctx.h, 3, offsets, n, item, staging, staging_bytes, lists,
                                    out_fnv, out_ret, g.cell(g.GRAN_WI, True, True), form, wg,
                                    None)
        assert fv() == -errno.ENODEV
        assert fv(item=64, staging_bytes=n * 64) == -errno.ENODEV
        for item in (0, 100, 4097, (1 << 20) + 64):
            assert fv(item=item) == -errno.EINVAL, item
        for wg in (0, 32, 96, 192, 2048):
            assert fv(wg=wg) == -errno.EINVAL, wg
        for k in ("offsets", "out_fnv", "out_ret"):
            assert fv(**{k: 0}) == -errno.EINVAL, k
        assert fv(n=(1 << 32) + 1) == -errno.EINVAL
        # the plain form stages every item; the persistent forms need two
        # work-groups' batches
        assert fv(staging_bytes=n * 4096 - 1) == -errno.EINVAL
        assert fv(staging_bytes=2 * 64 * 4096, form=g.PERSISTENT) == -errno.ENODEV
        assert fv(staging_bytes=2 * 64 * 4096 - 1, form=g.PERSISTENT) == -errno.EINVAL
        assert fv(staging=DEV) == -errno.EFAULT
        assert fv(n=n + 1, staging_bytes=(n + 1) * 4096) == -errno.EFAULT   # past staging
        assert fv(lists=DEV) == -errno.EFAULT
    finally:
        st.free()
        li.free()


def test_cpu_only_context_launches_nothing(ctx, capfd):
    """A CPU-only context answers every valid call with -ENODEV and launches
    nothing (on a machine with a GPU the device addresses here are not
    mapped, so a launch would fault); the library reports every failed
    launch on stderr, and none is reported."""
    import numpy as np
    st = ctx.host_alloc(1 << 20)
    pa = ctx.host_alloc(2 * g.PATH_MAX)
    try:
        K = g.cell(g.GRAN_KERNEL, False, True)
        WG = g.cell(g.GRAN_WG, True, True)
        sigma = np.arange(1024, dtype=np.uint16)
        tau = np.arange(64, dtype=np.uint8)
        calls = {
            "kv_build": lambda: g.lib.gsys_kv_build(ctx.h, DEV, 16, 0, 0, 0, 0, None),
            "fnv4k kernel cell": lambda: g.lib.gsys_fnv4k(ctx.h, 3, DEV, 16, 4096, st.dev, 16 * 4096,
                                                          st.dev, DEV, DEV, K, g.PLAIN, 64, None),
            "fnv4k persistent": lambda: g.lib.gsys_fnv4k(ctx.h, 3, DEV, 16, 4096, st.dev, 16 * 4096,
                                                         st.dev, DEV, DEV, 0, g.PERSISTENT, 64,
                                                         None),
            "fnv4k graph": lambda: g.lib.gsys_fnv4k(ctx.h, 3, DEV, 16, 4096, st.dev, 16 * 4096,
                                                    st.dev, DEV, DEV, 0, g.GRAPH, 64, None),
            "consume": lambda: g.lib.gsys_fnv4k_consume(ctx.h, DEV, DEV, 16, 4096, DEV, 64, 0, None),
            "canary": lambda: g.lib.gsys_canary(ctx.h, 3, st.dev, 64, 1, DEV, K, 64, None),
            "permute": lambda: g.lib.gsys_permute(ctx.h, 3, DEV, sigma.ctypes.data, tau.ctypes.data,
                                                  1, 0, st.dev, 0, DEV, WG, None),
            "roundtrip": lambda: roundtrip(ctx, staging=st.dev, paths=pa.dev),
            "kernel io": lambda: g.lib.gsys_file_kernel_io(ctx.h, 3, g.NR_WRITE, DEV, 4096, st.dev,
                                                           DEV, DEV, 4, None),
            "wordscan": lambda: g.lib.gsys_wordscan(ctx.h, DEV, 4, 4096, DEV, DEV, 1, DEV, 2,
                                                    st.dev, st.nbytes, g.PERSISTENT, 1, None),
            "wordcount_open": lambda: g.lib.gsys_wordcount_open(
                ctx.h, 3, pa.dev, 2, DEV, DEV, 1, DEV, DEV, 4096, st.dev, st.nbytes, 0, 0, None),
        }
        capfd.readouterr()
        for name, call in calls.items():
            assert call() == -errno.ENODEV, name
        assert "launch" not in capfd.readouterr().err
    finally:
        st.free()
        pa.free()


def test_launch_descriptor_checks(ctx):
    """gsys_launch checks its descriptor before anything else: no kernel, an
    empty grid, more than 1,024 work-items, an unknown mode or a persistent
    grid of more than one dimension is -EINVAL; a valid descriptor on a
    CPU-only context is -ENODEV (nothing launched, the kernel address here
    is not a kernel)."""
    import ctypes as C
    d = g.gsys_launch_desc()
    assert g.lib.gsys_launch(ctx.h, C.byref(d), None) == -errno.EINVAL       # no kernel
    d.kernel = DEV
    d.block[0] = 64
    assert g.lib.gsys_launch(ctx.h, C.byref(d), None) == -errno.EINVAL       # no work-groups
    d.grid[0] = 4
    for mode in (g.PLAIN, g.PERSISTENT, g.GRAPH):
        d.mode = mode
        assert g.lib.gsys_launch(ctx.h, C.byref(d), None) == -errno.ENODEV, mode
    d.mode = 7
    assert g.lib.gsys_launch(ctx.h, C.byref(d), None) == -errno.EINVAL
    d.mode = g.PLAIN
    d.block[0], d.block[1] = 64, 32                                          # 2,048 work-items
    assert g.lib.gsys_launch(ctx.h, C.byref(d), None) == -errno.EINVAL
    d.block[1] = 1
    d.grid[1] = 2
    assert g.lib.gsys_launch(ctx.h, C.byref(d), None) == -errno.ENODEV       # plain: 2-D is fine
    for mode in (g.PERSISTENT, g.GRAPH):
        d.mode = mode
        assert g.lib.gsys_launch(ctx.h, C.byref(d), None) == -errno.EINVAL, mode


def test_kv_build_checks(ctx):
    def kb(table=DEV, cap=16, keys=DEV, voff=DEV, vlen=DEV, n=4):
        return g.lib.gsys_kv_build(ctx.h, table, cap, keys, voff, vlen, n, None)
    assert kb() == -errno.ENODEV
    assert kb(keys=0, voff=0, vlen=0, n=0) == -errno.ENODEV   # an empty table
    for k in ("table", "keys", "voff", "vlen"):
        assert kb(**{k: 0}) == -errno.EINVAL, k
    assert kb(cap=0, n=0) == -errno.EINVAL
    assert kb(cap=3, n=4) == -errno.EINVAL                    # more keys than buckets
    assert kb(cap=(1 << 40) + 1) == -errno.EINVAL
    assert kb(cap=1 << 40) == -errno.ENODEV
