"""Property tests (Hypothesis) of the host pool's descriptor-list calls and
of the oracle's pread plumbing, on small random files (CPU only).

A group call carries a list of transfers; the pool runs it in list order and
folds runs that are contiguous both in the file and in the buffer into one
pread.  Whatever the list, every descriptor's result and the final buffer
must equal what individual preads issued one by one in list order give
(pread(2): min(len, max(0, size - off)) bytes from off)."""
import os

import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
import paper_1705_06965_amd as g
import gsys_hooks as hooks

BUF = 1 << 16


@pytest.fixture(scope="module")
def pool(tmp_path_factory):
    d = tmp_path_factory.mktemp("props")
    ctx = g.Context(flags=g.CFG_NO_DEVICE | g.CFG_NO_PIN, service_threads=3, ring_slots=64)
    buf = ctx.host_alloc(BUF)
    lst = ctx.host_alloc(64 * 16)
    yield ctx, buf, lst, str(d)
    ctx.shutdown()


# a transfer either continues the previous one in file and buffer (so the
# pool may fold it in) or starts anywhere
_seg = st.tuples(st.booleans(), st.integers(0, 6000), st.integers(0, 700), st.integers(0, BUF - 700))


@settings(max_examples=150, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(data=st.binary(max_size=5000), segs=st.lists(_seg, min_size=1, max_size=40))
def test_list_calls_equal_individual_preads(pool, data, segs):
    ctx, buf, lst, d = pool
    path = os.path.join(d, "f.bin")
    with open(path, "wb") as f:
        f.write(data)
    descs = []
    for cont, off, ln, boff in segs:
        if cont and descs:
            poff, pboff, pln = descs[-1]
            off, boff = poff + pln, pboff + pln
            if boff + ln > BUF:
                boff, ln = BUF - ln if ln <= BUF else 0, ln
        descs.append((off, boff, ln))
    fd = os.open(path, os.O_RDONLY)
    try:
        ctx.allow_fd(fd, g.FD_READ)
        buf.array[:] = 0xAB
        L = np.zeros(len(descs), dtype=[("off", "<u8"), ("buf_off", "<u4"), ("len_ret", "<i4")])
        for i, (off, boff, ln) in enumerate(descs):
            L[i] = (off, boff, ln)
        lst.array[:L.nbytes] = L.view(np.uint8)
        a = np.array([fd, lst.dev, len(descs), buf.dev, 0, 0], dtype=np.uint64)
        r = np.zeros(1, dtype=np.int64)
        assert hooks.lib.gsys_test_raw_call(
            ctx.h, g.NR_PREAD64, g.F_LIST | g.F_BLOCKING | (g.GRAN_WG << 4), a.ctypes.data,
            r.ctypes.data, 5_000_000_000) == 0
        got = lst.array[:L.nbytes].view(L.dtype)["len_ret"]
        # the model: preads one by one, in list order
        want_buf = bytearray(b"\xab" * BUF)
        total = 0
        for i, (off, boff, ln) in enumerate(descs):
            n = max(0, min(ln, len(data) - off))
            want_buf[boff:boff + n] = data[off:off + n]
            assert got[i] == n, (i, descs[i], len(data))
            total += n
        assert int(r[0]) == total
        assert bytes(buf.array) == bytes(want_buf)
    finally:
        ctx.allow_fd(fd, 0)
        os.close(fd)


@settings(max_examples=200, deadline=None)
@given(data=st.binary(max_size=3000),
       reads=st.lists(st.tuples(st.integers(0, 3500), st.integers(0, 4096)), min_size=1,
                      max_size=20))
def test_oracle_pread_equals_slicing(tmp_path_factory, data, reads):
    d = tmp_path_factory.mktemp("oprops")
    path = os.path.join(str(d), "f.bin")
    with open(path, "wb") as f:
        f.write(data)
    for off, ln in reads:
        fnv, ret = oracle.pread_fnv(path, np.array([off], dtype=np.uint64), max(ln, 1))
        n = max(0, min(max(ln, 1), len(data) - off))
        assert int(ret[0]) == n
        assert int(fnv[0]) == oracle.fnv1a64(np.frombuffer(data[off:off + n], dtype=np.uint8))


def test_contiguous_list_is_one_pread(pool):
    """Eight transfers contiguous in file and buffer run as one pread (seven
    folded), and each still gets its own 512 bytes back."""
    ctx, buf, lst, d = pool
    path = os.path.join(d, "g.bin")
    data = np.random.default_rng(1).integers(0, 256, 8192, dtype=np.uint8)
    data.tofile(path)
    fd = os.open(path, os.O_RDONLY)
    try:
        ctx.allow_fd(fd, g.FD_READ)
        L = np.zeros(8, dtype=[("off", "<u8"), ("buf_off", "<u4"), ("len_ret", "<i4")])
        for i in range(8):
            L[i] = (1000 + 512 * i, 512 * i, 512)
        lst.array[:L.nbytes] = L.view(np.uint8)
        s0 = ctx.stats()
        a = np.array([fd, lst.dev, 8, buf.dev, 0, 0], dtype=np.uint64)
        r = np.zeros(1, dtype=np.int64)
        assert hooks.lib.gsys_test_raw_call(ctx.h, g.NR_PREAD64, g.F_LIST | g.F_BLOCKING | (g.GRAN_WG << 4),
                                        a.ctypes.data, r.ctypes.data, 5_000_000_000) == 0
        s1 = ctx.stats()
        assert int(r[0]) == 4096
        assert (lst.array[:L.nbytes].view(L.dtype)["len_ret"] == 512).all()
        assert s1["merged"] - s0["merged"] == 7 and s1["host_calls"] - s0["host_calls"] == 1
        assert (buf.array[:4096] == data[1000:5096]).all()
    finally:
        ctx.allow_fd(fd, 0)
        os.close(fd)
