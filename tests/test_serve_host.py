"""Serving entry point on the CPU: every job record is checked on the host
before anything is launched.  A CPU-only context (GSYS_CFG_NO_DEVICE) gets
-EINVAL for a bad record and -ENODEV once every record passes (the launch
itself needs a GPU)."""
import ctypes as C
import errno

import numpy as np
import pytest

import paper_1705_06965_amd as g
from paper_1705_06965_amd.serve import JOB_DTYPE, JOB_PWRITE, JOB_RELEASE, JOB_SCAN

N_DIGESTS = 1024          # digests the call is told about
CONTENT = 1 << 20         # content bytes the call is told about
ARENA = 64 << 20          # 32 release blocks of 2 MiB


@pytest.fixture(scope="module")
def ctx():
    c = g.Context(flags=g.CFG_NO_DEVICE | g.CFG_NO_PIN, service_threads=1, arena_bytes=ARENA)
    yield c
    c.shutdown()


def good_jobs():
    j = np.zeros(3, dtype=JOB_DTYPE)
    j[0] = (JOB_SCAN, 3, 0, 4096 * N_DIGESTS, 0, 0, 0, 0, 0, 0)      # every digest
    j[1] = (JOB_PWRITE, 4, 0, CONTENT, 0, 0, 0, 0, 0, 0)              # the whole pool, 1 MiB
    j[2] = (JOB_RELEASE, 4, 0, ARENA // (2 << 20) - 1, 0, 3, 511, 0, 0, 0)
    return j


def call(ctx, jobs, **over):
    n = len(jobs)
    rec = ctx.host_alloc(max(64, 64 * n))
    rec.array[:64 * n] = jobs.view(np.uint8)
    staging = ctx.host_alloc(2 << 20)
    arrival = np.zeros(max(1, n), dtype=np.uint64)
    lat = np.zeros(max(1, n), dtype=np.uint64)
    P = g.gsys_serve_params(form=g.PERSISTENT, n=n, jobs_dev=rec.dev, jobs_host=rec.host,
                            arrival_ns=arrival.ctypes.data, latency_ns=lat.ctypes.data,
                            max_inflight=4, digests=0x1000, n_digests=N_DIGESTS,
                            content=0x2000, content_bytes=CONTENT, staging=staging.dev,
                            staging_bytes=staging.nbytes)
    for k, v in over.items():
        setattr(P, k, v)
    rc = g.lib.gsys_serve_run(ctx.h, C.byref(P), None)
    rec.free()
    staging.free()
    return rc


def test_valid_records_reach_the_launch(ctx):
    assert call(ctx, good_jobs()) == -errno.ENODEV
    assert call(ctx, good_jobs(), form=g.PLAIN) == -errno.ENODEV
    assert call(ctx, good_jobs()[:0]) == -errno.ENODEV


@pytest.mark.parametrize("field,index,value", [
    ("kind", 0, 3),                                  # unknown kind
    ("len", 0, 4096 * N_DIGESTS + 4096),             # digests past n_digests
    ("len", 0, 4095),                                # not a multiple of 4 KiB
    ("src", 0, 1),                                   # src + len / 4096 > n_digests
    ("src", 0, 2**64 - 1),                           # wraps
    ("len", 1, CONTENT + 1),                         # pwrite longer than one staging buffer
    ("src", 1, 16),                                  # content past content_bytes
    ("len", 2, ARENA // (2 << 20)),                  # arena block past the arena
    ("page", 2, 512),                                # page past the 2 MiB block
])
def test_bad_record_is_refused(ctx, field, index, value):
    j = good_jobs()
    j[field][index] = value
    assert call(ctx, j) == -errno.EINVAL


def test_bad_parameters_are_refused(ctx):
    assert call(ctx, good_jobs(), form=7) == -errno.EINVAL
    assert call(ctx, good_jobs(), max_inflight=0) == -errno.EINVAL
    assert call(ctx, good_jobs(), digests=0) == -errno.EINVAL
    assert call(ctx, good_jobs(), staging_bytes=(2 << 20) - 1) == -errno.EINVAL
    assert call(ctx, good_jobs(), staging=0x10) == -errno.EFAULT
    assert call(ctx, good_jobs(), jobs_dev=0x10) == -errno.EFAULT


def test_release_needs_an_arena():
    c = g.Context(flags=g.CFG_NO_DEVICE | g.CFG_NO_PIN, service_threads=1)
    try:
        assert call(c, good_jobs()) == -errno.EINVAL
        assert call(c, good_jobs()[:2]) == -errno.ENODEV
    finally:
        c.shutdown()
