"""The allocation-free serving entry point (gsys_serve_run_noalloc) against
the allocating one (gsys_serve_run), through the C ABI: the same job stream
gives the same results, scan digests and output-file bytes, bit for bit, on
two calls in a row, the second with fewer jobs than the first (the shared
scratch array keeps the first call's records, which the second must not
see).  Plus the size limit, checked on the CPU."""
import ctypes as C
import errno
import os
import sys

import numpy as np
import pytest

import synth
import paper_1705_06965_amd as g
from paper_1705_06965_amd.serve import JOB_DTYPE

SCRATCH_JOBS = 65536


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_size_limit_on_cpu():
    """n above the scratch array is refused with -E2BIG before anything
    runs; n at the limit passes the checks (a CPU-only context then stops
    at -ENODEV)."""
    c = g.Context(flags=g.CFG_NO_DEVICE | g.CFG_NO_PIN, service_threads=1)
    try:
        rec = c.host_alloc(64 * (SCRATCH_JOBS + 1))
        rec.array[:] = 0                               # empty scans: valid records
        staging = c.host_alloc(2 << 20)
        arr = np.zeros(SCRATCH_JOBS + 1, dtype=np.uint64)
        lat = np.zeros(SCRATCH_JOBS + 1, dtype=np.uint64)
        for n, want in ((SCRATCH_JOBS + 1, -errno.E2BIG), (SCRATCH_JOBS, -errno.ENODEV)):
            P = g.gsys_serve_params(form=g.PERSISTENT, n=n, jobs_dev=rec.dev, jobs_host=rec.host,
                                    arrival_ns=arr.ctypes.data, latency_ns=lat.ctypes.data,
                                    max_inflight=8, staging=staging.dev,
                                    staging_bytes=staging.nbytes)
            assert g.lib.gsys_serve_run_noalloc(c.h, C.byref(P), None) == want
        assert g.lib.gsys_strerror(-errno.E2BIG) == b"more jobs than the allocation-free scratch holds"
    finally:
        c.shutdown()


def sub_stream(js, n):
    return synth.JobStream(kind=js.kind[:n], arrival_ns=js.arrival_ns[:n], arg_off=js.arg_off[:n],
                           arg_len=js.arg_len[:n], content_off=js.content_off[:n],
                           content=js.content)


@pytest.mark.gpu
def test_noalloc_equals_allocating_entry_point(tmpdata):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1705_06965_amd.serve import ServeRun
    os.environ.setdefault("GSYS_DATA_DIR", tmpdata)
    in_path = synth.random_file(5, 64 << 20, name="c5_in_64m.bin")
    # scans up to 16 MiB, so the 4 MiB task size below splits some of them
    js = synth.job_stream(n_jobs=500, rate_per_s=20000, scan_file_bytes=64 << 20,
                          scan_max_log2_pages=12, pwrite_max_pages=64, arena_blocks=8192)
    ctx = g.Context(ring_slots=1 << 16, device_timeout_ns=60_000_000_000, arena_bytes=16 << 30)
    os.environ["GSYS_SERVE_SPLIT_MIB"] = "4"
    try:
        for n in (500, 173):  # the second call is smaller than the first
            sj = sub_stream(js, n)
            out = {}
            for name, entry in (("alloc", g.lib.gsys_serve_run),
                                ("noalloc", g.lib.gsys_serve_run_noalloc)):
                path = os.path.join(tmpdata, "noalloc_%s_%d.bin" % (name, n))
                sr = ServeRun(ctx, sj, in_path, path)
                say("serve", name, "jobs", n)
                res, dig, lat = sr.run(g.PERSISTENT, max_inflight=64,
                                       staging_bytes=(2 << 20) * 32, entry=entry)
                sr.close()
                assert (lat != np.uint64(2**64 - 1)).all(), name
                out[name] = (res, dig, np.fromfile(path, dtype=np.uint8))
            a, b = out["alloc"], out["noalloc"]
            assert (a[0] == b[0]).all(), n                 # results per job
            assert (a[1] == b[1]).all(), n                 # scan digests
            assert a[2].shape == b[2].shape and (a[2] == b[2]).all(), n  # output file
            kinds = np.bincount(sj.kind, minlength=3)
            assert kinds.min() > 0
            # every scan read its whole range
            s = sj.kind == 0
            assert (b[0][s] == sj.arg_len[s].astype(np.int64)).all()
        # the plain form through the allocation-free entry point too
        sj = sub_stream(js, 60)
        path = os.path.join(tmpdata, "noalloc_plain.bin")
        sr = ServeRun(ctx, sj, in_path, path)
        res_p, dig_p, _ = sr.run(g.PLAIN, max_inflight=16, staging_bytes=(2 << 20) * 4,
                                 entry=g.lib.gsys_serve_run_noalloc)
        sr.close()
        path2 = os.path.join(tmpdata, "alloc_plain.bin")
        sr2 = ServeRun(ctx, sj, in_path, path2)
        res_q, dig_q, _ = sr2.run(g.PLAIN, max_inflight=16, staging_bytes=(2 << 20) * 4)
        sr2.close()
        assert (res_p == res_q).all() and (dig_p == dig_q).all()
        assert (np.fromfile(path, dtype=np.uint8) == np.fromfile(path2, dtype=np.uint8)).all()
    finally:
        del os.environ["GSYS_SERVE_SPLIT_MIB"]
        assert ctx.shutdown() == 0
