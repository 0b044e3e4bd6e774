"""Driver of the serving mix: turns a job stream into gsys_job records and
runs it through gsys_serve_run (continuous batching on the GPU, or one launch
per job)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import FD_READ, FD_WRITE, check, gsys_serve_params, lib, _stream

JOB_SCAN, JOB_PWRITE, JOB_RELEASE = 0, 1, 2
JOB_DTYPE = np.dtype([("kind", "<u4"), ("fd", "<i4"), ("off", "<u8"), ("len", "<u8"),
                      ("src", "<u8"), ("aux_fd", "<i4"), ("page", "<u4"), ("done", "<u8"),
                      ("result", "<i8"), ("pad", "<u8")])
assert JOB_DTYPE.itemsize == 64
RELEASE_BLOCK = 2 << 20
RELEASE_OUT = 128


class ServeRun:
    """One serving session over a job stream (synth.JobStream).

    in_path: the file scans read and release jobs take their stamps from;
    out_path: where pwrite jobs write (at their offsets) and release jobs
    write their 128-byte readbacks (after the pwrite region)."""

    def __init__(self, ctx, stream, in_path: str, out_path: str, device: str = "cuda",
                 arena_blocks: int = 8192):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.js = stream
        n = len(stream.kind)
        self.n = n
        self.in_fd = os.open(in_path, os.O_RDONLY)
        self.out_fd = os.open(out_path, os.O_RDWR | os.O_CREAT | os.O_TRUNC, 0o600)
        ctx.allow_fd(self.in_fd, FD_READ)
        ctx.allow_fd(self.out_fd, FD_WRITE)
        in_size = os.fstat(self.in_fd).st_size
        kind = stream.kind
        jobs = np.zeros(n, dtype=JOB_DTYPE)
        jobs["kind"] = kind
        # scans
        s = kind == JOB_SCAN
        if (stream.arg_len[s] % 4096).any():
            raise ValueError("scan lengths must be multiples of 4096")
        blocks = np.where(s, stream.arg_len // 4096, 0).astype(np.uint64)
        self.digest_start = (np.cumsum(blocks) - blocks).astype(np.uint64)
        self.n_digests = int(blocks.sum())
        jobs["fd"][s] = self.in_fd
        jobs["off"][s] = stream.arg_off[s]
        jobs["len"][s] = stream.arg_len[s]
        jobs["src"][s] = self.digest_start[s]
        # pwrites
        w = kind == JOB_PWRITE
        jobs["fd"][w] = self.out_fd
        jobs["off"][w] = stream.arg_off[w]
        jobs["len"][w] = stream.arg_len[w]
        jobs["src"][w] = stream.content_off[w]
        self.pwrite_end = int((stream.arg_off[w] + stream.arg_len[w]).max()) if w.any() else 0
        # releases: readbacks after the pwrite region; stamps from the input file
        r = kind == JOB_RELEASE
        ridx = np.cumsum(r) - 1
        self.release_base = (self.pwrite_end + 4095) // 4096 * 4096
        jobs["fd"][r] = self.out_fd
        jobs["off"][r] = self.release_base + RELEASE_OUT * ridx[r].astype(np.uint64)
        jobs["len"][r] = (ridx[r] % arena_blocks).astype(np.uint64)
        jobs["src"][r] = (ridx[r].astype(np.uint64) * np.uint64(7 * 4096 + 64)) % \
            np.uint64(max(1, in_size - RELEASE_BLOCK))
        jobs["aux_fd"][r] = self.in_fd
        jobs["page"][r] = (ridx[r] * 37 % 512).astype(np.uint32)
        self.jobs_np = jobs
        self.jobs = ctx.host_alloc(max(64, n * 64))
        self.jobs.view(np.uint8)[:n * 64] = jobs.view(np.uint8)
        self.arrival = np.ascontiguousarray(stream.arrival_ns, dtype=np.uint64)
        self.digests = torch.zeros(max(1, self.n_digests), dtype=torch.int64, device=device)
        self.content = torch.from_numpy(stream.content if len(stream.content) else
                                        np.zeros(16, dtype=np.uint8)).to(device)
        self.latency = np.zeros(n, dtype=np.uint64)

    def params(self, form, max_inflight: int = 512, grid: int = 0, staging_bytes: int = 0,
               timeout_ns: int = 120_000_000_000, max_inflight_bytes: int = 0):
        """The gsys_serve_params of one session (staging allocated on first use)."""
        staging_bytes = staging_bytes or (2 << 20) * 256
        if not hasattr(self, "staging") or self.staging.nbytes < staging_bytes:
            self.staging = self.ctx.host_alloc(staging_bytes)
        # reset records (results, done flags) between runs
        self.jobs.view(np.uint8)[:self.n * 64] = self.jobs_np.view(np.uint8)
        return gsys_serve_params(
            form=form, n=self.n, jobs_dev=self.jobs.dev, jobs_host=self.jobs.host,
            arrival_ns=self.arrival.ctypes.data, latency_ns=self.latency.ctypes.data,
            max_inflight=max_inflight, grid=grid, max_inflight_bytes=max_inflight_bytes,
            digests=self.digests.data_ptr(), n_digests=self.digests.numel(),
            content=self.content.data_ptr(), content_bytes=self.content.numel(),
            staging=self.staging.dev, staging_bytes=self.staging.nbytes, timeout_ns=timeout_ns)

    def run(self, form, max_inflight: int = 512, grid: int = 0, staging_bytes: int = 0,
            timeout_ns: int = 120_000_000_000, stream=None, max_inflight_bytes: int = 0,
            entry=None):
        """One session through gsys_serve_run (or `entry`, an entry point of the
        same signature); returns (results, digests, latencies)."""
        P = self.params(form, max_inflight, grid, staging_bytes, timeout_ns, max_inflight_bytes)
        fn = entry or lib.gsys_serve_run
        check(fn(self.ctx.h, C.byref(P), _stream(stream)), fn.__name__)
        self.peak_inflight_bytes = P.peak_inflight_bytes
        self.torch.cuda.synchronize()
        rc = self.ctx.wait(30_000_000_000)
        if rc:
            raise RuntimeError("drain failed: %d" % rc)
        rec = self.jobs.view(np.uint8)[:self.n * 64].copy().view(JOB_DTYPE)
        return rec["result"].copy(), self.digests.cpu().numpy().view(np.uint64).copy(), \
            self.latency.copy()

    def close(self):
        for fd in (self.in_fd, self.out_fd):
            self.ctx.allow_fd(fd, 0)
            os.close(fd)
