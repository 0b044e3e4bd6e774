"""Driver of the per-item pread + FNV-1a workload (pread microbenchmark of
section 6, Fig. 5).  Allocates the buffers the kernels need and launches them
through the C ABI; device memory and streams come from PyTorch."""
from __future__ import annotations

import os

import numpy as np

from . import (Context, FD_READ, PLAIN, PERSISTENT, GRAPH, check, lib, cell_code,
               _stream)


class FnvRunner:
    def __init__(self, ctx: Context, path: str, offsets: np.ndarray, item_bytes: int = 4096,
                 wg_size: int = 256, device: str = "cuda", staging_bytes: int = 0):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.path = path
        self.fd = os.open(path, os.O_RDONLY)
        ctx.allow_fd(self.fd, FD_READ)
        self.n = int(len(offsets))
        self.item_bytes = item_bytes
        self.wg_size = wg_size
        self.staging_bytes = staging_bytes or max(1, self.n * item_bytes)
        self.staging = ctx.host_alloc(self.staging_bytes)
        self.lists = ctx.host_alloc(max(16, self.n * 16))
        offs = np.ascontiguousarray(offsets, dtype=np.uint64)
        self.offsets = torch.from_numpy(offs.view(np.int64)).to(device)
        self.out_fnv = torch.zeros(max(1, self.n), dtype=torch.int64, device=device)
        self.out_ret = torch.zeros(max(1, self.n), dtype=torch.int64, device=device)

    def launch(self, cell: int = 0, form: int = PLAIN, stream=None):
        return check(lib.gsys_fnv4k(self.ctx.h, self.fd, self.offsets.data_ptr(), self.n,
                                    self.item_bytes, self.staging.dev, self.staging_bytes,
                                    self.lists.dev,
                                    self.out_fnv.data_ptr(), self.out_ret.data_ptr(), cell, form,
                                    self.wg_size, _stream(stream)), "gsys_fnv4k")

    def run(self, g="WI", o="strong", b="block", form=PLAIN, stream=None):
        """Launch, wait for the GPU and drain the host pool."""
        self.out_fnv.zero_()
        self.out_ret.fill_(-12345)
        self.launch(cell_code(g, o, b), form, stream)
        self.torch.cuda.synchronize()
        rc = self.ctx.wait(60_000_000_000)
        if rc:
            raise RuntimeError("drain failed: %d" % rc)
        return self.result()

    def result(self):
        f = self.out_fnv.cpu().numpy().view(np.uint64)[:self.n].copy()
        r = self.out_ret.cpu().numpy()[:self.n].copy()
        return f, r

    def host_pread_rate(self, threads: int, reps: int = 3) -> float:
        """GB/s at which `threads` host threads make this runner's preads into
        its staging with no GPU work (gsys_host_pread_rate): the host's side
        of the sweep's roofline."""
        import ctypes as C
        offs = np.ascontiguousarray(self.offsets.cpu().numpy().view(np.uint64))
        fds = np.full(self.n, self.fd, dtype=np.int32)
        lens = np.full(self.n, self.item_bytes, dtype=np.uint32)
        out = C.c_double()
        check(lib.gsys_host_pread_rate(fds.ctypes.data, offs.ctypes.data, lens.ctypes.data,
                                       self.n, self.staging.host, self.item_bytes,
                                       self.staging_bytes // self.item_bytes, threads, reps,
                                       C.byref(out)), "gsys_host_pread_rate")
        return out.value

    def close(self):
        """Revoke and close the file, free the staging and list buffers."""
        self.ctx.allow_fd(self.fd, 0)
        os.close(self.fd)
        self.staging.free()
        self.lists.free()


def consume(ctx: Context, staging: int, rets, item_bytes: int, out, wg_size: int = 256,
            grid: int = 0, stream=None) -> int:
    """Kernel-split form (gsys_fnv4k_consume): out[i] = FNV-1a-64 of the first
    rets[i] bytes of staging + i * item_bytes.  `staging` is a device-readable
    address; `rets` (int64) and `out` (int64) are device tensors of one length."""
    n = int(rets.numel())
    if int(out.numel()) < n:
        raise ValueError("out holds %d items, rets %d" % (out.numel(), n))
    return check(lib.gsys_fnv4k_consume(ctx.h, staging, rets.data_ptr(), n, item_bytes,
                                        out.data_ptr(), wg_size, grid, _stream(stream)),
                 "gsys_fnv4k_consume")
