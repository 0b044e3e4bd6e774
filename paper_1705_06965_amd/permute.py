"""Driver of the block-permutation + pwrite workload (the ordering / blocking
microbenchmark of section 6, Fig. 6).  Allocates the input array in HBM, the
host staging the blocks are written from, and launches ``gsys_permute``
through the C ABI; device memory and streams come from PyTorch."""
from __future__ import annotations

import os

import numpy as np

from . import Context, FD_WRITE, check, lib, cell_code, _stream

BLOCK = 8192
WG_CELLS = [("WG", "strong", "block"), ("WG", "strong", "nonblock"),
            ("WG", "relaxed", "block"), ("WG", "relaxed", "nonblock")]


class PermuteRunner:
    def __init__(self, ctx: Context, path: str, data: np.ndarray, sigma: np.ndarray,
                 tau: np.ndarray, device: str = "cuda", file_off: int = 0):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.path = path
        d = np.ascontiguousarray(data, dtype=np.uint64)
        if d.size % (BLOCK // 8):
            raise ValueError("data is not a whole number of 8 KiB blocks")
        self.n = d.size // (BLOCK // 8)
        self.sigma = np.ascontiguousarray(sigma, dtype=np.uint16)
        self.tau = np.ascontiguousarray(tau, dtype=np.uint8)
        self.file_off = file_off
        self.fd = os.open(path, os.O_RDWR | os.O_CREAT, 0o600)
        ctx.allow_fd(self.fd, FD_WRITE)
        self.data = torch.from_numpy(d.view(np.int64)).to(device)
        self.staging = ctx.host_alloc(max(1, self.n) * BLOCK)
        self.out_ret = torch.zeros(max(1, self.n), dtype=torch.int64, device=device)

    def launch(self, iters: int, cell: int, stream=None):
        return check(lib.gsys_permute(self.ctx.h, self.fd, self.data.data_ptr(),
                                      self.sigma.ctypes.data, self.tau.ctypes.data, self.n,
                                      iters, self.staging.dev, self.file_off,
                                      self.out_ret.data_ptr(), cell, _stream(stream)),
                     "gsys_permute")

    def run(self, iters: int, g="WG", o="strong", b="block", stream=None):
        """Launch, wait for the GPU, drain the host pool; per-block results
        (pwrite's return value for blocking cells)."""
        self.out_ret.fill_(-12345)
        self.launch(iters, cell_code(g, o, b), stream)
        self.torch.cuda.synchronize()
        rc = self.ctx.wait(60_000_000_000)
        if rc:
            raise RuntimeError("drain failed: %d" % rc)
        return self.out_ret.cpu().numpy()[:self.n].copy()

    def file_bytes(self) -> np.ndarray:
        return np.fromfile(self.path, dtype=np.uint8)[self.file_off:self.file_off + self.n * BLOCK]

    def close(self):
        self.ctx.allow_fd(self.fd, 0)
        os.close(self.fd)
        self.staging.free()
