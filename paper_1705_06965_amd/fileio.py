"""Drivers of the stateful file calls (gsys_file_roundtrip,
gsys_file_kernel_io): device memory and streams come from PyTorch, every call
goes through the C ABI."""
from __future__ import annotations

import os

import numpy as np

from . import (FD_DIR, FD_READ, FD_WRITE, NR_READ, NR_WRITE, PATH_MAX, _stream, cell_code,
               check, lib)


class FileRoundtrip:
    """Work-group f writes file `names[f]` beneath `directory` in pieces,
    reads it back and compares."""

    def __init__(self, ctx, directory: str, names, device: str = "cuda"):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.dirfd = os.open(directory, os.O_RDONLY | os.O_DIRECTORY)
        ctx.allow_fd(self.dirfd, FD_READ | FD_WRITE | FD_DIR)
        self.nfiles = len(names)
        self.device = device
        self.paths = ctx.host_alloc(max(1, self.nfiles) * PATH_MAX)
        self.paths.array[:] = 0
        for i, n in enumerate(names):
            b = n.encode() if isinstance(n, str) else bytes(n)
            if len(b) >= PATH_MAX:
                raise ValueError("path %r: at most %d bytes" % (n, PATH_MAX - 1))
            self.paths.array[i * PATH_MAX:i * PATH_MAX + len(b)] = np.frombuffer(b, dtype=np.uint8)
        self.staging = None

    @staticmethod
    def area(file_bytes: int) -> int:
        return (max(file_bytes, 16) + 15) // 16 * 16

    def prepare(self, data: np.ndarray, piece: int):
        """Upload data of shape (nfiles, file_bytes), size and clear staging."""
        torch = self.torch
        data = np.ascontiguousarray(data, dtype=np.uint8).reshape(self.nfiles, -1)
        self.fb = fb = data.shape[1]
        self.piece = piece
        self.k = (fb + piece - 1) // piece
        self.a = a = self.area(fb)
        self.need = need = max(1, self.nfiles) * 2 * a
        if self.staging is None or self.staging.nbytes < need:
            if self.staging is not None:
                self.staging.free()
            self.staging = self.ctx.host_alloc(need)
        self.staging.array[:need] = 0
        self.d = torch.from_numpy(data.reshape(-1).copy()).to(self.device) if fb else \
            torch.zeros(1, dtype=torch.uint8, device=self.device)
        self.rets = torch.full((max(1, self.nfiles), 2 * self.k + 5), -12345, dtype=torch.int64,
                               device=self.device)
        self.mism = torch.zeros(max(1, self.nfiles), dtype=torch.int64, device=self.device)

    def launch(self, o: str = "strong", stream=None):
        check(lib.gsys_file_roundtrip(self.ctx.h, self.dirfd, self.paths.dev, self.nfiles,
                                      self.d.data_ptr(), self.fb, self.piece, self.staging.dev,
                                      self.need, self.rets.data_ptr(), self.mism.data_ptr(),
                                      cell_code("WG", o, "block"), _stream(stream)),
              "gsys_file_roundtrip")

    def finish(self):
        """Wait for the GPU and the host pool; (rets[f, 2K + 5], mismatch[f],
        read areas[f, file_bytes])."""
        self.torch.cuda.synchronize()
        rc = self.ctx.wait(60_000_000_000)
        if rc:
            raise RuntimeError("drain failed: %d" % rc)
        n, a, fb = max(1, self.nfiles), self.a, self.fb
        back = self.staging.array[:self.need].reshape(n, 2 * a)[:self.nfiles, a:a + fb]
        return (self.rets.cpu().numpy()[:self.nfiles].copy(),
                self.mism.cpu().numpy()[:self.nfiles].copy(), back.copy())

    def run(self, data: np.ndarray, piece: int, o: str = "strong", stream=None):
        """prepare + launch + finish."""
        self.prepare(data, piece)
        self.launch(o, stream)
        return self.finish()

    def close(self):
        self.ctx.allow_fd(self.dirfd, 0)
        os.close(self.dirfd)
        self.paths.free()
        if self.staging is not None:
            self.staging.free()


def kernel_io(ctx, fd: int, nr: int, data: np.ndarray, grid: int = 8, staging=None,
              device: str = "cuda", stream=None):
    """One kernel-granularity write (nr = NR_WRITE) or read (NR_READ) of
    len(data) bytes through `fd`; returns (ret, mismatch)."""
    import torch
    if nr not in (NR_WRITE, NR_READ):
        raise ValueError("nr must be NR_WRITE or NR_READ")
    data = np.ascontiguousarray(data, dtype=np.uint8)
    own = staging is None
    stg = ctx.host_alloc(len(data)) if own else staging
    try:
        d = torch.from_numpy(data.copy()).to(device)
        ret = torch.full((1,), -12345, dtype=torch.int64, device=device)
        mism = torch.zeros(1, dtype=torch.int64, device=device)
        check(lib.gsys_file_kernel_io(ctx.h, fd, nr, d.data_ptr(), len(data), stg.dev,
                                      ret.data_ptr(), mism.data_ptr(), grid, _stream(stream)),
              "gsys_file_kernel_io")
        torch.cuda.synchronize()
        rc = ctx.wait(60_000_000_000)
        if rc:
            raise RuntimeError("drain failed: %d" % rc)
        return int(ret.cpu()[0]), int(mism.cpu()[0])
    finally:
        if own:
            stg.free()
