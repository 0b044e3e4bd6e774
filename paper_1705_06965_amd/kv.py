"""Driver of the key-value GET workload (network case study, section 7.3):
builds the GPU-resident table, binds the loopback UDP socket, launches the
persistent server kernel and drives it with the native load generator."""
from __future__ import annotations

import ctypes as C
import socket

import numpy as np

from . import FD_SOCK, KV_BLOCKING, check, lib, _stream

REQ_LEN = 32
REPLY_STRIDE = 1040


def make_requests(req_keys: np.ndarray, ids: np.ndarray | None = None) -> np.ndarray:
    """Request datagrams: u64 id; u8 op = 1; u8 pad[7]; u8 key[16] (id k+1 for row k)."""
    n = len(req_keys)
    r = np.zeros((n, REQ_LEN), dtype=np.uint8)
    ids = np.arange(1, n + 1, dtype=np.uint64) if ids is None else ids.astype(np.uint64)
    r[:, :8] = ids.view(np.uint8).reshape(n, 8)
    r[:, 8] = 1
    r[:, 16:] = req_keys
    return r


def padded_heap(val_off: np.ndarray, val_len: np.ndarray, heap: np.ndarray):
    """Copy every value to a 16-byte aligned offset (the GPU copies replies in
    16-byte pieces)."""
    plen = (val_len.astype(np.uint64) + np.uint64(15)) // np.uint64(16) * np.uint64(16)
    poff = np.cumsum(plen) - plen
    out = np.zeros(int(plen.sum()) + 16, dtype=np.uint8)
    starts = val_off.astype(np.int64)
    lens = val_len.astype(np.int64)
    # byte b of value i goes from heap[val_off[i] + b] to out[poff[i] + b]
    b = np.arange(int(lens.sum())) - np.repeat(np.cumsum(lens) - lens, lens)
    src = np.repeat(starts, lens) + b
    dst = np.repeat(poff.astype(np.int64), lens) + b
    out[dst] = heap[src]
    return poff.astype(np.uint64), out


class KVServer:
    def __init__(self, ctx, keys, val_off, val_len, heap, cap: int | None = None,
                 grid: int = 16, batch: int = 256, device: str = "cuda",
                 pipelined: bool = True):
        import torch
        self.torch = torch
        self.ctx = ctx
        n = len(keys)
        self.cap = int(cap or max(1, 2 * n))   # an empty store still has one bucket
        poff, pheap = padded_heap(val_off, val_len, heap)
        self.keys = torch.from_numpy(np.ascontiguousarray(keys).reshape(-1)).to(device)
        self.voff = torch.from_numpy(poff.view(np.int64)).to(device)
        self.vlen = torch.from_numpy(val_len.astype(np.uint32).view(np.int32)).to(device)
        self.heap = torch.from_numpy(pheap).to(device)
        self.table = torch.zeros(self.cap * 32, dtype=torch.uint8, device=device)
        check(lib.gsys_kv_build(ctx.h, self.table.data_ptr(), self.cap, self.keys.data_ptr(),
                                self.voff.data_ptr(), self.vlen.data_ptr(), n, 0), "gsys_kv_build")
        torch.cuda.synchronize()
        self.sock = socket.socket(socket.AF_INET, socket.SOCK_DGRAM)
        for opt in (socket.SO_RCVBUF, socket.SO_SNDBUF):
            self.sock.setsockopt(socket.SOL_SOCKET, opt, 8 << 20)
        self.sock.bind(("127.0.0.1", 0))
        self.sock.setblocking(False)
        self.port = self.sock.getsockname()[1]
        ctx.allow_fd(self.sock.fileno(), FD_SOCK)
        self.grid = grid
        self.batch = batch
        self.flags = 0 if pipelined else KV_BLOCKING
        self.io_bytes = int(lib.gsys_kv_io_bytes()) * grid
        self.io = ctx.host_alloc(self.io_bytes)
        self.ctl = ctx.host_alloc(64)
        self.served = torch.zeros(1, dtype=torch.int64, device=device)
        self.running = False

    def start(self, stream=None, lifetime_ms: int = 120_000):
        self.ctl.view(np.uint64)[0] = 0
        check(lib.gsys_kv_serve(self.ctx.h, self.sock.fileno(), self.table.data_ptr(), self.cap,
                                self.heap.data_ptr(), self.io.dev, self.io_bytes, self.ctl.dev,
                                self.served.data_ptr(), self.batch, self.grid, self.flags,
                                lifetime_ms,
                                _stream(stream)), "gsys_kv_serve")
        self.running = True

    def stop(self):
        if self.running:
            self.ctl.view(np.uint64)[0] = 1
            self.torch.cuda.synchronize()
            rc = self.ctx.wait(30_000_000_000)
            self.running = False
            if rc:
                raise RuntimeError("drain failed: %d" % rc)

    def close(self):
        self.stop()
        self.ctx.allow_fd(self.sock.fileno(), 0)
        self.sock.close()


def loadgen(port: int, reqs: np.ndarray, threads: int = 4, window: int = 64,
            rto_ns: int = 20_000_000, timeout_ns: int = 60_000_000_000):
    """Run the native UDP load generator; returns (answered, replies[n,1040],
    reply_len[n], lat_ns[n], retransmits)."""
    n = len(reqs)
    reqs = np.ascontiguousarray(reqs, dtype=np.uint8)
    replies = np.zeros((n, REPLY_STRIDE), dtype=np.uint8)
    rlen = np.zeros(n, dtype=np.uint32)
    lat = np.zeros(n, dtype=np.uint64)
    rt = C.c_uint64(0)
    got = lib.gsys_kv_loadgen(port, reqs.ctypes.data, REQ_LEN, n, threads, window, rto_ns,
                              timeout_ns, replies.ctypes.data, REPLY_STRIDE, rlen.ctypes.data,
                              lat.ctypes.data, C.byref(rt))
    return int(got), replies, rlen, lat, int(rt.value)
