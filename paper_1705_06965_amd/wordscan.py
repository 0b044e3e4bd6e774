"""Driver of the word-search workload (wordcount case study, section 7.1):
builds the chunk table, allocates staging and launches gsys_wordscan."""
from __future__ import annotations

import os

import numpy as np

from . import FD_READ, PERSISTENT, PLAIN, check, lib, _stream

CHUNK_DTYPE = np.dtype([("fd", "<i4"), ("file", "<u4"), ("off", "<u8"), ("len", "<u4"),
                        ("pad", "<u4")])


def chunk_table(fds, sizes, chunk_max: int) -> np.ndarray:
    """Every file cut into chunks of at most chunk_max bytes covering it
    exactly, in file order (an empty file has no chunk)."""
    rows = []
    for f, (fd, size) in enumerate(zip(fds, sizes)):
        size = int(size)
        off = 0
        while off < size:
            ln = min(chunk_max, size - off)
            rows.append((int(fd), f, off, ln, 0))
            off += ln
    return np.array(rows, dtype=CHUNK_DTYPE)


def staging_bytes(chunk_max: int, n_buffers: int) -> int:
    return ((chunk_max + 64 + 15) // 16 * 16) * n_buffers


class WordScanRunner:
    def __init__(self, ctx, paths, queries, chunk_max: int = 1 << 20, device: str = "cuda",
                 persistent_buffers: int = 0):
        import torch
        self.torch = torch
        self.ctx = ctx
        self.fds = [os.open(p, os.O_RDONLY) for p in paths]
        for fd in self.fds:
            ctx.allow_fd(fd, FD_READ)
        self.sizes = np.array([os.fstat(fd).st_size for fd in self.fds], dtype=np.uint64)
        self.nfiles = len(paths)
        self.nq = len(queries)
        self.chunk_max = chunk_max
        tab = chunk_table(self.fds, self.sizes, chunk_max)
        self.n_chunks = len(tab)
        self.total_bytes = int(self.sizes.sum())
        self.chunks = torch.from_numpy(tab.view(np.uint8).copy()).to(device)
        q = np.zeros((self.nq, 16), dtype=np.uint8)
        ql = np.zeros(self.nq, dtype=np.uint32)
        for i, w in enumerate(queries):
            if not 1 <= len(w) <= 16 or b" " in w or b"\n" in w:
                raise ValueError("query %r: 1..16 bytes without delimiters" % (w,))
            q[i, :len(w)] = np.frombuffer(w, dtype=np.uint8)
            ql[i] = len(w)
        self.queries = torch.from_numpy(q).to(device)
        self.qlens = torch.from_numpy(ql.view(np.int32)).to(device)
        self.counts = torch.zeros(max(1, self.nfiles * self.nq), dtype=torch.int32, device=device)
        if not persistent_buffers:
            persistent_buffers = int(os.environ.get("GSYS_WS_BUFFERS", "128"))
        self.persistent_bytes = staging_bytes(chunk_max, min(persistent_buffers,
                                                             2 * max(1, self.n_chunks)))
        self.plain_bytes = staging_bytes(chunk_max, max(1, self.n_chunks))
        self.staging_p = ctx.host_alloc(self.persistent_bytes)
        self.staging_w = None

    def launch(self, form=PERSISTENT, stream=None, passes: int = 1):
        """One launch; the persistent forms scan the corpus `passes` times in
        it (counts add up)."""
        if form == PLAIN:
            if self.staging_w is None:
                self.staging_w = self.ctx.host_alloc(self.plain_bytes)
            st, sb = self.staging_w, self.plain_bytes
        else:
            st, sb = self.staging_p, self.persistent_bytes
        return check(lib.gsys_wordscan(self.ctx.h, self.chunks.data_ptr(), self.n_chunks,
                                       self.chunk_max, self.queries.data_ptr(),
                                       self.qlens.data_ptr(), self.nq, self.counts.data_ptr(),
                                       self.nfiles, st.dev, sb, form, passes, _stream(stream)),
                     "gsys_wordscan")

    def run(self, form=PERSISTENT, stream=None, passes: int = 1):
        self.launch(form, stream, passes)
        self.torch.cuda.synchronize()
        rc = self.ctx.wait(60_000_000_000)
        if rc:
            raise RuntimeError("drain failed: %d" % rc)
        return self.result()

    def result(self):
        return self.counts.cpu().numpy().view(np.uint32)[:self.nfiles * self.nq] \
            .reshape(self.nfiles, self.nq).copy()

    def close(self):
        for fd in self.fds:
            self.ctx.allow_fd(fd, 0)
            os.close(fd)
        self.fds = []


def host_pread_rate(runner: "WordScanRunner", threads: int, reps: int = 3,
                    passes: int = 10) -> float:
    """GB/s at which `threads` host threads pread the runner's chunks, `passes`
    times over, into its persistent staging with no GPU work
    (gsys_host_pread_rate): the host's side of the file scan's roofline."""
    import ctypes as C
    tab = chunk_table(runner.fds, runner.sizes, runner.chunk_max)
    fds = np.ascontiguousarray(np.tile(tab["fd"], passes), dtype=np.int32)
    offs = np.ascontiguousarray(np.tile(tab["off"], passes), dtype=np.uint64)
    lens = np.ascontiguousarray(np.tile(tab["len"], passes), dtype=np.uint32)
    slot = staging_bytes(runner.chunk_max, 1)
    out = C.c_double()
    check(lib.gsys_host_pread_rate(fds.ctypes.data, offs.ctypes.data, lens.ctypes.data, len(lens),
                                   runner.staging_p.host, slot, runner.persistent_bytes // slot,
                                   threads, reps, C.byref(out)), "gsys_host_pread_rate")
    return out.value


def open_buffer_bytes(chunk: int) -> int:
    """Bytes of one of a work-group's two piece buffers in the open form."""
    return int(lib.gsys_wordcount_open_buffer_bytes(chunk))


class WordOpenRunner:
    """The open / read / close form of the word search (gsys_wordcount_open):
    the GPU opens every file beneath `directory` by its name, reads it with
    read() in `chunk`-byte pieces and closes it."""

    def __init__(self, ctx, directory, names, queries, chunk: int = 1 << 20,
                 device: str = "cuda", groups: int = 256):
        import torch
        from . import FD_DIR, PATH_MAX
        self.torch = torch
        self.ctx = ctx
        self.dirfd = os.open(directory, os.O_RDONLY | os.O_DIRECTORY)
        ctx.allow_fd(self.dirfd, FD_READ | FD_DIR)
        self.nfiles = len(names)
        self.nq = len(queries)
        self.chunk = chunk
        self.paths = ctx.host_alloc(max(1, self.nfiles) * PATH_MAX)
        self.paths.array[:max(1, self.nfiles) * PATH_MAX] = 0
        for i, n in enumerate(names):
            b = n.encode() if isinstance(n, str) else bytes(n)
            if len(b) >= PATH_MAX:
                raise ValueError("path %r: at most %d bytes" % (n, PATH_MAX - 1))
            self.paths.array[i * PATH_MAX:i * PATH_MAX + len(b)] = np.frombuffer(b, dtype=np.uint8)
        q = np.zeros((self.nq, 16), dtype=np.uint8)
        ql = np.zeros(self.nq, dtype=np.uint32)
        for i, w in enumerate(queries):
            if not 1 <= len(w) <= 16 or b" " in w or b"\n" in w:
                raise ValueError("query %r: 1..16 bytes without delimiters" % (w,))
            q[i, :len(w)] = np.frombuffer(w, dtype=np.uint8)
            ql[i] = len(w)
        self.queries = torch.from_numpy(q).to(device)
        self.qlens = torch.from_numpy(ql.view(np.int32)).to(device)
        self.counts = torch.zeros(max(1, self.nfiles * self.nq), dtype=torch.int32, device=device)
        self.file_ret = torch.zeros(max(1, self.nfiles), dtype=torch.int64, device=device)
        self.groups = max(1, min(groups, self.nfiles))
        self.staging_bytes = 2 * open_buffer_bytes(chunk) * self.groups
        self.staging = ctx.host_alloc(self.staging_bytes)
        # per work-group progress records (host memory the kernel writes at
        # system scope): where each work-group is, readable while it runs
        self.progress = ctx.host_alloc(16 * self.groups)
        self.progress.array[:16 * self.groups] = 0

    def launch(self, stream=None):
        return check(lib.gsys_wordcount_open(self.ctx.h, self.dirfd, self.paths.dev, self.nfiles,
                                             self.queries.data_ptr(), self.qlens.data_ptr(),
                                             self.nq, self.counts.data_ptr(),
                                             self.file_ret.data_ptr(), self.chunk,
                                             self.staging.dev, self.staging_bytes,
                                             self.progress.dev, self.groups,
                                             _stream(stream)), "gsys_wordcount_open")

    def progress_records(self):
        """One (file or -1, phase, piece, ticket low bits) per work-group."""
        w = self.progress.array[:16 * self.groups].view(np.uint64).reshape(self.groups, 2)
        return [(int(a >> 32) - 1, int(a & 0xffffffff), int(b >> 32), int(b & 0xffffffff))
                for a, b in w.tolist()]

    def run(self, stream=None, timeout_s: float = 0.0):
        """(counts[f, q], bytes read per file or -errno).  With timeout_s the
        launch is awaited with a host-side deadline; past it the work-groups'
        progress records are raised in the error."""
        import time
        self.file_ret.fill_(-12345)
        self.progress.array[:16 * self.groups] = 0
        ev = self.torch.cuda.Event()
        self.launch(stream)
        ev.record()
        if timeout_s:
            t0 = time.monotonic()
            while not ev.query():
                if time.monotonic() - t0 > timeout_s:
                    raise TimeoutError("open-form launch still running after %.0f s; "
                                       "progress (file, phase, piece, ticket) per work-group: %r"
                                       % (timeout_s, self.progress_records()))
                time.sleep(0.002)
        self.torch.cuda.synchronize()
        rc = self.ctx.wait(60_000_000_000)
        if rc:
            raise RuntimeError("drain failed: %d" % rc)
        return self.result()

    def result(self):
        c = self.counts.cpu().numpy().view(np.uint32)[:self.nfiles * self.nq] \
            .reshape(self.nfiles, self.nq).copy()
        return c, self.file_ret.cpu().numpy()[:self.nfiles].copy()

    def close(self):
        self.ctx.allow_fd(self.dirfd, 0)
        os.close(self.dirfd)
        self.paths.free()
        self.staging.free()
        self.progress.free()
