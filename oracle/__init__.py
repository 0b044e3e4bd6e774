"""ctypes wrapper of the CPU oracle.  TEST INFRASTRUCTURE ONLY.

The oracle issues the whitelisted POSIX calls directly on the CPU and computes
the consumers' outputs byte by byte (see ``gsys_oracle.c``).  Only the tests,
the smoke check and the benchmark's CPU-baseline leg use it; the GPU path
neither imports nor links it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(_HERE, "gsys_oracle.c")
LIB = os.path.join(_HERE, "liboracle.so")


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no vectorisation flags)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared",
                               "-fPIC", "-pthread", SRC, "-o", tmp])
        os.replace(tmp, LIB)
    return LIB


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            build(force=False)
        L = C.CDLL(LIB)
        u8p = C.POINTER(C.c_uint8)
        L.oracle_fnv1a64.restype = C.c_uint64
        L.oracle_fnv1a64.argtypes = [C.c_void_p, C.c_uint64]
        L.oracle_pread_fnv.restype = C.c_int
        L.oracle_pread_fnv.argtypes = [C.c_int, C.c_void_p, C.c_uint64, C.c_uint32,
                                       C.c_void_p, C.c_void_p, C.c_int]
        L.oracle_wordcount.restype = C.c_int
        L.oracle_wordcount.argtypes = [C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p,
                                       C.c_void_p, C.c_uint32, C.c_uint32, C.c_void_p,
                                       C.c_int]
        L.oracle_file_roundtrip.restype = C.c_int
        L.oracle_file_roundtrip.argtypes = [C.c_int, C.c_void_p, C.c_uint32, C.c_uint32,
                                            C.c_void_p, C.c_uint64, C.c_uint32, C.c_void_p,
                                            C.c_void_p, C.c_int]
        L.oracle_kv_build.restype = C.c_void_p
        L.oracle_kv_build.argtypes = [C.c_void_p, C.c_uint64]
        L.oracle_kv_free.restype = None
        L.oracle_kv_free.argtypes = [C.c_void_p]
        L.oracle_kv_find.restype = C.c_int64
        L.oracle_kv_find.argtypes = [C.c_void_p, C.c_void_p]
        L.oracle_kv_reply.restype = C.c_uint32
        L.oracle_kv_reply.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_uint32, C.c_void_p]
        L.oracle_kv_serve.restype = C.c_int64
        L.oracle_kv_serve.argtypes = [C.c_void_p, C.c_int, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_uint64]
        L.oracle_release.restype = C.c_int
        L.oracle_release.argtypes = [C.c_uint64, C.c_void_p, C.c_void_p, C.c_void_p]
        L.oracle_release_job.restype = C.c_int
        L.oracle_release_job.argtypes = [C.c_int, C.c_uint64, C.c_uint32, C.c_int, C.c_uint64,
                                         C.c_void_p]
        L.oracle_wordcount_open.restype = C.c_int
        L.oracle_wordcount_open.argtypes = [C.c_int, C.c_void_p, C.c_uint32, C.c_uint32,
                                            C.c_uint32, C.c_void_p, C.c_void_p, C.c_uint32,
                                            C.c_uint32, C.c_void_p, C.c_void_p, C.c_int]
        L.oracle_permute.restype = C.c_int
        L.oracle_permute.argtypes = [C.c_int, C.c_void_p, C.c_uint64, C.c_void_p, C.c_void_p,
                                     C.c_uint32, C.c_uint64, C.c_void_p, C.c_int]
        del u8p
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def fnv1a64(data: bytes | np.ndarray) -> int:
    a = np.frombuffer(bytes(data), dtype=np.uint8) if not isinstance(data, np.ndarray) else data
    a = np.ascontiguousarray(a, dtype=np.uint8)
    return int(lib().oracle_fnv1a64(_p(a) if a.size else None, a.size))


def pread_fnv(path: str, offsets: np.ndarray, item_bytes: int = 4096, threads: int = 1):
    """(fnv[u64], ret[i64]) of pread(fd, item_bytes, off) per offset."""
    offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    out = np.zeros(len(offs), dtype=np.uint64)
    ret = np.zeros(len(offs), dtype=np.int64)
    fd = os.open(path, os.O_RDONLY)
    try:
        rc = lib().oracle_pread_fnv(fd, _p(offs), len(offs), item_bytes, _p(out), _p(ret),
                                    threads)
    finally:
        os.close(fd)
    if rc:
        raise OSError(-rc, "oracle_pread_fnv")
    return out, ret


def pack_queries(queries, stride: int = 16):
    q = np.zeros((len(queries), stride), dtype=np.uint8)
    ql = np.zeros(len(queries), dtype=np.uint32)
    for i, w in enumerate(queries):
        if len(w) > stride:
            raise ValueError("query longer than stride")
        q[i, :len(w)] = np.frombuffer(w, dtype=np.uint8)
        ql[i] = len(w)
    return q, ql


def wordcount(paths, queries, threads: int = 1) -> np.ndarray:
    """counts[f, q]: tokens of file f equal to query q (uint32)."""
    q, ql = pack_queries(queries)
    fds = np.array([os.open(p, os.O_RDONLY) for p in paths], dtype=np.int32)
    sizes = np.array([os.fstat(int(fd)).st_size for fd in fds], dtype=np.uint64)
    counts = np.zeros((len(paths), len(queries)), dtype=np.uint32)
    try:
        rc = lib().oracle_wordcount(_p(fds), _p(sizes), len(paths), _p(q), _p(ql),
                                    len(queries), q.shape[1], _p(counts), threads)
    finally:
        for fd in fds:
            os.close(int(fd))
    if rc:
        raise OSError(-rc, "oracle_wordcount")
    return counts


def pack_paths(names, stride: int = 256) -> np.ndarray:
    """NUL-terminated byte strings `stride` bytes apart."""
    out = np.zeros((len(names), stride), dtype=np.uint8)
    for i, n in enumerate(names):
        b = n.encode() if isinstance(n, str) else bytes(n)
        if len(b) >= stride:
            raise ValueError("path longer than stride - 1")
        out[i, :len(b)] = np.frombuffer(b, dtype=np.uint8)
    return out


def wordcount_open(directory: str, names, queries, chunk: int = 1 << 20, threads: int = 1):
    """(counts[f, q], rets[f]): each file opened beneath `directory` by name,
    read with read() in `chunk`-byte pieces, closed, and its tokens counted."""
    q, ql = pack_queries(queries)
    paths = pack_paths(names)
    counts = np.zeros((len(names), len(queries)), dtype=np.uint32)
    rets = np.zeros(len(names), dtype=np.int64)
    dfd = os.open(directory, os.O_RDONLY | os.O_DIRECTORY)
    try:
        rc = lib().oracle_wordcount_open(dfd, _p(paths), len(names), paths.shape[1], chunk, _p(q),
                                         _p(ql), len(queries), q.shape[1], _p(counts), _p(rets),
                                         threads)
    finally:
        os.close(dfd)
    if rc:
        raise OSError(-rc, "oracle_wordcount_open")
    return counts, rets


def file_roundtrip(directory: str, names, data: np.ndarray, piece: int, threads: int = 1):
    """(rets[f, 2K + 5], back[f, file_bytes]): each file created beneath
    `directory`, written with write() in `piece`-byte pieces, closed, opened
    read-only, read back with read() in the same pieces plus a 16-byte read at
    the end, closed.  `data` is nfiles x file_bytes."""
    data = np.ascontiguousarray(data, dtype=np.uint8).reshape(len(names), -1)
    fb = data.shape[1]
    k = (fb + piece - 1) // piece
    paths = pack_paths(names)
    rets = np.zeros((len(names), 2 * k + 5), dtype=np.int64)
    back = np.zeros_like(data)
    dfd = os.open(directory, os.O_RDONLY | os.O_DIRECTORY)
    try:
        rc = lib().oracle_file_roundtrip(dfd, _p(paths), len(names), paths.shape[1], _p(data), fb,
                                         piece, _p(rets), _p(back), threads)
    finally:
        os.close(dfd)
    if rc:
        raise OSError(-rc, "oracle_file_roundtrip")
    return rets, back


class KVIndex:
    """Sorted key index plus reply builder of the key-value GET server."""

    def __init__(self, keys: np.ndarray, val_off: np.ndarray, val_len: np.ndarray,
                 heap: np.ndarray):
        self.keys = np.ascontiguousarray(keys, dtype=np.uint8)
        self.val_off = np.ascontiguousarray(val_off, dtype=np.uint64)
        self.val_len = np.ascontiguousarray(val_len, dtype=np.uint32)
        self.heap = np.ascontiguousarray(heap, dtype=np.uint8)
        self.h = lib().oracle_kv_build(_p(self.keys), len(self.keys))
        if not self.h:
            raise MemoryError("oracle_kv_build")

    def close(self):
        if self.h:
            lib().oracle_kv_free(self.h)
            self.h = None

    def __del__(self):
        self.close()

    def find(self, key: bytes) -> int:
        k = np.frombuffer(key, dtype=np.uint8).copy()
        return int(lib().oracle_kv_find(self.h, _p(k)))

    def reply(self, req: bytes) -> bytes:
        r = np.frombuffer(req, dtype=np.uint8).copy()
        out = np.zeros(16 + 65536, dtype=np.uint8)
        n = lib().oracle_kv_reply(self.h, _p(self.val_off), _p(self.val_len), _p(self.heap),
                                  _p(r), len(r), _p(out))
        return out[:n].tobytes()

    def serve(self, sock_fd: int, n_req: int) -> int:
        return int(lib().oracle_kv_serve(self.h, sock_fd, _p(self.val_off), _p(self.val_len),
                                         _p(self.heap), n_req))


def release(nbytes: int, stamp: bytes):
    """(rc, before[pages,64], after[pages,64]) of the mmap/stamp/madvise cycle."""
    pages = nbytes // 4096
    s = np.frombuffer(stamp, dtype=np.uint8).copy()
    before = np.zeros((pages, 64), dtype=np.uint8)
    after = np.zeros((pages, 64), dtype=np.uint8)
    rc = lib().oracle_release(nbytes, _p(s), _p(before), _p(after))
    return rc, before, after


def release_job(stamp_fd: int, stamp_off: int, page: int, out_fd: int, out_off: int):
    """(rc, rets[6]) of one serving-mix memory-release job on the CPU."""
    rets = np.zeros(6, dtype=np.int64)
    rc = lib().oracle_release_job(stamp_fd, stamp_off, page, out_fd, out_off, _p(rets))
    return rc, rets


def permute(fd: int, data: np.ndarray, sigma: np.ndarray, tau: np.ndarray, iters: int,
            file_off: int = 0, threads: int = 1) -> np.ndarray:
    """ret[b] of pwrite(fd, permute^iters(block b), 8192, file_off + 8192 b)."""
    d = np.ascontiguousarray(data, dtype=np.uint64)
    if d.size % 1024:
        raise ValueError("data is not a whole number of 8 KiB blocks")
    s = np.ascontiguousarray(sigma, dtype=np.uint16)
    t = np.ascontiguousarray(tau, dtype=np.uint8)
    if s.size != 1024 or t.size != 64:
        raise ValueError("sigma needs 1024 entries and tau 64")
    n = d.size // 1024
    ret = np.zeros(n, dtype=np.int64)
    rc = lib().oracle_permute(fd, _p(d), n, _p(s), _p(t), iters, file_off, _p(ret), threads)
    if rc:
        raise OSError(-rc, "oracle_permute")
    return ret
