"""gsys: GPU-issued system calls on MI355X, serviced by a host pool.

Thin ctypes binding of libgsys.so.  Functions keep the C names
(``gsys_init``, ``gsys_allow_fd``, ``gsys_register_buffer``, ``gsys_launch``,
``gsys_wait``, ``gsys_shutdown``, ``gsys_fnv4k``, ...); :class:`Context` wraps
them for Python callers.  This module only marshals arguments: every step of
the path runs in the native library and its gfx950 kernels.  PyTorch is used
by callers only for device memory and streams.

The library must have been built (``python -m paper_1705_06965_amd.build`` or
``__graft_entry__.build()``); importing this module raises if it is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("GSYS_LIB") or os.path.join(_HERE, "libgsys.so")

ABI_VERSION = 3

# slot flags / states / call numbers (mirror include/gsys_abi.h)
ST_FREE, ST_POPULATING, ST_READY, ST_PROCESSING, ST_FINISHED = 0, 1, 2, 3, 4
NR_READ, NR_WRITE, NR_CLOSE, NR_MMAP, NR_MUNMAP = 0, 1, 3, 9, 11
NR_PREAD64, NR_PWRITE64, NR_MADVISE, NR_SENDTO, NR_RECVFROM, NR_OPENAT = 17, 18, 28, 44, 45, 257
PATH_MAX = 256
F_BLOCKING, F_LIST, F_PRODUCER, F_STRONG = 0x1, 0x2, 0x4, 0x8
GRAN_WI, GRAN_WG, GRAN_KERNEL = 0, 1, 2
CELL_STRONG, CELL_BLOCKING = 0x4, 0x8
PLAIN, PERSISTENT, GRAPH = 0, 1, 2
CFG_LEDGER, CFG_NO_DEVICE, CFG_NO_PIN, CFG_SHARED_FDS, CFG_DOORBELL = 0x1, 0x2, 0x4, 0x8, 0x10
KV_BLOCKING = 0x1  # gsys_kv_serve: blocking receive-then-send loop
FD_READ, FD_WRITE, FD_SOCK, FD_DIR = 0x1, 0x2, 0x4, 0x8
BUF_HOST, BUF_DEVICE = 1, 2
NOT_WAITED = -115   # a non-blocking call's result slot before anyone waited


def cell(gran: int, strong: bool, blocking: bool) -> int:
    return gran | (CELL_STRONG if strong else 0) | (CELL_BLOCKING if blocking else 0)


# the 8 legal granularity x ordering x blocking cells (section 4.1)
LEGAL_CELLS = [
    ("WI", "strong", "block"), ("WI", "strong", "nonblock"),
    ("WG", "strong", "block"), ("WG", "strong", "nonblock"),
    ("WG", "relaxed", "block"), ("WG", "relaxed", "nonblock"),
    ("K", "relaxed", "block"), ("K", "relaxed", "nonblock"),
]
_GRAN = {"WI": GRAN_WI, "WG": GRAN_WG, "K": GRAN_KERNEL}


def cell_code(g: str, o: str, b: str) -> int:
    return cell(_GRAN[g], o == "strong", b == "block")


class gsys_config(C.Structure):
    _fields_ = [("abi_version", C.c_uint32), ("device", C.c_int32),
                ("ring_slots", C.c_uint32), ("service_threads", C.c_uint32),
                ("coalesce_max", C.c_uint32), ("coalesce_window_ns", C.c_uint32),
                ("stripe", C.c_uint32), ("flags", C.c_uint32),
                ("arena_bytes", C.c_uint64), ("device_timeout_ns", C.c_uint64),
                ("first_cpu", C.c_int32), ("ledger_capacity", C.c_uint32),
                ("sleep_max", C.c_uint32), ("doorbell_idle_us", C.c_uint32),
                ("reserved", C.c_uint32 * 2)]


class gsys_stats(C.Structure):
    _fields_ = [(n, C.c_uint64) for n in (
        "requests", "host_calls", "bytes_in", "bytes_out", "errors", "rejected", "bundles",
        "merged", "idle_polls", "retired_lo", "claimed", "service_ns")] + [
        ("bundle_hist", C.c_uint64 * 8), ("errno_hist", C.c_uint64 * 8),
        ("doorbell_sleeps", C.c_uint64)]


class gsys_dev_ctx(C.Structure):
    _fields_ = [("ring", C.c_uint64), ("comp", C.c_uint64), ("tail", C.c_uint64),
                ("retired_lo", C.c_uint64), ("ring_mask", C.c_uint64),
                ("comp_mask", C.c_uint64), ("timeout_ticks", C.c_uint64),
                ("sleep_max", C.c_uint32), ("flags", C.c_uint32),
                ("arena", C.c_uint64), ("arena_bytes", C.c_uint64),
                ("doorbell", C.c_uint64), ("sleepers", C.c_uint64),
                ("ksites", C.c_uint64), ("n_ksites", C.c_uint32), ("pad", C.c_uint32)]


class gsys_serve_params(C.Structure):
    _fields_ = [("form", C.c_uint32), ("n", C.c_uint32), ("jobs_dev", C.c_uint64),
                ("jobs_host", C.c_void_p), ("arrival_ns", C.c_void_p),
                ("latency_ns", C.c_void_p), ("max_inflight", C.c_uint32), ("grid", C.c_uint32),
                ("max_inflight_bytes", C.c_uint64), ("digests", C.c_uint64),
                ("n_digests", C.c_uint64), ("content", C.c_uint64),
                ("content_bytes", C.c_uint64), ("staging", C.c_uint64),
                ("staging_bytes", C.c_uint64), ("timeout_ns", C.c_uint64),
                ("peak_inflight_bytes", C.c_uint64)]


class gsys_launch_desc(C.Structure):
    _fields_ = [("kernel", C.c_void_p), ("grid", C.c_uint32 * 3), ("block", C.c_uint32 * 3),
                ("lds_bytes", C.c_uint32), ("mode", C.c_uint32), ("args", C.c_void_p)]


_P = C.c_void_p
_SIGS = {
    "gsys_init": (C.c_int, [C.POINTER(gsys_config), C.POINTER(C.c_void_p)]),
    "gsys_allow_fd": (C.c_int, [_P, C.c_int, C.c_uint32]),
    "gsys_register_buffer": (C.c_int, [_P, C.c_uint64, _P, C.c_uint64, C.c_uint32,
                                       C.POINTER(C.c_uint32)]),
    "gsys_unregister_buffer": (C.c_int, [_P, C.c_uint32]),
    "gsys_host_alloc": (C.c_int, [_P, C.c_uint64, C.POINTER(C.c_void_p),
                                  C.POINTER(C.c_uint64), C.POINTER(C.c_uint32)]),
    "gsys_host_free": (C.c_int, [_P, _P]),
    "gsys_device_ctx": (C.c_int, [_P, C.POINTER(gsys_dev_ctx)]),
    "gsys_launch": (C.c_int, [_P, C.POINTER(gsys_launch_desc), _P]),
    "gsys_wait": (C.c_int, [_P, C.c_uint64]),
    "gsys_stats_get": (C.c_int, [_P, C.POINTER(gsys_stats), C.c_int]),
    "gsys_ledger": (C.c_int64, [_P, _P, C.c_uint64, C.c_int]),
    "gsys_shutdown": (C.c_int, [_P, C.c_uint64]),
    "gsys_strerror": (C.c_char_p, [C.c_int]),
    "gsys_fnv4k": (C.c_int, [_P, C.c_int, C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint64,
                             C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32,
                             C.c_uint32, C.c_uint32, _P]),
    "gsys_fnv4k_consume": (C.c_int, [_P, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32,
                                     C.c_uint64, C.c_uint32, C.c_uint32, _P]),
    "gsys_wordscan": (C.c_int, [_P, C.c_uint64, C.c_uint32, C.c_uint32, C.c_uint64, C.c_uint64,
                                C.c_uint32, C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64,
                                C.c_uint32, C.c_uint32, _P]),
    "gsys_kv_build": (C.c_int, [_P, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64,
                                C.c_uint64, _P]),
    "gsys_kv_io_bytes": (C.c_uint64, []),
    "gsys_kv_serve": (C.c_int, [_P, C.c_int, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64,
                                C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32, C.c_uint32,
                                C.c_uint32, C.c_uint64, _P]),
    "gsys_kv_loadgen": (C.c_int64, [C.c_uint32, _P, C.c_uint32, C.c_uint64, C.c_uint32,
                                    C.c_uint32, C.c_uint64, C.c_uint64, _P, C.c_uint32, _P, _P,
                                    _P]),
    "gsys_wordcount_open_buffer_bytes": (C.c_uint64, [C.c_uint32]),
    "gsys_host_pread_rate": (C.c_int, [_P, _P, _P, C.c_uint64, C.c_uint64, C.c_uint64,
                                       C.c_uint64, C.c_uint32, C.c_uint32,
                                       C.POINTER(C.c_double)]),
    "gsys_serve_run": (C.c_int, [_P, C.POINTER(gsys_serve_params), _P]),
    "gsys_serve_run_noalloc": (C.c_int, [_P, C.POINTER(gsys_serve_params), _P]),
    "gsys_canary": (C.c_int, [_P, C.c_int, C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint64,
                              C.c_uint32, C.c_uint32, _P]),
    "gsys_wordcount_open": (C.c_int, [_P, C.c_int, C.c_uint64, C.c_uint32, C.c_uint64,
                                      C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64,
                                      C.c_uint32, C.c_uint64, C.c_uint64, C.c_uint64,
                                      C.c_uint32, _P]),
    "gsys_permute": (C.c_int, [_P, C.c_int, C.c_uint64, _P, _P, C.c_uint64, C.c_uint32,
                               C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32, _P]),
    "gsys_file_roundtrip": (C.c_int, [_P, C.c_int, C.c_uint64, C.c_uint32, C.c_uint64,
                                      C.c_uint64, C.c_uint32, C.c_uint64, C.c_uint64,
                                      C.c_uint64, C.c_uint64, C.c_uint32, _P]),
    "gsys_file_kernel_io": (C.c_int, [_P, C.c_int, C.c_uint32, C.c_uint64, C.c_uint64,
                                      C.c_uint64, C.c_uint64, C.c_uint64, C.c_uint32, _P]),
}

if not os.path.exists(LIB_PATH):
    raise ImportError("libgsys.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
lib = C.CDLL(LIB_PATH, mode=C.RTLD_GLOBAL)
for _name, (_res, _args) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.restype = _res
    _f.argtypes = _args
    globals()[_name] = _f


class GsysError(OSError):
    pass


def check(rc: int, what: str = "") -> int:
    if rc < 0:
        msg = lib.gsys_strerror(rc).decode()
        raise GsysError(-rc, "%s: %s" % (what, msg) if what else msg)
    return rc


def _ptr(a) -> int:
    if a is None:
        return 0
    if isinstance(a, int):
        return a
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    if hasattr(a, "data_ptr"):
        return int(a.data_ptr())
    raise TypeError("cannot take the address of %r" % type(a))


def _stream(stream) -> int:
    if stream is None:
        return 0
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)


class HostBuffer:
    """Fine-grained host-coherent memory from gsys_host_alloc (registered)."""

    def __init__(self, ctx: "Context", nbytes: int):
        self.ctx = ctx
        h = C.c_void_p()
        d = C.c_uint64()
        i = C.c_uint32()
        check(lib.gsys_host_alloc(ctx.h, nbytes, C.byref(h), C.byref(d), C.byref(i)),
              "gsys_host_alloc")
        self.host = h.value
        self.dev = d.value
        self.id = i.value
        self.nbytes = nbytes
        self.array = np.ctypeslib.as_array((C.c_uint8 * nbytes).from_address(self.host))

    def view(self, dtype, count=None, offset=0):
        a = self.array[offset:]
        if count is not None:
            a = a[:count * np.dtype(dtype).itemsize]
        return a.view(dtype)

    def free(self):
        if self.host and self.ctx.h:
            check(lib.gsys_host_free(self.ctx.h, self.host), "gsys_host_free")
        self.host = None
        self.array = None


class Context:
    """One gsys context: slot ring, completion records, service pool."""

    def __init__(self, ring_slots=0, service_threads=0, coalesce_max=1, coalesce_window_ns=0,
                 stripe=0, flags=0, arena_bytes=0, device_timeout_ns=0, first_cpu=-1, device=0,
                 ledger_capacity=0, sleep_max=0, doorbell_idle_us=0):
        cfg = gsys_config()
        cfg.abi_version = ABI_VERSION
        cfg.device = device
        cfg.ring_slots = ring_slots
        cfg.service_threads = service_threads
        cfg.coalesce_max = coalesce_max
        cfg.coalesce_window_ns = coalesce_window_ns
        cfg.stripe = stripe
        cfg.flags = flags
        cfg.arena_bytes = arena_bytes
        cfg.device_timeout_ns = device_timeout_ns
        cfg.first_cpu = first_cpu
        cfg.ledger_capacity = ledger_capacity
        cfg.sleep_max = sleep_max
        cfg.doorbell_idle_us = doorbell_idle_us
        h = C.c_void_p()
        check(lib.gsys_init(C.byref(cfg), C.byref(h)), "gsys_init")
        self.h = h.value
        self.cfg = cfg
        self._bufs = []

    # whitelist -----------------------------------------------------------
    def allow_fd(self, fd: int, perms: int = FD_READ):
        return check(lib.gsys_allow_fd(self.h, fd, perms), "gsys_allow_fd")

    def register_buffer(self, dev_addr: int, host_addr: int | None, nbytes: int,
                        kind: int = BUF_HOST) -> int:
        i = C.c_uint32()
        check(lib.gsys_register_buffer(self.h, dev_addr, host_addr, nbytes, kind, C.byref(i)),
              "gsys_register_buffer")
        return i.value

    def unregister_buffer(self, bid: int):
        return check(lib.gsys_unregister_buffer(self.h, bid), "gsys_unregister_buffer")

    def host_alloc(self, nbytes: int) -> HostBuffer:
        b = HostBuffer(self, nbytes)
        self._bufs.append(b)
        return b

    # servicing -----------------------------------------------------------
    def device_ctx(self) -> gsys_dev_ctx:
        d = gsys_dev_ctx()
        check(lib.gsys_device_ctx(self.h, C.byref(d)), "gsys_device_ctx")
        return d

    def wait(self, timeout_ns: int = 0) -> int:
        return lib.gsys_wait(self.h, timeout_ns)

    def stats(self, reset: bool = False) -> dict:
        s = gsys_stats()
        check(lib.gsys_stats_get(self.h, C.byref(s), int(reset)), "gsys_stats_get")
        d = {n: getattr(s, n) for n, _ in gsys_stats._fields_[:12]}
        d["bundle_hist"] = list(s.bundle_hist)
        d["errno_hist"] = list(s.errno_hist)
        d["doorbell_sleeps"] = s.doorbell_sleeps
        return d

    def ledger(self, max_records: int = 1 << 22, reset: bool = False) -> np.ndarray:
        out = np.zeros((max_records, 6), dtype=np.uint64)
        n = check(int(lib.gsys_ledger(self.h, out.ctypes.data, max_records, int(reset))),
                  "gsys_ledger")
        return out[:n]

    def shutdown(self, timeout_ns: int = 5_000_000_000) -> int:
        if not self.h:
            return 0
        for b in self._bufs:
            b.host = None
            b.array = None
        rc = lib.gsys_shutdown(self.h, timeout_ns)
        self.h = None
        return rc

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.shutdown()

    # workloads -------------------------------------------------------------
    def fnv4k(self, fd, offsets, n_items, item_bytes, staging, staging_bytes, lists, out_fnv,
              out_ret, cell=0, form=PLAIN, wg_size=256, stream=None):
        return check(lib.gsys_fnv4k(self.h, fd, _ptr(offsets), n_items, item_bytes,
                                    _ptr(staging), staging_bytes, _ptr(lists), _ptr(out_fnv),
                                    _ptr(out_ret), cell, form, wg_size, _stream(stream)),
                     "gsys_fnv4k")


def exported_symbols():
    """Names of the C functions declared in include/*.h."""
    import re
    inc = os.path.join(os.path.dirname(_HERE), "include")
    names = []
    for fn in sorted(os.listdir(inc)):
        if fn.endswith(".h"):
            src = open(os.path.join(inc, fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_ ]*?[\s*]+(gsys_\w+)\s*\(",
                                src, flags=re.M)
    return sorted(set(names))
