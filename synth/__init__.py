"""Seeded synthetic inputs for the GPU system-call workloads.

This module is shared by the oracle and the GPU path and therefore holds only
input generation: random bytes, offsets, file sizes, token streams, key/value
records and job streams.  It contains none of the arithmetic that the method
computes (no checksums, no tokenisation, no hashing, no lookups).

Every stream is ``numpy.random.default_rng([MASTER_SEED, config, stream])``.
Files go to a tmpfs directory (``/dev/shm/gsys`` by default, overridable with
``GSYS_DATA_DIR``) so that they are page-cache resident for both sides.

The workload shapes follow the paper's evaluation: the pread microbenchmarks
of section 6 (Fig. 5, files on tmpfs), the wordcount case study of section 7.1
(64 search strings over many files), the UDP server of section 7.3, the
madvise memory-release use of section 7.2 and the block-permutation array of
section 6 (Fig. 6).  The paper's own datasets (a Linux
source tree on an SSD, miniAMR's input, a NIC) are not available; these
synthetic inputs stand in for them.
"""
from __future__ import annotations

import hashlib
import json
import os
from dataclasses import dataclass, field

import numpy as np

MASTER_SEED = 170506965
PAGE = 4096


def rng(config: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([MASTER_SEED, config, stream])


def data_dir() -> str:
    d = os.environ.get("GSYS_DATA_DIR", "/dev/shm/gsys")
    os.makedirs(d, exist_ok=True)
    return d


def _write_file(path: str, chunks) -> None:
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "wb") as f:
        for c in chunks:
            f.write(memoryview(c))
    os.replace(tmp, path)


def _manifest_ok(path: str, key: dict) -> bool:
    m = path + ".manifest.json"
    if not (os.path.exists(path) and os.path.exists(m)):
        return False
    try:
        with open(m) as f:
            return json.load(f) == key
    except (OSError, ValueError):
        return False


def _manifest_write(path: str, key: dict) -> None:
    with open(path + ".manifest.json", "w") as f:
        json.dump(key, f)


# ---------------------------------------------------------------------------
# pread microbenchmark files (tiny case and the 1 GiB sweep)
# ---------------------------------------------------------------------------

def random_file(config: int, size: int, name: str | None = None,
                piece: int = 64 << 20) -> str:
    """A file of ``size`` seeded uniform random bytes, stream 0 of ``config``.

    Bytes are drawn in pieces of ``piece`` bytes from one generator, so the
    content depends on (config, size, piece) only.
    """
    name = name or "rand_c%d_%d.bin" % (config, size)
    path = os.path.join(data_dir(), name)
    key = {"kind": "random", "config": config, "size": size, "piece": piece,
           "seed": MASTER_SEED}
    if _manifest_ok(path, key) and os.path.getsize(path) == size:
        return path
    g = rng(config, 0)

    def chunks():
        left = size
        while left > 0:
            n = min(piece, left)
            yield np.frombuffer(g.bytes(n), dtype=np.uint8)
            left -= n

    _write_file(path, chunks())
    _manifest_write(path, key)
    return path


def file_bytes(path: str) -> np.ndarray:
    return np.fromfile(path, dtype=np.uint8)


def tiny_offsets(n_items: int = 64, item_bytes: int = PAGE) -> np.ndarray:
    """Item i reads ``item_bytes`` at ``item_bytes * i``."""
    return (np.arange(n_items, dtype=np.uint64) * np.uint64(item_bytes))


def sweep_offsets(n_items: int, n_blocks: int, config: int = 2,
                  item_bytes: int = PAGE) -> np.ndarray:
    """Uniform random ``item_bytes``-aligned offsets (stream 1)."""
    blk = rng(config, 1).integers(0, n_blocks, n_items, dtype=np.int64)
    return blk.astype(np.uint64) * np.uint64(item_bytes)


# ---------------------------------------------------------------------------
# wordcount corpus (section 7.1 stand-in)
# ---------------------------------------------------------------------------

@dataclass
class Corpus:
    paths: list
    sizes: np.ndarray            # uint64 per file
    queries: list                # list of bytes, 64 distinct
    vocab_size: int
    total_bytes: int
    info: dict = field(default_factory=dict)


def _vocabulary(n_words: int, g: np.random.Generator):
    seen = set()
    words = []
    while len(words) < n_words:
        k = n_words - len(words)
        lens = g.integers(3, 13, k)
        letters = g.integers(ord("a"), ord("z") + 1, (k, 12), dtype=np.uint8)
        for i in range(k):
            w = letters[i, :lens[i]].tobytes()
            if w not in seen:
                seen.add(w)
                words.append(w)
    return words


def zipf_cdf(n: int, s: float) -> np.ndarray:
    """Inverse-CDF table of the finite Zipf(s) law over ranks 1..n."""
    w = np.arange(1, n + 1, dtype=np.float64) ** (-s)
    c = np.cumsum(w)
    return c / c[-1]


def zipf_sample(cdf: np.ndarray, u: np.ndarray) -> np.ndarray:
    """0-based ranks for uniforms ``u`` (rank 0 is the most frequent)."""
    r = np.searchsorted(cdf, u, side="right")
    return np.minimum(r, len(cdf) - 1)


def _tokens_to_bytes(ranks, seps, vocab_arr, vocab_len):
    wl = vocab_len[ranks]
    tl = wl + 1
    total = int(tl.sum())
    starts = np.cumsum(tl) - tl
    tok = np.repeat(np.arange(len(ranks)), tl)
    pos = np.arange(total) - starts[tok]
    out = vocab_arr[ranks[tok], np.minimum(pos, 11)]
    sep_mask = pos >= wl[tok]
    out[sep_mask] = seps[tok[sep_mask]]
    return out


def wordcount_corpus(n_files: int = 2000, median_bytes: int = 65536,
                     sigma: float = 1.0, cap_bytes: int = 8 << 20,
                     n_vocab: int = 50000, zipf_s: float = 1.1,
                     config: int = 3, tag: str = "full") -> Corpus:
    """Files of space/newline separated words drawn Zipf(s) from a seeded
    vocabulary; log-normal file sizes; 64 query words."""
    d = os.path.join(data_dir(), "wc_%s" % tag)
    os.makedirs(d, exist_ok=True)
    key = {"kind": "wordcount", "n_files": n_files, "median": median_bytes,
           "sigma": sigma, "cap": cap_bytes, "n_vocab": n_vocab,
           "s": zipf_s, "config": config, "seed": MASTER_SEED, "v": 2}
    g_vocab = rng(config, 0)
    vocab = _vocabulary(n_vocab, g_vocab)
    vocab_len = np.array([len(w) for w in vocab], dtype=np.int64)
    vocab_arr = np.zeros((n_vocab, 12), dtype=np.uint8)
    for i, w in enumerate(vocab):
        vocab_arr[i, :len(w)] = np.frombuffer(w, dtype=np.uint8)

    g_size = rng(config, 1)
    z = g_size.standard_normal(n_files)
    sizes = np.clip(np.round(np.exp(np.log(median_bytes) + sigma * z)),
                    1, cap_bytes).astype(np.uint64)

    g_q = rng(config, 3)
    vset = set(vocab)
    bands = [(0, min(100, n_vocab), 16), (min(100, n_vocab), min(5000, n_vocab), 24),
             (min(5000, n_vocab), n_vocab, 16)]
    chosen = []
    for lo, hi, k in bands:
        pool = np.arange(lo, hi)
        k = min(k, len(pool))
        chosen.extend(int(x) for x in g_q.choice(pool, k, replace=False))
    queries = [vocab[i] for i in chosen]
    # non-vocabulary strings: 4 lower-case misses and 4 with upper-case letters
    while len(queries) < 60:
        ln = int(g_q.integers(3, 13))
        w = g_q.integers(ord("a"), ord("z") + 1, ln, dtype=np.uint8).tobytes()
        if w not in vset and w not in queries:
            queries.append(w)
    while len(queries) < 64:
        ln = int(g_q.integers(3, 13))
        w = g_q.integers(ord("A"), ord("Z") + 1, ln, dtype=np.uint8).tobytes()
        if w not in queries:
            queries.append(w)

    paths = [os.path.join(d, "f%05d.txt" % i) for i in range(n_files)]
    mpath = os.path.join(d, "corpus")
    if not _manifest_ok(mpath, key) or not all(os.path.exists(p) for p in paths):
        cdf = zipf_cdf(n_vocab, zipf_s)
        g_tok = rng(config, 2)
        for i, p in enumerate(paths):
            sz = int(sizes[i])
            ntok = max(4, int(sz / 7.0) + 16)
            buf = np.zeros(0, dtype=np.uint8)
            parts = []
            have = 0
            while have < sz:
                ranks = zipf_sample(cdf, g_tok.random(ntok))
                seps = np.where(g_tok.random(ntok) < 1.0 / 16, 10, 32).astype(np.uint8)
                b = _tokens_to_bytes(ranks, seps, vocab_arr, vocab_len)
                parts.append(b)
                have += len(b)
            buf = np.concatenate(parts)[:sz]
            _write_file(p, [buf])
        with open(mpath, "w") as f:
            f.write("ok\n")
        _manifest_write(mpath, key)
    total = int(sizes.sum())
    return Corpus(paths=paths, sizes=sizes, queries=queries,
                  vocab_size=n_vocab, total_bytes=total,
                  info={"files": n_files, "bytes": total})


# ---------------------------------------------------------------------------
# key-value GET workload (section 7.3 stand-in)
# ---------------------------------------------------------------------------

@dataclass
class KVSet:
    keys: np.ndarray        # uint8 [n, 16]
    val_off: np.ndarray     # uint64 [n]  offset into heap
    val_len: np.ndarray     # uint32 [n]
    heap: np.ndarray        # uint8  [sum(len)]
    req_keys: np.ndarray    # uint8 [m, 16]  (some are planted misses)
    req_ids: np.ndarray     # uint64 [m]
    req_index: np.ndarray   # int64 [m]  index into keys, -1 for a planted miss


def kv_set(n_keys: int = 1_000_000, n_req: int = 4_000_000,
           vmin: int = 32, vmax: int = 1024, zipf_s: float = 0.99,
           miss_every: int = 64, config: int = 4) -> KVSet:
    g = rng(config, 0)
    keys = np.frombuffer(g.bytes(16 * n_keys), dtype=np.uint8).reshape(n_keys, 16).copy()
    # reject duplicate keys (redraw until distinct)
    while True:
        v = keys.view(np.dtype((np.void, 16))).ravel()
        _, first = np.unique(v, return_index=True)
        if len(first) == n_keys:
            break
        dup = np.setdiff1d(np.arange(n_keys), first)
        keys[dup] = np.frombuffer(g.bytes(16 * len(dup)), dtype=np.uint8).reshape(-1, 16)
    gv = rng(config, 1)
    val_len = gv.integers(vmin, vmax + 1, n_keys).astype(np.uint32)
    val_off = (np.cumsum(val_len.astype(np.uint64)) - val_len).astype(np.uint64)
    heap = np.frombuffer(gv.bytes(int(val_len.sum())), dtype=np.uint8).copy()
    gr = rng(config, 2)
    cdf = zipf_cdf(n_keys, zipf_s)
    rank = zipf_sample(cdf, gr.random(n_req))
    perm = rng(config, 3).permutation(n_keys)
    idx = perm[rank].astype(np.int64)
    req_keys = keys[idx].copy()
    if miss_every:
        gm = rng(config, 4)
        miss = np.arange(0, n_req, miss_every)
        mk = np.frombuffer(gm.bytes(16 * len(miss)), dtype=np.uint8).reshape(-1, 16).copy()
        kview = keys.view(np.dtype((np.void, 16))).ravel()
        mview = mk.view(np.dtype((np.void, 16))).ravel()
        if np.isin(mview, kview).any():
            raise RuntimeError("planted miss key collides with a stored key")
        req_keys[miss] = mk
        idx[miss] = -1
    ids = np.arange(1, n_req + 1, dtype=np.uint64)
    return KVSet(keys=keys, val_off=val_off, val_len=val_len, heap=heap,
                 req_keys=req_keys, req_ids=ids, req_index=idx)


# ---------------------------------------------------------------------------
# serving job stream (mixed scan / pwrite / mmap-release jobs)
# ---------------------------------------------------------------------------

JOB_SCAN, JOB_PWRITE, JOB_RELEASE = 0, 1, 2


@dataclass
class JobStream:
    kind: np.ndarray        # uint8
    arrival_ns: np.ndarray  # uint64, scheduled arrival time from t0
    arg_off: np.ndarray     # uint64: scan file offset / pwrite file offset / arena block index
    arg_len: np.ndarray     # uint64: scan bytes / pwrite bytes / release bytes
    content_off: np.ndarray # uint64: offset of pwrite content in the content pool
    content: np.ndarray     # uint8 pool holding all pwrite contents


def job_stream(n_jobs: int = 55_000, rate_per_s: float = 20_000.0,
               mix=(0.10, 0.60, 0.30), scan_file_bytes: int = 1 << 30,
               scan_max_log2_pages: int = 14, pwrite_max_pages: int = 64,
               arena_blocks: int = 8192, release_bytes: int = 2 << 20,
               config: int = 5) -> JobStream:
    g = rng(config, 0)
    gaps = g.exponential(1e9 / rate_per_s, n_jobs)
    arrival = np.cumsum(gaps).astype(np.uint64)
    gk = rng(config, 1)
    u = gk.random(n_jobs)
    kind = np.where(u < mix[0], JOB_SCAN,
                    np.where(u < mix[0] + mix[1], JOB_PWRITE, JOB_RELEASE)).astype(np.uint8)
    ga = rng(config, 2)
    scan_pages = np.round(2.0 ** ga.uniform(0, scan_max_log2_pages, n_jobs)).astype(np.uint64)
    pw_pages = np.round(2.0 ** ga.uniform(0, np.log2(pwrite_max_pages), n_jobs)).astype(np.uint64)
    file_pages = scan_file_bytes // PAGE
    scan_start = (ga.random(n_jobs) * (file_pages - scan_pages + 1)).astype(np.uint64)
    arg_off = np.zeros(n_jobs, dtype=np.uint64)
    arg_len = np.zeros(n_jobs, dtype=np.uint64)
    content_off = np.zeros(n_jobs, dtype=np.uint64)
    s = kind == JOB_SCAN
    arg_off[s] = scan_start[s] * PAGE
    arg_len[s] = scan_pages[s] * PAGE
    w = kind == JOB_PWRITE
    arg_len[w] = pw_pages[w] * PAGE
    # each pwrite job writes its own disjoint range of the output file
    arg_off[w] = np.cumsum(arg_len[w]) - arg_len[w]
    content_off[w] = arg_off[w]
    r = kind == JOB_RELEASE
    arg_off[r] = (np.arange(int(r.sum())) % arena_blocks).astype(np.uint64)
    arg_len[r] = release_bytes
    total_w = int(arg_len[w].sum())
    content = np.frombuffer(rng(config, 3).bytes(total_w), dtype=np.uint8).copy()
    return JobStream(kind=kind, arrival_ns=arrival, arg_off=arg_off, arg_len=arg_len,
                     content_off=content_off, content=content)


# ---------------------------------------------------------------------------
# block permutation + pwrite (the ordering / blocking microbenchmark)
# ---------------------------------------------------------------------------

PERM_BLOCK = 8192          # bytes per block: 1024 little-endian 64-bit words
PERM_WORDS = PERM_BLOCK // 8


@dataclass
class PermuteSet:
    data: np.ndarray   # uint64[n_blocks * 1024], the pre-loaded random array
    sigma: np.ndarray  # uint16[1024]: a permutation of the word positions
    tau: np.ndarray    # uint8[64]: a permutation of the bit positions


def permute_set(n_blocks: int = 8192, config: int = 6) -> PermuteSet:
    """Random array of 8 KiB blocks and the two random shuffles (word order
    and bit order) that one permutation round applies."""
    data = rng(config, 0).integers(0, 1 << 64, n_blocks * PERM_WORDS, dtype=np.uint64,
                                   endpoint=False)
    sigma = rng(config, 1).permutation(PERM_WORDS).astype(np.uint16)
    tau = rng(config, 2).permutation(64).astype(np.uint8)
    return PermuteSet(data=data, sigma=sigma, tau=tau)


def digest(*arrays) -> str:
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).view(np.uint8).tobytes())
    return h.hexdigest()[:16]
