"""Pins of the CPU oracle against facts outside the oracle itself.

- FNV-1a 64: the published test vectors (tests/golden/fnv1a64_vectors.txt).
- pread plumbing: every (offset, length) pair on tiny files, including EOF
  and zero-length reads, against slicing the file's bytes; bad fds -> -EBADF.
- word counts: a hand-counted fixture (tests/golden/wordcount_small.json),
  Python's bytes.split() counter on generated corpora, planted tokens.
- key-value GET: a Python dict built from the same keys.
- memory release: Linux madvise(2) semantics (zero pages after DONTNEED on
  private anonymous memory).
"""
import collections
import errno
import json
import os
import re

import numpy as np
import pytest

import oracle
import synth

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _vectors():
    out = []
    with open(os.path.join(GOLDEN, "fnv1a64_vectors.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            m = re.match(r'^"(.*)"\s+([0-9a-f]{16})$', line)
            assert m, line
            out.append((m.group(1).encode(), int(m.group(2), 16)))
    return out


@pytest.fixture(scope="module", autouse=True)
def _built():
    oracle.build(force=False)


def test_fnv_published_vectors():
    vec = _vectors()
    assert len(vec) >= 10
    for data, want in vec:
        assert oracle.fnv1a64(data) == want, data


def test_fnv_is_order_sensitive_and_distinguishes_fnv1():
    # FNV-1 (multiply before xor) of "a" is 0xaf63bd4c8601b7be; FNV-1a differs.
    assert oracle.fnv1a64(b"a") != 0xaf63bd4c8601b7be
    assert oracle.fnv1a64(b"ab") != oracle.fnv1a64(b"ba")


def _write(tmpdata, name, data: bytes) -> str:
    p = os.path.join(tmpdata, name)
    with open(p, "wb") as f:
        f.write(data)
    return p


@pytest.mark.parametrize("size", [0, 1, 100, 4095, 4096, 5000])
def test_pread_bruteforce_tiny_files(tmpdata, size):
    data = np.random.default_rng(size + 7).integers(0, 256, size, dtype=np.uint8).tobytes()
    p = _write(tmpdata, "tiny_%d.bin" % size, data)
    offs = np.arange(0, size + 6, dtype=np.uint64)
    for ln in (0, 1, 7, 64, 4096):
        fnv, ret = oracle.pread_fnv(p, offs, ln, threads=3)
        for i, o in enumerate(offs.tolist()):
            want = data[o:o + ln]
            assert ret[i] == len(want), (o, ln)
            assert fnv[i] == oracle.fnv1a64(want), (o, ln)


def test_pread_tiny_config_matches_file_slices(tmpdata):
    os.environ.setdefault("GSYS_DATA_DIR", tmpdata)
    p = synth.random_file(1, 262144, name="pin_c1.bin")
    data = synth.file_bytes(p)
    offs = synth.tiny_offsets(64)
    fnv, ret = oracle.pread_fnv(p, offs, 4096)
    assert (ret == 4096).all()
    for i in range(64):
        assert fnv[i] == oracle.fnv1a64(data[4096 * i:4096 * (i + 1)])
    # distinct blocks of random data: all checksums distinct
    assert len(set(fnv.tolist())) == 64


def test_pread_bad_fd_gives_ebadf():
    lib = oracle.lib()
    offs = np.zeros(2, dtype=np.uint64)
    out = np.zeros(2, dtype=np.uint64)
    ret = np.zeros(2, dtype=np.int64)
    rc = lib.oracle_pread_fnv(987654, offs.ctypes.data, 2, 16, out.ctypes.data,
                              ret.ctypes.data, 1)
    assert rc == 0
    assert (ret == -errno.EBADF).all()
    assert (out == 0xcbf29ce484222325).all()


def test_wordcount_hand_fixture(tmpdata):
    doc = json.load(open(os.path.join(GOLDEN, "wordcount_small.json")))
    p = _write(tmpdata, "wc_hand.txt", doc["text"].encode())
    qs = [k.encode() for k in doc["expected"]]
    counts = oracle.wordcount([p], qs)
    assert counts[0].tolist() == list(doc["expected"].values())


def test_wordcount_vs_bytes_split(tmpdata):
    os.environ["GSYS_DATA_DIR"] = tmpdata
    c = synth.wordcount_corpus(n_files=12, median_bytes=8192, n_vocab=300, tag="pin12")
    counts = oracle.wordcount(c.paths, c.queries, threads=4)
    for f, p in enumerate(c.paths):
        data = open(p, "rb").read()
        assert set(data) <= set(b"abcdefghijklmnopqrstuvwxyz \n")
        cnt = collections.Counter(data.split())
        assert counts[f].tolist() == [cnt.get(q, 0) for q in c.queries]
    # 8 of the 64 queries are not vocabulary words; upper-case ones never match
    assert counts[:, 60:].sum() == 0


def test_wordcount_planted_tokens(tmpdata):
    # a token is counted once wherever it sits: file start, end, next to
    # newlines or runs of delimiters, or straddling a 4 KiB boundary
    q = b"needle"
    body = bytearray(b"x " * 5000)
    for pos in (0, 4093, 8190, len(body) - 6):
        body[pos:pos + 6] = q
    data = bytes(body[:len(body) - 6]) + b"\n" + q  # last token ends at EOF
    p = _write(tmpdata, "planted.txt", data)
    want = collections.Counter(data.split())[q]
    counts = oracle.wordcount([p], [q, b"needl", b"eedle", b"x"])
    assert counts[0, 0] == want
    assert counts[0, 1] == 0 and counts[0, 2] == 0
    assert counts[0, 3] == collections.Counter(data.split())[b"x"]


def test_wordcount_empty_and_delimiter_only_files(tmpdata):
    p0 = _write(tmpdata, "empty.txt", b"")
    p1 = _write(tmpdata, "delims.txt", b" \n \n\n  ")
    counts = oracle.wordcount([p0, p1], [b"a", b" "])
    assert counts.sum() == 0


def test_kv_lookup_vs_dict():
    kv = synth.kv_set(n_keys=2000, n_req=3000, miss_every=16)
    ix = oracle.KVIndex(kv.keys, kv.val_off, kv.val_len, kv.heap)
    d = {kv.keys[i].tobytes(): i for i in range(len(kv.keys))}
    for j in range(len(kv.req_keys)):
        k = kv.req_keys[j].tobytes()
        want = d.get(k, -1)
        assert ix.find(k) == want
        assert want == kv.req_index[j]
        req = int(kv.req_ids[j]).to_bytes(8, "little") + bytes([1]) + bytes(7) + k
        rep = ix.reply(req)
        assert rep[:8] == req[:8]
        if want < 0:
            assert rep[8] == 1 and len(rep) == 16
        else:
            ln = int(kv.val_len[want])
            off = int(kv.val_off[want])
            assert rep[8] == 0
            assert int.from_bytes(rep[10:12], "little") == ln
            assert rep[16:] == kv.heap[off:off + ln].tobytes()
    # a malformed request (wrong op) is answered with status 2
    bad = (5).to_bytes(8, "little") + bytes([7]) + bytes(23)
    assert ix.reply(bad)[8] == 2
    ix.close()


def test_kv_reply_shapes_and_empty_index():
    """The request format fixes every malformed reply: status 2, the id from
    the first 8 bytes (0 when the datagram is shorter), 16 bytes and no value;
    an index of no keys answers every well-formed GET with a miss."""
    kv = synth.kv_set(n_keys=100, n_req=10, miss_every=0)
    ix = oracle.KVIndex(kv.keys, kv.val_off, kv.val_len, kv.heap)
    good = (77).to_bytes(8, "little") + bytes([1]) + bytes(7) + kv.keys[3].tobytes()
    assert ix.reply(good)[8] == 0
    for req in (b"", b"\x01", good[:7], good[:8], good[:31], good + b"\x00", good * 2,
                good[:8] + bytes([2]) + good[9:]):
        rep = ix.reply(req)
        want_id = req[:8] if len(req) >= 8 else bytes(8)
        assert len(rep) == 16 and rep[:8] == want_id and rep[8] == 2, req
        assert rep[9:] == bytes(7)
    ix.close()
    empty = oracle.KVIndex(np.zeros((0, 16), np.uint8), np.zeros(0, np.uint64),
                           np.zeros(0, np.uint32), np.zeros(0, np.uint8))
    for k in range(5):
        key = kv.keys[k].tobytes()
        assert empty.find(key) == -1
        rep = empty.reply(good[:16] + key)
        assert rep[8] == 1 and len(rep) == 16 and rep[:8] == good[:8]
    empty.close()


def test_release_zero_pages_after_dontneed():
    stamp = bytes(range(64))
    rc, before, after = oracle.release(2 << 20, stamp)
    assert rc == 0
    pages = (2 << 20) // 4096
    for p in range(pages):
        want = bytearray(stamp)
        want[0] ^= p & 0xFF
        assert before[p].tobytes() == bytes(want)
    assert not after.any()


def test_release_job_stamp_then_zeros(tmpdata):
    """mmap / pread / pwrite / madvise(MADV_DONTNEED) / pwrite / munmap: the
    output file holds the stamped bytes of the chosen page, then zeros."""
    stamp = np.random.default_rng(21).integers(0, 256, 3 << 20, dtype=np.uint8).tobytes()
    sp = _write(tmpdata, "stamp.bin", stamp)
    op = os.path.join(tmpdata, "rel_out.bin")
    sfd = os.open(sp, os.O_RDONLY)
    ofd = os.open(op, os.O_RDWR | os.O_CREAT | os.O_TRUNC, 0o600)
    try:
        for page, soff, ooff in ((0, 0, 0), (511, 4096 * 7, 128), (37, 12345, 4096)):
            rc, rets = oracle.release_job(sfd, soff, page, ofd, ooff)
            assert rc == 0
            assert rets.tolist() == [0, 2 << 20, 64, 0, 64, 0]
            got = os.pread(ofd, 128, ooff)
            assert got[:64] == stamp[soff + 4096 * page: soff + 4096 * page + 64]
            assert got[64:] == bytes(64)
        # a stamp read past EOF reads fewer bytes; the readback shows it
        rc, rets = oracle.release_job(sfd, len(stamp) - 4096, 1, ofd, 8192)
        assert rets[1] == 4096
        assert os.pread(ofd, 64, 8192) == bytes(64)
    finally:
        os.close(sfd)
        os.close(ofd)


# --------------------------------------------------------------- permutation

def _bits_round(bits: np.ndarray, sigma: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """One round as a gather over the flat bit index 64*i + j of a block
    (numpy's unpackbits on little-endian words numbers the bits that way)."""
    idx = (sigma.astype(np.int64)[:, None] * 64 + tau.astype(np.int64)[None, :]).ravel()
    return bits.reshape(-1, 65536)[:, idx].ravel()


def _permute_file(tmpdata, name, data, sigma, tau, iters, threads=2, file_off=0):
    p = os.path.join(tmpdata, name)
    fd = os.open(p, os.O_RDWR | os.O_CREAT | os.O_TRUNC, 0o600)
    try:
        ret = oracle.permute(fd, data, sigma, tau, iters, file_off=file_off, threads=threads)
    finally:
        os.close(fd)
    return ret, np.fromfile(p, dtype=np.uint8)[file_off:]


@pytest.mark.parametrize("iters", [0, 1, 3])
def test_permute_vs_flat_bit_gather(tmpdata, iters):
    ps = synth.permute_set(n_blocks=3)
    ret, got = _permute_file(tmpdata, "perm_gather.bin", ps.data, ps.sigma, ps.tau, iters)
    assert ret.tolist() == [8192] * 3
    bits = np.unpackbits(ps.data.astype("<u8").view(np.uint8), bitorder="little")
    for _ in range(iters):
        bits = _bits_round(bits, ps.sigma, ps.tau)
    want = np.packbits(bits, bitorder="little")
    assert np.array_equal(got, want)
    if iters == 0:
        assert got.tobytes() == ps.data.astype("<u8").tobytes()


def test_permute_byte_reversal_is_bswap(tmpdata):
    data = synth.permute_set(n_blocks=2).data
    sigma = np.arange(1024, dtype=np.uint16)
    tau = np.array([8 * (7 - j // 8) + j % 8 for j in range(64)], dtype=np.uint8)
    _, got = _permute_file(tmpdata, "perm_bswap.bin", data, sigma, tau, 1)
    assert got.view("<u8").tolist() == data.byteswap().tolist()
    _, got2 = _permute_file(tmpdata, "perm_bswap2.bin", data, sigma, tau, 2)
    assert got2.view("<u8").tolist() == data.tolist()


@pytest.mark.parametrize("r,k", [(1, 1), (5, 3), (1000, 7)])
def test_permute_rotation_closed_form(tmpdata, r, k):
    data = synth.permute_set(n_blocks=2).data
    sigma = ((np.arange(1024) + r) % 1024).astype(np.uint16)
    tau = np.arange(64, dtype=np.uint8)
    _, got = _permute_file(tmpdata, "perm_rot.bin", data, sigma, tau, k)
    want = np.concatenate([np.roll(blk, -k * r) for blk in data.reshape(2, 1024)])
    assert got.view("<u8").tolist() == want.tolist()


def test_permute_order_returns_identity(tmpdata):
    # sigma: 3-cycles on words 0..299, 2-cycles on words 300..499, fixed
    # elsewhere (order 6); tau: 4-cycles on the 64 bits (order 4) -> the
    # round has order lcm(6, 4) = 12: 12 rounds give back the block, 6 and 4
    # rounds do not.
    sigma = np.arange(1024)
    for a in range(0, 300, 3):
        sigma[a:a + 3] = [a + 1, a + 2, a]
    for a in range(300, 500, 2):
        sigma[a:a + 2] = [a + 1, a]
    tau = np.arange(64).reshape(16, 4)[:, [1, 2, 3, 0]].ravel()
    data = synth.permute_set(n_blocks=1).data
    for iters, same in ((12, True), (24, True), (6, False), (4, False)):
        _, got = _permute_file(tmpdata, "perm_order.bin", data, sigma.astype(np.uint16),
                               tau.astype(np.uint8), iters)
        assert (got.view("<u8").tolist() == data.tolist()) == same, iters


def test_permute_keeps_popcounts_and_threads_agree(tmpdata):
    ps = synth.permute_set(n_blocks=9)
    _, a = _permute_file(tmpdata, "perm_t1.bin", ps.data, ps.sigma, ps.tau, 5, threads=1)
    _, b = _permute_file(tmpdata, "perm_t4.bin", ps.data, ps.sigma, ps.tau, 5, threads=4)
    assert np.array_equal(a, b)
    pc = lambda w: np.unpackbits(w.astype("<u8").view(np.uint8)).reshape(-1, 64).sum(1)
    assert sorted(pc(a.view("<u8")).tolist()) == sorted(pc(ps.data).tolist())


def test_permute_offset_bad_fd_and_bad_tables(tmpdata):
    ps = synth.permute_set(n_blocks=2)
    ret, got = _permute_file(tmpdata, "perm_off.bin", ps.data, ps.sigma, ps.tau, 0,
                             file_off=4096)
    assert ret.tolist() == [8192, 8192] and got.tobytes() == ps.data.astype("<u8").tobytes()
    assert oracle.permute(987654, ps.data, ps.sigma, ps.tau, 1).tolist() == [-errno.EBADF] * 2
    bad = ps.sigma.copy()
    bad[3] = 1024
    with pytest.raises(OSError):
        oracle.permute(987654, ps.data, bad, ps.tau, 1)


# ------------------------------------------- wordcount with open/read/close

@pytest.mark.parametrize("chunk", [1, 7, 4096, 1 << 20])
def test_wordcount_open_vs_bytes_split(tmpdata, chunk):
    """Files opened by name and read with read() in pieces of any size give
    the bytes.split() counts and their sizes as byte counts."""
    os.environ["GSYS_DATA_DIR"] = tmpdata
    c = synth.wordcount_corpus(n_files=6, median_bytes=6000, n_vocab=200, tag="pinopen")
    d = os.path.dirname(c.paths[0])
    names = [os.path.basename(p) for p in c.paths]
    counts, rets = oracle.wordcount_open(d, names, c.queries, chunk=chunk, threads=3)
    for f, p in enumerate(c.paths):
        data = open(p, "rb").read()
        assert rets[f] == len(data)
        cnt = collections.Counter(data.split())
        assert counts[f].tolist() == [cnt.get(q, 0) for q in c.queries]


def test_wordcount_open_missing_file_and_subdirectory(tmpdata):
    d = os.path.join(tmpdata, "open_pin")
    os.makedirs(os.path.join(d, "s"), exist_ok=True)
    open(os.path.join(d, "s", "a.txt"), "wb").write(b"x y\nx")
    counts, rets = oracle.wordcount_open(d, ["s/a.txt", "nope.txt"], [b"x", b"y"])
    assert rets.tolist() == [5, -errno.ENOENT]
    assert counts.tolist() == [[2, 1], [0, 0]]


@pytest.mark.parametrize("fb,piece", [(0, 4096), (1, 4096), (15, 7), (4096, 4096), (4097, 4096),
                                      (100_000, 1000), (65_537, 1 << 20)])
def test_file_roundtrip_vs_closed_form(tmpdata, fb, piece):
    """Every write and read returns its piece's length (min(piece, fb - p *
    piece)), the read at the end returns 0, both closes 0; the file holds the
    bytes in piece order (read with Python's own file API) and the read-back
    equals them."""
    d = os.path.join(tmpdata, "rt_%d_%d" % (fb, piece))
    os.makedirs(d, exist_ok=True)
    names = ["f%d.bin" % i for i in range(5)]
    data = np.random.default_rng([fb, piece]).integers(0, 256, (len(names), fb), dtype=np.uint8)
    rets, back = oracle.file_roundtrip(d, names, data, piece, threads=3)
    k = (fb + piece - 1) // piece
    lens = [min(piece, fb - p * piece) for p in range(k)]
    for f, n in enumerate(names):
        r = rets[f].tolist()
        assert r[0] >= 0 and r[k + 2] >= 0                       # the two openat
        assert r[1:k + 1] == lens and r[k + 1] == 0              # writes, close
        assert r[k + 3:2 * k + 3] == lens                        # reads
        assert r[2 * k + 3] == 0 and r[2 * k + 4] == 0           # end of file, close
        with open(os.path.join(d, n), "rb") as fh:
            assert fh.read() == data[f].tobytes()
        assert (back[f] == data[f]).all()


def test_file_roundtrip_failed_openat_ends_the_sequence(tmpdata):
    """A name in a missing subdirectory: openat fails with -ENOENT and no
    later call is made for that file (its entries keep their initial 0)."""
    d = os.path.join(tmpdata, "rt_missing")
    os.makedirs(d, exist_ok=True)
    data = np.full((2, 100), 7, dtype=np.uint8)
    rets, back = oracle.file_roundtrip(d, ["ok.bin", "nodir/x.bin"], data, 64)
    assert rets[1, 0] == -errno.ENOENT and not rets[1, 1:].any()
    assert rets[0, 0] >= 0 and rets[0, 1:3].tolist() == [64, 36]
    assert (back[0] == 7).all() and not back[1].any()
