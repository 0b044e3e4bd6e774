"""GPU parity of the open / read / close word search (the wordcount as the
case study of section 7.1 issues it) against the oracle, through the C ABI
(gsys_wordcount_open): every work-group opens its files by name beneath an
allowed directory, reads them with read() and closes them."""
import collections
import errno
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

# Device waits give up after 5 s (a lost request ends as -ETIMEDOUT in
# file_ret), and every launch is awaited with a host deadline that reports
# each work-group's progress record (file, phase, piece, ticket) if it passes.
DEVICE_TIMEOUT_NS = 5_000_000_000
LAUNCH_DEADLINE_S = 60.0


@pytest.fixture(scope="module")
def gs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_06965_amd as g
    ctx = g.Context(ring_slots=1 << 14, device_timeout_ns=DEVICE_TIMEOUT_NS, flags=g.CFG_LEDGER,
                    ledger_capacity=1 << 20)
    yield g, ctx
    assert ctx.shutdown() == 0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def small(tmpdata):
    os.environ["GSYS_DATA_DIR"] = tmpdata
    c = synth.wordcount_corpus(n_files=40, median_bytes=20000, n_vocab=400, tag="gpuopen")
    return c, os.path.dirname(c.paths[0]), [os.path.basename(p) for p in c.paths]


@pytest.mark.parametrize("chunk", [64, 4096, 65536, 1 << 20])
def test_counts_match_oracle(gs, small, chunk):
    g, ctx = gs
    from paper_1705_06965_amd.wordscan import WordOpenRunner
    c, d, names = small
    want, want_ret = oracle.wordcount_open(d, names, c.queries, chunk=chunk, threads=8)
    assert (want == oracle.wordcount(c.paths, c.queries, threads=8)).all()
    r = WordOpenRunner(ctx, d, names, c.queries, chunk=chunk)
    ctx.ledger(reset=True)
    say("wordopen chunk", chunk)
    got, ret = r.run(timeout_s=LAUNCH_DEADLINE_S)
    assert (ret == want_ret).all()
    assert (got == want).all()
    # per file: one openat, reads until one comes back short, one close
    led = ctx.ledger(reset=True)
    nr = collections.Counter(led[:, 1].tolist())
    sizes = np.array([os.path.getsize(p) for p in c.paths])
    assert nr[g.NR_OPENAT] == len(names) and nr[g.NR_CLOSE] == len(names)
    assert nr[g.NR_READ] == int((sizes // chunk + 1).sum())
    assert (led[led[:, 1] == g.NR_CLOSE, 2] == 0).all()
    # every work-group ran out of files (phase 5)
    assert all(p[1] == 5 for p in r.progress_records()), r.progress_records()
    r.close()


def test_piece_edges_eof_and_errors(gs, tmpdata):
    g, ctx = gs
    from paper_1705_06965_amd.wordscan import WordOpenRunner
    d = os.path.join(tmpdata, "wordopen_edges")
    os.makedirs(os.path.join(d, "sub"), exist_ok=True)
    q = b"needle"
    files = {}
    body = bytearray(b"ab " * 3000)
    for pos in (0, 4090, 4093, 8186, 8189, 12282):     # around 4 KiB piece edges
        body[pos:pos + 6] = q
    files["edges.txt"] = bytes(body)
    files["exact.txt"] = (b"x " * 2047 + b"ne") + (b"edle " + b"y " * 2045 + b"z")[:4096]
    files["empty.txt"] = b""
    files["one.txt"] = q
    files["eof.txt"] = b"a " * 2046 + b"q" + q               # token ends at EOF
    files["long.txt"] = b"needleneedleneedleneedle " + q + b"\n" + q * 3
    files["sub/nested.txt"] = b" \n".join([q] * 5000)
    for n, b in files.items():
        open(os.path.join(d, n), "wb").write(b)
    link = os.path.join(d, "escape.txt")
    if not os.path.lexists(link):
        os.symlink(os.path.join(tmpdata, "..", "x.txt"), link)
    names = list(files) + ["missing.txt", "escape.txt", "../wordopen_edges/one.txt"]
    queries = [q, b"ab", b"x", b"y", b"z", b"a", b"needleneedleneedl"[:16]]
    r = WordOpenRunner(ctx, d, names, queries, chunk=4096)
    say("wordopen edges")
    got, ret = r.run(timeout_s=LAUNCH_DEADLINE_S)
    n = len(files)
    want, want_ret = oracle.wordcount_open(d, names[:n], queries, chunk=4096)
    assert (got[:n] == want).all()
    assert ret[:n].tolist() == [len(b) for b in files.values()]
    for f, b in enumerate(files.values()):
        cnt = collections.Counter(b.split())
        assert got[f].tolist() == [cnt.get(x, 0) for x in queries], names[f]
    assert ret[n] == -errno.ENOENT
    assert ret[n + 1] in (-errno.EXDEV, -errno.ELOOP)
    assert ret[n + 2] == -errno.EXDEV
    assert not got[n:].any()
    r.close()


def test_full_corpus(gs):
    """The benchmark's corpus: 2,000 files, 1 MiB pieces, the whole count
    matrix against the oracle."""
    g, ctx = gs
    from paper_1705_06965_amd.wordscan import WordOpenRunner
    c = synth.wordcount_corpus()
    d = os.path.dirname(c.paths[0])
    names = [os.path.basename(p) for p in c.paths]
    r = WordOpenRunner(ctx, d, names, c.queries, chunk=1 << 20)
    ctx.ledger(reset=True)
    say("wordopen full corpus")
    got, ret = r.run(timeout_s=LAUNCH_DEADLINE_S)
    ctx.ledger(reset=True)
    assert ret.tolist() == [os.path.getsize(p) for p in c.paths]
    assert (got == oracle.wordcount(c.paths, c.queries, threads=16)).all()
    r.close()
