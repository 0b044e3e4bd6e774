"""GPU parity of the word-search workload (section 7.1 wordcount) against the
oracle: uint32 counts bit-exact, for several chunk sizes (a token belongs to
the chunk in which it starts), both forms."""
import json
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def gs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_06965_amd as g
    ctx = g.Context(ring_slots=1 << 14, device_timeout_ns=60_000_000_000)
    yield g, ctx
    assert ctx.shutdown() == 0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def corpus(gs):
    c = synth.wordcount_corpus(n_files=48, median_bytes=24 << 10, cap_bytes=3 << 20,
                               n_vocab=2000, tag="gpu48")
    want = oracle.wordcount(c.paths, c.queries, threads=8)
    return c, want


@pytest.mark.parametrize("chunk", [1 << 20, 4096, 777])
@pytest.mark.parametrize("form", ["persistent", "plain"])
def test_corpus_counts_match_oracle(gs, corpus, chunk, form):
    g, ctx = gs
    from paper_1705_06965_amd.wordscan import WordScanRunner
    c, want = corpus
    r = WordScanRunner(ctx, c.paths, c.queries, chunk_max=chunk)
    say("wordscan", form, "chunk", chunk, "chunks", r.n_chunks)
    got = r.run(g.PERSISTENT if form == "persistent" else g.PLAIN)
    assert got.shape == want.shape
    assert (got == want).all()
    assert want.sum() > 0
    r.close()


def test_hand_fixture_and_tiny_chunks(gs, tmpdata):
    g, ctx = gs
    from paper_1705_06965_amd.wordscan import WordScanRunner
    doc = json.load(open(os.path.join(GOLDEN, "wordcount_small.json")))
    p = os.path.join(tmpdata, "wc_hand_gpu.txt")
    open(p, "wb").write(doc["text"].encode())
    qs = [k.encode() for k in doc["expected"]]
    want = list(doc["expected"].values())
    for chunk in (1, 2, 3, 7, 13, 4096):
        r = WordScanRunner(ctx, [p], qs, chunk_max=chunk)
        for form in (g.PERSISTENT, g.GRAPH, g.PLAIN):
            say("hand", chunk, form)
            assert r.run(form)[0].tolist() == want
        r.close()


def test_planted_tokens_across_chunk_edges(gs, tmpdata):
    g, ctx = gs
    from paper_1705_06965_amd.wordscan import WordScanRunner
    q = b"needle"
    body = bytearray(b"ab " * 30000)
    pos = [0, 4093, 8190, 16380, 16381 + 9, 65533, len(body) - 6]
    for p_ in pos:
        body[p_:p_ + 6] = q
    body = bytes(body)
    p = os.path.join(tmpdata, "planted_gpu.txt")
    open(p, "wb").write(body)
    qs = [q, b"needl", b"eedle", b"ab", b"abab", b"x" * 16]
    want = oracle.wordcount([p], qs)
    for chunk in (4096, 16384, 65536, 1 << 20):
        r = WordScanRunner(ctx, [p], qs, chunk_max=chunk)
        got = r.run(g.PERSISTENT)
        assert (got == want).all(), (chunk, got, want)
        r.close()


def test_empty_files_and_long_tokens(gs, tmpdata):
    g, ctx = gs
    from paper_1705_06965_amd.wordscan import WordScanRunner
    files = {"e0.txt": b"", "e1.txt": b" \n \n", "l.txt": b"a" * 40 + b" " + b"a" * 16 + b"\n" +
             b"a" * 17 + b" aaaaaaaaaaaaaaaa"}
    paths = []
    for name, data in files.items():
        p = os.path.join(tmpdata, name)
        open(p, "wb").write(data)
        paths.append(p)
    qs = [b"a" * 16, b"a" * 15, b"a"]
    want = oracle.wordcount(paths, qs)
    for chunk in (5, 16, 4096):
        r = WordScanRunner(ctx, paths, qs, chunk_max=chunk)
        for form in (g.PERSISTENT, g.PLAIN):
            assert (r.run(form) == want).all()
        r.close()
