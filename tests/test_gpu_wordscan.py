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


def test_largest_chunks(gs, tmpdata):
    """Chunks of 64 MiB, the largest the entry point takes: an 80 MiB file in
    two chunks, the second starting inside a planted token, in every form."""
    g, ctx = gs
    from paper_1705_06965_amd.wordscan import WordScanRunner
    rng = np.random.default_rng([170506965, 78])
    vocab = [b"w%d" % i for i in range(300)] + [b"needle", b"x" * 16]
    words = rng.integers(0, len(vocab), 200_000)
    seps = rng.integers(0, 2, 200_000)
    block = b"".join(vocab[w] + (b" " if s_ else b"\n") for w, s_ in zip(words, seps))
    body = bytearray(block * ((80 << 20) // len(block) + 1))
    cut = 64 << 20
    body[cut - 4:cut + 4] = b" needle "          # straddles the chunk edge
    p = os.path.join(tmpdata, "largest_chunks.txt")
    open(p, "wb").write(body)
    qs = [b"needle", b"w7", b"w299", b"x" * 16, b"nee", b"dle"]
    want = oracle.wordcount([p], qs)
    assert want[0, 0] > 0
    r = WordScanRunner(ctx, [p], qs, chunk_max=64 << 20)
    assert r.n_chunks == 2
    for form in (g.PERSISTENT, g.GRAPH, g.PLAIN):
        say("64 MiB chunks", form)
        assert (r.run(form) == want).all(), form
    r.close()


def test_corpus_without_chunks(gs, tmpdata):
    """Files that are all empty give no chunks: every form only zeroes the
    counts (filled with garbage first), and no files at all is a valid call."""
    g, ctx = gs
    from paper_1705_06965_amd.wordscan import WordScanRunner
    paths = []
    for k in range(3):
        p = os.path.join(tmpdata, "empty_%d.txt" % k)
        open(p, "wb").close()
        paths.append(p)
    for ps in (paths, []):
        r = WordScanRunner(ctx, ps, [b"a", b"bc"], chunk_max=4096)
        assert r.n_chunks == 0
        for form in (g.PERSISTENT, g.GRAPH, g.PLAIN):
            r.counts.fill_(-1)
            say("no chunks", len(ps), form)
            got = r.run(form)
            assert got.shape == (len(ps), 2)
            assert not got.any()
            assert not r.counts[:len(ps) * 2].any()
        r.close()


@pytest.mark.parametrize("form", ["persistent", "graph"])
@pytest.mark.parametrize("passes", [2, 5])
def test_passes_in_one_launch(gs, corpus, form, passes):
    """Several passes over the corpus in one persistent launch (the
    measurement form of section 7.1's scan): every count is `passes` times
    the oracle's; one pass of the same runner afterwards gives the oracle's."""
    g, ctx = gs
    from paper_1705_06965_amd.wordscan import WordScanRunner
    c, want = corpus
    r = WordScanRunner(ctx, c.paths, c.queries, chunk_max=65536, persistent_buffers=16)
    fm = g.PERSISTENT if form == "persistent" else g.GRAPH
    say("passes", passes, form)
    got = r.run(fm, passes=passes)
    assert (got == want * passes).all()
    assert (r.run(fm) == want).all()
    r.close()


def test_passes_refused_where_not_meaningful(gs, corpus):
    g, ctx = gs
    import errno
    from paper_1705_06965_amd.wordscan import WordScanRunner
    c, _ = corpus
    r = WordScanRunner(ctx, c.paths[:2], c.queries, chunk_max=65536)
    for form, passes in ((g.PERSISTENT, 0), (g.PLAIN, 2)):
        with pytest.raises(g.GsysError) as e:
            r.launch(form, passes=passes)
        assert e.value.errno == errno.EINVAL
    r.close()


def test_full_corpus_in_the_benchmark_configuration(gs):
    """The benchmark's workload as it is timed: the 2,000-file corpus in
    1 MiB chunks, 128 chunk buffers (64 work-groups of 512), several passes in
    one persistent launch and in its graph form: every count is the passes
    times the oracle's, and a single pass equals the oracle's."""
    g, ctx = gs
    from paper_1705_06965_amd.wordscan import WordScanRunner
    c = synth.wordcount_corpus()
    want = oracle.wordcount(c.paths, c.queries, threads=16)
    r = WordScanRunner(ctx, c.paths, c.queries, chunk_max=1 << 20, persistent_buffers=128)
    say("full corpus, one pass")
    assert (r.run(g.PERSISTENT) == want).all()
    for fm, passes in ((g.PERSISTENT, 3), (g.GRAPH, 2)):
        say("full corpus, passes", passes, fm)
        assert (r.run(fm, passes=passes) == want * passes).all()
    r.close()
