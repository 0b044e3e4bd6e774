"""GPU parity of the serving mix: every job's outputs (scan digests, pwrite
file bytes, release readbacks and return values) equal the oracle's, in the
mix and alone, in the persistent and plain forms."""
import os
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def gs():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_06965_amd as g
    ctx = g.Context(ring_slots=1 << 16, device_timeout_ns=60_000_000_000, arena_bytes=16 << 30)
    yield g, ctx
    assert ctx.shutdown() == 0


def sub_stream(js, idx):
    idx = np.asarray(idx)
    arr = js.arrival_ns[idx] - js.arrival_ns[idx[0]]
    return synth.JobStream(kind=js.kind[idx], arrival_ns=arr, arg_off=js.arg_off[idx],
                           arg_len=js.arg_len[idx], content_off=js.content_off[idx],
                           content=js.content)


def check_outputs(sr, js, res, dig, in_path, out_path, label):
    data = synth.file_bytes(in_path)
    out = np.fromfile(out_path, dtype=np.uint8)
    jobs = sr.jobs_np
    n_scan = n_pw = n_rel = 0
    for i in range(len(js.kind)):
        k = int(js.kind[i])
        if k == 0:
            ln, off = int(jobs["len"][i]), int(jobs["off"][i])
            assert res[i] == ln, (label, i, res[i])
            nb = ln // 4096
            offs = off + 4096 * np.arange(nb, dtype=np.uint64)
            want, _ = oracle.pread_fnv(in_path, offs, 4096)
            d0 = int(sr.digest_start[i])
            assert (dig[d0:d0 + nb] == want).all(), (label, i)
            n_scan += 1
        elif k == 1:
            ln, off, src = int(jobs["len"][i]), int(jobs["off"][i]), int(jobs["src"][i])
            assert res[i] == ln, (label, i, res[i])
            assert (out[off:off + ln] == js.content[src:src + ln]).all(), (label, i)
            n_pw += 1
        else:
            assert res[i] == 0, (label, i, res[i])
            off, src, pg = int(jobs["off"][i]), int(jobs["src"][i]), int(jobs["page"][i])
            stamp = data[src + 4096 * pg: src + 4096 * pg + 64]
            assert (out[off:off + 64] == stamp).all(), (label, i)
            assert not out[off + 64:off + 128].any(), (label, i)
            n_rel += 1
    return n_scan, n_pw, n_rel


@pytest.fixture(scope="module")
def mix(gs, tmpdata):
    in_path = synth.random_file(5, 64 << 20, name="c5_in_64m.bin")
    js = synth.job_stream(n_jobs=600, rate_per_s=20000, scan_file_bytes=64 << 20,
                          scan_max_log2_pages=8, pwrite_max_pages=64, arena_blocks=8192)
    return js, in_path


@pytest.mark.parametrize("form", ["persistent", "plain"])
def test_mix_matches_oracle(gs, mix, tmpdata, form):
    g, ctx = gs
    from paper_1705_06965_amd.serve import ServeRun
    js, in_path = mix
    out_path = os.path.join(tmpdata, "serve_out_%s.bin" % form)
    sr = ServeRun(ctx, js, in_path, out_path)
    say("serve", form, "jobs", sr.n)
    res, dig, lat = sr.run(g.PERSISTENT if form == "persistent" else g.PLAIN, max_inflight=64,
                           staging_bytes=(2 << 20) * 32)
    sr.close()
    counts = check_outputs(sr, js, res, dig, in_path, out_path, form)
    assert min(counts) > 0
    assert (lat != np.uint64(2**64 - 1)).all()


def test_default_grid_matches_oracle(gs, mix, tmpdata):
    """The library's default persistent grid (grid 0: 64 work-groups) with
    staging for 128: results equal the oracle's."""
    g, ctx = gs
    from paper_1705_06965_amd.serve import ServeRun
    js, in_path = mix
    out_path = os.path.join(tmpdata, "serve_out_default_grid.bin")
    sr = ServeRun(ctx, js, in_path, out_path)
    say("serve default grid, jobs", sr.n)
    res, dig, lat = sr.run(g.PERSISTENT, max_inflight=256, grid=0,
                           staging_bytes=(2 << 20) * 128)
    sr.close()
    counts = check_outputs(sr, js, res, dig, in_path, out_path, "persistent")
    assert min(counts) > 0
    assert (lat != np.uint64(2**64 - 1)).all()


def test_empty_session_then_a_session(gs, mix, tmpdata):
    """A session of no jobs is a valid call in both forms and through the
    allocation-free entry (the persistent work-groups start, find the stop
    flag and leave); a session run after it gives the oracle's results."""
    g, ctx = gs
    from paper_1705_06965_amd.serve import ServeRun
    js, in_path = mix
    empty = synth.job_stream(n_jobs=0, scan_file_bytes=64 << 20)
    sr = ServeRun(ctx, empty, in_path, os.path.join(tmpdata, "serve_out_empty.bin"))
    for form, entry in ((g.PERSISTENT, None), (g.PLAIN, None),
                        (g.PERSISTENT, g.lib.gsys_serve_run_noalloc)):
        say("serve empty session", form, entry is not None)
        res, dig, lat = sr.run(form, max_inflight=64, staging_bytes=(2 << 20) * 32, entry=entry)
        assert len(res) == 0 and len(lat) == 0
        assert not dig.any()
    sr.close()
    sub = sub_stream(js, np.arange(60))
    out_path = os.path.join(tmpdata, "serve_out_after_empty.bin")
    sr = ServeRun(ctx, sub, in_path, out_path)
    say("serve after empty, jobs", sr.n)
    res, dig, lat = sr.run(g.PERSISTENT, max_inflight=64, staging_bytes=(2 << 20) * 32)
    sr.close()
    counts = check_outputs(sr, sub, res, dig, in_path, out_path, "after empty")
    assert sum(counts) == 60
    assert (lat != np.uint64(2**64 - 1)).all()


def test_jobs_alone_equal_in_mix(gs, mix, tmpdata):
    g, ctx = gs
    from paper_1705_06965_amd.serve import ServeRun
    js, in_path = mix
    out_mix = os.path.join(tmpdata, "serve_mix.bin")
    sr = ServeRun(ctx, js, in_path, out_mix)
    res, dig, _ = sr.run(g.PERSISTENT, max_inflight=128, staging_bytes=(2 << 20) * 32)
    sr.close()
    out_m = np.fromfile(out_mix, dtype=np.uint8)
    for i in (0, 1, 2, 17, 101, 333, 599):
        one = sub_stream(js, [i])
        out1 = os.path.join(tmpdata, "serve_one_%d.bin" % i)
        s1 = ServeRun(ctx, one, in_path, out1)
        r1, d1, _ = s1.run(g.PERSISTENT, max_inflight=1, staging_bytes=(2 << 20) * 4)
        s1.close()
        assert r1[0] == res[i]
        k = int(js.kind[i])
        if k == 0:
            nb = int(js.arg_len[i]) // 4096
            d0 = int(sr.digest_start[i])
            assert (d1[:nb] == dig[d0:d0 + nb]).all()
        elif k == 1:
            off, ln = int(js.arg_off[i]), int(js.arg_len[i])
            o1 = np.fromfile(out1, dtype=np.uint8)
            assert (o1[off:off + ln] == out_m[off:off + ln]).all()
        else:
            o1 = np.fromfile(out1, dtype=np.uint8)
            j1 = s1.jobs_np[0]
            jm = sr.jobs_np[i]
            # the same stamp page and source offset read back the same bytes
            if int(j1["src"]) == int(jm["src"]) and int(j1["page"]) == int(jm["page"]):
                assert (o1[int(j1["off"]):int(j1["off"]) + 128] ==
                        out_m[int(jm["off"]):int(jm["off"]) + 128]).all()


def test_release_readback_matches_oracle_release_job(gs, mix, tmpdata):
    g, ctx = gs
    from paper_1705_06965_amd.serve import ServeRun
    js, in_path = mix
    rel = np.nonzero(js.kind == 2)[0][:5]
    sub = sub_stream(js, rel)
    out_g = os.path.join(tmpdata, "rel_gpu.bin")
    sr = ServeRun(ctx, sub, in_path, out_g)
    res, _, _ = sr.run(g.PERSISTENT, max_inflight=4, staging_bytes=(2 << 20) * 4)
    sr.close()
    out_o = os.path.join(tmpdata, "rel_oracle.bin")
    ifd = os.open(in_path, os.O_RDONLY)
    ofd = os.open(out_o, os.O_RDWR | os.O_CREAT | os.O_TRUNC, 0o600)
    try:
        for j in range(len(rel)):
            rec = sr.jobs_np[j]
            rc, rets = oracle.release_job(ifd, int(rec["src"]), int(rec["page"]), ofd,
                                          int(rec["off"]))
            assert rc == 0 and res[j] == 0
    finally:
        os.close(ifd)
        os.close(ofd)
    a = np.fromfile(out_g, dtype=np.uint8)
    b = np.fromfile(out_o, dtype=np.uint8)
    lo = int(sr.jobs_np["off"].min())
    assert (a[lo:] == b[lo:]).all()


@pytest.mark.parametrize("form", ["persistent", "plain"])
def test_split_scans_match_oracle(gs, tmpdata, form):
    """Scans up to 32 MiB: the persistent form cuts every scan longer than
    its task size (4 MiB here, 8 MiB by default) into tasks run by
    different work-groups (up to 8 per job); digests and return values must
    equal the oracle's, as in the plain form (one work-group per job)."""
    g, ctx = gs
    from paper_1705_06965_amd.serve import ServeRun
    in_path = synth.random_file(6, 64 << 20, name="c6_in_64m.bin")
    js = synth.job_stream(n_jobs=90, rate_per_s=5000, mix=(0.7, 0.2, 0.1),
                          scan_file_bytes=64 << 20, scan_max_log2_pages=13,
                          pwrite_max_pages=16, arena_blocks=64, config=6)
    big = int(((js.kind == 0) & (js.arg_len > (4 << 20))).sum())
    assert big >= 10
    out_path = os.path.join(tmpdata, "serve_split_%s.bin" % form)
    sr = ServeRun(ctx, js, in_path, out_path)
    say("split scans", form, "big", big)
    os.environ["GSYS_SERVE_SPLIT_MIB"] = "4"
    try:
        res, dig, lat = sr.run(g.PERSISTENT if form == "persistent" else g.PLAIN, max_inflight=32,
                               staging_bytes=(2 << 20) * 64)
    finally:
        del os.environ["GSYS_SERVE_SPLIT_MIB"]
    n_scan, n_pw, n_rel = check_outputs(sr, js, res, dig, in_path, out_path, "split-" + form)
    assert n_scan == int((js.kind == 0).sum()) and n_pw + n_rel == len(js.kind) - n_scan
    sr.close()


def test_byte_budget_admission(gs, mix, tmpdata):
    """Admission by buffer bytes: with a 6 MiB budget (three 2 MiB scan or
    release jobs, or many small pwrites) the admitted, unfinished jobs never
    hold more than the budget, and every output still equals the oracle's."""
    g, ctx = gs
    from paper_1705_06965_amd.serve import ServeRun
    js, in_path = mix
    budget = 6 << 20
    out_path = os.path.join(tmpdata, "serve_budget.bin")
    sr = ServeRun(ctx, js, in_path, out_path)
    say("serve byte budget", budget)
    res, dig, lat = sr.run(g.PERSISTENT, max_inflight=512, staging_bytes=(2 << 20) * 32,
                           max_inflight_bytes=budget)
    peak = sr.peak_inflight_bytes
    sr.close()
    assert 0 < peak <= budget, peak
    counts = check_outputs(sr, js, res, dig, in_path, out_path, "budget")
    assert min(counts) > 0
    assert (lat != np.uint64(2**64 - 1)).all()


def test_full_size_scans_default_split(gs, tmpdata):
    """The serving config's largest scans (64 MiB, and 64 MiB - 4 KiB at an
    unaligned-to-the-split offset) at the default 8 MiB task size, next to
    a pwrite and a release: digests, file bytes and return values equal the
    oracle's."""
    g, ctx = gs
    from paper_1705_06965_amd.serve import ServeRun
    in_path = synth.random_file(5, 64 << 20, name="c5_in_64m.bin")
    M = 1 << 20
    kind = np.array([0, 1, 0, 2, 0], dtype=np.uint8)
    content = synth.rng(5, 9).integers(0, 256, 8192, dtype=np.uint8)
    js = synth.JobStream(kind=kind,
                         arrival_ns=np.array([0, 10_000, 20_000, 30_000, 40_000], dtype=np.uint64),
                         arg_off=np.array([0, 0, 4096, 0, 12 * M], dtype=np.uint64),
                         arg_len=np.array([64 * M, 8192, 64 * M - 4096, 2 * M, 32 * M + 4096],
                                          dtype=np.uint64),
                         content_off=np.zeros(5, dtype=np.uint64), content=content)
    out_path = os.path.join(tmpdata, "serve_fullsize.bin")
    sr = ServeRun(ctx, js, in_path, out_path)
    say("serve 64 MiB scans at the default split")
    assert "GSYS_SERVE_SPLIT_MIB" not in os.environ
    res, dig, lat = sr.run(g.PERSISTENT, max_inflight=8, staging_bytes=(2 << 20) * 16)
    sr.close()
    n_scan, n_pw, n_rel = check_outputs(sr, js, res, dig, in_path, out_path, "full-size")
    assert (n_scan, n_pw, n_rel) == (3, 1, 1)


def test_full_session_in_the_benchmark_configuration(gs, tmpdata):
    """The benchmark's serving session as it is timed: 55,000 Poisson jobs at
    20k/s over the 1 GiB file (scans up to 64 MiB in 8 MiB tasks), 64
    work-groups, 256 staging buffers: every job returns what the oracle's
    calls return, every pwrite and release leaves the oracle's bytes in the
    output file, and a sample of 200 scans has the oracle's digests."""
    g, ctx = gs
    from paper_1705_06965_amd.serve import ServeRun
    in_path = synth.random_file(2, 1 << 30, name="c2_1g.bin")
    js = synth.job_stream(n_jobs=55_000, rate_per_s=20_000.0)
    out_path = os.path.join(tmpdata, "serve_out_full.bin")
    sr = ServeRun(ctx, js, in_path, out_path)
    say("serve full session, jobs", sr.n)
    res, dig, lat = sr.run(g.PERSISTENT, max_inflight=512, staging_bytes=(2 << 20) * 256,
                           timeout_ns=300_000_000_000)
    sr.close()
    assert (lat != np.uint64(2**64 - 1)).all()
    jobs = sr.jobs_np
    kind = js.kind
    scan, pw, rel = np.nonzero(kind == 0)[0], np.nonzero(kind == 1)[0], np.nonzero(kind == 2)[0]
    assert (res[scan] == jobs["len"][scan].astype(np.int64)).all()
    assert (res[pw] == jobs["len"][pw].astype(np.int64)).all()
    assert (res[rel] == 0).all()
    data = np.memmap(in_path, dtype=np.uint8, mode="r")
    out = np.memmap(out_path, dtype=np.uint8, mode="r")
    for i in pw:
        off, ln, src = int(jobs["off"][i]), int(jobs["len"][i]), int(jobs["src"][i])
        assert (out[off:off + ln] == js.content[src:src + ln]).all(), i
    for i in rel:
        off, src, pg = int(jobs["off"][i]), int(jobs["src"][i]), int(jobs["page"][i])
        assert (out[off:off + 64] == data[src + 4096 * pg:src + 4096 * pg + 64]).all(), i
        assert not out[off + 64:off + 128].any(), i
    for i in np.random.default_rng(5).choice(scan, 200, replace=False):
        nb = int(jobs["len"][i]) // 4096
        offs = int(jobs["off"][i]) + 4096 * np.arange(nb, dtype=np.uint64)
        want, _ = oracle.pread_fnv(in_path, offs, 4096, threads=8)
        d0 = int(sr.digest_start[i])
        assert (dig[d0:d0 + nb] == want).all(), i
