#!/usr/bin/env python3
"""Benchmark: GPU-issued system calls serviced by the host pool on one MI355X.

Workload (one step = one pass): the pread microbenchmark sweep of section 6 at
its full size -- 1024 work-groups x 256 work-items, each work-item's item a
4 KiB pread at a uniform random 4 KiB-aligned offset of a 1 GiB file of seeded
random bytes on tmpfs, followed by the GPU's FNV-1a-64 of the bytes read.  The
timed form is the persistent batched form (work-group list calls, relaxed,
non-blocking, double-buffered, replayed from a hipGraph); the plain form
(one launch, work-item granularity, strong, blocking) is timed beside it.

Prints one JSON line.  value = host pread calls executed for GPU requests per
second over the timed steps (inputs already resident: the file is in the page
cache, offsets in HBM).  The roofline object covers the dominant kernel (the
persistent kernel): algorithmic bytes are the 4 KiB payload of every call,
which crosses the host link once, over the kernel's average duration measured
with HIP events on its stream, against the PCIe 5.0 x16 per-direction link
(and beside it the measured pinned host-to-device copy rate).  The pool size
is chosen per box in the warm-up (tuned size, 12, all cores but one).

The same line carries the metric's other configurations as sub-objects under
"workloads", each with its own roofline or latency figures and CPU baseline:
tiny (64 blocking work-item preads in one launch: end-to-end and per-call
latency), file_scan (the word search over 2,000 files, GB/s), serving (the job mix at
20k jobs/s, jobs/s with p50/p99 from scheduled arrival) and kv (4M GETs over
loopback UDP, GET/s).  --sweep-only times the sweep alone.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

LINK_PEAK_GBPS = 63.0        # PCIe 5.0 x16: 32 GT/s x 16 lanes x 128/130 / 8, per direction
N_WG, WG, ITEM = 1024, 256, 4096
FILE_BYTES = 1 << 30


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--form", default="graph", choices=["graph", "persistent"])
    ap.add_argument("--no-plain", action="store_true", help="skip timing the plain form")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--service-threads", type=int, default=-1,
                    help="host pollers (-1: the autotuned value, 0: cores - 1)")
    ap.add_argument("--no-tuned", action="store_true",
                    help="sweep: ignore the autotuned knobs and use the defaults")
    ap.add_argument("--stripe", type=int, default=0,
                    help="sweep: tickets a poller takes per stripe (0 = the library default, 8)")
    ap.add_argument("--staging-mib", type=int, default=0,
                    help="persistent form: staging ring size (0 = one slot per item)")
    ap.add_argument("--only", default="", help="profiling aid: 'plain' or 'persistent' only")
    ap.add_argument("--kv-grid", type=int, default=0,
                    help="kv: server work-groups (0 = the autotuned value)")
    ap.add_argument("--kv-batch", type=int, default=0,
                    help="kv: datagrams per list call (0 = the autotuned value)")
    ap.add_argument("--kv-clients", type=int, default=4, help="kv: load generator threads")
    ap.add_argument("--kv-window", type=int, default=128, help="kv: outstanding per client")
    ap.add_argument("--kv-doorbell", action="store_true",
                    help="kv: idle pollers block on the GPU's interrupt doorbell")
    ap.add_argument("--serve-jobs", type=int, default=55000, help="serve: jobs in the stream")
    ap.add_argument("--ws-passes", type=int, default=50,
                    help="wordscan: passes over the corpus per persistent launch")
    ap.add_argument("--serve-rate", type=float, default=20000.0, help="serve: arrivals per second")
    ap.add_argument("--serve-inflight", type=int, default=512, help="serve: admission limit")
    ap.add_argument("--serve-ledger", action="store_true",
                    help="serve: record every call and report host service times by call")
    ap.add_argument("--serve-grid", type=int, default=0,
                    help="serve: persistent work-groups (0 = the autotuned value)")
    ap.add_argument("--serve-sleep-max", type=int, default=0,
                    help="serve: cap of the device waiters' backoff (s_sleep steps, 0 = default)")
    ap.add_argument("--serve-ledger-out", default="",
                    help="serve: also save the raw ledger (numpy .npy, one row per call)")
    ap.add_argument("--serve-sweep", default="",
                    help="serve: offered loads (jobs/s, comma-separated) to sweep after the "
                         "main run, about 2.75 s of arrivals each")
    ap.add_argument("--perm-iters", default="1,4,16,64,256,1024,2048,4096",
                    help="permute: permutation rounds per block before the pwrite")
    ap.add_argument("--sweep-only", action="store_true",
                    help="default run: time only the sweep, not the word search, key-value "
                         "and serving configurations beside it")
    ap.add_argument("--workload", default="sweep",
                    choices=["sweep", "tiny", "wordscan", "kv", "serve", "permute",
                             "granularity", "coalesce", "wordopen", "doorbell", "fileio"],
                    help="sweep: the pread microbenchmark sweep (headline); wordscan: the "
                         "word search over 2,000 files")
    ap.add_argument("--db-gap-us", type=int, default=2000,
                    help="doorbell: GPU idle time before each tiny launch")
    ap.add_argument("--db-serve-rate", type=float, default=2000.0,
                    help="doorbell: offered load of the low-load serving run (0 = skip)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy (counter calibration)")
    return ap.parse_args()


COMMON_SOURCES = ["include/gsys_device.hpp", "include/gsys_abi.h"]
PROFILES = {
    "sweep": ("profiles/fnv4k_persistent_pread_sweep_1g.md",
              ["paper_1705_06965_amd/csrc/k_fnv.hip", "paper_1705_06965_amd/csrc/fnv_wave.hpp"]),
    "wordscan": ("profiles/wordscan_persistent_corpus_2000.md",
                 ["paper_1705_06965_amd/csrc/k_wordscan.hip"]),
    "permute": ("profiles/permute_pwrite_64m.md", ["paper_1705_06965_amd/csrc/k_permute.hip"]),
    "tiny": ("profiles/fnv4k_plain_tiny_64.md",
             ["paper_1705_06965_amd/csrc/k_fnv.hip", "paper_1705_06965_amd/csrc/fnv_wave.hpp"]),
    "serve": ("profiles/serve_persistent_mix_20k.md",
              ["paper_1705_06965_amd/csrc/k_serve.hip", "paper_1705_06965_amd/csrc/fnv_wave.hpp"]),
    "kv": ("profiles/kv_serve_get_4m.md", ["paper_1705_06965_amd/csrc/k_kv.hip"]),
}


def profile_traffic(workload):
    """HBM + link bytes per launch of the workload's dominant kernel from the
    committed rocprofv3 counter summary, or None when the kernel sources
    changed since the counters were taken."""
    import hashlib
    prof, sources = PROFILES[workload]
    h = hashlib.sha256()
    for f in sources + COMMON_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    try:
        with open(os.path.join(ROOT, prof)) as fh:
            line = [l for l in fh if l.startswith("machine-readable:")][0]
        d = json.loads(line.split(":", 1)[1])
    except (OSError, IndexError, ValueError):
        return None
    return d["traffic_bytes"] if d.get("source_sha") == h.hexdigest()[:16] else None


def oracle_leg(args):
    """The oracle, for the CPU-baseline leg only: its timed runs and the
    comparison of its results with the GPU's.  None with --no-cpu, so that
    no other part of a run loads it."""
    if args.no_cpu:
        return None
    import oracle
    return oracle


def percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return None
    k = min(len(xs) - 1, max(0, int(round(q / 100.0 * (len(xs) - 1)))))
    return xs[k]


def main():
    args = parse()
    # the pool (and the host pread probe) give every poller its own open file
    # description of every allowed file: 2,000 files x 15 threads need more
    # descriptors than a default soft limit allows
    import resource
    soft, hard = resource.getrlimit(resource.RLIMIT_NOFILE)
    want = hard if hard != resource.RLIM_INFINITY else 1 << 20
    if soft != resource.RLIM_INFINITY and soft < want:
        resource.setrlimit(resource.RLIMIT_NOFILE, (min(want, 1 << 20), hard))
    if args.gpus != 1:
        print("bench.py measures one GPU: a gsys context drives one GPU, and there is no "
              "multi-GPU path (each GPU would run its own ring and host pool); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    if args.copy_calibration:
        a = torch.empty(1 << 30, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": 1 << 30, "copies": 3}))
        return
    if args.workload == "wordscan":
        return run_wordscan(args)
    if args.workload == "kv":
        return run_kv(args)
    if args.workload == "serve":
        return run_serve(args)
    if args.workload == "permute":
        return run_permute(args)
    if args.workload == "tiny":
        return run_tiny(args)
    if args.workload == "wordopen":
        return run_wordopen(args)
    if args.workload == "granularity":
        return run_granularity(args)
    if args.workload == "doorbell":
        return run_doorbell(args)
    if args.workload == "fileio":
        return run_fileio(args)
    if args.workload == "coalesce":
        return run_coalesce(args)
    res = run_sweep(args)
    if not args.sweep_only:
        # the other four configurations of the metric, each with its own
        # roofline (or latency figures) and CPU baseline, in the same line
        peak = measure_h2d()
        res["roofline"]["peak_measured_h2d"] = peak
        res["roofline"]["frac_of_measured_h2d"] = round(res["roofline"]["achieved"] / peak, 4)
        res["workloads"] = {}
        # serving before key-value: right after the key-value phase (every
        # core busy for ~15 s) a serving session measured p99 13 ms against
        # 1.7-1.8 ms on its own on the same box
        for name, fn in (("tiny", run_tiny), ("file_scan", run_wordscan), ("serving", run_serve),
                         ("kv", run_kv)):
            sub = fn(args, sub=True)
            if "roofline" in sub and sub["roofline"].get("unit") == "GB/s":
                sub["roofline"]["peak_measured_h2d"] = peak
                sub["roofline"]["frac_of_measured_h2d"] = \
                    round(sub["roofline"]["achieved"] / peak, 4)
            res["workloads"][name] = sub
            print("%s done" % name, file=sys.stderr, flush=True)
    print(json.dumps(res), flush=True)


SUB_DROP = ("metric", "n_gpus", "higher_is_better", "scaling", "vs_baseline", "data", "dtype")


def emit(res, sub):
    """Print a workload's line, or hand it back as a sub-object."""
    if sub:
        return {k: v for k, v in res.items() if k not in SUB_DROP}
    print(json.dumps(res), flush=True)
    return res


def measure_h2d(nbytes=1 << 30, reps=5):
    """Host-to-device copy rate of pinned host memory (GB/s), the measured
    ceiling beside the link's nominal 63 GB/s."""
    import torch
    h = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    d = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    d.copy_(h, non_blocking=True)
    torch.cuda.synchronize()
    best = 0.0
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        d.copy_(h, non_blocking=True)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del h, d
    return round(best, 2)


def run_sweep(args):
    """The headline: the pread sweep (see the module docstring)."""
    import numpy as np
    import torch
    import synth
    import paper_1705_06965_amd as g
    from paper_1705_06965_amd.fnv import FnvRunner

    t_setup = time.time()
    path = synth.random_file(2, FILE_BYTES, name="c2_1g.bin")
    n = N_WG * WG
    offs = synth.sweep_offsets(n, FILE_BYTES // ITEM)
    # warm the page cache
    with open(path, "rb") as f:
        while f.read(64 << 20):
            pass
    print("setup %.1fs" % (time.time() - t_setup), file=sys.stderr, flush=True)

    from paper_1705_06965_amd import autotune
    tp = dict(autotune.DEFAULTS) if args.no_tuned else autotune.load("sweep")
    cores = len(os.sched_getaffinity(0))
    pool_trials = None
    if args.service_threads >= 0:
        tp["service_threads"] = args.service_threads
    elif not args.no_tuned and args.form == "graph":
        # The pool size that suits this host, chosen in the warm-up: the
        # host's pread cost differs between machines of one type, and the
        # tuned size came from one of them.
        stream0 = torch.cuda.current_stream()
        pool_trials = {}
        for P in sorted({int(tp["service_threads"]) or cores - 1, 12, 14, cores - 1}):
            if not 1 <= P <= cores - 1:
                continue
            c0 = g.Context(ring_slots=tp["ring_slots"], service_threads=P,
                           sleep_max=tp["sleep_max"], device_timeout_ns=60_000_000_000)
            r0 = FnvRunner(c0, path, offs, ITEM, wg_size=tp["wg_size"])
            rates = []
            for k in range(6):
                t0 = time.perf_counter()
                r0.launch(0, g.GRAPH, stream0)
                torch.cuda.synchronize()
                if c0.wait(60_000_000_000):
                    raise RuntimeError("drain failed")
                if k >= 2:
                    rates.append(n / (time.perf_counter() - t0))
            r0.close()
            c0.shutdown()
            # the median of four launches: one lucky launch does not pick P
            pool_trials[P] = round(float(np.median(rates)), 1)
        tp["service_threads"] = max(pool_trials, key=pool_trials.get)
        print("pool trials %s -> %d pollers" % (pool_trials, tp["service_threads"]),
              file=sys.stderr, flush=True)
    ctx = g.Context(ring_slots=tp["ring_slots"], service_threads=tp["service_threads"],
                    coalesce_max=tp["coalesce_max"], coalesce_window_ns=tp["coalesce_window_ns"],
                    sleep_max=tp["sleep_max"], stripe=max(0, args.stripe),
                    device_timeout_ns=60_000_000_000)
    r = FnvRunner(ctx, path, offs, ITEM, wg_size=tp["wg_size"],
                  staging_bytes=args.staging_mib << 20)
    rp = r if (not args.staging_mib and tp["wg_size"] == WG) else \
        FnvRunner(ctx, path, offs, ITEM, wg_size=WG)
    stream = torch.cuda.current_stream()
    form = g.GRAPH if args.form == "graph" else g.PERSISTENT

    def step(cell, fm, ev=None, on=None):
        runner = on if on is not None else (r if fm != g.PLAIN else rp)
        if ev:
            ev[0].record(stream)
        runner.launch(cell, fm, stream)
        if ev:
            ev[1].record(stream)
        torch.cuda.synchronize()
        rc = runner.ctx.wait(60_000_000_000)
        if rc:
            raise RuntimeError("drain failed %d" % rc)

    def timed(cell, fm, steps, warmup, on=None):
        c = on.ctx if on is not None else ctx
        for _ in range(warmup):
            step(cell, fm, on=on)
        torch.cuda.synchronize()
        c.stats(reset=True)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        wall = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            s0 = time.perf_counter()
            step(cell, fm, evs[i], on=on)
            wall.append(time.perf_counter() - s0)
        torch.cuda.synchronize()
        total = time.perf_counter() - t0
        kern_ms = [a.elapsed_time(b) for a, b in evs]
        st = c.stats()
        return total, wall, kern_ms, st

    out = {}
    persistent_cell = 0
    if args.only != "plain":
        total, wall, kern_ms, st = timed(persistent_cell, form, args.steps, args.warmup)
        f, ret = r.result()
        if not (ret == ITEM).all():
            raise RuntimeError("persistent form: unexpected return values")
        out["persistent"] = (total, wall, kern_ms, st)
        print("persistent: %.2f ms/step, kernel %.2f ms, host calls %d" %
              (1e3 * total / args.steps, np.mean(kern_ms), st["host_calls"]),
              file=sys.stderr, flush=True)
    plain_cell = g.cell_code("WI", "strong", "block")
    if not args.no_plain and args.only != "persistent":
        psteps = max(3, args.steps // 2)
        total, wall, kern_ms, st = timed(plain_cell, g.PLAIN, psteps, 1)
        f2, ret2 = rp.result()
        out["plain"] = (total, wall, kern_ms, st)
        print("plain: %.2f ms/step, kernel %.2f ms" % (1e3 * total / psteps, np.mean(kern_ms)),
              file=sys.stderr, flush=True)
        if "persistent" in out and not ((f2 == f).all() and (ret2 == ret).all()):
            raise RuntimeError("plain and persistent forms disagree")
        if tp["service_threads"] not in (0, len(os.sched_getaffinity(0)) - 1):
            # the plain form may prefer a different pool size than the
            # tuned persistent one: time it on the full pool as well
            ctx2 = g.Context(ring_slots=tp["ring_slots"], sleep_max=tp["sleep_max"],
                             device_timeout_ns=60_000_000_000)
            rp2 = FnvRunner(ctx2, path, offs, ITEM, wg_size=WG)
            out["plain_full"] = timed(plain_cell, g.PLAIN, psteps, 1, on=rp2)
            f3, ret3 = rp2.result()
            if not ((f3 == f2).all() and (ret3 == ret2).all()):
                raise RuntimeError("plain form differs between pools")
            rp2.close()
            ctx2.shutdown()

    cpu = None
    oracle = oracle_leg(args)
    if oracle:
        threads = len(os.sched_getaffinity(0))
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            of, orr = oracle.pread_fnv(path, offs, ITEM, threads=threads)
        dt = time.perf_counter() - t0
        if "persistent" in out and not (of == f).all():
            raise RuntimeError("GPU checksums differ from the oracle")
        # the same oracle on one thread, over the first eighth of the items
        n1 = max(1, n // 8)
        t0 = time.perf_counter()
        of1, _ = oracle.pread_fnv(path, offs[:n1], ITEM, threads=1)
        dt1 = time.perf_counter() - t0
        if "persistent" in out and not (of1 == f[:n1]).all():
            raise RuntimeError("GPU checksums differ from the oracle")
        cpu = {"value": round(reps * n / dt, 1), "unit": "syscalls/s", "cores": threads,
               "kind": "oracle",
               "sample": "%d full passes of the sweep (%d preads of 4 KiB + FNV-1a each), "
                         "items split over %d POSIX threads" % (reps, n, threads),
               "one_thread": {"value": round(n1 / dt1, 1), "unit": "syscalls/s",
                              "sample": "the first %d items on one thread" % n1}}

    key = "persistent" if "persistent" in out else "plain"
    total, wall, kern_ms, st = out[key]
    steps = len(wall)
    calls_per_step = n
    value = calls_per_step * steps / total
    gbps = calls_per_step * ITEM * steps / total / 1e9
    kavg_ms = float(np.mean(kern_ms))
    achieved = calls_per_step * ITEM / (kavg_ms * 1e-3) / 1e9
    res = {
        "metric": "GPU-issued syscalls/s + pread-scan GB/s (frac of link roofline); p99 latency",
        "value": round(value, 1),
        "unit": "syscalls/s",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(1e3 * total / steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "pread sweep: 1024 work-groups x 256 work-items, one 4 KiB pread "
                               "each at uniform random 4 KiB-aligned offsets of a 1 GiB "
                               "seeded random file on tmpfs + FNV-1a-64 per item",
                   "form": "persistent batched (%s)" % args.form,
                   "calls_per_step": calls_per_step,
                   "service_threads": int(ctx.cfg.service_threads) or
                   len(os.sched_getaffinity(0)) - 1,
                   "staging_bytes": r.staging_bytes,
                   "tuned": {k: v for k, v in tp.items()},
                   "pool_trials_calls_per_s": pool_trials,
                   "stripe": min(64, max(int(ctx.cfg.stripe) or 8,
                                         min(64, int(ctx.cfg.coalesce_max)))),
                   "ring_slots": int(ctx.cfg.ring_slots)},
        "pread_GBps": round(gbps, 2),
        "link_frac": round(gbps / LINK_PEAK_GBPS, 4),
        "step_ms_p50": round(1e3 * percentile(wall, 50), 3),
        "step_ms_p99": round(1e3 * percentile(wall, 99), 3),
        "roofline": {"bound": "host-link", "achieved": round(achieved, 2),
                     "peak": LINK_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / LINK_PEAK_GBPS, 4),
                     "traffic": profile_traffic("sweep") if key == "persistent" else None,
                     "kernel": "fnv4k_persistent", "kernel_ms": round(kavg_ms, 3),
                     "bytes_per_launch": calls_per_step * ITEM},
        "host": {"calls": st["host_calls"] // steps, "requests": st["requests"] // steps,
                 "merged": st["merged"] // steps,
                 "service_us_per_call": round(st["service_ns"] / max(1, st["host_calls"]) / 1e3, 3),
                 "pool_busy_frac": round(st["service_ns"] / 1e9 / max(1e-9, total) /
                                         max(1, int(ctx.cfg.service_threads) or
                                             len(os.sched_getaffinity(0)) - 1), 3)},
    }
    if "plain" in out and "persistent" in out:
        pt, pw, pk, _ = out["plain"]
        pv = calls_per_step * len(pw) / pt
        res["plain_form"] = {"value": round(pv, 1), "unit": "syscalls/s",
                             "ms_per_step": round(1e3 * pt / len(pw), 3),
                             "kernel_ms": round(float(np.mean(pk)), 3)}
        res["persistent_over_plain"] = round(value / pv, 3)
        # the plain form on all the pollers it can have (its best pool): the
        # same run when the persistent form's pool is already all of them
        res["persistent_over_best_plain"] = res["persistent_over_plain"]
        if "plain_full" in out:
            qt, qw, qk, _ = out["plain_full"]
            qv = calls_per_step * len(qw) / qt
            res["plain_form_full_pool"] = {"value": round(qv, 1), "unit": "syscalls/s",
                                           "service_threads": len(os.sched_getaffinity(0)) - 1,
                                           "ms_per_step": round(1e3 * qt / len(qw), 3)}
            res["persistent_over_best_plain"] = round(value / max(pv, qv), 3)
    # the host's side of the roofline: the same preads into the same staging
    # on as many host threads as the pool has, without the GPU
    hp = r.host_pread_rate(res["config"]["service_threads"])
    res["roofline"]["host_pread_GBps"] = round(hp, 2)
    res["roofline"]["host_pread_calls_per_s"] = round(hp * 1e9 / ITEM, 1)
    res["roofline"]["frac_of_host_pread"] = round(achieved / hp, 4)
    # context: the kernel-split model (section 2, Fig. 1 left).  The host
    # has just read every item into staging (the probe above, item i at
    # staging + i * 4 KiB); one kernel then checksums them all.  Its time is
    # the host's reads followed by that kernel, nothing overlapped.
    if r.staging_bytes >= calls_per_step * ITEM:
        from paper_1705_06965_amd.fnv import consume
        rets = torch.full((calls_per_step,), ITEM, dtype=torch.int64, device="cuda")
        out_split = torch.zeros(calls_per_step, dtype=torch.int64, device="cuda")
        ks = []
        for _ in range(4):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            consume(ctx, r.staging.dev, rets, ITEM, out_split, stream=stream)
            e1.record(stream)
            torch.cuda.synchronize()
            ks.append(e0.elapsed_time(e1))
        if not torch.equal(out_split, r.out_fnv):
            raise RuntimeError("kernel-split checksums differ from the persistent form's")
        host_ms = calls_per_step * ITEM / (hp * 1e9) * 1e3
        kms = float(np.median(ks[1:]))
        res["kernel_split"] = {"value": round(calls_per_step / ((host_ms + kms) * 1e-3), 1),
                               "unit": "syscalls/s", "host_pread_ms": round(host_ms, 3),
                               "kernel_ms": round(kms, 3)}
    if cpu:
        res["cpu_baseline"] = cpu
    r.close()
    if rp is not r:
        rp.close()
    ctx.shutdown()
    return res


def run_wordscan(args, sub=False):
    """Word search: 2,000 files (log-normal sizes, median 64 KiB, cap 8 MiB) of
    Zipf(1.1) words from a 50k-word vocabulary; 64 queries; 1 MiB chunks.
    value = scanned file bytes per second (GB/s) over the timed passes."""
    import numpy as np
    import torch
    import synth
    import paper_1705_06965_amd as g
    from paper_1705_06965_amd.wordscan import WordScanRunner
    t0 = time.time()
    c = synth.wordcount_corpus()
    for p in c.paths:
        with open(p, "rb") as f:
            f.read()
    print("corpus %d files %.1f MiB, setup %.1fs" % (len(c.paths), c.total_bytes / 2**20,
                                                     time.time() - t0), file=sys.stderr, flush=True)
    from paper_1705_06965_amd import autotune
    tw_ = autotune.load("wordscan")
    pollers = args.service_threads if args.service_threads >= 0 else tw_["service_threads"]
    ctx = g.Context(ring_slots=1 << 16, service_threads=pollers, sleep_max=tw_["sleep_max"],
                    device_timeout_ns=60_000_000_000)
    r = WordScanRunner(ctx, c.paths, c.queries, chunk_max=1 << 20,
                       persistent_buffers=tw_["buffers"])
    stream = torch.cuda.current_stream()

    def timed(form, steps, warmup, passes=1):
        for _ in range(warmup):
            r.launch(form, stream, passes)
            torch.cuda.synchronize()
            ctx.wait(60_000_000_000)
        ctx.stats(reset=True)
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(steps)]
        wall = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            s0 = time.perf_counter()
            evs[i][0].record(stream)
            r.launch(form, stream, passes)
            evs[i][1].record(stream)
            torch.cuda.synchronize()
            if ctx.wait(60_000_000_000):
                raise RuntimeError("drain failed")
            wall.append(time.perf_counter() - s0)
        total = time.perf_counter() - t0
        return total, wall, [a.elapsed_time(b) for a, b in evs], ctx.stats()

    # the persistent form scans the corpus `passes` times per launch (work-groups
    # go from pass to pass without draining); single-pass launches beside it
    passes = max(1, args.ws_passes)
    single = timed(g.PERSISTENT, args.steps, args.warmup)
    counts = r.result()
    tp = timed(g.PERSISTENT, max(3, args.steps // 4), 1, passes)
    if not (r.result() == counts * passes).all():
        raise RuntimeError("multi-pass counts are not passes x the single-pass counts")
    tw = None
    if not args.no_plain:
        tw = timed(g.PLAIN, max(3, args.steps // 2), 1)
        if not (r.result() == counts).all():
            raise RuntimeError("plain and persistent forms disagree")
    cpu = None
    oracle = oracle_leg(args)
    if oracle:
        threads = len(os.sched_getaffinity(0))
        t1 = time.perf_counter()
        want = oracle.wordcount(c.paths, c.queries, threads=threads)
        dt = time.perf_counter() - t1
        if not (want == counts).all():
            raise RuntimeError("GPU counts differ from the oracle")
        cpu = {"value": round(c.total_bytes / dt / 1e9, 3), "unit": "GB/s", "cores": threads,
               "kind": "oracle", "sample": "one full pass over the 2,000-file corpus "
                                           "(files split over %d POSIX threads)" % threads}
    total, wall, kern_ms, st = tp
    steps = len(wall)
    gbps = c.total_bytes * passes * steps / total / 1e9
    kavg = float(np.mean(kern_ms))
    link_bytes = st["bytes_in"] / steps        # bytes the host delivered per pass
    achieved = link_bytes / (kavg * 1e-3) / 1e9
    res = {
        "metric": "GPU-issued syscalls/s + pread-scan GB/s (frac of link roofline); p99 latency",
        "value": round(gbps, 3), "unit": "GB/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * total / steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "word search: 2,000 files, log-normal sizes (median 64 KiB, "
                               "sigma 1, cap 8 MiB), Zipf(1.1) words from a 50k vocabulary, "
                               "64 queries, 1 MiB chunk preads", "form": "persistent",
                   "passes_per_launch": passes,
                   "files": len(c.paths), "bytes": c.total_bytes, "chunks": r.n_chunks,
                   "service_threads": int(ctx.cfg.service_threads) or
                   max(1, len(os.sched_getaffinity(0)) - 1),
                   "tuned": tw_},
        "link_frac": round(gbps / LINK_PEAK_GBPS, 4),
        "syscalls_per_s": round(st["host_calls"] / total, 1),
        "step_ms_p50": round(1e3 * percentile(wall, 50), 3),
        "step_ms_p99": round(1e3 * percentile(wall, 99), 3),
        "roofline": {"bound": "host-link", "achieved": round(achieved, 2), "peak": LINK_PEAK_GBPS,
                     "unit": "GB/s", "frac": round(achieved / LINK_PEAK_GBPS, 4),
                     "traffic": profile_traffic("wordscan"), "kernel": "wordscan_persistent", "kernel_ms": round(kavg, 3),
                     "bytes_per_launch": int(link_bytes)},
    }
    # the host's side of the roofline: the same chunk preads, same threads,
    # same staging, without the GPU
    from paper_1705_06965_amd.wordscan import host_pread_rate
    hp = round(host_pread_rate(r, res["config"]["service_threads"]), 2)
    res["roofline"]["host_pread_GBps"] = hp
    res["roofline"]["frac_of_host_pread"] = round(achieved / hp, 4)
    ot, ow, ok_, ost = single
    ok_avg = float(np.mean(ok_))
    res["single_pass"] = {"value": round(c.total_bytes * len(ow) / ot / 1e9, 3), "unit": "GB/s",
                          "ms_per_step": round(1e3 * ot / len(ow), 3),
                          "kernel_ms": round(ok_avg, 3),
                          "link_frac": round(ost["bytes_in"] / len(ow) / (ok_avg * 1e-3) / 1e9
                                             / LINK_PEAK_GBPS, 4)}
    if tw:
        pt, pw, pk, _ = tw
        res["plain_form"] = {"value": round(c.total_bytes * len(pw) / pt / 1e9, 3), "unit": "GB/s",
                             "ms_per_step": round(1e3 * pt / len(pw), 3)}
    if cpu:
        res["cpu_baseline"] = cpu
    r.close()
    ctx.shutdown()
    return emit(res, sub)


def run_kv(args, sub=False):
    """Key-value GET: 1M keys, values 32..1024 B, 4M GETs (Zipf 0.99, every
    64th a planted miss) over loopback UDP.  One step = all 4M GETs answered.
    value = GETs per second; p50/p99 latency from the client's first send."""
    import socket
    import struct
    import threading
    import numpy as np
    import torch
    import synth
    import paper_1705_06965_amd as g
    from paper_1705_06965_amd.kv import KVServer, loadgen, make_requests
    t0 = time.time()
    kv = synth.kv_set()
    reqs = make_requests(kv.req_keys)
    print("kv set %d keys, %d requests, setup %.1fs" % (len(kv.keys), len(reqs), time.time() - t0),
          file=sys.stderr, flush=True)
    if not sub:
        return emit(_kv_run(args, kv, reqs, args.kv_clients, sub), sub)
    # beside the sweep: 4 load-generator threads with the tuned list size, the
    # same with the configuration's 256-datagram lists, and 8 threads
    res = _kv_run(args, kv, reqs, 4, sub)
    res["batch256"] = {k: v for k, v in _kv_run(args, kv, reqs, 4, sub, batch=256,
                                                with_cpu=False).items()
                       if k not in SUB_DROP + ("steps", "warmup")}
    res["clients8"] = {k: v for k, v in _kv_run(args, kv, reqs, 8, sub).items()
                       if k not in SUB_DROP + ("steps", "warmup")}
    return emit(res, sub)


def _kv_run(args, kv, reqs, clients, sub, batch=0, with_cpu=True):
    """One key-value measurement with `clients` load-generator threads; the
    pool's knobs come from the cache entry tuned for that client count
    (`batch`, when given, sets the datagrams per list call instead).
    with_cpu=False leaves out the oracle server's run."""
    import socket
    import struct
    import threading
    import numpy as np
    import paper_1705_06965_amd as g
    from paper_1705_06965_amd.kv import KVServer, loadgen
    from paper_1705_06965_amd import autotune
    tk_ = autotune.load("kv8" if clients == 8 else "kv")
    tuned = dict(tk_)   # the cache entry, before any override below
    if args.kv_grid:
        tk_["grid"] = args.kv_grid
    if args.kv_batch:
        tk_["batch"] = args.kv_batch
    if batch:
        tk_["batch"] = batch
    pollers = args.service_threads if args.service_threads >= 0 else tk_["service_threads"]
    ctx = g.Context(ring_slots=1 << 16, service_threads=pollers,
                    device_timeout_ns=60_000_000_000,
                    flags=g.CFG_DOORBELL if args.kv_doorbell else 0)
    srv = KVServer(ctx, kv.keys, kv.val_off, kv.val_len, kv.heap, grid=tk_["grid"],
                   batch=tk_["batch"], pipelined=bool(tk_.get("pipelined", 1)))
    # beside the sweep: one warm-up pass and two timed passes of the 4M GETs
    warmup = 1 if sub else args.warmup
    steps = 2 if sub else max(1, min(args.steps, 3))
    res_steps = []
    for st in range(warmup + steps):
        ctx.stats(reset=True)
        srv.start(lifetime_ms=300_000)
        t1 = time.perf_counter()
        got, replies, rlen, lat, rt = loadgen(srv.port, reqs, threads=clients,
                                              window=args.kv_window, timeout_ns=120_000_000_000)
        dt = time.perf_counter() - t1
        srv.stop()
        stt = ctx.stats()
        if got != len(reqs):
            raise RuntimeError("kv: %d of %d answered" % (got, len(reqs)))
        if st >= warmup:
            res_steps.append((dt, lat.copy(), rt, stt))
        print("kv step %d: %.3f s, %.0f GET/s, retransmits %d" % (st, dt, len(reqs) / dt, rt),
              file=sys.stderr, flush=True)
    # CPU-baseline leg: the oracle's replies for a sample of requests
    oracle = oracle_leg(args)
    if oracle:
        ix = oracle.KVIndex(kv.keys, kv.val_off, kv.val_len, kv.heap)
        for k in np.random.default_rng(9).choice(len(reqs), 4096, replace=False):
            want = ix.reply(reqs[k].tobytes())
            if replies[k, :rlen[k]].tobytes() != want:
                raise RuntimeError("kv reply %d differs from the oracle" % k)
    cpu = None
    if oracle and with_cpu:
        # the oracle as a CPU server on the same loopback path, same client
        n_cpu = 1_000_000
        threads = max(1, len(os.sched_getaffinity(0)) - clients)
        sock = socket.socket(socket.AF_INET, socket.SOCK_DGRAM)
        for opt in (socket.SO_RCVBUF, socket.SO_SNDBUF):
            sock.setsockopt(socket.SOL_SOCKET, opt, 8 << 20)
        sock.setsockopt(socket.SOL_SOCKET, socket.SO_RCVTIMEO, struct.pack("ll", 0, 300000))
        sock.bind(("127.0.0.1", 0))
        ths = [threading.Thread(target=ix.serve, args=(sock.fileno(), 1 << 40))
               for _ in range(threads)]
        for t in ths:
            t.start()
        t1 = time.perf_counter()
        gc, rc_, rl_, lat_c, _ = loadgen(sock.getsockname()[1], reqs[:n_cpu],
                                         threads=clients, window=args.kv_window)
        dtc = time.perf_counter() - t1
        for t in ths:
            t.join()
        sock.close()
        cpu = {"value": round(gc / dtc, 1), "unit": "GET/s", "cores": threads, "kind": "oracle",
               "sample": "first 1,000,000 GETs against the oracle's CPU UDP server (sorted "
                         "index + bsearch), %d server threads on one socket, same load "
                         "generator" % threads}
    if oracle:
        ix.close()
    dts = [d for d, _, _, _ in res_steps]
    dt_med = float(np.median(dts))
    lat_all = np.concatenate([l for _, l, _, _ in res_steps]).astype(np.float64)
    stt = res_steps[-1][3]
    reply_bytes = int(rlen.sum())
    res = {
        "metric": "GPU-issued syscalls/s + pread-scan GB/s (frac of link roofline); p99 latency",
        "value": round(len(reqs) / dt_med, 1), "unit": "GET/s", "n_gpus": 1,
        "steps": len(res_steps), "warmup": warmup, "ms_per_step": round(1e3 * dt_med, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "key-value GET over loopback UDP: 1M 16-byte keys, values "
                               "32-1024 B, 4M GETs Zipf(0.99), table load 0.5, %d-datagram "
                               "recvfrom/sendto list calls per work-group" % tk_["batch"],
                   "server_workgroups": tk_["grid"], "batch": tk_["batch"],
                   "server_loop": "pipelined" if tk_.get("pipelined", 1) else "blocking",
                   "tuned": tuned, "client_threads": clients,
                   "service_threads": pollers,
                   "client_window": args.kv_window, "doorbell": bool(args.kv_doorbell)},
        # calls the GPU's lists asked for (datagrams received or sent) and the
        # kernel entries the host used for them (recvmmsg / sendmmsg batches)
        "syscalls_per_s": round((stt["host_calls"] + stt["merged"]) / dts[-1], 1),
        "host_kernel_calls_per_s": round(stt["host_calls"] / dts[-1], 1),
        "pool_busy_frac": round(stt["service_ns"] / 1e9 / max(1e-9, dts[-1]) / max(1, pollers), 3),
        "latency_us_p50": round(float(np.percentile(lat_all, 50)) / 1e3, 1),
        "latency_us_p99": round(float(np.percentile(lat_all, 99)) / 1e3, 1),
        "reply_GBps": round(reply_bytes / dt_med / 1e9, 3),
        "retransmits": res_steps[-1][2],
        "roofline": {"bound": "host-cpu",
                     "achieved": round((stt["host_calls"] + stt["merged"]) / dts[-1], 1),
                     "peak": None, "unit": "syscalls/s", "frac": None,
                     "traffic": profile_traffic("kv") if clients == 4 else None,
                     "kernel": "kv_serve"},
    }
    if cpu:
        res["cpu_baseline"] = cpu
        res["over_cpu_baseline"] = round(res["value"] / cpu["value"], 3)
    srv.close()
    ctx.shutdown()
    return res


def run_serve(args, sub=False):
    """Serving mix: Poisson arrivals (mean 20k/s) of scan (4 KiB-64 MiB
    log-uniform reads of the 1 GiB file, per-4 KiB FNV digests), pwrite
    (4-256 KiB) and release (mmap / madvise(MADV_DONTNEED) of 2 MiB blocks of
    a 16 GiB arena) jobs; 55,000 jobs, the first 5,000 are warm-up.  One
    step = the whole stream.  value = jobs per second; p50/p99 latency from
    each job's scheduled arrival to the host seeing it done."""
    import concurrent.futures as cf
    import numpy as np
    import torch
    import synth
    import paper_1705_06965_amd as g
    from paper_1705_06965_amd.serve import ServeRun
    t0 = time.time()
    in_path = synth.random_file(2, FILE_BYTES, name="c2_1g.bin")
    js = synth.job_stream(n_jobs=args.serve_jobs, rate_per_s=args.serve_rate)
    with open(in_path, "rb") as f:
        while f.read(64 << 20):
            pass
    out_path = os.path.join(synth.data_dir(), "serve_out.bin")
    print("job stream %d jobs (%s), setup %.1fs" % (len(js.kind), np.bincount(js.kind).tolist(),
                                                   time.time() - t0), file=sys.stderr, flush=True)
    from paper_1705_06965_amd import autotune
    ts_ = autotune.load("serve")
    if args.serve_grid:
        ts_["grid"] = args.serve_grid
    if args.serve_sleep_max:
        ts_["sleep_max"] = args.serve_sleep_max
    if args.service_threads >= 0:
        ts_["service_threads"] = args.service_threads
    ctx = g.Context(ring_slots=1 << 16, service_threads=ts_["service_threads"],
                    device_timeout_ns=60_000_000_000, arena_bytes=16 << 30,
                    flags=g.CFG_LEDGER if args.serve_ledger else 0, ledger_capacity=1 << 22,
                    sleep_max=ts_["sleep_max"])
    sr = ServeRun(ctx, js, in_path, out_path)
    warm = min(5000, len(js.kind) // 10)

    def session(form, inflight, n_limit=None):
        t1 = time.perf_counter()
        res, dig, lat = sr.run(form, max_inflight=inflight, staging_bytes=(2 << 20) * 256,
                               grid=ts_["grid"] if form == g.PERSISTENT else 0,
                               timeout_ns=300_000_000_000)
        dt = time.perf_counter() - t1
        return res, dig, lat, dt

    if args.warmup > 0:
        # a warm-up session on the stream's first 20,000 jobs (1 s at 20k/s):
        # the host's first huge-page allocations for the arena and its first
        # calls of each kind happen here, not in the timed session
        n_w = min(len(js.kind), 20000)
        wjs = synth.JobStream(kind=js.kind[:n_w], arrival_ns=js.arrival_ns[:n_w],
                              arg_off=js.arg_off[:n_w], arg_len=js.arg_len[:n_w],
                              content_off=js.content_off[:n_w], content=js.content)
        wr = ServeRun(ctx, wjs, in_path, out_path)
        wr.run(g.PERSISTENT, max_inflight=args.serve_inflight, staging_bytes=(2 << 20) * 256,
               grid=ts_["grid"], timeout_ns=300_000_000_000)
        wr.close()
    res, dig, lat, dt = session(g.PERSISTENT, args.serve_inflight)
    lat_s = lat[warm:].astype(np.float64) / 1e3
    span_s = (float(js.arrival_ns[-1]) - float(js.arrival_ns[warm])) / 1e9 + \
        float(np.median(lat_s)) / 1e6
    # CPU-baseline leg: the oracle's results for a sample of jobs
    oracle = oracle_leg(args)
    data = np.memmap(in_path, dtype=np.uint8, mode="r")
    out = np.memmap(out_path, dtype=np.uint8, mode="r")
    jobs = sr.jobs_np
    sample = np.random.default_rng(11).choice(len(js.kind), 300, replace=False) if oracle else []
    for i in sample:
        k = int(js.kind[i])
        if k == 0:
            nb = int(jobs["len"][i]) // 4096
            offs = int(jobs["off"][i]) + 4096 * np.arange(min(nb, 256), dtype=np.uint64)
            want, _ = oracle.pread_fnv(in_path, offs, 4096)
            d0 = int(sr.digest_start[i])
            ok = res[i] == int(jobs["len"][i]) and (dig[d0:d0 + len(offs)] == want).all()
        elif k == 1:
            off, ln, src = int(jobs["off"][i]), int(jobs["len"][i]), int(jobs["src"][i])
            ok = res[i] == ln and (out[off:off + ln] == js.content[src:src + ln]).all()
        else:
            off, src, pg = int(jobs["off"][i]), int(jobs["src"][i]), int(jobs["page"][i])
            ok = res[i] == 0 and (out[off:off + 64] == data[src + 4096 * pg:src + 4096 * pg + 64]).all() \
                and not out[off + 64:off + 128].any()
        if not ok:
            raise RuntimeError("serving job %d differs from the oracle" % i)
    plain = None
    if not args.no_plain:
        # the plain form: one launch per job, on the first 4,000 jobs only
        sub = synth.JobStream(kind=js.kind[:4000], arrival_ns=js.arrival_ns[:4000],
                              arg_off=js.arg_off[:4000], arg_len=js.arg_len[:4000],
                              content_off=js.content_off[:4000], content=js.content)
        sp = ServeRun(ctx, sub, in_path, out_path + ".plain")
        t1 = time.perf_counter()
        _, _, lp, dtp = None, None, None, None
        rp, dp, lp = sp.run(g.PLAIN, max_inflight=args.serve_inflight,
                            staging_bytes=(2 << 20) * 4, timeout_ns=300_000_000_000)
        dtp = time.perf_counter() - t1
        lps = lp[400:].astype(np.float64) / 1e3
        plain = {"jobs": 4000, "jobs_per_s": round(4000 / dtp, 1),
                 "latency_us_p50": round(float(np.percentile(lps, 50)), 1),
                 "latency_us_p99": round(float(np.percentile(lps, 99)), 1)}
        sp.close()
    cpu = None
    if oracle:
        # the oracle runs the first 5,000 jobs on a thread pool, as fast as it can
        threads = len(os.sched_getaffinity(0))
        ofd = os.open(out_path + ".cpu", os.O_RDWR | os.O_CREAT | os.O_TRUNC, 0o600)
        ifd = os.open(in_path, os.O_RDONLY)

        def one(i):
            k = int(js.kind[i])
            if k == 0:
                nb = int(jobs["len"][i]) // 4096
                offs = int(jobs["off"][i]) + 4096 * np.arange(nb, dtype=np.uint64)
                oracle.pread_fnv(in_path, offs, 4096)
            elif k == 1:
                off, ln, src = int(jobs["off"][i]), int(jobs["len"][i]), int(jobs["src"][i])
                os.pwrite(ofd, js.content[src:src + ln].tobytes(), off)
            else:
                oracle.release_job(ifd, int(jobs["src"][i]), int(jobs["page"][i]), ofd,
                                   int(jobs["off"][i]))
        t1 = time.perf_counter()
        with cf.ThreadPoolExecutor(threads) as ex:
            list(ex.map(one, range(5000)))
        dtc = time.perf_counter() - t1
        os.close(ofd)
        os.close(ifd)
        cpu = {"value": round(5000 / dtc, 1), "unit": "jobs/s", "cores": threads, "kind": "oracle",
               "sample": "the first 5,000 jobs run back to back by the oracle on a pool of %d "
                         "threads (closed loop: capacity, not latency)" % threads}
    kinds = {}
    for k, nm in ((0, "scan"), (1, "pwrite"), (2, "release")):
        lk = lat_s[js.kind[warm:] == k]
        if len(lk):
            kinds[nm] = {"jobs": int(len(lk)), "p50": round(float(np.percentile(lk, 50)), 1),
                         "p99": round(float(np.percentile(lk, 99)), 1)}
    sweep = []
    for rate in [float(x) for x in args.serve_sweep.split(",") if x]:
        n_r = max(2000, int(rate * 2.75))
        jr = synth.job_stream(n_jobs=n_r, rate_per_s=rate)
        srr = ServeRun(ctx, jr, in_path, out_path + ".sweep")
        t1 = time.perf_counter()
        rr, _, lr = srr.run(g.PERSISTENT, max_inflight=args.serve_inflight,
                            staging_bytes=(2 << 20) * 256, timeout_ns=300_000_000_000)
        dtr = time.perf_counter() - t1
        w_r = n_r // 10
        lrs = lr[w_r:].astype(np.float64) / 1e3
        span_r = (float(jr.arrival_ns[-1]) - float(jr.arrival_ns[w_r])) / 1e9 + \
            float(np.median(lrs)) / 1e6
        sweep.append({"offered_jobs_per_s": rate, "jobs": n_r,
                      "jobs_per_s": round((n_r - w_r) / span_r, 1),
                      "latency_us_p50": round(float(np.percentile(lrs, 50)), 1),
                      "latency_us_p99": round(float(np.percentile(lrs, 99)), 1),
                      "session_s": round(dtr, 3)})
        srr.close()
        print("sweep %.0f/s done" % rate, file=sys.stderr, flush=True)
    st = ctx.stats()
    host_us = None
    if args.serve_ledger:
        # host service time per call kind (claim to completion), microseconds
        led = ctx.ledger(reset=True)
        if args.serve_ledger_out:
            np.save(args.serve_ledger_out, led)
        svc = ((led[:, 5] >> np.uint64(8)).astype(np.int64) - led[:, 4].astype(np.int64)) / 1e3
        host_us = {}
        for nr, nm in ((g.NR_PREAD64, "pread"), (g.NR_PWRITE64, "pwrite"), (g.NR_MMAP, "mmap"),
                       (g.NR_MADVISE, "madvise"), (g.NR_MUNMAP, "munmap")):
            m = led[:, 1] == nr
            if m.any():
                host_us[nm] = {"calls": int(m.sum()), "p50": round(float(np.percentile(svc[m], 50)), 1),
                               "p99": round(float(np.percentile(svc[m], 99)), 1),
                               "max": round(float(svc[m].max()), 1),
                               "busy_s": round(float(svc[m].sum()) / 1e6, 3)}
        pollers = int(ctx.cfg.service_threads) or max(1, len(os.sched_getaffinity(0)) - 1)
        host_us["pool_busy_frac"] = round(float(svc.sum()) / 1e6 / (pollers * dt), 3)
    res_j = {
        "metric": "GPU-issued syscalls/s + pread-scan GB/s (frac of link roofline); p99 latency",
        "value": round((len(js.kind) - warm) / span_s, 1), "unit": "jobs/s", "n_gpus": 1,
        "steps": 1, "warmup": 0, "ms_per_step": round(1e3 * dt, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "serving mix: Poisson arrivals at %.0f/s of scan (4 KiB-64 MiB "
                               "log-uniform, per-4 KiB FNV), pwrite (4-256 KiB) and "
                               "mmap/madvise release (2 MiB of a 16 GiB arena) jobs, "
                               "10/60/30%%" % args.serve_rate,
                   "jobs": len(js.kind), "warmup_jobs": warm, "max_inflight": args.serve_inflight,
                   "form": "persistent (continuous batching)",
                   "persistent_workgroups": ts_["grid"], "tuned": ts_},
        "latency_us_p50": round(float(np.percentile(lat_s, 50)), 1),
        "latency_us_p99": round(float(np.percentile(lat_s, 99)), 1),
        "offered_jobs_per_s": args.serve_rate,
        "latency_us_by_kind": kinds,
        "scan_GBps": round(float(js.arg_len[js.kind == 0].sum()) / dt / 1e9, 3),
        "host_calls": st["host_calls"],
    }
    if sweep:
        res_j["offered_load_sweep"] = sweep
    if host_us:
        res_j["host_service_us"] = host_us
    if plain:
        res_j["plain_form"] = plain
    if cpu:
        res_j["cpu_baseline"] = cpu
    sr.close()
    ctx.shutdown()
    return emit(res_j, sub)




def run_permute(args):
    """Block permutation + pwrite (section 6, Fig. 6): a 64 MiB array of
    random words in 8,192 blocks of 8 KiB; a 1024-wide work-group permutes a
    block `iters` times and writes it with one work-group pwrite, under each
    of strong / relaxed x blocking / non-blocking.  One step = one launch
    over the whole array, timed from launch until the host pool has written
    every block.  Reported per cell and iteration count: time per iteration
    (step time / iters, lower is better).  value = pwrite calls per second of
    the fastest cell at the smallest iteration count."""
    import numpy as np
    import torch
    import synth
    import paper_1705_06965_amd as g
    from paper_1705_06965_amd.permute import PermuteRunner, WG_CELLS
    n_blocks = 8192
    iters_list = [int(x) for x in args.perm_iters.split(",") if x]
    ps = synth.permute_set(n_blocks=n_blocks)
    path = os.path.join(synth.data_dir(), "permute_out.bin")
    ctx = g.Context(ring_slots=1 << 14, service_threads=max(0, args.service_threads),
                    device_timeout_ns=60_000_000_000)
    r = PermuteRunner(ctx, path, ps.data, ps.sigma, ps.tau)
    stream = torch.cuda.current_stream()
    name = {("WG", "strong", "block"): "strong-block", ("WG", "strong", "nonblock"):
            "strong-nonblock", ("WG", "relaxed", "block"): "weak-block",
            ("WG", "relaxed", "nonblock"): "weak-nonblock"}
    pick = np.array([0, 1, 4095, 8191])
    curves, kern = {}, {}
    total_steps, total_t = 0, 0.0
    for cell in WG_CELLS:
        code = g.cell_code(*cell)
        curves[name[cell]], kern[name[cell]] = {}, {}
        for it in iters_list:
            for _ in range(max(1, args.warmup)):
                r.launch(it, code, stream)
                torch.cuda.synchronize()
                if ctx.wait(60_000_000_000):
                    raise RuntimeError("drain failed")
            wall, kms = [], []
            for _ in range(args.steps):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                e0.record(stream)
                r.launch(it, code, stream)
                e1.record(stream)
                torch.cuda.synchronize()
                if ctx.wait(60_000_000_000):
                    raise RuntimeError("drain failed")
                wall.append(time.perf_counter() - t0)
                kms.append(e0.elapsed_time(e1))
            total_steps += len(wall)
            total_t += sum(wall)
            med = float(np.median(wall))
            curves[name[cell]][it] = round(med / it * 1e6, 2)      # us per iteration
            kern[name[cell]][it] = round(float(np.median(kms)), 4)  # ms per launch
        # the file now holds the last iteration count's blocks: the CPU-
        # baseline leg spot-checks them against the oracle
        oracle = oracle_leg(args)
        if oracle:
            got = r.file_bytes().reshape(n_blocks, 8192)[pick].ravel()
            sub = ps.data.reshape(n_blocks, 1024)[pick].ravel()
            chk = os.path.join(synth.data_dir(), "permute_check.bin")
            fd = os.open(chk, os.O_RDWR | os.O_CREAT | os.O_TRUNC, 0o600)
            oracle.permute(fd, sub, ps.sigma, ps.tau, iters_list[-1], threads=4)
            os.close(fd)
            if not np.array_equal(got, np.fromfile(chk, dtype=np.uint8)):
                raise RuntimeError("GPU blocks differ from the oracle (%s)" % name[cell])
        print("cell %s done" % name[cell], file=sys.stderr, flush=True)
    lo = iters_list[0]
    best = min(curves, key=lambda c: curves[c][lo])
    step_s = curves[best][lo] * lo / 1e6
    calls_per_s = n_blocks / step_s
    # the link roofline of the launch whose duration is GPU work alone (the
    # relaxed non-blocking cell at the smallest iteration count): 8 KiB per
    # block written to host memory (the HBM read of the same bytes is
    # negligible)
    link_bytes = n_blocks * 8192
    kms = kern["weak-nonblock"][lo]
    achieved = link_bytes / (kms * 1e-3) / 1e9
    # LDS work per round: per word one 8-byte gather, eight 8-byte table
    # reads and one 8-byte store
    hi = iters_list[-1]
    lds_bytes = n_blocks * 1024 * 80 * hi
    lds_peak = 128 * 256 * 2.4e9 / 1e12      # 128 B/clk per CU, 256 CUs, 2.4 GHz
    lds_tbs = lds_bytes / (kern["weak-nonblock"][hi] * 1e-3) / 1e12
    cpu = None
    oracle = oracle_leg(args)
    if oracle:
        threads = len(os.sched_getaffinity(0))
        chk = os.path.join(synth.data_dir(), "permute_cpu.bin")
        fd = os.open(chk, os.O_RDWR | os.O_CREAT | os.O_TRUNC, 0o600)
        t1 = time.perf_counter()
        reps = 3
        for _ in range(reps):
            oracle.permute(fd, ps.data, ps.sigma, ps.tau, lo, threads=threads)
        dt = (time.perf_counter() - t1) / reps
        os.close(fd)
        cpu = {"value": round(n_blocks / dt, 1), "unit": "calls/s", "cores": threads,
               "kind": "oracle", "sample": "the whole 8,192-block array at %d round(s), "
                                           "%d repetitions, blocks split over %d POSIX "
                                           "threads" % (lo, reps, threads)}
    res = {
        "metric": "GPU-issued syscalls/s + pread-scan GB/s (frac of link roofline); p99 latency",
        "value": round(calls_per_s, 1), "unit": "calls/s", "n_gpus": 1,
        "steps": total_steps, "warmup": args.warmup,
        "ms_per_step": round(1e3 * total_t / max(1, total_steps), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "block permutation + work-group pwrite: 64 MiB of random "
                               "words, 8,192 blocks of 8 KiB, 1024-wide work-groups",
                   "iters": iters_list, "best_cell": best},
        "us_per_iteration": curves,
        "kernel_ms": kern,
        # 1 - t(cell) / t(strong-block): how much of the blocking, strongly
        # ordered cell's time the other cells save, per iteration count
        "gain_vs_strong_block": {c: {it: round(1 - curves[c][it] / curves["strong-block"][it], 4)
                                     for it in iters_list}
                                 for c in curves if c != "strong-block"},
        # the host writes every block to one file, and writes to one file are
        # serialised by the kernel: this is the floor of every step
        "host_pwrite_GBps": round(link_bytes / step_s / 1e9, 3),
        "roofline": {"bound": "host-link", "achieved": round(achieved, 2),
                     "peak": LINK_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(achieved / LINK_PEAK_GBPS, 4),
                     "traffic": profile_traffic("permute"),
                     "kernel": "permute<relaxed, non-blocking>", "kernel_ms": kms,
                     "bytes_per_launch": link_bytes},
        "lds_roofline_at_%d" % hi: {"achieved": round(lds_tbs, 2), "peak": round(lds_peak, 2),
                                     "unit": "TB/s", "frac": round(lds_tbs / lds_peak, 4)},
    }
    if cpu:
        res["cpu_baseline"] = cpu
    r.close()
    ctx.shutdown()
    print(json.dumps(res), flush=True)


def run_tiny(args, sub=False):
    """Plain form, tiny: one work-group of 64 work-items, each a blocking
    pread of 4 KiB at 4096 i from a 256 KiB file of random bytes (work-item,
    strong), FNV-1a per item.  Latency only, no roofline: per launch the
    end-to-end time (launch until the host pool has drained), the kernel's
    duration, and per call the time from the launch to the end of its
    service on the host and the service itself (ledger timestamps, the same
    CLOCK_MONOTONIC).  value = 64 calls / median end-to-end time."""
    import numpy as np
    import torch
    import synth
    import paper_1705_06965_amd as g
    from paper_1705_06965_amd.fnv import FnvRunner
    path = synth.random_file(1, 262144, name="c1_256k.bin")
    offs = synth.tiny_offsets(64)
    oracle = oracle_leg(args)
    # the sweep's tuned pool: with pollers spinning on all cores but one,
    # this thread shares the last core with the runtime's threads, and about
    # one launch in a hundred took 1-5 ms end to end (the kernel did not)
    from paper_1705_06965_amd import autotune
    pollers = args.service_threads if args.service_threads >= 0 else \
        int(autotune.load("sweep")["service_threads"]) or 12
    ctx = g.Context(ring_slots=1 << 10, service_threads=pollers,
                    device_timeout_ns=10_000_000_000, flags=g.CFG_LEDGER)
    r = FnvRunner(ctx, path, offs, 4096, wg_size=64)
    stream = torch.cuda.current_stream()
    cell = g.cell_code("WI", "strong", "block")
    reps = max(200, args.steps)   # enough launches for a p99 that is not the maximum
    for _ in range(max(1, args.warmup)):
        r.launch(cell, g.PLAIN, stream)
        torch.cuda.synchronize()
        ctx.wait(10_000_000_000)
    ctx.ledger(reset=True)
    e2e, kern, to_done, service = [], [], [], []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0 = time.monotonic_ns()
        e0.record(stream)
        r.launch(cell, g.PLAIN, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        if ctx.wait(10_000_000_000):
            raise RuntimeError("drain failed")
        e2e.append((time.monotonic_ns() - t0) / 1e3)
        kern.append(e0.elapsed_time(e1) * 1e3)
        led = ctx.ledger(reset=True)
        if len(led) != 64:
            raise RuntimeError("expected 64 serviced calls, got %d" % len(led))
        t_end = (led[:, 5] >> np.uint64(8)).astype(np.int64)
        to_done.extend(((t_end - t0) / 1e3).tolist())
        service.extend(((t_end - led[:, 4].astype(np.int64)) / 1e3).tolist())
    f, ret = r.result()
    if not (ret == 4096).all():
        raise RuntimeError("a tiny-case pread returned %s" % ret[ret != 4096][:4])
    cpu = None
    if oracle:
        # CPU-baseline leg: the oracle's checksums, then its latency
        want, _ = oracle.pread_fnv(path, offs, 4096)
        if not (f == want).all():
            raise RuntimeError("GPU checksums differ from the oracle")
        n_cpu = 2000
        ts = []
        for _ in range(n_cpu):
            t1 = time.perf_counter()
            oracle.pread_fnv(path, offs, 4096, threads=1)
            ts.append(time.perf_counter() - t1)
        cpu = {"value": round(64 / float(np.median(ts)), 1), "unit": "calls/s", "cores": 1,
               "kind": "oracle", "latency_us_p50": round(1e6 * float(np.median(ts)), 2),
               "sample": "the same 64 preads + checksums, one thread, median of %d runs "
                         "(includes opening the file)" % n_cpu}
    med = float(np.median(e2e))
    pc = lambda xs, q: round(float(np.percentile(xs, q)), 2)
    res = {
        "metric": "GPU-issued syscalls/s + pread-scan GB/s (frac of link roofline); p99 latency",
        "value": round(64 / (med * 1e-6), 1), "unit": "calls/s", "n_gpus": 1, "steps": reps,
        "warmup": args.warmup, "ms_per_step": round(med / 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "tiny plain form: 1 work-group x 64 work-items, blocking 4 KiB "
                               "pread at 4096 i of a 256 KiB file, work-item / strong",
                   "form": "plain", "service_threads": pollers, "launches": reps},
        "end_to_end_us": {"p50": pc(e2e, 50), "p99": pc(e2e, 99), "min": round(min(e2e), 2)},
        "kernel_us": {"p50": pc(kern, 50), "p99": pc(kern, 99)},
        "per_call_launch_to_serviced_us": {"p50": pc(to_done, 50), "p99": pc(to_done, 99)},
        "per_call_service_us": {"p50": pc(service, 50), "p99": pc(service, 99)},
    }
    if cpu:
        res["cpu_baseline"] = cpu
    r.close()
    ctx.shutdown()
    return emit(res, sub)


def _spot_check(args, path, offs, item, f, ret, k=64):
    """CPU-baseline leg: recompute k evenly spaced items with the oracle
    (nothing with --no-cpu)."""
    import numpy as np
    oracle = oracle_leg(args)
    if not oracle:
        return
    pick = np.unique(np.linspace(0, len(offs) - 1, k).astype(np.int64))
    want_f, want_r = oracle.pread_fnv(path, offs[pick], item)
    if not ((f[pick] == want_f).all() and (ret[pick] == want_r).all()):
        raise RuntimeError("GPU checksums differ from the oracle")


def _time_runs(runner, ctx, cell, form, steps, warmup):
    import numpy as np
    import torch
    for _ in range(warmup):
        runner.launch(cell, form)
        torch.cuda.synchronize()
        if ctx.wait(120_000_000_000):
            raise RuntimeError("drain failed")
    ts = []
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        runner.launch(cell, form)
        torch.cuda.synchronize()
        if ctx.wait(120_000_000_000):
            raise RuntimeError("drain failed")
        ts.append(time.perf_counter() - t0)
    return float(np.median(ts))


def run_granularity(args):
    """Invocation granularity (section 6, Fig. 5).  Left: the time to read
    the first S bytes of the file in 4 KiB preads (one per work-item, items
    in file order, 64-wide work-groups, one plain launch), for every legal
    granularity x ordering x blocking cell.  Right: work-group granularity
    (relaxed, blocking) as the work-group grows from 64 to 1024 work-items.
    Adjacent reads of a group's descriptor list merge into one host pread,
    so a work-group call reads its whole range at once and a kernel call
    reads the file as one pread on one host thread.  value = calls/s of the
    fastest cell at the largest size."""
    import numpy as np
    import synth
    import paper_1705_06965_amd as g
    from paper_1705_06965_amd.fnv import FnvRunner
    path = synth.random_file(2, FILE_BYTES, name="c2_1g.bin")
    with open(path, "rb") as fh:
        while fh.read(64 << 20):
            pass
    sizes = [4 << 20, 64 << 20, 1 << 30]
    ctx = g.Context(ring_slots=1 << 18, service_threads=max(0, args.service_threads),
                    device_timeout_ns=120_000_000_000)
    steps = max(1, min(args.steps, 3))
    left = {}
    best = (0.0, None)
    for S in sizes:
        n = S // ITEM
        offs = (np.arange(n, dtype=np.uint64) * ITEM)
        r = FnvRunner(ctx, path, offs, ITEM, wg_size=64)
        left[S] = {}
        for cell in g.LEGAL_CELLS:
            code = g.cell_code(*cell)
            t = _time_runs(r, ctx, code, g.PLAIN, steps, 1)
            f, ret = r.result()
            _spot_check(args, path, offs, ITEM, f, ret)
            name = "/".join(cell)
            left[S][name] = round(1e3 * t, 3)
            if S == sizes[-1] and n / t > best[0]:
                best = (n / t, name)
        r.close()
        print("size %d MiB done" % (S >> 20), file=sys.stderr, flush=True)
    S = sizes[-1]
    n = S // ITEM
    offs = (np.arange(n, dtype=np.uint64) * ITEM)
    right = {}
    for wg in (64, 128, 256, 512, 1024):
        r = FnvRunner(ctx, path, offs, ITEM, wg_size=wg)
        t = _time_runs(r, ctx, g.cell_code("WG", "relaxed", "block"), g.PLAIN, steps, 1)
        f, ret = r.result()
        _spot_check(args, path, offs, ITEM, f, ret)
        st = ctx.stats()
        right[wg] = round(1e3 * t, 3)
        r.close()
    ctx.shutdown()
    res = {
        "metric": "GPU-issued syscalls/s + pread-scan GB/s (frac of link roofline); p99 latency",
        "value": round(best[0], 1), "unit": "syscalls/s", "n_gpus": 1, "steps": steps,
        "warmup": 1, "ms_per_step": round(1e3 * n / best[0], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "invocation granularity: read the first S bytes of a 1 GiB "
                               "random file in 4 KiB preads, plain launch",
                   "sizes": sizes, "best_cell_at_1g": best[1]},
        "read_ms_by_size_and_cell": {str(k): v for k, v in left.items()},
        "read_ms_1g_by_wg_size": {str(k): v for k, v in right.items()},
    }
    print(json.dumps(res), flush=True)


def run_coalesce(args):
    """Coalescing (section 6, Fig. 7): 16,384 work-items (64 work-groups of
    256) each pread one contiguous piece of the file, so the piece size is
    the file size / 16,384; work-item granularity, strong, blocking, one
    plain launch.  Host pool without coalescing (K = 1) and with bundles of
    up to K = 8 calls gathered for up to T = 10 us; a bundle's calls that
    continue each other in the file and in memory become one pread.
    Reported: time per requested byte.  value = calls/s of the best setting
    at the smallest piece."""
    import numpy as np
    import synth
    import paper_1705_06965_amd as g
    from paper_1705_06965_amd.fnv import FnvRunner
    path = synth.random_file(2, FILE_BYTES, name="c2_1g.bin")
    with open(path, "rb") as fh:
        while fh.read(64 << 20):
            pass
    n = 16384
    pieces = [64, 256, 1024, 4096, 16384, 65536]
    steps = max(1, min(args.steps, 5))
    cell = g.cell_code("WI", "strong", "block")
    out = {}
    best = (0.0, None)
    for K, T in ((1, 0), (8, 10_000)):
        ctx = g.Context(ring_slots=1 << 16, service_threads=max(0, args.service_threads),
                        coalesce_max=K, coalesce_window_ns=T, device_timeout_ns=60_000_000_000)
        key = "K%d" % K
        out[key] = {}
        for piece in pieces:
            offs = np.arange(n, dtype=np.uint64) * np.uint64(piece)
            r = FnvRunner(ctx, path, offs, piece, wg_size=256)
            t = _time_runs(r, ctx, cell, g.PLAIN, steps, 1)
            f, ret = r.result()
            _spot_check(args, path, offs, piece, f, ret)
            st = ctx.stats(reset=True)
            out[key][piece] = {"ms": round(1e3 * t, 3),
                               "ns_per_byte": round(1e9 * t / (n * piece), 4),
                               "merged_per_launch": st["merged"] // (steps + 1)}
            if piece == pieces[0] and n / t > best[0]:
                best = (n / t, key)
            r.close()
        ctx.shutdown()
        print("coalescing %s done" % key, file=sys.stderr, flush=True)
    res = {
        "metric": "GPU-issued syscalls/s + pread-scan GB/s (frac of link roofline); p99 latency",
        "value": round(best[0], 1), "unit": "syscalls/s", "n_gpus": 1, "steps": steps,
        "warmup": 1, "ms_per_step": round(1e3 * n / best[0], 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "coalescing: 16,384 work-items each pread one contiguous piece "
                               "of a 1 GiB random file, work-item / strong / blocking",
                   "pieces": pieces, "coalescing": {"K1": "off", "K8": "K = 8, T = 10 us"},
                   "best_at_64B": best[1]},
        "by_setting_and_piece": {k: {str(p): v for p, v in d.items()} for k, d in out.items()},
    }
    print(json.dumps(res), flush=True)


def run_wordopen(args):
    """Word search as section 7.1 issues it: the same 2,000-file corpus, each
    file opened by name on the GPU, read front to back with read() in 1 MiB
    pieces and closed (work-group granularity, relaxed).  value = scanned
    file bytes per second; the pread form on the same corpus is timed
    beside it."""
    import numpy as np
    import torch
    import synth
    import paper_1705_06965_amd as g
    from paper_1705_06965_amd.wordscan import WordOpenRunner, WordScanRunner
    c = synth.wordcount_corpus()
    for p in c.paths:
        with open(p, "rb") as fh:
            fh.read()
    d = os.path.dirname(c.paths[0])
    names = [os.path.basename(p) for p in c.paths]
    ctx = g.Context(ring_slots=1 << 16, service_threads=max(0, args.service_threads),
                    device_timeout_ns=60_000_000_000)
    r = WordOpenRunner(ctx, d, names, c.queries, chunk=1 << 20)
    stream = torch.cuda.current_stream()

    def timed(run, steps, warmup):
        for _ in range(warmup):
            run()
        ctx.stats(reset=True)
        wall, kms = [], []
        t0 = time.perf_counter()
        for _ in range(steps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            s0 = time.perf_counter()
            e0.record(stream)
            run(e1)
            wall.append(time.perf_counter() - s0)
            kms.append(e0.elapsed_time(e1))
        return time.perf_counter() - t0, wall, kms, ctx.stats()

    def run_open(e1=None):
        r.launch(stream)
        if e1 is not None:
            e1.record(stream)
        torch.cuda.synchronize()
        if ctx.wait(60_000_000_000):
            raise RuntimeError("drain failed")

    total, wall, kms, st = timed(run_open, args.steps, args.warmup)
    counts, ret = r.result()
    if not (ret == np.array([os.path.getsize(p) for p in c.paths])).all():
        raise RuntimeError("unexpected byte counts")
    pread_gbps = None
    if not args.no_plain:
        ws = WordScanRunner(ctx, c.paths, c.queries, chunk_max=1 << 20)

        def run_pread(e1=None):
            ws.launch(g.PERSISTENT, stream)
            if e1 is not None:
                e1.record(stream)
            torch.cuda.synchronize()
            if ctx.wait(60_000_000_000):
                raise RuntimeError("drain failed")
        pt, pw, _, _ = timed(run_pread, args.steps, 1)
        if not (ws.result() == counts).all():
            raise RuntimeError("open and pread forms disagree")
        pread_gbps = c.total_bytes * len(pw) / pt / 1e9
        ws.close()
    cpu = None
    oracle = oracle_leg(args)
    if oracle:
        threads = len(os.sched_getaffinity(0))
        t1 = time.perf_counter()
        want, _ = oracle.wordcount_open(d, names, c.queries, chunk=1 << 20, threads=threads)
        dt = time.perf_counter() - t1
        if not (want == counts).all():
            raise RuntimeError("GPU counts differ from the oracle")
        cpu = {"value": round(c.total_bytes / dt / 1e9, 3), "unit": "GB/s", "cores": threads,
               "kind": "oracle", "sample": "one pass over the 2,000-file corpus with openat / "
                                           "read / close, files split over %d POSIX threads"
                                           % threads}
    steps = len(wall)
    gbps = c.total_bytes * steps / total / 1e9
    kavg = float(np.mean(kms))
    res = {
        "metric": "GPU-issued syscalls/s + pread-scan GB/s (frac of link roofline); p99 latency",
        "value": round(gbps, 3), "unit": "GB/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * total / steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "word search with GPU openat / read / close: 2,000 files, "
                               "log-normal sizes (median 64 KiB, sigma 1, cap 8 MiB), 64 "
                               "queries, 1 MiB reads", "files": len(c.paths),
                   "bytes": c.total_bytes},
        "link_frac": round(gbps / LINK_PEAK_GBPS, 4),
        "syscalls_per_s": round(st["host_calls"] / total, 1),
        "calls_per_step": st["host_calls"] // steps,
        "roofline": {"bound": "host-link", "achieved": round(c.total_bytes / (kavg * 1e-3) / 1e9, 2),
                     "peak": LINK_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(c.total_bytes / (kavg * 1e-3) / 1e9 / LINK_PEAK_GBPS, 4),
                     "traffic": None, "kernel": "wordopen_persistent",
                     "kernel_ms": round(kavg, 3), "bytes_per_launch": c.total_bytes},
    }
    if pread_gbps is not None:
        res["pread_form_GBps"] = round(pread_gbps, 3)
    if cpu:
        res["cpu_baseline"] = cpu
    r.close()
    ctx.shutdown()
    print(json.dumps(res), flush=True)



def _cpu_s():
    import resource
    ru = resource.getrusage(resource.RUSAGE_SELF)
    return ru.ru_utime + ru.ru_stime


def run_doorbell(args):
    """Host cost of waiting for a quiet GPU: spinning pollers against the
    doorbell (idle pollers block on an HSA interrupt signal the kernels
    raise).  Per mode: the host CPU time the whole process burns per second
    of wall time while the GPU is idle, and the tiny case (one work-group x
    64 blocking 4 KiB preads) launched after `--db-gap-us` of idleness each
    time, end-to-end latency and CPU per second; then the serving mix at a
    low offered load (`--db-serve-rate`), latency and CPU per second.
    value = 64 calls / median tiny latency with the doorbell."""
    import numpy as np
    import torch
    import synth
    import paper_1705_06965_amd as g
    from paper_1705_06965_amd.fnv import FnvRunner
    from paper_1705_06965_amd.serve import ServeRun
    path = synth.random_file(1, 262144, name="c1_256k.bin")
    offs = synth.tiny_offsets(64)
    oracle = oracle_leg(args)
    want = oracle.pread_fnv(path, offs, 4096)[0] if oracle else None
    reps = max(50, args.steps)
    cell = g.cell_code("WI", "strong", "block")
    stream = torch.cuda.current_stream()
    modes = {}
    js = None
    if args.db_serve_rate > 0:
        in_path = synth.random_file(2, FILE_BYTES, name="c2_1g.bin")
        out_path = os.path.join(synth.data_dir(), "serve_out_db.bin")
        n_jobs = max(2000, int(args.db_serve_rate * 3))
        js = synth.job_stream(n_jobs=n_jobs, rate_per_s=args.db_serve_rate)
    for mode, flags in (("spin", 0), ("doorbell", g.CFG_DOORBELL)):
        ctx = g.Context(ring_slots=1 << 16, service_threads=max(0, args.service_threads),
                        device_timeout_ns=60_000_000_000, flags=flags,
                        arena_bytes=(16 << 30) if js is not None else 0)
        r = FnvRunner(ctx, path, offs, 4096, wg_size=64)
        for _ in range(max(1, args.warmup)):
            r.launch(cell, g.PLAIN, stream)
            torch.cuda.synchronize()
            ctx.wait(10_000_000_000)
        # idle: nothing launched for one second
        c0, w0 = _cpu_s(), time.perf_counter()
        time.sleep(1.0)
        idle_cores = (_cpu_s() - c0) / (time.perf_counter() - w0)
        s0 = ctx.stats()["doorbell_sleeps"]
        e2e = []
        c0, w0 = _cpu_s(), time.perf_counter()
        for _ in range(reps):
            time.sleep(args.db_gap_us * 1e-6)
            t0 = time.perf_counter()
            r.launch(cell, g.PLAIN, stream)
            torch.cuda.synchronize()
            if ctx.wait(10_000_000_000):
                raise RuntimeError("drain failed")
            e2e.append((time.perf_counter() - t0) * 1e6)
        tiny_cores = (_cpu_s() - c0) / (time.perf_counter() - w0)
        f, ret = r.result()
        if not ((ret == 4096).all() and (want is None or (f == want).all())):
            raise RuntimeError("GPU checksums differ from the oracle (%s)" % mode)
        m = {"idle_host_cores_busy": round(idle_cores, 3),
             "tiny_after_gap": {"gap_us": args.db_gap_us, "runs": reps,
                                "latency_us_p50": round(float(np.percentile(e2e, 50)), 1),
                                "latency_us_p99": round(float(np.percentile(e2e, 99)), 1),
                                "host_cores_busy": round(tiny_cores, 3)},
             "pollers_blocked": ctx.stats()["doorbell_sleeps"] - s0}
        r.close()
        if js is not None:
            sr = ServeRun(ctx, js, in_path, out_path)
            c0, w0 = _cpu_s(), time.perf_counter()
            res, _, lat = sr.run(g.PERSISTENT, max_inflight=args.serve_inflight,
                                 staging_bytes=(2 << 20) * 256, timeout_ns=300_000_000_000)
            cores = (_cpu_s() - c0) / (time.perf_counter() - w0)
            w = len(js.kind) // 10
            ls = lat[w:].astype(np.float64) / 1e3
            if (res < 0).any():
                raise RuntimeError("serving job failed (%s)" % mode)
            m["serve_low_load"] = {"offered_jobs_per_s": args.db_serve_rate, "jobs": len(js.kind),
                                   "latency_us_p50": round(float(np.percentile(ls, 50)), 1),
                                   "latency_us_p99": round(float(np.percentile(ls, 99)), 1),
                                   "host_cores_busy": round(cores, 3)}
            sr.close()
        modes[mode] = m
        ctx.shutdown()
        print("doorbell bench: %s done" % mode, file=sys.stderr, flush=True)
    med = modes["doorbell"]["tiny_after_gap"]["latency_us_p50"]
    res_j = {
        "metric": "GPU-issued syscalls/s + pread-scan GB/s (frac of link roofline); p99 latency",
        "value": round(64 / (med * 1e-6), 1), "unit": "calls/s", "n_gpus": 1, "steps": reps,
        "warmup": args.warmup, "ms_per_step": round(med / 1e3, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "doorbell against spinning pollers: tiny plain form (1 x 64 "
                               "blocking 4 KiB preads) after %d us of GPU idleness, and the "
                               "serving mix at %.0f jobs/s" % (args.db_gap_us, args.db_serve_rate),
                   "form": "plain (tiny), persistent (serving)"},
        "modes": modes,
    }
    print(json.dumps(res_j), flush=True)


def run_fileio(args):
    """Stateful file calls from the GPU.  Work-group round trip: 64
    work-groups each create a 4 MiB file on tmpfs, write it with write() in
    1 MiB pieces (strong), close it, reopen it, read it back in 1 MiB pieces
    plus an end-of-file read, close it and compare; one step = one launch
    (640 calls, 512 MiB moved each way).  value = bytes written + read per
    second.  Kernel granularity: 64 launches each appending 1 MiB through one
    descriptor with one kernel-wide write(), then 64 launches consuming it
    with one kernel-wide read(); per-launch latency."""
    import numpy as np
    import torch
    import synth
    import paper_1705_06965_amd as g
    from paper_1705_06965_amd.fileio import FileRoundtrip, kernel_io
    nf, fb, piece = 64, 4 << 20, 1 << 20
    base = os.path.join(synth.data_dir(), "fileio")
    d = os.path.join(base, "gpu")
    os.makedirs(d, exist_ok=True)
    names = ["f%02d.bin" % i for i in range(nf)]
    data = np.random.default_rng(170506965).integers(0, 256, (nf, fb), dtype=np.uint8)
    ctx = g.Context(ring_slots=1 << 12, service_threads=max(0, args.service_threads),
                    device_timeout_ns=60_000_000_000, flags=g.CFG_LEDGER)
    r = FileRoundtrip(ctx, d, names)
    k = fb // piece
    steps = max(1, args.steps)
    ts = []
    r.prepare(data, piece)
    for st in range(args.warmup + steps):
        r.rets.fill_(-12345)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r.launch("strong")
        torch.cuda.synchronize()
        if ctx.wait(60_000_000_000):
            raise RuntimeError("drain failed")
        dt = time.perf_counter() - t0
        rets, mism, back = r.finish()
        if mism.any() or not (rets[:, 1:k + 1] == piece).all() or \
                not (rets[:, k + 3:2 * k + 3] == piece).all() or rets[:, 2 * k + 3].any():
            raise RuntimeError("file round trip differs from the expected results")
        if st >= args.warmup:
            ts.append(dt)
    with open(os.path.join(d, names[-1]), "rb") as fh:
        if fh.read() != data[-1].tobytes():
            raise RuntimeError("file contents differ from the data")
    led = ctx.ledger(reset=True)
    svc = ((led[:, 5] >> np.uint64(8)).astype(np.int64) - led[:, 4].astype(np.int64)) / 1e3
    by_nr = {}
    for nr, nm in ((g.NR_WRITE, "write"), (g.NR_READ, "read"), (g.NR_OPENAT, "openat"),
                   (g.NR_CLOSE, "close")):
        m = led[:, 1] == nr
        if m.any():
            by_nr[nm] = round(float(np.median(svc[m])), 1)
    r.close()
    med = float(np.median(ts))
    # kernel granularity: append then consume through one description
    p = os.path.join(base, "append.bin")
    part = np.random.default_rng(5).integers(0, 256, 1 << 20, dtype=np.uint8)
    stg = ctx.host_alloc(1 << 20)
    wfd = os.open(p, os.O_WRONLY | os.O_CREAT | os.O_TRUNC, 0o600)
    ctx.allow_fd(wfd, g.FD_WRITE)
    lw = []
    for _ in range(64):
        t0 = time.perf_counter()
        ret, mm = kernel_io(ctx, wfd, g.NR_WRITE, part, grid=64, staging=stg)
        lw.append((time.perf_counter() - t0) * 1e6)
        if ret != len(part):
            raise RuntimeError("kernel-granularity write returned %d" % ret)
    ctx.allow_fd(wfd, 0)
    os.close(wfd)
    rfd = os.open(p, os.O_RDONLY)
    ctx.allow_fd(rfd, g.FD_READ)
    lr = []
    for _ in range(64):
        t0 = time.perf_counter()
        ret, mm = kernel_io(ctx, rfd, g.NR_READ, part, grid=64, staging=stg)
        lr.append((time.perf_counter() - t0) * 1e6)
        if ret != len(part) or mm:
            raise RuntimeError("kernel-granularity read returned %d (%d differ)" % (ret, mm))
    ctx.allow_fd(rfd, 0)
    os.close(rfd)
    stg.free()
    ctx.shutdown()
    cpu = None
    oracle = oracle_leg(args)
    if oracle:
        threads = len(os.sched_getaffinity(0))
        dc = os.path.join(base, "cpu")
        os.makedirs(dc, exist_ok=True)
        tc = []
        for _ in range(3):
            t0 = time.perf_counter()
            oracle.file_roundtrip(dc, names, data, piece, threads=threads)
            tc.append(time.perf_counter() - t0)
        cpu = {"value": round(2 * nf * fb / float(np.median(tc)) / 1e9, 3), "unit": "GB/s",
               "cores": threads, "kind": "oracle",
               "sample": "the same 64-file round trip issued by the oracle on %d threads, "
                         "median of 3" % threads}
    res = {
        "metric": "GPU-issued syscalls/s + pread-scan GB/s (frac of link roofline); p99 latency",
        "value": round(2 * nf * fb / med / 1e9, 3), "unit": "GB/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": round(1e3 * med, 3), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u8", "data": "synthetic",
        "config": {"workload": "stateful file round trip: 64 work-groups x (openat create, 4 x "
                               "1 MiB write, close, openat, 4 x 1 MiB read + end-of-file read, "
                               "close) on tmpfs, strong blocking work-group calls",
                   "form": "plain"},
        "calls_per_s": round(nf * (2 * k + 5) / med, 1),
        "host_service_us_median": by_nr,
        "kernel_append_1mib_us": {"p50": round(float(np.percentile(lw, 50)), 1),
                                  "p99": round(float(np.percentile(lw, 99)), 1)},
        "kernel_consume_1mib_us": {"p50": round(float(np.percentile(lr, 50)), 1),
                                   "p99": round(float(np.percentile(lr, 99)), 1)},
    }
    if cpu:
        res["cpu_baseline"] = cpu
    print(json.dumps(res), flush=True)

if __name__ == "__main__":
    main()
