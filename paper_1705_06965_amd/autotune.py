"""Autotuner of the batching and serving forms: picks the host pool and
launch knobs of each workload by measurement and caches them as JSON keyed by
workload, device and host core count, with every trial it measured.

Knobs are searched one at a time (coordinate search), each keeping the best
value so far; a new value must beat the best by 1% to replace it.
  sweep     service_threads P, wg_size W (descriptors per ring entry),
            sleep_max (GPU wait backoff cap), ring_slots D, coalescing (K, T)
            (section 4.2); objective: host calls per second
  wordscan  service_threads, buffers (two per persistent work-group, so also
            the grid), sleep_max; objective: scanned GB/s over launches of
            several passes (the form the benchmark times)
  serve     grid (persistent work-groups), sleep_max, service_threads;
            objective: p99 latency at the offered load, among settings that
            keep up with it
  kv, kv8   grid (server work-groups), batch (datagrams per list call),
            service_threads, and for kv the server loop (pipelined or
            blocking), with 4 (kv) or 8 (kv8) load-generator threads on the
            same host; objective: GETs per second
"""
from __future__ import annotations

import json
import os
import time

CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tuned.json")
DEFAULTS = {"service_threads": 0, "wg_size": 256, "sleep_max": 64, "ring_slots": 1 << 18,
            "coalesce_max": 1, "coalesce_window_ns": 0}
SPACE = [("service_threads", [8, 10, 12, 14, 15]),
         ("wg_size", [64, 128, 256]),
         ("sleep_max", [16, 64, 256, 1024]),
         ("ring_slots", [1 << 12, 1 << 16, 1 << 18]),
         ("coalesce", [(1, 0), (8, 2000), (32, 5000)])]


DEFAULTS_BY = {
    "sweep": DEFAULTS,
    "wordscan": {"service_threads": 12, "buffers": 128, "sleep_max": 64},
    "serve": {"grid": 64, "sleep_max": 64, "service_threads": 0},
    "kv": {"grid": 16, "batch": 256, "service_threads": 12, "pipelined": 1},
    "kv8": {"grid": 16, "batch": 256, "service_threads": 8, "pipelined": 0},
}
SPACE_BY = {
    "wordscan": [("service_threads", [8, 10, 12, 14, 15]), ("buffers", [96, 128, 160, 256]),
                 ("sleep_max", [16, 64, 256])],
    "serve": [("grid", [32, 48, 64, 96]), ("sleep_max", [16, 64, 256]),
              ("service_threads", [12, 14, 15])],
    "kv": [("pipelined", [0, 1]), ("grid", [8, 16, 32]), ("batch", [64, 128, 256]),
           ("service_threads", [8, 10, 12])],
    # with 8 load-generator threads the host's cores are all busy, and the
    # pipelined loop's second receive per work-group splits the datagrams
    # over more kernel calls (0.8x the blocking loop at 8 groups, 128-datagram
    # lists): the blocking loop only
    "kv8": [("grid", [4, 8, 16, 32]), ("service_threads", [6, 7, 8]),
            ("batch", [128, 256])],
}


def host_key(workload: str) -> str:
    try:
        import torch
        dev = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    except Exception:  # noqa: BLE001 - no GPU: key without a device name
        dev = "nodev"
    return "%s/%s/cores%d" % (workload, dev, len(os.sched_getaffinity(0)))


def load(workload: str = "sweep") -> dict:
    base = DEFAULTS_BY.get(workload, DEFAULTS)
    try:
        with open(CACHE) as f:
            d = json.load(f)
        return dict(base, **d.get(host_key(workload), {}).get("params", {}))
    except (OSError, ValueError):
        return dict(base)


def coordinate_search(measure, defaults: dict, space, log=print, lower_is_better=False):
    """One knob at a time from the defaults; returns (best params, best value,
    every trial as {"params", "value"})."""
    better = (lambda a, b: a < b * 0.99) if lower_is_better else (lambda a, b: a > b * 1.01)
    best = dict(defaults)
    best_v = measure(best)
    log("defaults %s: %s" % (best, best_v))
    trials = [{"params": dict(best), "value": best_v}]
    for knob, values in space:
        for v in values:
            p = dict(best)
            p[knob] = v
            if p == best:
                continue
            val = measure(p)
            trials.append({"params": dict(p), "value": val})
            log("%s=%s: %s" % (knob, v, val))
            if val is not None and (best_v is None or better(val, best_v)):
                best, best_v = p, val
    return best, best_v, trials


def measure_sweep(params: dict, path: str, offs, steps: int = 3) -> float:
    """Host calls per second of the persistent sweep with `params`."""
    import torch
    import paper_1705_06965_amd as g
    from paper_1705_06965_amd.fnv import FnvRunner
    ctx = g.Context(ring_slots=params["ring_slots"], service_threads=params["service_threads"],
                    coalesce_max=params["coalesce_max"],
                    coalesce_window_ns=params["coalesce_window_ns"],
                    sleep_max=params["sleep_max"], device_timeout_ns=60_000_000_000)
    try:
        r = FnvRunner(ctx, path, offs, 4096, wg_size=params["wg_size"])
        for _ in range(2):
            r.launch(0, g.GRAPH)
            torch.cuda.synchronize()
            ctx.wait()
        t = time.perf_counter()
        for _ in range(steps):
            r.launch(0, g.GRAPH)
            torch.cuda.synchronize()
            ctx.wait()
        dt = time.perf_counter() - t
        r.close()
        return len(offs) * steps / dt
    finally:
        ctx.shutdown()


def tune_sweep(path: str, offs, log=print) -> dict:
    best = dict(DEFAULTS)
    best_v = measure_sweep(best, path, offs)
    log("defaults: %.0f calls/s" % best_v)
    trials = [{"params": dict(best), "value": round(best_v, 1)}]
    for knob, values in SPACE:
        for v in values:
            p = dict(best)
            if knob == "coalesce":
                p["coalesce_max"], p["coalesce_window_ns"] = v
            else:
                p[knob] = v
            if p == best:
                continue
            val = measure_sweep(p, path, offs)
            trials.append({"params": dict(p), "value": round(val, 1)})
            log("%s=%s: %.0f calls/s" % (knob, v, val))
            if val > best_v * 1.01:
                best, best_v = p, val
    return {"params": best, "calls_per_s": round(best_v, 1), "trials": trials,
            "tuned_at": time.strftime("%Y-%m-%d %H:%M:%S")}


def measure_wordscan(params: dict, corpus, launches: int = 2, passes: int = 10) -> float:
    """Scanned GB/s of the persistent word search with `params`, over
    `launches` launches of `passes` passes each (after two warm-up launches)."""
    import torch
    import paper_1705_06965_amd as g
    from paper_1705_06965_amd.wordscan import WordScanRunner
    ctx = g.Context(ring_slots=1 << 16, service_threads=params["service_threads"],
                    sleep_max=params["sleep_max"], device_timeout_ns=60_000_000_000)
    try:
        r = WordScanRunner(ctx, corpus.paths, corpus.queries, chunk_max=1 << 20,
                           persistent_buffers=params["buffers"])
        for k in range(2 + launches):
            if k == 2:
                t = time.perf_counter()
            r.launch(g.PERSISTENT, passes=passes)
            torch.cuda.synchronize()
            ctx.wait()
        dt = time.perf_counter() - t
        r.close()
        return round(corpus.total_bytes * passes * launches / dt / 1e9, 3)
    finally:
        ctx.shutdown()


def measure_serve(params: dict, jobs, in_path: str, out_path: str, rate: float) -> float:
    """p99 latency (us, from scheduled arrival) of a persistent serving
    session with `params`; None if it did not keep up with the offered load."""
    import numpy as np
    import paper_1705_06965_amd as g
    from paper_1705_06965_amd.serve import ServeRun
    ctx = g.Context(ring_slots=1 << 16, service_threads=params["service_threads"],
                    sleep_max=params["sleep_max"], device_timeout_ns=60_000_000_000,
                    arena_bytes=16 << 30)
    try:
        sr = ServeRun(ctx, jobs, in_path, out_path)
        _, _, lat = sr.run(g.PERSISTENT, max_inflight=512, grid=params["grid"],
                           staging_bytes=(2 << 20) * 256)
        sr.close()
        warm = len(lat) // 10
        lat_us = lat[warm:].astype(np.float64) / 1e3
        span = (float(jobs.arrival_ns[-1]) - float(jobs.arrival_ns[warm])) / 1e9 + \
            float(np.median(lat_us)) / 1e6
        served = (len(lat) - warm) / span
        if served < 0.98 * rate:
            return None
        return round(float(np.percentile(lat_us, 99)), 1)
    finally:
        ctx.shutdown()


def measure_kv(params: dict, kv, reqs, clients: int = 4) -> float:
    """GETs per second of the key-value server with `params`."""
    import paper_1705_06965_amd as g
    from paper_1705_06965_amd.kv import KVServer, loadgen
    ctx = g.Context(ring_slots=1 << 16, service_threads=params["service_threads"],
                    device_timeout_ns=60_000_000_000)
    srv = None
    try:
        srv = KVServer(ctx, kv.keys, kv.val_off, kv.val_len, kv.heap, grid=params["grid"],
                       batch=params["batch"], pipelined=bool(params.get("pipelined", 1)))
        best = 0.0
        for _ in range(2):
            srv.start(lifetime_ms=120_000)
            t = time.perf_counter()
            got, *_ = loadgen(srv.port, reqs, threads=clients, window=128)
            dt = time.perf_counter() - t
            srv.stop()
            if got != len(reqs):
                return None
            best = max(best, len(reqs) / dt)
        return round(best, 1)
    finally:
        if srv is not None:
            srv.close()
        ctx.shutdown()


def tune(workload: str, log=print) -> dict:
    """Tune one of wordscan, serve, kv, kv8 on this machine; returns the cache entry."""
    import synth
    if workload == "wordscan":
        corpus = synth.wordcount_corpus()
        for p in corpus.paths:
            with open(p, "rb") as f:
                f.read()
        measure = lambda p: measure_wordscan(p, corpus)  # noqa: E731
        unit, low = "GBps", False
    elif workload == "serve":
        in_path = synth.random_file(2, 1 << 30, name="c2_1g.bin")
        jobs = synth.job_stream(n_jobs=12_000, rate_per_s=20_000.0)
        out_path = os.path.join(synth.data_dir(), "tune_serve_out.bin")
        measure = lambda p: measure_serve(p, jobs, in_path, out_path, 20_000.0)  # noqa: E731
        unit, low = "p99_us", True
    elif workload in ("kv", "kv8"):
        from paper_1705_06965_amd.kv import make_requests
        kv = synth.kv_set(n_req=1_000_000)
        reqs = make_requests(kv.req_keys)
        clients = 8 if workload == "kv8" else 4
        measure = lambda p: measure_kv(p, kv, reqs, clients)  # noqa: E731
        unit, low = "GET_per_s", False
    else:
        raise ValueError(workload)
    best, best_v, trials = coordinate_search(measure, DEFAULTS_BY[workload], SPACE_BY[workload],
                                             log=log, lower_is_better=low)
    return {"params": best, unit: best_v, "trials": trials,
            "tuned_at": time.strftime("%Y-%m-%d %H:%M:%S")}


def save(workload: str, result: dict, path: str | None = None) -> None:
    """Merge `result` into the cache (or into `path`, e.g. a copy to ship)."""
    path = path or CACHE
    d = {}
    for src in (path, CACHE):  # entries already written there, else the shipped cache
        try:
            with open(src) as f:
                d = json.load(f)
            break
        except (OSError, ValueError):
            continue
    d[host_key(workload)] = result
    with open(path, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)


if __name__ == "__main__":
    import sys
    import synth
    which = sys.argv[1:] or ["sweep", "wordscan", "serve", "kv"]
    for w in which:
        if w == "sweep":
            path = synth.random_file(2, 1 << 30, name="c2_1g.bin")
            offs = synth.sweep_offsets(262144, 262144)
            res = tune_sweep(path, offs, log=lambda s: print(s, flush=True))
        else:
            res = tune(w, log=lambda s, w=w: print(w, s, flush=True))
        save(w, res, os.environ.get("GSYS_TUNE_OUT"))
        print(w, json.dumps({k: v for k, v in res.items() if k != "trials"}), flush=True)
