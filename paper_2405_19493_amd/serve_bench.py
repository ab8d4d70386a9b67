"""Open-loop serving benchmark of the zg_server loop.

Requests arrive as a Poisson process (rate `rate` per second, inter-arrival
times from numpy PCG64(5)); sizes are log-uniform in [16, 2^24] variates;
70% FP64, 30% FP32; each request draws from one of a pool of counter handles
(SplitMix64 streams; 70% of the pool serves FP64 requests, the rest FP32,
since a handle's counter serves one output mode), so a stream's requests
continue where its previous one stopped.  Outputs go to the server's device arena and are released as soon as
they complete (the admission cap bounds the bytes in flight).  Latency is
completion time minus the scheduled arrival time, on the server clock.

The same arrival trace runs once in batched mode and once in per-request mode
(every request launched alone through the same path).  A sample of completed
requests is then regenerated alone with zg_fill at the first index the server
gave them, and must match bit for bit (alone-vs-mix).
"""
import sys
import threading
import time

import numpy as np
import torch

import paper_2405_19493_amd as Z


def make_trace(rate, duration_s, n_handles, seed=5, min_n=16, max_n=1 << 24):
    rng = np.random.Generator(np.random.PCG64(seed))
    count = int(rate * duration_s * 1.2) + 16
    gaps = rng.exponential(1.0 / rate, count)
    t = np.cumsum(gaps)
    t = t[t < duration_s]
    m = t.size
    sizes = np.exp(rng.uniform(np.log(min_n), np.log(max_n), m)).astype(np.int64)
    sizes = np.clip(sizes, min_n, max_n)
    dtypes = np.where(rng.uniform(0, 1, m) < 0.7, Z.ZG_F64, Z.ZG_F32)
    # a handle serves one dtype: the first 70% of the pool FP64, the rest FP32
    n64 = handle_split(n_handles)
    u = rng.uniform(0, 1, m)
    handles = np.where(dtypes == Z.ZG_F64, (u * n64).astype(np.int64),
                       n64 + (u * (n_handles - n64)).astype(np.int64))
    return t, sizes, dtypes, handles


def handle_split(n_handles):
    """Handles [0, n64) of the pool serve FP64 requests, the rest FP32."""
    return max(1, min(n_handles - 1, (7 * n_handles) // 10))


def open_handles(ctx, n_handles):
    n64 = handle_split(n_handles)
    return [ctx.zg_stream_open(1000 + h, h, Z.ZG_SPLITMIX64,
                               dtype=Z.ZG_F64 if h < n64 else Z.ZG_F32)
            for h in range(n_handles)]


def run_mode(ctx, mode, trace, handles, mem_cap, sample, sample_n_max, seed_base, window_us,
             n_streams=2):
    t_arr, sizes, dtypes, hidx = trace
    srv = Z.Server(ctx, mem_cap_bytes=mem_cap, max_inflight=8192, max_batch=4096,
                   batch_window_us=window_us, n_streams=n_streams, mode=mode)
    tickets = [None] * len(t_arr)
    keep = {}
    done_evt = threading.Event()
    errors = []

    def consumer():
        try:
            for k in range(len(t_arr)):
                while tickets[k] is None:
                    time.sleep(0.0001)
                c = srv.wait(tickets[k], 120.0)
                if c["status"] != Z.ZG_OK:
                    errors.append((k, c["status"]))
                if k in sample and sizes[k] <= sample_n_max:
                    n = int(sizes[k])
                    tdt = torch.float64 if dtypes[k] == Z.ZG_F64 else torch.float32
                    v = srv.output(c, n, int(dtypes[k]))
                    keep[k] = (c["first_index"], v.clone())
                    assert keep[k][1].dtype == tdt
                srv.release(tickets[k])
        except Exception as e:  # surfaced by the caller
            errors.append(("consumer", repr(e)))
        finally:
            done_evt.set()

    th = threading.Thread(target=consumer, daemon=True)
    th.start()
    base = srv.now() + 0.05
    for k in range(len(t_arr)):
        at = base + float(t_arr[k])
        while True:
            d = at - srv.now()
            if d <= 0:
                break
            if d > 0.0005:
                time.sleep(d - 0.0003)
        tickets[k] = srv.submit(handles[int(hidx[k])], int(sizes[k]), int(dtypes[k]),
                                Z.ZG_ZIGGURAT, at)
    done_evt.wait(600)
    srv.drain()
    st = srv.stats()
    srv.close()
    torch.cuda.synchronize()
    span = st["last_complete_s"] - st["first_arrival_s"]
    res = {
        "requests": int(st["completed"]), "batches": int(st["batches"]),
        "variates": int(st["variates"]),
        "variates_per_s": st["variates"] / span if span > 0 else 0.0,
        "p50_latency_ms": st["p50_latency_s"] * 1e3, "p99_latency_ms": st["p99_latency_s"] * 1e3,
        "max_latency_ms": st["max_latency_s"] * 1e3,
        "peak_inflight_bytes": int(st["peak_inflight_bytes"]), "errors": len(errors),
    }
    return res, keep, errors


def alone_vs_mix(ctx, keep, trace, seed_of_handle, stream_of_handle):
    """Regenerates each kept request alone at its recorded first index."""
    _, sizes, dtypes, hidx = trace
    bad = 0
    for k, (first, got) in keep.items():
        h = int(hidx[k])
        out = torch.empty_like(got)
        ctx.zg_fill(out, kind=Z.ZG_SPLITMIX64, seed=seed_of_handle(h), stream=stream_of_handle(h),
                    first_index=first)
        torch.cuda.synchronize()
        if not torch.equal(out.view(torch.uint8), got.view(torch.uint8)):
            bad += 1
    return bad


def replay_mode(ctx, mode, trace, handles, mem_cap, window_us, n_streams=2):
    """C-driven open-loop replay of the trace; returns the server's figures."""
    t_arr, sizes, dtypes, hidx = trace
    srv = Z.Server(ctx, mem_cap_bytes=mem_cap, max_inflight=8192, max_batch=4096,
                   batch_window_us=window_us, n_streams=n_streams, mode=mode)
    hs = np.asarray(handles, dtype=np.int64)[hidx]
    t0 = time.perf_counter()
    srv.replay(hs, sizes, dtypes, t_arr, timeout_s=600.0)
    wall = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    span = st["last_complete_s"] - st["first_arrival_s"]
    return {"requests": int(st["completed"]), "batches": int(st["batches"]),
            "variates_per_s": st["variates"] / span if span > 0 else 0.0,
            "p50_latency_ms": st["p50_latency_s"] * 1e3, "p99_latency_ms": st["p99_latency_s"] * 1e3,
            "max_latency_ms": st["max_latency_s"] * 1e3,
            "peak_inflight_bytes": int(st["peak_inflight_bytes"]), "wall_s": wall}


def run(ctx, duration_s=5.0, rate=20000.0, n_handles=65536, mem_cap=64 << 30, window_us=0,
        check_s=1.0, sweep=(20000, 50000, 100000, 200000, 400000), sweep_s=1.0,
        sample_every=97, sample_n_max=1 << 20):
    """The serving figures for the bench line: the trace at `rate` replayed
    in both modes (headline p50/p99 and variates/s), an alone-vs-mix bit check
    on sampled requests, and a rate sweep to saturation."""
    free, _total = torch.cuda.mem_get_info()
    mem_cap = int(min(mem_cap, free * 0.6)) & ~255
    out = {"offered_rate_per_s": rate, "duration_s": duration_s, "arena_bytes": mem_cap,
           "batch_window_us": window_us}
    modes = (("batched", Z.ZG_SERVE_BATCHED), ("per_request", Z.ZG_SERVE_PER_REQUEST))
    handles = open_handles(ctx, n_handles)
    try:
        trace = make_trace(rate, duration_s, n_handles)
        out["requests"] = len(trace[0])
        out["mean_request_variates"] = float(trace[1].mean()) if len(trace[0]) else 0.0
        for name, mode in modes:
            print(f"serve: {name}, {duration_s:.0f} s at {rate:.0f} requests/s", file=sys.stderr,
                  flush=True)
            out[name] = replay_mode(ctx, mode, trace, handles, mem_cap, window_us)
        # alone-vs-mix: a shorter trace driven from Python so outputs can be kept
        ctrace = make_trace(rate, check_s, n_handles, seed=6)
        sample = set(range(0, len(ctrace[0]), sample_every))
        for name, mode in modes:
            _res, keep, errors = run_mode(ctx, mode, ctrace, handles, mem_cap, sample,
                                          sample_n_max, 1000, window_us)
            out[name]["alone_vs_mix_checked"] = len(keep)
            out[name]["alone_vs_mix_mismatch"] = alone_vs_mix(ctx, keep, ctrace,
                                                              lambda h: 1000 + h, lambda h: h)
            out[name]["errors"] = len(errors)
        rows = []
        print("serve: rate sweep", file=sys.stderr, flush=True)
        for r in sweep:
            tr = make_trace(float(r), sweep_s, n_handles, seed=7)
            row = {"rate_per_s": r}
            for name, mode in modes:
                res = replay_mode(ctx, mode, tr, handles, mem_cap, window_us)
                row[name] = {k: res[k] for k in ("variates_per_s", "p50_latency_ms",
                                                 "p99_latency_ms", "batches")}
            rows.append(row)
        out["sweep"] = rows
        # the lowest offered rate of the sweep at which the batched mode's p99
        # beats the per-request mode's (None: not within the sweep)
        out["p99_crossover_rate_per_s"] = next(
            (row["rate_per_s"] for row in rows
             if row["batched"]["p99_latency_ms"] < row["per_request"]["p99_latency_ms"]), None)
    finally:
        for h in handles:
            ctx.zg_stream_close(h)
    return out
