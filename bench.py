"""Benchmark: FP64 Gaussian variates/s against the HBM-write roofline.

Workload (the configuration the metric is quoted on): the original 128-layer
ziggurat and the Marsaglia polar method side by side, 2^28 FP64 standard
normals each, SplitMix64 uniforms with seed 7 and 65536 independent stream ids
of 4096 variates, written to one contiguous float64 buffer (2 GiB).  A step is
one ziggurat fill of the whole buffer; the polar fill is timed the same way and
reported beside it.  Inputs are synthetic (seeds only).

Prints one JSON line.  --gpus N > 1 exits: the benchmark runs on one GPU (every
variate is a pure function of its key, so GPUs would split the streams with no
communication; that path is a design, not code).
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "FP64 Gaussian variates/s vs HBM-write roofline; p50/p99 request latency"
HBM_PEAK_GBS = 8000.0
N_STREAMS = 65536
N_PER = 4096
SEED = 7


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--cpu-seconds", type=float, default=10.0,
                   help="approximate CPU work of the oracle baseline sample")
    p.add_argument("--only", choices=["zig", "polar", "mz", "f32", "lcg", "mutate", "ea", "c4",
                                      "all"],
                   default="all",
                   help="restrict the timed kernels (for profiling runs; c4: only the batch row, "
                        "printed as its own JSON line)")
    p.add_argument("--serve-seconds", type=float, default=60.0,
                   help="serving-loop run per mode (open-loop Poisson, 20k requests/s); 0 = skip")
    p.add_argument("--autotune", action="store_true",
                   help="run the launch-shape autotuner (zg_autotune) first; by default the "
                        "library's default shapes are timed (chosen from a sweep of every "
                        "candidate shape on these workloads)")
    p.add_argument("--no-extra", action="store_true",
                   help="skip the LCG, batch and mutation rows (profiling runs)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run three plain 1 GiB device copies (the known-size kernel "
                        "that scales the HBM byte counters) and exit")
    return p.parse_args()


def copy_calibration(torch):
    """Three device-to-device copies of 2^27 float64 (1 GiB read + 1 GiB written
    each): what FETCH_SIZE and WRITE_SIZE read for them calibrates those
    counters for the fill kernels."""
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": a.numel() * 8, "launches": 3}), flush=True)


def time_kernel(fn, steps, warmup, torch):
    """Average ms per launch with HIP events on the current stream (the stream
    the kernels are launched on), bracketed by device syncs."""
    for _ in range(warmup):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        fn()
        b.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [a.elapsed_time(b) for a, b in ev]
    return sum(ms) / len(ms), ms, wall


def time_kernel_back_to_back(fn, launches, warmup, torch):
    """Average ms per launch of `launches` launches between one pair of HIP
    events: for kernels of tens of microseconds, where events around every
    launch would also time the host's launch gap."""
    for _ in range(warmup):
        fn()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    a.record()
    for _ in range(launches):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / launches


def median_ci(xs, z=3.29):
    """Median of the per-launch times and a distribution-free 99.9% confidence
    interval for it (order statistics at n/2 -+ z sqrt(n)/2)."""
    v = sorted(xs)
    n = len(v)
    med = v[n // 2] if n % 2 else 0.5 * (v[n // 2 - 1] + v[n // 2])
    half = z * (n ** 0.5) / 2.0
    lo = max(0, int(n / 2.0 - half))
    hi = min(n - 1, int(n / 2.0 + half + 0.999))
    return med, [v[lo], v[hi]]


def note(msg):
    """A progress line on stderr (stdout carries only the JSON line)."""
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def cpu_baseline(seconds):
    """The oracle (oracle/zg_oracle.c) on a bounded sample of the same workload:
    whole streams of 4096 variates, seed 7, SplitMix64, in batches of streams
    whose variates the oracle's own threads share (one thread per host core,
    capped at 16, the CPU share of one GPU), until about `seconds` of wall time
    have passed."""
    from oracle import coracle as orc
    orc.build(force=False)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(cores, 16))
    per_batch = 256 * cores

    def one(s):
        orc.fill_f64(orc.SM64, SEED, s, 0, N_PER, nthreads=1)

    s = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds and s < N_STREAMS:
        b = min(per_batch, N_STREAMS - s)
        orc.fill_streams_f64(orc.SM64, SEED, s, b, 0, N_PER, nthreads=cores)
        s += b
    dt = time.perf_counter() - t0
    done = s * N_PER
    # one core, to set beside per-call times on a CPU (ns per variate)
    k = 0
    t1 = time.perf_counter()
    while time.perf_counter() - t1 < min(3.0, seconds) and k < N_STREAMS:
        one(k)
        k += 1
    dt1 = time.perf_counter() - t1
    cpu = {}
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if ":" in line:
                    key, val = (x.strip() for x in line.split(":", 1))
                    if key in ("model name", "cpu family", "model", "stepping", "cpu MHz",
                               "cache size") and key not in cpu:
                        cpu[key] = val
    except OSError:
        pass
    rows = cpu_rows(orc, cores)
    return {"value": done / dt, "unit": "variates/s", "cores": cores, "kind": "oracle",
            "cpu": cpu.get("model name", ""), "cpu_id": cpu,
            "nproc": os.cpu_count(),
            "affinity": len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None,
            "threads_note": "the oracle's threads are capped at 16, the host CPU share of one "
                            "GPU on these machines, whatever nproc shows",
            "sample": f"streams 0..{s - 1} of the 65536 x 4096 FP64 ziggurat variates "
                      f"(SplitMix64 seed 7): {done} variates in {dt:.1f} s",
            "one_core": {"value": k * N_PER / dt1, "unit": "variates/s",
                         "ns_per_variate": dt1 * 1e9 / (k * N_PER),
                         "sample": f"streams 0..{k - 1}, one thread"},
            "rows": rows}


def cpu_rows(orc, cores):
    """The oracle on a bounded sample of each other row's workload, with the
    same threads: rates to set beside the GPU rows."""
    import numpy as np
    out = {}

    def timed(name, fn, units, unit, sample):
        t0 = time.perf_counter()
        fn()
        dt = time.perf_counter() - t0
        out[name] = {"value": units / dt, "unit": unit, "cores": cores, "sample": sample,
                     "seconds": dt}

    ns = 16384   # a quarter of the 65536 streams of 4096
    timed("mcfarland", lambda: orc.fill_streams_mz(orc.SM64, SEED, 0, ns, 0, N_PER, nthreads=cores),
          ns * N_PER, "variates/s", f"modified ziggurat, streams 0..{ns - 1} x 4096, seed 7")
    timed("polar", lambda: orc.fill_streams_polar(orc.SM64, SEED, 0, ns, 0, N_PER, nthreads=cores),
          ns * N_PER, "variates/s", f"polar, streams 0..{ns - 1} x 4096, seed 7")
    timed("f32", lambda: orc.fill_streams_f32(orc.SM64, SEED, 0, ns, 0, N_PER, nthreads=cores),
          ns * N_PER, "variates/s", f"FP32 ziggurat, streams 0..{ns - 1} x 4096, seed 7")
    n_lcg = 1 << 26
    timed("c3_lcg", lambda: orc.fill_f64(orc.LCG48, 123456789, 0, 0, n_lcg, nthreads=cores),
          n_lcg, "variates/s", "FP64 ziggurat, LCG48 seed 123456789, the first 2^26 of the stream")
    pop, genes = 16384, 1024
    g = np.random.Generator(np.random.PCG64(7))
    P = g.uniform(-5.0, 5.0, (pop, genes))
    F = (P * P).sum(axis=1)
    timed("ea_step", lambda: orc.ea_step(P, F, 2, 2024, 100, 3, 0.05, 0.1, -5.0, 5.0,
                                         nthreads=cores),
          pop * genes, "genes/s", "one EA generation, 16384 x 1024 genes (the whole row)")
    return out


def c3_lcg(ctx, Z, torch, steps, warmup):
    """FP64 ziggurat over 2^28 variates of one LCG48 stream (seed 123456789)."""
    n = 1 << 28
    out = torch.empty(n, dtype=torch.float64, device="cuda")

    def go():
        ctx.zg_fill(out, kind=Z.ZG_JAVA_LCG48, seed=123456789, stream=0, first_index=0)

    ms, _, _ = time_kernel(go, steps, warmup, torch)
    del out
    t = ctx.zg_get_tune(Z.ZG_TUNE_FILL_F64)
    kernel = ("k_zigws" if t[4] else "k_zig") + "<OP_ZIG64, LCG48>"
    return {"workload": "ziggurat fill, 2^28 FP64, LCG48 seed 123456789, stream 0",
            "value": n / (ms * 1e-3), "unit": "variates/s", "kernel_ms": ms,
            "roofline": {"bound": "hbm", "achieved": 8.0 * n / (ms * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": 8.0 * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         "kernel": kernel, "traffic": read_traffic(kernel)}}


def sequential_row(ctx, Z, torch, steps, warmup):
    """Sequential consumption: the variates successive nextGaussian(random)
    calls take from one SplitMix64 generator (seed 7, stream 0), at the
    largest size checked on the device (all four passes timed together)."""
    n = Z.ZG_SEQ_MAX_N
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    work = torch.empty(Z.zg_sequential_workspace(n), dtype=torch.uint8, device="cuda")

    def go():
        ctx.zg_fill_sequential(out, kind=Z.ZG_SPLITMIX64, seed=7, stream=0, first_word=0,
                               work=work)

    ms, _, _ = time_kernel(go, steps, warmup, torch)
    del out, work
    return {"workload": f"sequential consumption, {n} FP64 variates from one SplitMix64 "
                        "generator (seed 7, stream 0)",
            "capped": {"size_run": n, "benchmark_size": N_STREAMS * N_PER,
                       "reason": "the path refuses more than ZG_SEQ_MAX_N variates: every device "
                                 "run above 1024 workgroups faulted, cause not shown"},
            "value": n / (ms * 1e-3), "unit": "variates/s", "ms": ms,
            "roofline": {"bound": "hbm", "achieved": 8.0 * n / (ms * 1e-3) / 1e9,
                         "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": 8.0 * n / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                         # the path is several launches (chain maps, scan, write pass),
                         # timed as a whole; no counter pass covers it
                         "kernel": "zg_fill_sequential (all its launches)", "traffic": None}}


def f32_row(ctx, Z, torch, steps, warmup):
    """The c2 layout in FP32 output (2^28 variates, 1 GiB; 4 B per variate)."""
    n = N_STREAMS * N_PER
    out = torch.empty(n, dtype=torch.float32, device="cuda")

    def go():
        ctx.zg_fill_streams(out, N_PER, N_STREAMS, method=Z.ZG_ZIGGURAT, kind=Z.ZG_SPLITMIX64,
                            seed=SEED, stream0=0, first_index=0)

    ms, _, _ = time_kernel(go, steps, warmup, torch)
    del out
    gbs = 4.0 * n / (ms * 1e-3) / 1e9
    t = ctx.zg_get_tune(Z.ZG_TUNE_FILL_F32)
    kernel = ("k_zigws" if t[4] else "k_zig") + "<OP_ZIG32>"
    return {"workload": "ziggurat fill, 2^28 FP32, SplitMix64 seed 7, 65536 streams x 4096",
            "value": n / (ms * 1e-3), "unit": "variates/s", "kernel_ms": ms,
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "kernel": kernel,
                         "traffic": read_traffic(kernel)}}


def c4_recipe():
    """The c4 request set: 10^4 sizes clamp(floor(2^(20u)), 1, 2^20) and FP64
    with probability 0.7, u from numpy PCG64(4); request k is seed 1000 + k,
    stream k, from index 0.  Plus one mutation of 4096 x 1024 genes (seed 999,
    stream 0, sigma 0.1) whose initial genes are -5 + 10 U, U from the uniform
    words of (seed 1, stream 65535)."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(4))
    m = 10000
    u = rng.uniform(0.0, 1.0, m)
    sizes = np.clip(np.floor(2.0 ** (20 * u)).astype(np.int64), 1, 1 << 20)
    is64 = rng.uniform(0.0, 1.0, m) < 0.7
    return sizes, is64, 4096 * 1024


def c4_batch(ctx, Z, torch, reps):
    """10^4 uneven requests (sizes clamp(2^(20u)), 70% FP64) plus one mutation
    of 4096 x 1024 genes: one persistent batch launch against the same
    requests issued one by one to the plain kernels."""
    import numpy as np
    sizes, is64, genes = c4_recipe()
    m = sizes.size
    nbytes = [int(n) * (8 if f else 4) for n, f in zip(sizes, is64)]
    offs = np.concatenate([[0], np.cumsum([(b + 255) // 256 * 256 for b in nbytes])])
    pool = torch.empty(int(offs[-1]) + genes * 8 + 256, dtype=torch.uint8, device="cuda")
    views = []
    for k in range(m):
        v = pool[int(offs[k]):int(offs[k]) + nbytes[k]]
        views.append(v.view(torch.float64) if is64[k] else v.view(torch.float32))
    g0 = int(offs[-1])
    x = pool[g0:g0 + genes * 8].view(torch.float64)
    # initial genes: -5 + 10 U from the uniform words of (seed 1, stream 65535)
    w = torch.empty(genes, dtype=torch.int64, device="cuda")
    ctx.zg_uniform_words(w, kind=Z.ZG_SPLITMIX64, seed=1, stream=65535)
    x0 = -5.0 + 10.0 * ((w >> 11).to(torch.float64) * 2.0 ** -53)
    del w
    reqs = [{"out": views[k], "n": int(sizes[k]), "seed": 1000 + k, "stream": k,
             "dtype": Z.ZG_F64 if is64[k] else Z.ZG_F32} for k in range(m)]
    reqs.append({"out": x, "n": genes, "seed": 999, "stream": 0, "op": Z.ZG_OP_MUTATE,
                 "sigma": 0.1, "dtype": Z.ZG_F64})

    creqs = ctx.zg_batch_prepare(reqs)

    def batched():
        x.copy_(x0)
        ctx.zg_batch(creqs)

    def plain():
        # the same requests as 10^4 + 1 plain launches from one C loop
        x.copy_(x0)
        ctx.zg_fill_each(creqs)

    variates = int(sizes.sum()) + genes
    total_bytes = int(sum(nbytes)) + 16 * genes   # outputs written, genes read and written
    out = {"workload": "10^4 requests, sizes clamp(2^(20u),1,2^20), 70% FP64 / 30% FP32, "
                       "plus a 4096x1024-gene mutation (sigma 0.1)", "variates": variates,
           "per_request_form": "zg_fill_each: one plain launch per request, from a C loop"}
    kept = None
    same = True
    for name, fn in (("batched", batched), ("per_request", plain)):
        # one call at a time (the latency of one call, host planning included),
        # and calls back to back (the throughput of a stream of such calls: the
        # host plans the next while the device runs this one)
        ms, _, _ = time_kernel(fn, reps, 1, torch)
        ms_b2b = time_kernel_back_to_back(fn, 2 * reps, 0, torch)
        pool[:g0].zero_()
        fn()
        torch.cuda.synchronize()
        if kept is None:
            kept = pool[:g0 + genes * 8].clone()
        else:
            # every byte of every request and of the mutated genes
            same = bool(torch.equal(kept, pool[:g0 + genes * 8]))
        out[name] = {"ms": ms, "variates_per_s": variates / (ms * 1e-3),
                     "ms_back_to_back": ms_b2b,
                     "variates_per_s_back_to_back": variates / (ms_b2b * 1e-3),
                     "bytes_per_s_back_to_back": total_bytes / (ms_b2b * 1e-3)}
    del kept
    out["same_bits"] = same
    out["speedup"] = out["per_request"]["ms"] / out["batched"]["ms"]
    out["speedup_back_to_back"] = (out["per_request"]["ms_back_to_back"] /
                                   out["batched"]["ms_back_to_back"])
    out["mutation"] = mutation_row(ctx, torch, x, 20, 3)
    del pool, views, x, x0
    torch.cuda.empty_cache()
    return out


def mutation_row(ctx, torch, x, steps, warmup):
    """The c4 mutation alone (4096 x 1024 genes, sigma 0.1, seed 999), against
    its own roofline: 8 B read + 8 B written per gene."""
    genes = x.numel()
    ms = time_kernel_back_to_back(lambda: ctx.zg_mutate(x, 0.1, seed=999, stream=0),
                                  max(steps, 50), warmup, torch)
    gbs = 16.0 * genes / (ms * 1e-3) / 1e9
    t = ctx.zg_get_tune(3)
    kernel = ("k_zigws" if t[4] else "k_zig") + "<OP_MUTATE>"
    return {"genes": genes, "kernel_ms": ms, "timing": "back-to-back launches between two events",
            "genes_per_s": genes / (ms * 1e-3),
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "kernel": kernel,
                         "traffic": read_traffic(kernel)}}


def ea_row(ctx, Z, torch, steps, warmup):
    """One EA generation (zg_ea_step): 16384 genomes x 1024 genes, sphere
    fitness, binary tournament, per-gene rate 0.05, sigma 0.1, bounds [-5, 5];
    against the HBM roofline of 8 B read + 8 B written per gene."""
    pop, genes = 16384, 1024
    g = torch.Generator(device="cpu").manual_seed(7)
    P = (torch.rand((pop, genes), generator=g, dtype=torch.float64) * 10.0 - 5.0).cuda()
    F = (P * P).sum(dim=1)
    C = torch.empty_like(P)
    W = torch.empty(pop, dtype=torch.int32, device="cuda")

    def go():
        ctx.zg_ea_step(P, F, C, W, tournament=2, rate=0.05, sigma=0.1, lo=-5.0, hi=5.0,
                       seed=2024, stream=100, generation=3)

    ms = time_kernel_back_to_back(go, max(steps, 50), warmup, torch)
    cells = pop * genes
    gbs = 16.0 * cells / (ms * 1e-3) / 1e9
    del P, F, C, W
    return {"workload": "one EA generation: 16384 x 1024 genes, sphere fitness, tournament 2, "
                        "rate 0.05, sigma 0.1, bounds [-5, 5]",
            "kernel_ms": ms, "timing": "back-to-back launches between two events",
            "genes_per_s": cells / (ms * 1e-3),
            "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": gbs / HBM_PEAK_GBS, "kernel": "k_ea",
                         "traffic": read_traffic("k_ea")}}


def read_profile(kernel):
    """The committed rocprofv3 summary entry of a kernel (profiles/traffic.json),
    if it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            ent = json.load(fh).get(kernel)
    except (OSError, ValueError):
        return None
    if not ent:
        return None
    import hashlib
    src = os.path.join(ROOT, "paper_2405_19493_amd", "csrc", "zg_kernels.hip")
    with open(src, "rb") as fh:
        if ent.get("source_sha") != hashlib.sha256(fh.read()).hexdigest()[:16]:
            return None
    return ent


# VALU issue peak for FP64-heavy code: one wave-64 instruction per 4 cycles
# per SIMD (the published FP64 vector rate, 16 lanes per cycle), 256 CUs x 4
# SIMDs at 2.4 GHz.  Plain 32-bit integer instructions issue faster (about 2.6
# cycles measured) and 32-bit multiplies slower (about 4.8), so for integer
# work this is an estimate, not a ceiling.
VALU_PEAK_G = 256 * 4 * 2.4e9 / 4 / 1e9


def read_traffic(kernel):
    """HBM bytes per launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(path) as fh:
            doc = json.load(fh)
    except (OSError, ValueError):
        return None
    ent = doc.get(kernel)
    if not ent:
        return None
    import hashlib
    src = os.path.join(ROOT, "paper_2405_19493_amd", "csrc", "zg_kernels.hip")
    with open(src, "rb") as fh:
        digest = hashlib.sha256(fh.read()).hexdigest()[:16]
    if ent.get("source_sha") != digest:
        return None
    return ent.get("bytes_per_launch")


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: every configuration here fits one MI355X, "
              "and the path would shard by index range with no communication",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return
    import paper_2405_19493_amd as Z

    n = N_STREAMS * N_PER
    ctx = Z.Context(0)
    if args.autotune:
        # the launch shape that is fastest on this device, at this size; cached
        # per device so that later runs (a profiler's) time the same shape
        import tempfile
        cache = os.path.join(tempfile.gettempdir(), "zg_autotune_2p28.json")
        ctx.zg_autotune(cache, 8 * N_STREAMS * N_PER, use_cache=True)
    if args.only in ("f32", "lcg", "mutate", "ea"):
        # one row alone (short runs under a profiler)
        if args.only == "f32":
            row = f32_row(ctx, Z, torch, args.steps, args.warmup)
        elif args.only == "ea":
            row = ea_row(ctx, Z, torch, args.steps, args.warmup)
        elif args.only == "lcg":
            row = c3_lcg(ctx, Z, torch, args.steps, args.warmup)
        else:
            import numpy as np
            rng = np.random.Generator(np.random.PCG64(5))
            x = torch.from_numpy(rng.uniform(-5.0, 5.0, 4096 * 1024)).cuda()
            row = mutation_row(ctx, torch, x, args.steps, args.warmup)
        ctx.close()
        print(json.dumps({args.only: row}), flush=True)
        return
    if args.only == "c4":
        row = c4_batch(ctx, Z, torch, 3)
        row["batch_tune"] = list(ctx.zg_get_tune(Z.ZG_TUNE_BATCH))
        ctx.close()
        print(json.dumps({"c4_batch": row}), flush=True)
        return
    tune = ctx.zg_get_tune(Z.ZG_TUNE_FILL_F64)

    def launch_of(t):
        return {"kernel": "wave-specialised" if t[4] else "block-pooled", "tile": t[0],
                "waves_per_block": t[1], "persistent_blocks_per_cu": t[2], "drain_waves": t[4],
                "group_steps": t[5], "autotuned": bool(args.autotune)}
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    out.zero_()

    def zig():
        ctx.zg_fill_streams(out, N_PER, N_STREAMS, method=Z.ZG_ZIGGURAT, kind=Z.ZG_SPLITMIX64,
                            seed=SEED, stream0=0, first_index=0)

    def polar():
        ctx.zg_fill_streams(out, N_PER, N_STREAMS, method=Z.ZG_POLAR, kind=Z.ZG_SPLITMIX64,
                            seed=SEED, stream0=0, first_index=0)

    def mz():
        ctx.zg_fill_streams(out, N_PER, N_STREAMS, method=Z.ZG_MCFARLAND, kind=Z.ZG_SPLITMIX64,
                            seed=SEED, stream0=0, first_index=0)

    res = {}
    if args.only == "all":
        # a plain store-only kernel writing the same 2 GiB (torch fill_): the
        # write bandwidth this machine reaches with no compute at all
        res["store_only"] = time_kernel(lambda: out.fill_(0.5), args.steps, args.warmup, torch)
    if args.only in ("zig", "all"):
        note("ziggurat fill, 2^28 FP64")
        res["zig"] = time_kernel(zig, args.steps, args.warmup, torch)
    if args.only in ("polar", "all"):
        res["polar"] = time_kernel(polar, args.steps, args.warmup, torch)
    if args.only in ("mz", "all"):
        res["mz"] = time_kernel(mz, args.steps, args.warmup, torch)
    flags = ctx.zg_error_flags()
    if flags:
        raise SystemExit(f"device error flags {flags}")

    main_key = "zig" if "zig" in res else ("mz" if "mz" in res else "polar")
    ms, all_ms, wall = res[main_key]
    wall_ms = wall * 1e3 / args.steps
    med, ci = median_ci(all_ms)
    bytes_per = 8.0 * n
    achieved = bytes_per / (ms * 1e-3) / 1e9
    mz_tune = ctx.zg_get_tune(Z.ZG_TUNE_FILL_MZ)
    kname = lambda t, op: ("k_zigws" if t[4] else "k_zig") + f"<{op}>"
    kernel = {"zig": kname(tune, "OP_ZIG64"), "mz": kname(mz_tune, "OP_MZ64"),
              "polar": "k_polar"}[main_key]
    traffic = read_traffic(kernel)
    line = {
        "metric": METRIC,
        "value": n / (wall_ms * 1e-3),
        "unit": "variates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall_ms,
        "kernel_ms": ms,
        "kernel_ms_median": med,
        "kernel_ms_median_ci999": ci,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "ziggurat fill, 2^28 FP64 N(0,1), SplitMix64 seed 7, "
                               "65536 streams x 4096, contiguous float64 (2 GiB); "
                               "polar fill of the same shape timed beside it",
                   "method": {"zig": "ziggurat", "mz": "modified ziggurat",
                              "polar": "polar"}[main_key],
                   "launch": launch_of(tune),
                   "variates_per_step": n, "streams": N_STREAMS, "per_stream": N_PER},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel, "algorithmic_bytes_per_launch": bytes_per},
    }
    if "store_only" in res:
        sgbs = bytes_per / (res["store_only"][0] * 1e-3) / 1e9
        line["roofline"]["store_only_GBps"] = sgbs
        line["roofline"]["frac_of_store_only"] = achieved / sgbs
    if "polar" in res and main_key == "zig":
        pms = res["polar"][0]
        pwall = res["polar"][2] * 1e3 / args.steps
        pach = bytes_per / (pms * 1e-3) / 1e9
        line["polar"] = {"value": n / (pwall * 1e-3), "unit": "variates/s", "ms_per_step": pwall,
                         "kernel_ms": pms,
                         "roofline": {"bound": "hbm", "achieved": pach, "peak": HBM_PEAK_GBS,
                                      "unit": "GB/s", "frac": pach / HBM_PEAK_GBS,
                                      "kernel": "k_polar", "traffic": read_traffic("k_polar")}}
        prof = read_profile("k_polar")
        if prof:
            # polar is bound by VALU issue: its instruction rate against that peak
            rate = prof["valu_per_64"] * n / 64 / (pms * 1e-3) / 1e9
            line["polar"]["alu_view"] = {
                "bound": "alu", "achieved": rate, "peak": VALU_PEAK_G,
                "unit": "G VALU wave-instructions/s", "frac": rate / VALU_PEAK_G,
                "valu_per_64_variates": prof["valu_per_64"],
                "source": "profiles/polar_2p28.counters.txt (SQ_INSTS_VALU)"}
    if "mz" in res and main_key == "zig":
        # the modified ziggurat (McFarland's method) on the same workload: the
        # paper's comparator, measured 11.52% faster than the original on
        # SplittableRandom in Section 3
        mms = res["mz"][0]
        mwall = res["mz"][2] * 1e3 / args.steps
        mach = bytes_per / (mms * 1e-3) / 1e9
        line["mcfarland"] = {
            "workload": "modified ziggurat fill, 2^28 FP64, SplitMix64 seed 7, "
                        "65536 streams x 4096 (the same buffer and launch shape)",
            "value": n / (mwall * 1e-3), "unit": "variates/s", "ms_per_step": mwall,
            "kernel_ms": mms, "kernel_ms_median": median_ci(res["mz"][1])[0],
            "launch": launch_of(mz_tune),
            "ziggurat_over_mcfarland_kernel_time": ms / mms,
            "roofline": {"bound": "hbm", "achieved": mach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": mach / HBM_PEAK_GBS, "kernel": kname(mz_tune, "OP_MZ64"),
                         "traffic": read_traffic(kname(mz_tune, "OP_MZ64"))}}
    del out
    torch.cuda.empty_cache()
    if not args.no_extra:
        note("FP32, LCG, sequential and c4 rows")
        line["f32"] = f32_row(ctx, Z, torch, args.steps, args.warmup)
        line["c3_lcg"] = c3_lcg(ctx, Z, torch, args.steps, args.warmup)
        line["sequential"] = sequential_row(ctx, Z, torch, args.steps, args.warmup)
        line["c4_batch"] = c4_batch(ctx, Z, torch, 3)
        line["ea_step"] = ea_row(ctx, Z, torch, args.steps, args.warmup)
    if args.serve_seconds > 0:
        from paper_2405_19493_amd import serve_bench
        note(f"serving, {args.serve_seconds:.0f} s per mode")
        line["serving"] = serve_bench.run(ctx, duration_s=args.serve_seconds)
    if not args.no_cpu_baseline:
        note("CPU baseline (the oracle)")
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
