"""Benchmark: FP64 Gaussian variates/s against the HBM-write roofline.

Workload (the configuration the metric is quoted on): the original 128-layer
ziggurat and the Marsaglia polar method side by side, 2^28 FP64 standard
normals each, SplitMix64 uniforms with seed 7 and 65536 independent stream ids
of 4096 variates, written to one contiguous float64 buffer (2 GiB).  A step is
one ziggurat fill of the whole buffer; the polar fill is timed the same way and
reported beside it.  Inputs are synthetic (seeds only).

Prints one JSON line.  --gpus N > 1 exits: this build runs on one GPU.
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
    p.add_argument("--only", choices=["zig", "polar", "all"], default="all",
                   help="restrict the timed kernels (for profiling runs)")
    p.add_argument("--serve-seconds", type=float, default=0.0,
                   help="also run the serving loop for this long and report p50/p99")
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


def cpu_baseline(seconds):
    """The oracle (oracle/zg_oracle.c) on a bounded sample of the same workload:
    whole streams of 4096 variates, seed 7, SplitMix64, one stream per call, the
    calls spread over a thread pool of the host's cores (capped at 16, the CPU
    share of one GPU), until about `seconds` of wall time have passed."""
    from concurrent.futures import ThreadPoolExecutor
    from oracle import coracle as orc
    orc.build(force=False)
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    cores = max(1, min(cores, 16))
    per_batch = 64 * cores

    def one(s):
        orc.fill_f64(orc.SM64, SEED, s, 0, N_PER, nthreads=1)

    s = 0
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=cores) as pool:
        while time.perf_counter() - t0 < seconds and s < N_STREAMS:
            list(pool.map(one, range(s, min(s + per_batch, N_STREAMS))))
            s = min(s + per_batch, N_STREAMS)
    dt = time.perf_counter() - t0
    done = s * N_PER
    return {"value": done / dt, "unit": "variates/s", "cores": cores, "kind": "oracle",
            "sample": f"streams 0..{s - 1} of the 65536 x 4096 FP64 ziggurat variates "
                      f"(SplitMix64 seed 7): {done} variates in {dt:.1f} s"}


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
              "and the path shards by index range with no communication (see the design notes)",
              file=sys.stderr)
        sys.exit(2)
    import torch
    if args.copy_calibration:
        copy_calibration(torch)
        return
    import paper_2405_19493_amd as Z

    n = N_STREAMS * N_PER
    ctx = Z.Context(0)
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    out.zero_()

    def zig():
        ctx.zg_fill_streams(out, N_PER, N_STREAMS, method=Z.ZG_ZIGGURAT, kind=Z.ZG_SPLITMIX64,
                            seed=SEED, stream0=0, first_index=0)

    def polar():
        ctx.zg_fill_streams(out, N_PER, N_STREAMS, method=Z.ZG_POLAR, kind=Z.ZG_SPLITMIX64,
                            seed=SEED, stream0=0, first_index=0)

    res = {}
    if args.only in ("zig", "all"):
        res["zig"] = time_kernel(zig, args.steps, args.warmup, torch)
    if args.only in ("polar", "all"):
        res["polar"] = time_kernel(polar, args.steps, args.warmup, torch)
    flags = ctx.zg_error_flags()
    if flags:
        raise SystemExit(f"device error flags {flags}")

    main_key = "zig" if "zig" in res else "polar"
    ms, all_ms, wall = res[main_key]
    wall_ms = wall * 1e3 / args.steps
    bytes_per = 8.0 * n
    achieved = bytes_per / (ms * 1e-3) / 1e9
    kernel = "k_zig<OP_ZIG64>" if main_key == "zig" else "k_fill<OP_POLAR>"
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
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "ziggurat fill, 2^28 FP64 N(0,1), SplitMix64 seed 7, "
                               "65536 streams x 4096, contiguous float64 (2 GiB); "
                               "polar fill of the same shape timed beside it",
                   "method": "ziggurat" if main_key == "zig" else "polar",
                   "variates_per_step": n, "streams": N_STREAMS, "per_stream": N_PER},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": kernel, "algorithmic_bytes_per_launch": bytes_per},
    }
    if "polar" in res and main_key == "zig":
        pms = res["polar"][0]
        pwall = res["polar"][2] * 1e3 / args.steps
        pach = bytes_per / (pms * 1e-3) / 1e9
        line["polar"] = {"value": n / (pwall * 1e-3), "unit": "variates/s", "ms_per_step": pwall,
                         "kernel_ms": pms,
                         "roofline": {"bound": "hbm", "achieved": pach, "peak": HBM_PEAK_GBS,
                                      "unit": "GB/s", "frac": pach / HBM_PEAK_GBS}}
    if args.serve_seconds > 0:
        from paper_2405_19493_amd import serve_bench
        line["serving"] = serve_bench.run(ctx, duration_s=args.serve_seconds)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    ctx.close()
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
