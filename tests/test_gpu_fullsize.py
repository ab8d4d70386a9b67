"""Full-size GPU checks, in the launch configurations bench.py times:

- every variate of the benchmark's rows against the oracle: the c2 FP64
  ziggurat (in the launch shape the benchmark's autotuner picks), the c2 polar
  and FP32 fills, and the c3 LCG stream (2^28 each);
- sampled parity at 2^28 variates (c2 ziggurat and polar: 65536 streams x
  4096, SplitMix64 seed 7; c3: one LCG48 stream, seed 123456789): 2^16 random
  positions compared element by element with the oracle, under the rules of
  tests/parity.py;
- statistics of GPU output at 1e8: moments, Kolmogorov-Smirnov against Phi
  and the tail frequency erfc(r/sqrt 2), the same pins the oracle passes.
"""
import numpy as np
import pytest
import torch

from oracle import coracle as orc
from oracle import stats
from parity import compare, compare_mutated, mutation_z

pytestmark = pytest.mark.gpu

N_STREAMS, N_PER = 65536, 4096
SAMPLES = 1 << 16
Z_MAX = 5.0


def _sample_positions(n, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.unique(rng.integers(0, n, SAMPLES))


def _oracle_at(kind, seed, positions, n_per, method=0):
    """Oracle values and classes of single elements (stream = e // n_per)."""
    vals = np.empty(positions.size)
    cls = np.empty(positions.size, dtype=np.uint8)
    for k, e in enumerate(positions):
        s, v = divmod(int(e), n_per)
        if method == 1:
            p = v & ~1   # polar works on pairs: evaluate the pair, take the element
            x, c, _ = orc.fill_polar(kind, seed, s, p, 2, nthreads=1)
            vals[k], cls[k] = x[v - p], c[v - p]
        else:
            x, c, _ = orc.fill_f64(kind, seed, s, v, 1, nthreads=1)
            vals[k], cls[k] = x[0], c[0]
    return vals, cls


@pytest.mark.parametrize("shape", ["default", "pooled"])
def test_c2_full_parity_ziggurat(ctx, zg, shape):
    """Every one of the 2^28 FP64 ziggurat variates of the benchmark's workload
    against the oracle (its multi-stream routine on the host's cores), in the
    library's default launch shape, the one the benchmark times (the
    wave-specialised kernel), and in the block-pooled kernel at workgroup
    tiles of 1024 x 16 waves, at most 2 persistent workgroups per CU."""
    n = N_STREAMS * N_PER
    before = ctx.zg_get_tune(zg.ZG_TUNE_FILL_F64)
    if shape == "pooled":
        ctx.zg_set_tune(zg.ZG_TUNE_FILL_F64, 1024, 16, 2, 0, 0, 4)
    try:
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        ctx.zg_fill_streams(out, N_PER, N_STREAMS, kind=zg.ZG_SPLITMIX64, seed=7)
        got = out.cpu().numpy()
        del out
        torch.cuda.empty_cache()
    finally:
        ctx.zg_set_tune(zg.ZG_TUNE_FILL_F64, *before)
    want, cls, errs = orc.fill_streams_f64(orc.SM64, 7, 0, N_STREAMS, 0, N_PER, nthreads=16)
    assert errs == 0
    compare(got, want, cls, "c2 full")
    assert ctx.zg_error_flags() == 0


def _full_stream_fill(ctx, zg, dtype, method):
    tdt = torch.float32 if dtype == zg.ZG_F32 else torch.float64
    out = torch.empty(N_STREAMS * N_PER, dtype=tdt, device="cuda")
    ctx.zg_fill_streams(out, N_PER, N_STREAMS, method=method, kind=zg.ZG_SPLITMIX64, seed=7)
    got = out.cpu().numpy()
    del out
    torch.cuda.empty_cache()
    return got


def test_c2_full_parity_polar(ctx, zg):
    """Every polar variate of the benchmark's c2 workload (2^28), within 4 ulp."""
    got = _full_stream_fill(ctx, zg, zg.ZG_F64, zg.ZG_POLAR)
    want, cls, errs = orc.fill_streams_polar(orc.SM64, 7, 0, N_STREAMS, 0, N_PER, nthreads=16)
    assert errs == 0
    compare(got, want, cls, "c2 polar full", polar=True)
    assert ctx.zg_error_flags() == 0


def test_c2_full_parity_f32(ctx, zg):
    """Every FP32 variate of the benchmark's FP32 row (the c2 layout, 2^28)."""
    got = _full_stream_fill(ctx, zg, zg.ZG_F32, zg.ZG_ZIGGURAT)
    want, _, cls, errs = orc.fill_streams_f32(orc.SM64, 7, 0, N_STREAMS, 0, N_PER, nthreads=16)
    assert errs == 0
    compare(got, want, cls, "c2 f32 full")
    assert ctx.zg_error_flags() == 0


def test_c3_full_parity_lcg(ctx, zg):
    """Every variate of the c3 row: 2^28 FP64 variates of one LCG48 stream."""
    n = 1 << 28
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.zg_fill(out, kind=zg.ZG_JAVA_LCG48, seed=123456789, stream=0)
    got = out.cpu().numpy()
    del out
    torch.cuda.empty_cache()
    want, cls, errs = orc.fill_f64(orc.LCG48, 123456789, 0, 0, n, nthreads=16)
    assert errs == 0
    compare(got, want, cls, "c3 full")
    assert ctx.zg_error_flags() == 0


@pytest.mark.parametrize("method", [0, 1])
def test_c2_sampled_parity(ctx, zg, method):
    n = N_STREAMS * N_PER
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.zg_fill_streams(out, N_PER, N_STREAMS, method=method, kind=zg.ZG_SPLITMIX64, seed=7)
    pos = _sample_positions(n, 31 + method)
    got = out[torch.from_numpy(pos).cuda()].cpu().numpy()
    # the stream-boundary neighbourhood too: first and last element of some streams
    edge = np.array([s * N_PER + o for s in (0, 1, 4095, 65535) for o in (0, 1, N_PER - 2, N_PER - 1)])
    got_e = out[torch.from_numpy(edge).cuda()].cpu().numpy()
    del out
    torch.cuda.empty_cache()
    want, cls = _oracle_at(orc.SM64, 7, pos, N_PER, method)
    compare(got, want, cls, ("c2", method), polar=method == 1)
    want_e, cls_e = _oracle_at(orc.SM64, 7, edge, N_PER, method)
    compare(got_e, want_e, cls_e, ("c2 edges", method), polar=method == 1)
    assert ctx.zg_error_flags() == 0


def test_c3_lcg_sampled_parity(ctx, zg):
    n = 1 << 28
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.zg_fill(out, kind=zg.ZG_JAVA_LCG48, seed=123456789, stream=0)
    pos = _sample_positions(n, 33)
    got = out[torch.from_numpy(pos).cuda()].cpu().numpy()
    del out
    torch.cuda.empty_cache()
    want, cls = _oracle_at(orc.LCG48, 123456789, pos, n)
    compare(got, want, cls, "c3")


def _check_normal(x, r, label):
    z = stats.moment_zscores(x)
    assert all(abs(v) < Z_MAX for v in z.values()), (label, z)
    D = stats.ks_statistic(x)
    assert D < stats.ks_critical(x.size, 0.001), (label, D)
    tz, k, e = stats.tail_count_z(x, r)
    assert abs(tz) < Z_MAX, (label, k, e)


@pytest.mark.parametrize("dtype,kind", [(torch.float64, 1), (torch.float32, 1), (torch.float64, 2)])
def test_statistics_1e8(ctx, zg, dtype, kind):
    n = 10 ** 8
    out = torch.empty(n, dtype=dtype, device="cuda")
    ctx.zg_fill(out, kind=kind, seed=42, stream=3, first_index=1000)
    x = out.cpu().numpy().astype(np.float64)
    del out
    torch.cuda.empty_cache()
    assert np.all(np.isfinite(x))
    _check_normal(x, orc.table_dict()["r"], (str(dtype), kind))


def test_c4_full_parity_batch(ctx, zg):
    """The benchmark's c4 batch (10^4 uneven requests, 7.6e8 variates, plus the
    4096 x 1024-gene mutation) in one zg_batch launch: every variate of every
    request, and every mutated gene, against the oracle."""
    import bench
    sizes, is64, genes = bench.c4_recipe()
    m = sizes.size
    outs = [torch.empty(int(n), dtype=torch.float64 if f else torch.float32, device="cuda")
            for n, f in zip(sizes, is64)]
    # initial genes from the oracle's uniform words (the product's words equal them bit
    # for bit, test_uniform_words_bit_exact)
    w = orc.words(orc.SM64, 1, 65535, 0, 0, genes)
    x0 = -5.0 + 10.0 * ((w >> np.uint64(11)).astype(np.float64) * 2.0 ** -53)
    x = torch.from_numpy(x0.copy()).cuda()
    reqs = [{"out": outs[k], "n": int(sizes[k]), "seed": 1000 + k, "stream": k,
             "dtype": zg.ZG_F64 if is64[k] else zg.ZG_F32} for k in range(m)]
    reqs.append({"out": x, "n": genes, "seed": 999, "stream": 0, "op": zg.ZG_OP_MUTATE,
                 "sigma": 0.1, "dtype": zg.ZG_F64})
    ctx.zg_batch(ctx.zg_batch_prepare(reqs))
    torch.cuda.synchronize()
    assert ctx.zg_error_flags() == 0
    g64, w64, c64, g32, w32, c32 = [], [], [], [], [], []
    for k in range(m):
        got = outs[k].cpu().numpy()
        if is64[k]:
            want, cls, errs = orc.fill_f64(orc.SM64, 1000 + k, k, 0, int(sizes[k]),
                                           nthreads=16 if sizes[k] > 65536 else 1)
            g64.append(got); w64.append(want); c64.append(cls)
        else:
            want, _, cls, errs = orc.fill_f32(orc.SM64, 1000 + k, k, 0, int(sizes[k]),
                                              nthreads=16 if sizes[k] > 65536 else 1)
            g32.append(got); w32.append(want); c32.append(cls)
        assert errs == 0
    del outs
    compare(np.concatenate(g64), np.concatenate(w64), np.concatenate(c64), "c4 f64")
    compare(np.concatenate(g32), np.concatenate(w32), np.concatenate(c32), "c4 f32")
    xm = x.cpu().numpy()
    want, cls, errs = orc.mutate(x0, orc.SM64, 999, 0, 0, 0.1)
    assert errs == 0
    compare_mutated(xm, want, cls, mutation_z(orc, orc.SM64, 999, 0, 0), 0.1, "c4 mutation")
