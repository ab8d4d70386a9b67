"""The modified ziggurat (McFarland's method, ZG_MCFARLAND) on the GPU against
the oracle, through the C ABI.

Covered:
- fills of both word kinds at sizes that span many workgroup tiles, with
  ragged tails, unaligned starts and offset first indices;
- multi-stream jobs, including streams shorter than a step;
- both kernels (block-pooled and wave-specialised) in several launch shapes,
  which must give the same bits;
- the draw budget, and a forced tiny queue (the overflow path);
- the benchmark's workload (2^28 variates, 65536 streams of 4096, SplitMix64
  seed 7) compared in full with the oracle, in the launch shape the benchmark
  times, plus its statistics.

The rules are those of tests/parity.py. Layer variates must be bit-exact.
Overhang values are exact arithmetic on both sides, so they agree bit for bit
whenever the decision does. Tail values go through log, within 2 ulp.
Decision disagreements (exp or log on either side of a threshold) are at
most 1e-9 per variate.
"""
import numpy as np
import pytest
import torch

from oracle import coracle as orc
from oracle import stats
from parity import compare

pytestmark = pytest.mark.gpu

N_STREAMS, N_PER = 65536, 4096
Z_MAX = 5.0


def dev_empty(n, dtype, offset=0):
    base = torch.empty(n + offset + 8, dtype=dtype, device="cuda")
    return base[offset:offset + n]


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


@pytest.mark.parametrize("n,kind,seed,s,first,offset", [
    (1, 1, 1, 0, 0, 0), (2, 1, 1, 0, 5, 1), (127, 1, 3, 9, 0, 0), (129, 2, 3, 9, 0, 1),
    (100001, 1, 7, 65535, 2**40 - 100001, 1), (300007, 2, 11, 1, 12345, 0),
    (262144, 2, 123456789, 0, 0, 0), (4099, 1, 5, 5, 3, 1), (1 << 20, 1, 42, 0, 0, 0)])
def test_fill_mz(ctx, zg, n, kind, seed, s, first, offset):
    out = dev_empty(n, torch.float64, offset)
    out.fill_(float("nan"))
    ctx.zg_fill(out, method=zg.ZG_MCFARLAND, kind=kind, seed=seed, stream=s, first_index=first)
    got = host(out)
    want, cls, errs = orc.fill_mz(kind, seed, s, first, n)
    assert errs == 0
    rep = compare(got, want, cls, ("mz", n, kind, seed, s, first, offset))
    assert rep["disagreements"] == 0
    assert ctx.zg_error_flags() == 0


@pytest.mark.parametrize("n_per,n_streams,kind,first,offset", [
    (4096, 64, 1, 0, 0), (1000, 37, 1, 5, 1), (37, 301, 1, 0, 0), (37, 250, 2, 0, 1),
    (5, 1000, 1, 0, 1), (4096, 8, 2, 0, 0)])
def test_fill_streams_mz(ctx, zg, n_per, n_streams, kind, first, offset):
    out = dev_empty(n_per * n_streams, torch.float64, offset)
    ctx.zg_fill_streams(out, n_per, n_streams, method=zg.ZG_MCFARLAND, kind=kind, seed=77,
                        stream0=3, first_index=first)
    got = host(out)
    want, cls, errs = orc.fill_streams_mz(kind, 77, 3, n_streams, first, n_per)
    assert errs == 0
    compare(got, want, cls, ("mz streams", n_per, n_streams, kind))


def test_mz_rejects_f32_and_batches(ctx, zg):
    with pytest.raises(zg.ZgError) as e:
        ctx.zg_fill(torch.empty(10, dtype=torch.float32, device="cuda"), method=zg.ZG_MCFARLAND)
    assert e.value.status == zg.ZG_EINVAL
    with pytest.raises(zg.ZgError) as e:
        ctx.zg_stream_open(seed=1, stream=0, method=zg.ZG_MCFARLAND)
    assert e.value.status == zg.ZG_EINVAL


@pytest.mark.parametrize("kind", [1, 2])
def test_mz_launch_shapes_same_bits(ctx, zg, kind):
    """Block-pooled (one workgroup per tile or persistent, small or large
    tiles, 1 to 8 steps per group) and wave-specialised (1 to 8 drain waves)
    launches of the modified ziggurat: the same bits, equal to the oracle."""
    n_per, ns = 777, 240   # streams 7..246: within the LCG's 256
    saved = ctx.zg_get_tune(zg.ZG_TUNE_FILL_MZ)
    try:
        ref = None
        for tile, waves, res, dw, gs in [(1024, 16, 2, 0, 4), (256, 4, 0, 0, 1), (512, 8, 1, 0, 8),
                                         (4096, 16, 0, 0, 2), (1024, 16, 2, 1, 4),
                                         (1024, 16, 2, 4, 2), (1024, 16, 2, 8, 8),
                                         (1024, 8, 3, 2, 2), (512, 4, 4, 3, 1)]:
            ctx.zg_set_tune(zg.ZG_TUNE_FILL_MZ, tile, waves, res, 0, dw, gs)
            out = dev_empty(n_per * ns, torch.float64, 1)
            ctx.zg_fill_streams(out, n_per, ns, method=zg.ZG_MCFARLAND, kind=kind, seed=2,
                                stream0=7, first_index=33)
            got = host(out)
            if ref is None:
                ref = got.tobytes()
                want, cls, _ = orc.fill_streams_mz(kind, 2, 7, ns, 33, n_per)
                compare(got, want, cls, ("mz shapes", kind))
            assert got.tobytes() == ref, (tile, waves, res, dw, gs)
    finally:
        ctx.zg_set_tune(zg.ZG_TUNE_FILL_MZ, *saved)


@pytest.mark.parametrize("qcap", [1, 16])
def test_mz_queue_overflow(ctx, zg, qcap):
    saved = ctx.zg_get_tune(zg.ZG_TUNE_FILL_MZ)
    try:
        outs = []
        for cap in (0, qcap):
            ctx.zg_set_tune(zg.ZG_TUNE_FILL_MZ, saved[0], saved[1], saved[2], cap)
            out = dev_empty(100003, torch.float64, 1)
            ctx.zg_fill(out, method=zg.ZG_MCFARLAND, kind=1, seed=5, stream=2, first_index=7)
            outs.append(host(out).copy())
        assert outs[0].tobytes() == outs[1].tobytes()
        want, cls, _ = orc.fill_mz(1, 5, 2, 7, 100003)
        compare(outs[1], want, cls, ("mz overflow", qcap))
    finally:
        ctx.zg_set_tune(zg.ZG_TUNE_FILL_MZ, *saved)


@pytest.mark.parametrize("dmax", [1, 2, 3, 4, 5])
def test_mz_budget(ctx, zg, dmax):
    n = 200000
    try:
        ctx.zg_error_flags(clear=True)
        ctx.zg_set_test_knob(zg.ZG_KNOB_DMAX, dmax)
        out = torch.empty(n, dtype=torch.float64, device="cuda")
        ctx.zg_fill(out, method=zg.ZG_MCFARLAND, kind=1, seed=42, stream=0)
        got = host(out)
        want, cls, errs = orc.fill_mz(1, 42, 0, 0, n, dmax=dmax)
        compare(got, want, cls, ("mz budget", dmax))
        flags = ctx.zg_error_flags(clear=True)
        assert bool(flags & zg.ZG_FLAG_BUDGET) == (errs > 0)
        assert errs > 0
    finally:
        ctx.zg_set_test_knob(zg.ZG_KNOB_DMAX, 256)
    assert ctx.zg_error_flags() == 0


def test_mz_full_parity_2p28(ctx, zg):
    """Every one of the 2^28 variates of the benchmark's modified-ziggurat row
    (65536 streams x 4096, SplitMix64 seed 7) against the oracle, in the
    library's default launch shape for it (the one the benchmark times), and
    their statistics: moments, KS on a 1e7 subsample, the tail frequency
    erfc(X_0/sqrt 2)."""
    n = N_STREAMS * N_PER
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.zg_fill_streams(out, N_PER, N_STREAMS, method=zg.ZG_MCFARLAND, kind=zg.ZG_SPLITMIX64,
                        seed=7)
    got = out.cpu().numpy()
    del out
    torch.cuda.empty_cache()
    want, cls, errs = orc.fill_streams_mz(orc.SM64, 7, 0, N_STREAMS, 0, N_PER, nthreads=16)
    assert errs == 0
    rep = compare(got, want, cls, "mz 2^28 full")
    assert rep["disagreements"] == 0
    del want, cls
    assert np.all(np.isfinite(got))
    z = stats.moment_zscores(got)
    assert all(abs(v) < Z_MAX for v in z.values()), z
    sub = got[np.random.Generator(np.random.PCG64(9)).integers(0, n, 10**7)]
    assert stats.ks_statistic(sub) < stats.ks_critical(sub.size, 0.001)
    tz, k, e = stats.tail_count_z(got, orc.mz_table().x0)
    assert abs(tz) < Z_MAX, (k, e)
    assert ctx.zg_error_flags() == 0


def test_mz_lcg_2p24(ctx, zg):
    """2^24 variates of one java.util.Random stream (nextLong words): the
    low-order bits the method relies on are the LCG's weak ones, but the
    values must still be the oracle's, bit for bit on the layers."""
    n = 1 << 24
    out = torch.empty(n, dtype=torch.float64, device="cuda")
    ctx.zg_fill(out, method=zg.ZG_MCFARLAND, kind=zg.ZG_JAVA_LCG48, seed=123456789)
    got = host(out)
    want, cls, errs = orc.fill_mz(orc.LCG48, 123456789, 0, 0, n, nthreads=16)
    assert errs == 0
    compare(got, want, cls, "mz lcg 2^24")
