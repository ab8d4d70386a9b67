"""HIP path against the oracle, element by element, through the C ABI.

Sizes span many tiles and ragged tails; every case uses seeded synthetic
inputs.  Rules: tests/parity.py (fast path bit-exact, slow path <= 2 ulp,
decision disagreements <= 1e-9 per variate)."""
import numpy as np
import pytest
import torch

from oracle import coracle as orc
from parity import compare, compare_mutated, mutation_z

pytestmark = pytest.mark.gpu


def dev_empty(n, dtype, offset=0):
    """A device buffer of n elements starting `offset` elements into an
    allocation (to exercise unaligned heads)."""
    base = torch.empty(n + offset + 8, dtype=dtype, device="cuda")
    return base[offset:offset + n]


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def test_table_bits_match_oracle(ctx):
    t = ctx.zg_table()
    o = orc.table_dict()
    assert t.r == o["r"] and t.v == o["v"]
    for k in ("W", "y", "dy", "w53", "w24d", "k53", "k24"):
        assert list(getattr(t, k)) == o[k], k
    assert all(np.float32(t.w24[i]) == np.float32(o["w24f"][i] * 2.0 ** -24) for i in range(128))


@pytest.mark.parametrize("kind,seed,s,d,first,n", [
    (1, 0, 0, 0, 0, 1000), (1, 42, 7, 3, 123456789, 100003), (1, 2**64 - 1, 65535, 255, 2**40 - 5000, 5000),
    (2, 123456789, 0, 0, 0, 100003), (2, 5, 255, 255, 2147483547 - 777, 777), (2, 99, 3, 1, 1 << 30, 65537)])
def test_uniform_words_bit_exact(ctx, zg, kind, seed, s, d, first, n):
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    ctx.zg_uniform_words(out, kind=kind, seed=seed, stream=s, draw=d, first_index=first)
    got = host(out).view(np.uint64)
    want = orc.words(kind, seed, s, d, first, n)
    assert np.array_equal(got, want)


def test_lcg_stream_equals_sequential_random_2p28(ctx, zg):
    """Stream 0, draw 0 of the LCG kind is Random(123456789).nextDouble() in
    order, 2^28 doubles (2^29 LCG steps), against the sequential C generator."""
    n = 1 << 28
    out = torch.empty(n, dtype=torch.int64, device="cuda")
    ctx.zg_uniform_words(out, kind=zg.ZG_JAVA_LCG48, seed=123456789)
    got = host(out).view(np.uint64)
    del out
    seq = orc.lcg_seq_doubles(123456789, n)
    assert np.array_equal(got >> np.uint64(11), seq)
    assert np.all((got & np.uint64(0x7FF)) == 0)


def _fill_case(ctx, zg, n, dtype, method, kind, seed, s, first, offset):
    tdt = torch.float64 if dtype == zg.ZG_F64 else torch.float32
    out = dev_empty(n, tdt, offset)
    ctx.zg_fill(out, method=method, kind=kind, seed=seed, stream=s, first_index=first)
    got = host(out)
    if method == zg.ZG_POLAR:
        want, cls, _ = orc.fill_polar(kind, seed, s, first, n)
    elif dtype == zg.ZG_F64:
        want, cls, _ = orc.fill_f64(kind, seed, s, first, n)
    else:
        want, _, cls, _ = orc.fill_f32(kind, seed, s, first, n)
    return compare(got, want, cls, (n, dtype, method, kind, seed, s, first, offset),
                   polar=method == zg.ZG_POLAR)


def test_c1_config_full_parity(ctx, zg):
    """1e6 FP64 ziggurat variates, SplitMix64 seed 42 stream 0."""
    rep = _fill_case(ctx, zg, 10**6, zg.ZG_F64, zg.ZG_ZIGGURAT, zg.ZG_SPLITMIX64, 42, 0, 0, 0)
    assert rep["disagreements"] == 0


@pytest.mark.parametrize("n,kind,seed,s,first,offset", [
    (1, 1, 1, 0, 0, 0), (2, 1, 1, 0, 5, 1), (127, 1, 3, 9, 0, 0), (129, 2, 3, 9, 0, 1),
    (100001, 1, 7, 65535, 2**40 - 100001, 1), (300007, 2, 11, 1, 12345, 0),
    (262144, 2, 123456789, 0, 0, 0), (4099, 1, 5, 5, 3, 1)])
def test_fill_f64_ziggurat(ctx, zg, n, kind, seed, s, first, offset):
    _fill_case(ctx, zg, n, zg.ZG_F64, zg.ZG_ZIGGURAT, kind, seed, s, first, offset)


@pytest.mark.parametrize("n,kind,seed,s,first,offset", [
    (1, 1, 1, 0, 0, 0), (3, 1, 1, 0, 1, 1), (255, 1, 2, 4, 0, 2), (257, 2, 2, 4, 7, 3),
    (200003, 1, 9, 100, 1, 1), (200003, 1, 9, 100, 2, 0), (65536, 2, 31, 2, 99, 2)])
def test_fill_f32_ziggurat(ctx, zg, n, kind, seed, s, first, offset):
    _fill_case(ctx, zg, n, zg.ZG_F32, zg.ZG_ZIGGURAT, kind, seed, s, first, offset)


@pytest.mark.parametrize("n,kind,seed,s,first,offset", [
    (1, 1, 1, 0, 0, 0), (2, 1, 1, 0, 1, 1), (129, 1, 4, 2, 0, 1), (100001, 1, 7, 12, 3, 0),
    (100000, 2, 11, 2, 0, 1), (65536, 1, 7, 0, 0, 0)])
def test_fill_polar(ctx, zg, n, kind, seed, s, first, offset):
    _fill_case(ctx, zg, n, zg.ZG_F64, zg.ZG_POLAR, kind, seed, s, first, offset)


@pytest.mark.parametrize("n_per,n_streams,method,dtype,kind,first,offset", [
    (4096, 64, 0, 0, 1, 0, 0), (1000, 37, 0, 0, 1, 5, 1), (37, 301, 0, 0, 1, 0, 0), (37, 250, 0, 0, 2, 0, 1),
    (4096, 16, 1, 0, 1, 0, 0), (1001, 9, 1, 0, 2, 1, 1), (333, 50, 0, 1, 1, 3, 2),
    (4096, 8, 0, 1, 2, 0, 0), (5, 1000, 0, 1, 1, 0, 1)])
def test_fill_streams(ctx, zg, n_per, n_streams, method, dtype, kind, first, offset):
    tdt = torch.float64 if dtype == 0 else torch.float32
    out = dev_empty(n_per * n_streams, tdt, offset)
    s0 = 3
    ctx.zg_fill_streams(out, n_per, n_streams, method=method, kind=kind, seed=77, stream0=s0,
                        first_index=first)
    got = host(out).reshape(n_streams, n_per)
    for k in range(n_streams):
        if method == 1:
            want, cls, _ = orc.fill_polar(kind, 77, s0 + k, first, n_per)
        elif dtype == 0:
            want, cls, _ = orc.fill_f64(kind, 77, s0 + k, first, n_per)
        else:
            want, _, cls, _ = orc.fill_f32(kind, 77, s0 + k, first, n_per)
        compare(got[k], want, cls, ("streams", k), polar=method == 1)


@pytest.mark.parametrize("n,kind,offset", [(1, 1, 0), (4194304, 1, 0), (100003, 2, 1)])
def test_mutate(ctx, zg, n, kind, offset):
    rng = np.random.Generator(np.random.PCG64(4))
    x0 = rng.uniform(-5.0, 5.0, n)
    x = dev_empty(n, torch.float64, offset)
    x.copy_(torch.from_numpy(x0))
    ctx.zg_mutate(x, 0.1, kind=kind, seed=17, stream=2, first_index=10)
    got = host(x)
    want, cls, _ = orc.mutate(x0, kind, 17, 2, 10, 0.1)
    compare_mutated(got, want, cls, mutation_z(orc, kind, 17, 2, 10), 0.1, ("mutate", n))


def test_decide_words_boundaries(ctx, zg):
    t = orc.table_dict()
    J = (1 << 53) - 1
    words = []
    for i in range(128):
        k = t["k53"][i]
        for neg in (0, 1):
            for j in sorted({max(k - 1, 0), k, min(k + 1, J), 0, J}):
                words.append((i << 57) | (neg << 56) | (j << 3) | 5)
    rng = np.random.Generator(np.random.PCG64(8))
    words += [int(w) for w in rng.integers(0, 2**63, 4000, dtype=np.uint64) * np.uint64(2) + rng.integers(0, 2, 4000, dtype=np.uint64)]
    w = torch.tensor(np.array(words, dtype=np.uint64).view(np.int64), device="cuda")
    cls = torch.empty(len(words), dtype=torch.uint8, device="cuda")
    x = torch.empty(len(words), dtype=torch.float64, device="cuda")
    ctx.zg_decide_words(w, cls, x)
    gc, gx = host(cls), host(x)
    for k, W in enumerate(words):
        c, xv = orc.decide_word(W)
        assert gc[k] == c and np.float64(xv).tobytes() == gx[k].tobytes(), (k, hex(W))


@pytest.mark.parametrize("dmax", [1, 2, 3])
def test_budget_exhaustion(ctx, zg, dmax):
    n = 50000
    try:
        ctx.zg_error_flags(clear=True)
        ctx.zg_set_test_knob(zg.ZG_KNOB_DMAX, dmax)
        for method, dtype in ((0, 0), (0, 1), (1, 0)):
            tdt = torch.float64 if dtype == 0 else torch.float32
            out = torch.empty(n, dtype=tdt, device="cuda")
            ctx.zg_fill(out, method=method, kind=1, seed=42, stream=0)
            got = host(out)
            if method == 1:
                want, cls, errs = orc.fill_polar(1, 42, 0, 0, n, dmax=dmax)
            elif dtype == 0:
                want, cls, errs = orc.fill_f64(1, 42, 0, 0, n, dmax=dmax)
            else:
                want, _, cls, errs = orc.fill_f32(1, 42, 0, 0, n, dmax=dmax)
            compare(got, want, cls, ("budget", dmax, method, dtype), polar=method == 1)
            flags = ctx.zg_error_flags(clear=True)
            assert bool(flags & zg.ZG_FLAG_BUDGET) == (errs > 0)
            assert errs > 0
    finally:
        ctx.zg_set_test_knob(zg.ZG_KNOB_DMAX, 256)
    ctx.zg_fill(torch.empty(1000, dtype=torch.float64, device="cuda"), seed=1)
    assert ctx.zg_error_flags() == 0


def test_errors_are_reported(ctx, zg):
    out = torch.empty(10, dtype=torch.float64, device="cuda")
    with pytest.raises(zg.ZgError) as e:
        ctx.zg_fill(out, kind=3)
    assert e.value.status == zg.ZG_EINVAL
    with pytest.raises(zg.ZgError) as e:
        ctx.zg_fill(out, first_index=2**40 - 5)
    assert e.value.status == zg.ZG_ERANGE
    with pytest.raises(zg.ZgError) as e:
        ctx.zg_fill(out, kind=2, stream=256)
    assert e.value.status == zg.ZG_EINVAL
    with pytest.raises(zg.ZgError) as e:
        ctx.zg_fill(torch.empty(10, dtype=torch.float32, device="cuda"), method=zg.ZG_POLAR)
    assert e.value.status == zg.ZG_EINVAL
    with pytest.raises(zg.ZgError) as e:
        ctx.zg_fill(out, kind=2, first_index=zg.ZG_LCG_WINDOW - 9)
    assert e.value.status == zg.ZG_ERANGE
    ctx.zg_fill(out[:0])   # n == 0 is a no-op


@pytest.mark.parametrize("qcap", [1, 16, 200])
def test_queue_overflow_path(ctx, zg, qcap):
    """A workgroup queue too small for its slow elements (the same cap
    applies to the retry queue): elements that find a queue full are resolved
    by their own lane.  Output must not change (checked against the default
    capacity bit for bit, and against the oracle)."""
    cases = [(zg.ZG_TUNE_FILL_F64, torch.float64, 100003, 1), (zg.ZG_TUNE_FILL_F32, torch.float32, 100003, 3),
             (zg.ZG_TUNE_FILL_F64, torch.float64, 37 * 1000, 0)]
    saved = {c: ctx.zg_get_tune(c) for c in (zg.ZG_TUNE_FILL_F64, zg.ZG_TUNE_FILL_F32, zg.ZG_TUNE_MUTATE)}
    try:
        for cls_t, tdt, n, offset in cases:
            multi = n == 37 * 1000
            outs = []
            for cap in (0, qcap):
                tile, waves, bpc = saved[cls_t][:3]
                ctx.zg_set_tune(cls_t, tile, waves, bpc, cap)
                out = dev_empty(n, tdt, offset)
                out.fill_(float("nan"))
                if multi:
                    ctx.zg_fill_streams(out, 1000, 37, kind=1, seed=5, stream0=2, first_index=7)
                else:
                    ctx.zg_fill(out, kind=1, seed=5, stream=2, first_index=7)
                outs.append(host(out).copy())
            assert outs[0].tobytes() == outs[1].tobytes(), (cls_t, n, qcap)
            if multi:
                for k in range(37):
                    want, cls, _ = orc.fill_f64(1, 5, 2 + k, 7, 1000)
                    compare(outs[1][k * 1000:(k + 1) * 1000], want, cls, ("overflow streams", k))
            elif tdt == torch.float64:
                want, cls, _ = orc.fill_f64(1, 5, 2, 7, n)
                compare(outs[1], want, cls, ("overflow f64", qcap))
            else:
                want, _, cls, _ = orc.fill_f32(1, 5, 2, 7, n)
                compare(outs[1], want, cls, ("overflow f32", qcap))
        # mutation
        rng = np.random.Generator(np.random.PCG64(6))
        x0 = rng.uniform(-3.0, 3.0, 50001)
        tile, waves, bpc = saved[zg.ZG_TUNE_MUTATE][:3]
        ctx.zg_set_tune(zg.ZG_TUNE_MUTATE, tile, waves, bpc, qcap)
        x = dev_empty(x0.size, torch.float64, 1)
        x.copy_(torch.from_numpy(x0))
        ctx.zg_mutate(x, 0.25, kind=1, seed=3, stream=1, first_index=0)
        want, cls, _ = orc.mutate(x0, 1, 3, 1, 0, 0.25)
        compare_mutated(host(x), want, cls, mutation_z(orc, 1, 3, 1, 0), 0.25,
                        ("overflow mutate", qcap))
    finally:
        for c, t in saved.items():
            ctx.zg_set_tune(c, *t)


@pytest.mark.parametrize("cls_t,tdt,kind", [(0, torch.float64, 1), (1, torch.float32, 1),
                                            (3, torch.float64, 1), (0, torch.float64, 2)])
def test_launch_shape_never_changes_bits(ctx, zg, cls_t, tdt, kind):
    """One workgroup per tile or a persistent grid, small or large tiles,
    4 to 16 waves, 1 to 8 steps per group, the block-pooled or the
    wave-specialised kernel with 1 to 8 drain waves, workgroups of 2 to 16
    waves (down to one streaming wave) and up to 8 per compute unit: the same
    bits (every variate is keyed by its index).  Streams of 777 (SplitMix64)
    or 1001 (Java LCG, at most 256 streams) variates start inside steps, so
    steps taken singly, in pairs and across stream ends all occur."""
    n = 3 * 65536 + 4097
    n_per = 777 if kind == 1 else 1001
    saved = ctx.zg_get_tune(cls_t)
    rng = np.random.Generator(np.random.PCG64(12))
    x0 = torch.from_numpy(rng.uniform(-1, 1, n)).cuda() if cls_t == 3 else None
    try:
        ref = None
        for tile, waves, res, dw, gs in [(2048, 16, 2, 0, 4), (256, 4, 0, 0, 1), (512, 8, 1, 0, 8),
                                         (4096, 16, 0, 0, 2), (1024, 16, 4, 0, 4),
                                         (1024, 16, 2, 1, 4), (1024, 16, 2, 4, 2),
                                         (1024, 16, 2, 8, 8), (1024, 8, 3, 2, 2),
                                         (1024, 12, 2, 3, 4), (512, 4, 4, 3, 1),
                                         (1024, 2, 8, 1, 2)]:
            ctx.zg_set_tune(cls_t, tile, waves, res, 0, dw, gs)
            out = dev_empty(n, tdt, 1)
            if cls_t == 3:
                out.copy_(x0)
                ctx.zg_mutate(out, 0.5, kind=1, seed=2, stream=7, first_index=33)
            else:
                ctx.zg_fill_streams(out, n_per, n // n_per, kind=kind, seed=2, stream0=7,
                                    first_index=33)
                out = out[: (n // n_per) * n_per]
            got = host(out).tobytes()
            if ref is None:
                ref = got
            assert got == ref, (tile, waves, res, dw, gs)
    finally:
        ctx.zg_set_tune(cls_t, *saved)
