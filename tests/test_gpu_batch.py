"""Batch launch, device counters, checkpoint/resume and launch-shape
invariance, against the oracle and against the per-request calls."""
import numpy as np
import pytest
import torch

from oracle import coracle as orc
from parity import compare, compare_mutated, mutation_z

pytestmark = pytest.mark.gpu


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def _oracle_for(r):
    kind, seed, s, first, n = r["kind"], r["seed"], r["stream"], r["first_index"], r["n"]
    if r.get("op", 0) == 1:
        want, cls, _ = orc.mutate(r["x0"], kind, seed, s, first, r["sigma"])
        return want, cls, False
    if r.get("method", 0) == 1:
        want, cls, _ = orc.fill_polar(kind, seed, s, first, n)
        return want, cls, True
    if r["dtype"] == 0:
        want, cls, _ = orc.fill_f64(kind, seed, s, first, n)
    else:
        want, _, cls, _ = orc.fill_f32(kind, seed, s, first, n)
    return want, cls, False


def _uneven_requests(count, rng, max_log2=16, with_mutate=True):
    reqs = []
    for i in range(count):
        n = int(min(max(int(2 ** (max_log2 * rng.random())), 1), 2 ** max_log2))
        kind = 1 if rng.random() < 0.7 else 2
        dtype = 0 if rng.random() < 0.7 else 1
        method = 1 if (dtype == 0 and rng.random() < 0.15) else 0
        off = int(rng.integers(0, 4))
        tdt = torch.float64 if dtype == 0 else torch.float32
        buf = torch.empty(n + off, dtype=tdt, device="cuda")[off:]
        r = dict(out=buf, n=n, seed=int(rng.integers(0, 2**63)), stream=i % 256,
                 first_index=int(rng.integers(0, 2**20)), dtype=dtype, method=method, kind=kind, op=0)
        reqs.append(r)
    if with_mutate:
        n = 4096 * 64
        x0 = np.random.Generator(np.random.PCG64(3)).uniform(-5, 5, n)
        x = torch.from_numpy(x0).cuda()
        reqs.append(dict(out=x, n=n, seed=5, stream=9, first_index=0, dtype=0, method=0, kind=1,
                         op=1, sigma=0.1, x0=x0))
    return reqs


@pytest.mark.parametrize("count,seed", [(1, 1), (5, 4), (7, 5), (37, 2), (300, 3)])
def test_batch_matches_oracle(ctx, zg, count, seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    reqs = _uneven_requests(count, rng)
    ctx.zg_batch([{k: v for k, v in r.items() if k != "x0"} for r in reqs])
    torch.cuda.synchronize()
    for i, r in enumerate(reqs):
        want, cls, polar = _oracle_for(r)
        label = ("batch", i, r["n"], r["dtype"], r["method"], r["kind"])
        if r.get("op", 0) == 1:
            compare_mutated(host(r["out"]), want, cls,
                            mutation_z(orc, r["kind"], r["seed"], r["stream"], r["first_index"]),
                            r["sigma"], label)
        else:
            compare(host(r["out"]), want, cls, label, polar=polar)


def test_batch_equals_plain_calls_and_shapes(ctx, zg):
    """Same bits from one batch, from per-request calls, and under every
    launch shape (index keying leaves no room for a geometry dependence)."""
    rng = np.random.Generator(np.random.PCG64(11))
    reqs = _uneven_requests(120, rng, max_log2=15, with_mutate=False)
    ctx.zg_batch(reqs)
    ref = [host(r["out"]).copy() for r in reqs]
    saved = {c: ctx.zg_get_tune(c) for c in range(zg.ZG_TUNE_CLASSES)}
    try:
        # the batch classes block-pooled (0 drain waves) or wave-specialised
        shapes = [(1024, 4, 1, 1), (2048, 8, 2, 0), (4096, 16, 4, 2), (8192, 2, 1, 0),
                  (2048, 16, 1, 4), (1024, 8, 3, 7)]
        for tile, waves, bpc, bdrain in shapes:
            for c in (0, 2, 3):
                ctx.zg_set_tune(c, tile, waves, bpc)
            ctx.zg_set_tune(1, 2 * tile, waves, bpc)
            ctx.zg_set_tune(4, max(tile // 2, 256), min(waves, 8), bpc, 0, bdrain, 2)
            for r, want in zip(reqs, ref):
                r["out"].fill_(float("nan"))
            ctx.zg_batch(reqs)
            for r, want in zip(reqs, ref):
                assert host(r["out"]).tobytes() == want.tobytes(), (tile, waves, bpc, bdrain)
            for r, want in zip(reqs, ref):
                r["out"].fill_(float("nan"))
                o = r["out"]
                if r["dtype"] == 0 and r["method"] == 0:
                    ctx.zg_fill(o, kind=r["kind"], seed=r["seed"], stream=r["stream"], first_index=r["first_index"])
                elif r["method"] == 1:
                    ctx.zg_fill(o, method=1, kind=r["kind"], seed=r["seed"], stream=r["stream"], first_index=r["first_index"])
                else:
                    ctx.zg_fill(o, kind=r["kind"], seed=r["seed"], stream=r["stream"], first_index=r["first_index"])
                assert host(o).tobytes() == want.tobytes(), ("plain", tile, waves)
    finally:
        for c, t in saved.items():
            ctx.zg_set_tune(c, *t)


def test_counters_continue_and_checkpoint(ctx, zg):
    h = ctx.zg_stream_open(seed=123, stream=4, kind=zg.ZG_SPLITMIX64)
    try:
        a = torch.empty(1000, dtype=torch.float64, device="cuda")
        b = torch.empty(2501, dtype=torch.float64, device="cuda")
        ctx.zg_stream_fill(h, a)
        ctx.zg_stream_fill(h, b)
        assert ctx.zg_stream_get_counter(h) == 3501
        whole = torch.empty(3501, dtype=torch.float64, device="cuda")
        ctx.zg_fill(whole, seed=123, stream=4)
        w = host(whole)
        assert np.concatenate([host(a), host(b)]).tobytes() == w.tobytes()
        # checkpoint / resume: restore the counter and replay
        ctx.zg_stream_set_counter(h, 1000)
        ctx.zg_stream_fill(h, b)
        assert host(b).tobytes() == w[1000:].tobytes()
        # another mode would read the handle's words again: refused
        c = torch.empty(77, dtype=torch.float32, device="cuda")
        with pytest.raises(zg.ZgError) as e:
            ctx.zg_stream_fill(h, c)
        assert e.value.status == zg.ZG_EINVAL
        with pytest.raises(zg.ZgError) as e:
            ctx.zg_stream_fill(h, a, method=zg.ZG_POLAR)
        assert e.value.status == zg.ZG_EINVAL
        assert ctx.zg_stream_get_counter(h) == 3501
    finally:
        ctx.zg_stream_close(h)


def test_handle_modes(ctx, zg):
    """FP32 and polar handles: each continues its own index space, and a
    mutation goes through an FP64 ziggurat handle."""
    h32 = ctx.zg_stream_open(seed=5, stream=2, kind=zg.ZG_SPLITMIX64, dtype=zg.ZG_F32)
    hp = ctx.zg_stream_open(seed=6, stream=3, kind=zg.ZG_SPLITMIX64, method=zg.ZG_POLAR)
    with pytest.raises(zg.ZgError) as e:
        ctx.zg_stream_open(seed=6, stream=3, dtype=zg.ZG_F32, method=zg.ZG_POLAR)
    assert e.value.status == zg.ZG_EINVAL
    try:
        c = torch.empty(77, dtype=torch.float32, device="cuda")
        ctx.zg_stream_fill(h32, c)
        ctx.zg_stream_fill(h32, c)
        assert ctx.zg_stream_get_counter(h32) == 154
        want, _, cls, _ = orc.fill_f32(1, 5, 2, 77, 77)
        compare(host(c), want, cls, "handle f32")
        p = torch.empty(1001, dtype=torch.float64, device="cuda")
        ctx.zg_stream_fill(hp, p, method=zg.ZG_POLAR)
        ctx.zg_stream_fill(hp, p, method=zg.ZG_POLAR)
        whole = torch.empty(2002, dtype=torch.float64, device="cuda")
        ctx.zg_fill(whole, method=zg.ZG_POLAR, seed=6, stream=3)
        assert host(p).tobytes() == host(whole)[1001:].tobytes()
        with pytest.raises(zg.ZgError) as e:
            ctx.zg_batch([dict(out=p, n=1001, handle=h32, op=zg.ZG_OP_MUTATE, sigma=0.1)])
        assert e.value.status == zg.ZG_EINVAL
    finally:
        ctx.zg_stream_close(h32)
        ctx.zg_stream_close(hp)


def test_batch_counters_follow_submission_order(ctx, zg):
    hs = [ctx.zg_stream_open(seed=900 + k, stream=k, kind=1 + (k % 2)) for k in range(3)]
    try:
        sizes = [5, 300, 17, 1, 4096, 33, 250, 7]
        reqs = []
        for i, n in enumerate(sizes):
            out = torch.empty(n, dtype=torch.float64, device="cuda")
            reqs.append(dict(out=out, n=n, handle=hs[i % 3], dtype=0, method=0, op=0))
        first = ctx.zg_batch(reqs, want_first=True)
        expect = [0, 0, 0]
        for i, n in enumerate(sizes):
            assert first[i] == expect[i % 3]
            expect[i % 3] += n
        for k in range(3):
            assert ctx.zg_stream_get_counter(hs[k]) == expect[k]
        for i, r in enumerate(reqs):
            k = i % 3
            want, cls, _ = orc.fill_f64(1 + (k % 2), 900 + k, k, first[i], r["n"])
            compare(host(r["out"]), want, cls, ("ordered", i))
    finally:
        for h in hs:
            ctx.zg_stream_close(h)


def test_batch_range_error_is_flagged(ctx, zg):
    h = ctx.zg_stream_open(seed=1, stream=0, kind=zg.ZG_JAVA_LCG48)
    try:
        ctx.zg_stream_set_counter(h, zg.ZG_LCG_WINDOW - 10)
        out = torch.full((20,), 7.0, dtype=torch.float64, device="cuda")
        ctx.zg_error_flags(clear=True)
        ctx.zg_stream_fill(h, out)
        flags = ctx.zg_error_flags(clear=True)
        assert flags & zg.ZG_FLAG_RANGE
        assert np.all(host(out) == 7.0)    # skipped, untouched
    finally:
        ctx.zg_stream_close(h)
