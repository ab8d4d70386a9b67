"""The launch-shape autotuner (zg_autotune) through the C ABI: it picks a
valid shape for every class (block-pooled or wave-specialised kernel, tile,
waves, persistence, steps per group, drain waves), the shapes it picks give
the same bits as the default shapes, and its cache (keyed by architecture and
HIP runtime version) gives the same shapes back."""
import json
import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu


def _fills(ctx, zg):
    """FP64 and FP32 multi-stream fills with ragged streams and an unaligned
    start, and a mutation, as host bytes."""
    out = []
    n_per, ns = 1537, 211
    for tdt in (torch.float64, torch.float32):
        buf = torch.empty(n_per * ns + 3, dtype=tdt, device="cuda")[1:1 + n_per * ns]
        buf.fill_(float("nan"))
        ctx.zg_fill_streams(buf, n_per, ns, kind=zg.ZG_SPLITMIX64, seed=77, stream0=5,
                            first_index=9)
        out.append(buf.cpu().numpy().tobytes())
    x0 = np.random.Generator(np.random.PCG64(8)).uniform(-5, 5, 300001)
    x = torch.from_numpy(x0).cuda()
    ctx.zg_mutate(x, 0.1, kind=zg.ZG_JAVA_LCG48, seed=3, stream=4, first_index=11)
    out.append(x.cpu().numpy().tobytes())
    torch.cuda.synchronize()
    return out


def test_autotune_shapes_keep_bits_and_cache(ctx, zg, tmp_path):
    saved = {c: ctx.zg_get_tune(c) for c in range(zg.ZG_TUNE_CLASSES)}
    try:
        ref = _fills(ctx, zg)
        cache = str(tmp_path / "tune.json")
        print("autotune on 64 MiB", flush=True)
        ctx.zg_autotune(cache, 64 << 20, use_cache=False)
        tuned = {c: ctx.zg_get_tune(c) for c in range(zg.ZG_TUNE_CLASSES)}
        for c, (tile, waves, bpc, qcap, dw, gs) in tuned.items():
            assert qcap == 0 and gs in (1, 2, 4, 8) and 0 <= dw <= 8, (c, tuned[c])
            if dw == 0:
                assert tile >= 128 and 1 <= waves <= 16, (c, tuned[c])
        assert tuned[zg.ZG_TUNE_POLAR][4] == 0
        assert _fills(ctx, zg) == ref
        doc = json.load(open(cache))
        (key,) = doc.keys()
        assert " hip " in key
        assert len(doc[key]["fill_f64"]) == 5
        # the cache gives the same shapes back, without timing anything
        for c, t in saved.items():
            ctx.zg_set_tune(c, *t)
        ctx.zg_autotune(cache, 64 << 20, use_cache=True)
        assert {c: ctx.zg_get_tune(c) for c in range(zg.ZG_TUNE_CLASSES)} == tuned
    finally:
        for c, t in saved.items():
            ctx.zg_set_tune(c, *t)
    assert ctx.zg_error_flags() == 0


def test_tune_rejects_bad_shapes(ctx, zg):
    saved = ctx.zg_get_tune(zg.ZG_TUNE_FILL_F64)
    try:
        for bad in [(1024, 16, 2, 0, 9, 4), (1024, 16, 2, 0, 0, 3), (1024, 16, 2, 0, 0, 16),
                    (1000, 16, 2, 0, 0, 4), (1024, 17, 2, 0, 0, 4)]:
            with pytest.raises(zg.ZgError) as e:
                ctx.zg_set_tune(zg.ZG_TUNE_FILL_F64, *bad)
            assert e.value.status == zg.ZG_EINVAL, bad
    finally:
        ctx.zg_set_tune(zg.ZG_TUNE_FILL_F64, *saved)
