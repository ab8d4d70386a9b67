"""The sequential fill that allocates nothing (zg_fill_sequential_noalloc),
through the C ABI: the same bits and next position as zg_fill_sequential
with a caller workspace, on two calls in a row (the second smaller, so it
runs over what the first left in the library's resident workspace), and the
size limits refused before anything is launched."""
import numpy as np
import pytest
import torch

from parity import compare

pytestmark = pytest.mark.gpu


def _both(ctx, n, kind, seed, s, first):
    a = torch.empty(n, dtype=torch.float64, device="cuda")
    b = torch.empty(n, dtype=torch.float64, device="cuda")
    na = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    nb = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    ctx.zg_fill_sequential_noalloc(a, kind=kind, seed=seed, stream=s, first_word=first,
                                   next_word=na)
    ctx.zg_fill_sequential(b, kind=kind, seed=seed, stream=s, first_word=first, next_word=nb)
    torch.cuda.synchronize()
    return a.cpu().numpy(), b.cpu().numpy(), int(na.cpu()[0]), int(nb.cpu()[0])


def test_noalloc_matches_workspace_entry_point(ctx, zg, orc):
    calls = [(1_000_000, 1, 2**64 - 5, 9, 123), (70_001, 2, 123456789, 3, 77)]
    for n, kind, seed, s, first in calls:
        print(f"noalloc sequential n={n} kind={kind} seed={seed} s={s} first={first}", flush=True)
        got, ref, g_next, r_next = _both(ctx, n, kind, seed, s, first)
        assert np.array_equal(got.view(np.uint64), ref.view(np.uint64)), (n, kind)
        assert g_next == r_next
        o, cls, _starts, o_next, fails = orc.seq_f64(kind, seed, s, first, n)
        assert fails == 0
        compare(got, o, cls, label=f"noalloc {n}")
        assert g_next == o_next
    assert ctx.zg_error_flags() == 0


def test_noalloc_refuses_sizes_beyond_its_limits(ctx, zg):
    out = torch.empty(zg.ZG_SEQ_MAX_N + 1, dtype=torch.float64, device="cuda")
    with pytest.raises(zg.ZgError) as e:
        ctx.zg_fill_sequential_noalloc(out, kind=1)
    assert e.value.status == zg.ZG_EINVAL
    st = zg.lib.zg_fill_sequential_noalloc(ctx.h, out.data_ptr(), zg.ZG_SEQ_NOALLOC_MAX_N + 1,
                                           1, 0, 0, 0, None, None)
    assert st == zg.ZG_EINVAL
    ctx.zg_fill_sequential_noalloc(out[:0], kind=1)   # n = 0: nothing to do
    torch.cuda.synchronize()
