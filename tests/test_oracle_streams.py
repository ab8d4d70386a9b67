"""The oracle's multi-stream batch routine (used by the benchmark's CPU
baseline) gives exactly the per-stream variates, in stream-major order, for
any thread count."""
import numpy as np
import pytest


@pytest.mark.parametrize("kind,nthreads", [(1, 1), (1, 5), (2, 3)])
def test_fill_streams_matches_per_stream(orc, kind, nthreads):
    s0, ns, first, n_per = 9, 7, 123, 1001
    a, ca, ea = orc.fill_streams_f64(kind, 77, s0, ns, first, n_per, nthreads=nthreads)
    parts = [orc.fill_f64(kind, 77, s0 + i, first, n_per, nthreads=1) for i in range(ns)]
    b = np.concatenate([p[0] for p in parts])
    cb = np.concatenate([p[1] for p in parts])
    assert ea == 0
    assert np.array_equal(a.view(np.uint64), b.view(np.uint64))
    assert np.array_equal(ca, cb)


@pytest.mark.parametrize("kind", [1, 2])
def test_fill_streams_f32_and_polar_match_per_stream(orc, kind):
    s0, ns, first, n_per = 4, 5, 10, 998
    a, a64, ca, ea = orc.fill_streams_f32(kind, 5, s0, ns, first, n_per, nthreads=3)
    p = [orc.fill_f32(kind, 5, s0 + i, first, n_per, nthreads=1) for i in range(ns)]
    assert ea == 0
    assert np.array_equal(a.view(np.uint32), np.concatenate([x[0] for x in p]).view(np.uint32))
    assert np.array_equal(a64.view(np.uint64), np.concatenate([x[1] for x in p]).view(np.uint64))
    b, cb, eb = orc.fill_streams_polar(kind, 5, s0, ns, first, n_per, nthreads=4)
    q = [orc.fill_polar(kind, 5, s0 + i, first, n_per, nthreads=1) for i in range(ns)]
    assert eb == 0
    assert np.array_equal(b.view(np.uint64), np.concatenate([x[0] for x in q]).view(np.uint64))
    assert np.array_equal(cb, np.concatenate([x[1] for x in q]))
