"""The oracle's multi-stream batch driver (used by the benchmark's CPU
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
