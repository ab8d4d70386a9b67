"""The C oracle against its pure-Python twin (itself pinned by brute force):
identical bits on sampled indices that cover all three paths, both uniform
kinds, FP64, FP32, polar, mutation and the draw-budget error."""
import math
import random
import struct

import numpy as np
import pytest

from oracle import table_mp, twin


@pytest.fixture(scope="module")
def tables():
    L = table_mp.exact_layers("B", 128)
    return twin.TwinTable(128, 53, exact=L), twin.TwinTable(128, 24, exact=L)


def _bits(x):
    return struct.pack("<d", x)


def _word_fn(kind, seed, s, v):
    if kind == 1:
        return lambda d: twin.sm64_word(seed, s, v, d)
    return lambda d: twin.lcg_word(seed, s, v, d)


def _pick(cls, n_fast, n_slow, rng):
    idx = np.arange(cls.size)
    slow = idx[(cls & 3) != 0].tolist()
    multi = idx[(cls >> 2) > 0].tolist()
    fast = idx[cls == 0].tolist()
    return sorted(set(rng.sample(fast, n_fast) + rng.sample(slow, min(n_slow, len(slow))) + multi[:200]))


@pytest.mark.parametrize("kind,seed,s", [(1, 42, 0), (1, 7, 65535), (2, 123456789, 0), (2, 5, 255)])
def test_f64_matches_twin(orc, tables, kind, seed, s):
    T53, _ = tables
    n = 200000 if kind == 1 else 40000
    x, cls, errs = orc.fill_f64(kind, seed, s, 1000, n)
    assert errs == 0
    rng = random.Random(seed)
    for k in _pick(cls, 300, 300, rng):
        val, path, att = twin.variate(T53, twin.REAL, _word_fn(kind, seed, s, 1000 + k))
        assert _bits(val) == _bits(float(x[k])), k
        assert path == (cls[k] & 3) and att - 1 == min(cls[k] >> 2, 63)


@pytest.mark.parametrize("kind,seed,s", [(1, 42, 3), (2, 99, 1)])
def test_f32_matches_twin(orc, tables, kind, seed, s):
    T53, T24 = tables
    n = 100000 if kind == 1 else 30000
    first = 777
    x, x64, cls, errs = orc.fill_f32(kind, seed, s, first, n)
    assert errs == 0
    rng = random.Random(seed)
    for k in _pick(cls, 300, 300, rng):
        v = first + k
        pair = twin.sm64_word(seed, s, v >> 1, 0) if kind == 1 else None
        val, path, att = twin.variate_f32(T24, T53, _word_fn(kind, seed, s, v), pair, v)
        assert np.float32(val).tobytes() == x[k].tobytes(), k
        assert path == (cls[k] & 3)


def test_polar_matches_twin(orc):
    for kind, seed, s, first in [(1, 7, 12, 3), (2, 11, 2, 0)]:
        n = 20000
        x, cls, errs = orc.fill_polar(kind, seed, s, first, n)
        assert errs == 0
        for k in list(range(0, n, 97)) + [0, 1, n - 1]:
            v = first + k
            z1, z2, att = twin.polar_pair(_word_fn(kind, seed, s, v >> 1))
            assert _bits(z2 if v & 1 else z1) == _bits(float(x[k]))
            assert att - 1 == cls[k] >> 2


def test_mutation_is_x_plus_sigma_z(orc):
    rng = np.random.Generator(np.random.PCG64(1))
    x0 = rng.uniform(-5, 5, 50000)
    y, cls, errs = orc.mutate(x0, 1, 9, 4, 100, 0.1)
    z, _, _ = orc.fill_f64(1, 9, 4, 100, x0.size)
    assert errs == 0
    assert np.array_equal(y, x0 + 0.1 * z)


def test_budget_exhaustion_gives_nan_and_count(orc, tables):
    T53, _ = tables
    for dmax in (1, 2, 3):
        x, cls, errs = orc.fill_f64(1, 42, 0, 0, 50000, dmax=dmax)
        bad = (cls & 3) == 3
        assert errs == int(bad.sum()) > 0
        assert np.all(np.isnan(x[bad])) and not np.any(np.isnan(x[~bad]))
        assert np.all(x[bad].view(np.uint64) == np.uint64(0x7FF8000000000000))
        for k in np.flatnonzero(bad)[:50].tolist() + np.flatnonzero(~bad)[:50].tolist():
            val, path, _ = twin.variate(T53, twin.REAL, _word_fn(1, 42, 0, k), dmax=dmax)
            assert (path == 3) == bool(bad[k])
            if path != 3:
                assert _bits(val) == _bits(float(x[k]))
    # dmax = 1: exactly the slow first attempts fail
    x, cls, errs = orc.fill_f64(1, 42, 0, 0, 50000, dmax=1)
    x2, cls2, _ = orc.fill_f64(1, 42, 0, 0, 50000)
    assert np.array_equal((cls & 3) == 3, cls2 != 0)
