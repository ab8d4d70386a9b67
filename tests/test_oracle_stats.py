"""Statistical pins of the oracle: moments, Kolmogorov-Smirnov against Phi and
the tail frequency erfc(r/sqrt 2), at 1e8 samples for the FP64 ziggurat fed by
SplitMix64 (1e7 for the other modes), plus the conditional law of the tail and
the independence of streams and retry windows."""
import math

import numpy as np
import pytest

from oracle import stats

Z_MAX = 5.0


def _check_normal(x, r, label):
    z = stats.moment_zscores(x)
    assert all(abs(v) < Z_MAX for v in z.values()), (label, z)
    D = stats.ks_statistic(x)
    assert D < stats.ks_critical(x.size, 0.001), (label, D)
    tz, k, e = stats.tail_count_z(x, r)
    assert abs(tz) < Z_MAX, (label, k, e)


@pytest.mark.slow
def test_f64_sm64_1e8(orc):
    t = orc.table_dict()
    x, cls, errs = orc.fill_f64(orc.SM64, 42, 0, 0, 10**8)
    assert errs == 0
    _check_normal(x, t["r"], "f64 sm64")
    # path frequencies per variate against the table geometry
    p_fast = sum(t["k53"]) * 2.0 ** -53 / 128
    first_fast = np.count_nonzero(cls == 0) / x.size
    assert abs(first_fast - p_fast) < Z_MAX * math.sqrt(p_fast * (1 - p_fast) / x.size)
    # conditional law beyond r
    tail = np.abs(x[np.abs(x) > t["r"]])
    D = stats.ks_statistic(tail, stats.tail_conditional_cdf(t["r"]))
    assert D < stats.ks_critical(tail.size, 0.001)
    del x


@pytest.mark.parametrize("kind,seed,s", [(2, 123456789, 0), (1, 7, 65535), (2, 5, 255)])
def test_f64_1e7(orc, kind, seed, s):
    t = orc.table_dict()
    x, _, errs = orc.fill_f64(kind, seed, s, 12345, 10**7)
    assert errs == 0
    _check_normal(x, t["r"], (kind, seed, s))


def test_f32_1e7(orc):
    t = orc.table_dict()
    for kind in (1, 2):
        x, x64, cls, errs = orc.fill_f32(kind, 3, 1, 0, 10**7)
        assert errs == 0
        _check_normal(x.astype(np.float64), t["r"], ("f32", kind))
        # stated FP32 error against the FP64 value of the same uniform and
        # decision: the fast path rounds W to FP32 (relative 2^-24) and the
        # product (half an ulp), so |x32 - x64| <= ulp32/2 + 2^-24 |x| (at most
        # 1.5 ulp_f32); the slow path is the correctly rounded FP64 value.
        ulp = np.spacing(np.abs(x)).astype(np.float64)
        err = np.abs(x.astype(np.float64) - x64)
        fast = (cls & 3) == 0
        assert np.all(err[fast] <= 0.5 * ulp[fast] + np.abs(x64[fast]) * 2.0 ** -24 * (1 + 2.0 ** -20))
        assert np.max(err[fast] / ulp[fast]) <= 1.5
        assert np.array_equal(x[~fast], x64[~fast].astype(np.float32))


def test_polar_1e7(orc):
    t = orc.table_dict()
    for kind in (1, 2):
        x, cls, errs = orc.fill_polar(kind, 7, 3, 0, 10**7)
        assert errs == 0
        _check_normal(x, t["r"], ("polar", kind))
        att = (cls >> 2).astype(np.float64) + 1
        # attempts per pair are geometric with success pi/4
        assert abs(att.mean() - 4 / math.pi) < Z_MAX * math.sqrt((1 - math.pi / 4)) / (math.pi / 4) / math.sqrt(x.size / 2)


@pytest.mark.parametrize("kind", [1, 2])
def test_streams_and_windows_are_uncorrelated(orc, kind):
    """Same index in neighbouring streams, and the first word against the words
    of later draws, show no linear or layer-level dependence."""
    n = 10**6
    a, _, _ = orc.fill_f64(kind, 99, 0, 0, n)
    b, _, _ = orc.fill_f64(kind, 99, 1, 0, n)
    assert abs(np.corrcoef(a, b)[0, 1]) * math.sqrt(n) < Z_MAX
    assert abs(np.corrcoef(a * a, b * b)[0, 1]) * math.sqrt(n) < Z_MAX
    w0 = orc.words(kind, 99, 0, 0, 0, n)
    for d in (1, 2):
        wd = orc.words(kind, 99, 0, d, 0, n)
        u0 = (w0 >> np.uint64(11)).astype(np.float64)
        ud = (wd >> np.uint64(11)).astype(np.float64)
        assert abs(np.corrcoef(u0, ud)[0, 1]) * math.sqrt(n) < Z_MAX
        # layer of the first word against the top 8 bits of the retry word
        obs = np.zeros((128, 8))
        np.add.at(obs, ((w0 >> np.uint64(57)).astype(np.int64), (wd >> np.uint64(61)).astype(np.int64)), 1)
        expct = obs.sum(1, keepdims=True) * obs.sum(0, keepdims=True) / n
        chi2 = float(((obs - expct) ** 2 / expct).sum())
        dof = 127 * 7
        assert (chi2 - dof) / math.sqrt(2 * dof) < Z_MAX
