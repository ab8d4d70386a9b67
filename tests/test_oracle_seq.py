"""Pins of the oracle's sequential-consumption routine: the variates that
successive nextGaussian(random) calls take from one generator in order
(Section 2, Listing 2).  Each attempt reads one word, a wedge test one more
and the base strip two more; a rejected attempt is followed by an attempt at
the next unread word.

The pins come from outside the routine: crafted word lists whose outcomes the
table geometry fixes, the keyed oracle (separately pinned) at positions where
the first attempt is fast, continuation across calls, and the mean number of
words per variate against its closed form (Wald's identity with the
per-attempt acceptance sqrt(pi/2) / (128 v))."""
import math

import numpy as np
import pytest

from oracle import stats

TOP = 2 ** 53
ALL1 = 2 ** 64 - 1


def _word(i, neg, j):
    return (i << 57) | (neg << 56) | (j << 3)


def test_crafted_consumption(orc):
    """Fast, wedge accept, wedge reject, tail accept and tail reject, each with
    the words it must read and the value the definitions give."""
    t = orc.table_dict()
    k53, w53, r = t["k53"], t["w53"], t["r"]
    jf3, jf9, jf2 = k53[3] // 2, k53[9] // 3, k53[2] // 5
    jw5, jw7 = (k53[5] + TOP) // 2, (k53[7] + TOP) // 2   # middle of the wedge part
    words = [
        _word(3, 0, jf3),               # v0: fast
        _word(5, 0, jw5), 0,            # v1: wedge, U = 0 accepts (y = y[4] < f(x))
        _word(7, 0, jw7), ALL1,         # v2: wedge, U ~ 1 rejects (y ~ y[7] > f(x)) ...
        _word(9, 1, jf9),               #     ... then a fast attempt
        _word(0, 0, k53[0]), ALL1, 0,   # v3: base strip, U1+ = 1 (a = 0), U2 = 0 accepts: x = r
        _word(0, 1, k53[0] + 5), 0, ALL1,   # v4: base strip, U1+ = 2^-53, U2 ~ 1 rejects ...
        _word(2, 0, jf2),               #     ... then a fast attempt
    ]
    out, cls, starts, nxt, fails = orc.seq_f64(0, 0, 0, 0, 5, words=words)
    want = [float(jf3) * w53[3], float(jw5) * w53[5], -(float(jf9) * w53[9]), r,
            float(jf2) * w53[2]]
    assert fails == 0
    assert out.tolist() == want
    assert starts.tolist() == [0, 1, 3, 6, 9]
    assert nxt == 13
    # path of the accepting attempt (low 2 bits) and rejected attempts before it
    assert [(c & 3, c >> 2) for c in cls.tolist()] == [(0, 0), (1, 0), (0, 1), (2, 0), (0, 1)]
    # a stream that ends inside a variate: that variate fails, nothing else
    out, cls, starts, nxt, fails = orc.seq_f64(0, 0, 0, 0, 4, words=words[:8])
    assert fails == 1 and np.isnan(out[3]) and out[:3].tolist() == want[:3] and nxt == 8


@pytest.mark.parametrize("kind", [1, 2])
def test_fast_starts_match_keyed(orc, kind):
    """Stream s word p is the keyed word W(s, p, 0): where a variate's first
    attempt is fast, it equals keyed variate v = p of the same stream."""
    n, first, s = 20000, 777, 3
    out, cls, starts, nxt, fails = orc.seq_f64(kind, 99, s, first, n)
    assert fails == 0 and starts[0] == first
    assert np.all(np.diff(starts.astype(np.int64)) >= 1)
    fast = cls == 0
    assert fast.mean() > 0.95
    keyed, kcls, _ = orc.fill_f64(kind, 99, s, int(starts[0]), int(starts[-1] - starts[0] + 1))
    idx = (starts[fast] - starts[0]).astype(np.int64)
    assert np.array_equal(out[fast].view(np.uint64), keyed[idx].view(np.uint64))
    assert np.all(kcls[idx] == 0)
    # a variate accepted at its first attempt read 1 word (fast), 2 (wedge)
    # or 3 (base strip)
    per = np.diff(np.append(starts.astype(np.int64), nxt))
    one = (cls >> 2) == 0
    assert np.array_equal(per[one], (cls[one] & 3).astype(np.int64) + 1)


@pytest.mark.parametrize("kind", [1, 2])
def test_continuation(orc, kind):
    """n1 + n2 variates in one call equal n1, then n2 from the returned position."""
    a, _, _, nxt_a, _ = orc.seq_f64(kind, 5, 0, 10, 30001)
    b1, _, _, nxt1, _ = orc.seq_f64(kind, 5, 0, 10, 12345)
    b2, _, _, nxt2, _ = orc.seq_f64(kind, 5, 0, nxt1, 30001 - 12345)
    assert np.array_equal(a.view(np.uint64), np.concatenate([b1, b2]).view(np.uint64))
    assert nxt2 == nxt_a


def test_words_per_variate_closed_form(orc):
    """Mean words per variate = E[words per attempt] / P(accept per attempt).
    E[words per attempt] = 1 + (1/128) sum_i (1 - k_i 2^-53) (2 if i = 0
    else 1); P(accept) = sqrt(pi/2) / (128 v), v = r f(r) + f(r)/r."""
    t = orc.table_dict()
    r = t["r"]
    f = math.exp(-0.5 * r * r)
    v = r * f + f / r
    p_acc = math.sqrt(math.pi / 2) / (128 * v)
    e_w = 1.0 + sum((1.0 - t["k53"][i] / TOP) * (2 if i == 0 else 1) for i in range(128)) / 128
    mean = e_w / p_acc
    n = 10 ** 7
    out, cls, starts, nxt, fails = orc.seq_f64(1, 2024, 0, 0, n)
    assert fails == 0
    per = np.diff(np.append(starts.astype(np.int64), nxt))
    z = (per.mean() - mean) / (per.std() / math.sqrt(n))
    assert abs(z) < 5.0, (per.mean(), mean, z)
    # every rejected attempt read at least 2 words (a wedge or the base strip)
    attempts = (cls >> 2).astype(np.int64) + 1
    assert np.all(per >= 2 * attempts - 1)


def test_sequential_normal(orc):
    """Sequential consumption changes which words a variate reads, not its law."""
    t = orc.table_dict()
    out, cls, starts, nxt, fails = orc.seq_f64(2, 31337, 0, 0, 10 ** 6)
    assert fails == 0
    z = stats.moment_zscores(out)
    assert all(abs(v) < 5.0 for v in z.values()), z
    assert stats.ks_statistic(out) < stats.ks_critical(out.size, 0.001)
