"""Pins of the oracle's uniform sources against published outputs.

SplittableRandom and Random are the PRNGs of Section 2 and Table 1; their
index-keyed forms must reduce to the sequential generators at stream 0, draw 0.
"""
import json
import os
import random

import numpy as np

from conftest import GOLDEN
from oracle import twin


def _load(name):
    with open(os.path.join(GOLDEN, name)) as fh:
        return json.load(fh)


def test_splitmix64_published_outputs(orc):
    pins = _load("splitmix64_pins.json")
    got = [orc.word(orc.SM64, pins["seed"], 0, v, 0) for v in range(3)]
    assert got == [int(h, 16) for h in pins["values"]]
    assert [twin.sm64_word(pins["seed"], 0, v, 0) for v in range(3)] == got


def test_java_random_published_outputs(orc):
    pins = _load("java_random_pins.json")
    ints = orc.lcg_seq_ints(pins["nextInt"]["seed"], len(pins["nextInt"]["values"]))
    assert ints.tolist() == pins["nextInt"]["values"]
    for case in pins["nextDouble"]:
        vals = orc.lcg_seq_doubles(case["seed"], len(case["values"]))
        assert [float(m) * 2.0 ** -53 for m in vals] == [float(x) for x in case["values"]]


def test_polar_core_reproduces_java_nextgaussian(orc):
    """Random(0).nextGaussian(): polar attempts on consecutive nextDouble pairs."""
    pins = _load("java_random_pins.json")["nextGaussian"]
    u = orc.lcg_seq_doubles(pins["seed"], 64).astype(np.float64) * 2.0 ** -53
    k = 0
    while True:
        ok, z1, z2 = orc.polar_core(u[k], u[k + 1])
        k += 2
        if ok:
            break
    assert [z1, z2] == [float(x) for x in pins["values"]]
    # the pure-Python twin of the polar attempt gives the same pair
    words = {d: int(m) << 11 for d, m in enumerate(orc.lcg_seq_doubles(pins["seed"], 64))}
    t1, t2, _ = twin.polar_pair(lambda d: words[d])
    assert (t1, t2) == (z1, z2)


def test_keyed_words_equal_sequential_streams(orc):
    """Stream 0, draw 0 words are the sequential generator outputs."""
    n = 20000
    for seed in (0, 7, 123456789, 2**64 - 1):
        seq = orc.lcg_seq_doubles(seed, n)
        keyed = orc.words(orc.LCG48, seed, 0, 0, 0, n)
        assert np.array_equal(keyed >> np.uint64(11), seq)
    # SplittableRandom(seed).nextLong() k-th = mix64(seed + (k+1) gamma)
    w = orc.words(orc.SM64, 42, 0, 0, 0, 1000)
    assert all(int(w[k]) == twin.sm64_word(42, 0, k, 0) for k in range(0, 1000, 37))


def test_lcg_jump_equals_stepping(orc):
    rng = random.Random(5)
    seed = 123456789
    S = orc.lib().orc_lcg_state0(seed)
    states = [S]
    for _ in range(5000):
        S = orc.lib().orc_lcg_step(S)
        states.append(S)
    for k in [0, 1, 2, 3, 4999, 5000] + [rng.randrange(5000) for _ in range(50)]:
        assert orc.lib().orc_lcg_state(seed, k) == states[k]
    # the twin sums the geometric series in exact integers: a different route
    for k in [rng.randrange(2**48) for _ in range(50)] + [2**47, 2**48 - 1]:
        assert orc.lib().orc_lcg_state(seed, k) == twin.lcg_state(seed, k)
    # composition law of affine maps
    M = (1 << 48) - 1
    for _ in range(50):
        a, b = rng.randrange(2**46), rng.randrange(2**46)
        A1, C1 = orc.lcg_affine(a)
        A2, C2 = orc.lcg_affine(b)
        A, C = orc.lcg_affine(a + b)
        assert A == (A2 * A1) & M and C == (A2 * C1 + C2) & M
    # period 2^48: the map of 2^48 steps is the identity
    assert orc.lcg_affine(2**48) == (1, 0)


def test_keyed_words_match_twin(orc):
    rng = random.Random(11)
    for _ in range(300):
        seed = rng.randrange(2**64)
        s, d = rng.randrange(2**8), rng.randrange(2**8)
        v = rng.randrange(twin.LCG_WINDOW)
        assert orc.word(orc.LCG48, seed, s, v, d) == twin.lcg_word(seed, s, v, d)
        s16, v40 = rng.randrange(2**16), rng.randrange(2**40)
        assert orc.word(orc.SM64, seed, s16, v40, d) == twin.sm64_word(seed, s16, v40, d)


def test_keyed_index_windows_are_disjoint():
    """Distinct (s, d, v) within the limits never share a counter / LCG index."""
    rng = random.Random(3)
    seen_sm, seen_lcg = {}, {}
    for _ in range(20000):
        s, d = rng.randrange(2**16), rng.randrange(2**8)
        v = rng.randrange(2**40)
        ctr = 1 + (s << 48) + (d << 40) + v
        assert ctr < 2**64
        assert seen_sm.setdefault(ctr, (s, d, v)) == (s, d, v)
        s8, v31 = rng.randrange(2**8), rng.randrange(twin.LCG_WINDOW)
        m = s8 * twin.LCG_STREAM + d * twin.LCG_WINDOW + v31
        assert 2 * m + 2 < 2**48
        assert seen_lcg.setdefault(m, (s8, d, v31)) == (s8, d, v31)
    # the largest SplitMix64 counter wraps to 0, which no other key reaches
    assert 1 + ((2**16 - 1) << 48) + ((2**8 - 1) << 40) + (2**40 - 1) == 2**64
    # LCG windows of one stream, and streams, do not overlap; all fit the period
    assert 256 * twin.LCG_WINDOW <= twin.LCG_STREAM and 256 * twin.LCG_STREAM <= 2**47


def _nu2(mult, m=2**48):
    """Length of the shortest vector of the 2-D lattice x + mult y = 0 (mod m)
    (Gauss reduction): the spectral test figure of the pair (S, mult S + c)."""
    u, v = (m, 0), ((-mult) % m, 1)
    norm = lambda w: w[0] * w[0] + w[1] * w[1]
    if norm(u) < norm(v):
        u, v = v, u
    while True:
        t = round((u[0] * v[0] + u[1] * v[1]) / norm(v))
        w = (u[0] - t * v[0], u[1] - t * v[1])
        if norm(w) >= norm(v):
            return norm(v) ** 0.5
        u, v = v, w


def test_lcg_window_jumps_pass_spectral_test():
    """Words of one variate in windows d and d+k, and of streams s and s+1, are
    related by the multiplier a^(2 jump); its 2-D figure must be within a factor
    2 of consecutive doubles (a^2), unlike power-of-two spacings."""
    a, M = 0x5DEECE66D, 2**48
    ref = _nu2(pow(a, 2, M))
    for k in (1, 2, 3):
        assert _nu2(pow(a, 2 * k * twin.LCG_WINDOW, M)) > ref / 2
    assert _nu2(pow(a, 2 * twin.LCG_STREAM, M)) > ref / 2
    # the power-of-two layout fails this by orders of magnitude
    assert _nu2(pow(a, 2**32, M)) < ref / 500 and _nu2(pow(a, 2**40, M)) < ref / 1e5
