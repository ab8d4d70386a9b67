"""Pins of the oracle's 128-layer table (the original ziggurat of Section 1 /
Section 2, ported from GSL) against published constants, closed forms and
its defining geometry, re-checked in plain float arithmetic."""
import json
import math
import os

import numpy as np
from mpmath import mp, mpf
import mpmath

from conftest import GOLDEN
from oracle import table_mp


def _consts():
    with open(os.path.join(GOLDEN, "published_constants.json")) as fh:
        return json.load(fh)


def test_reading_a_reproduces_marsaglia_tsang_constants():
    """The same bisection/recurrence with the base area of Marsaglia-Tsang gives
    their printed r and v (their v is v(r) at their 13-digit r)."""
    c = _consts()["marsaglia_tsang_2000"]
    with mp.workdps(60):
        r = table_mp.solve_r("A")
        assert abs(r - mpf(c["r"])) < mpf("3e-12")   # printed to 12 places
        v_at_printed_r = table_mp.base_area(mpf(c["r"]), "A")
        assert abs(v_at_printed_r - mpf(c["v"])) < mpf("1e-17")


def test_reading_b_reproduces_gsl_constant():
    c = _consts()["gsl_ziggurat"]
    t = table_mp.load_table()
    assert abs(t["r"] - float(c["r"])) < 5e-12


def test_stored_table_is_regenerable():
    t, _ = table_mp.build_table("B")
    s = table_mp.load_table()
    for key in ("r", "v", "W", "y", "dy", "k53", "k24", "w24f", "w53", "w24", "w24d"):
        assert s[key] == t[key], key


def test_equal_areas_closure_and_tail_constant_in_float():
    t = table_mp.load_table()
    r, v = t["r"], t["v"]
    W, y, dy = np.array(t["W"]), np.array(t["y"]), np.array(t["dy"])
    # every rectangle has area v (base: virtual box W0 x f(r))
    assert abs(W[0] * y[0] - v) <= 1e-12 * v
    areas = W[1:] * dy[1:]
    assert np.max(np.abs(areas - v)) <= 1e-12 * v
    # closure: the top layer [0, b_126] x [f(b_126), 1] has area v
    assert abs(W[127] * (1.0 - y[126]) - v) <= 1e-12 * v
    # closed-form tail constant: v - r f(r) = f(r)/r (exponential majorant mass)
    fr = math.exp(-r * r / 2)
    assert abs((v - r * fr) - fr / r) <= 1e-12 * (fr / r)
    assert abs(y[0] - fr) <= 1e-15
    # corners lie on the curve: y_i = f(b_i) with b_i = W_{i+1}
    b = W[1:]
    assert np.max(np.abs(y[:127] - np.exp(-b * b / 2)) / y[:127]) <= 1e-13
    assert y[127] == 1.0
    # dy is the difference of heights
    assert np.max(np.abs(dy[1:] - (y[1:] - y[:-1])) / dy[1:]) <= 1e-13
    # monotone geometry
    assert np.all(np.diff(W[1:]) < 0) and W[0] > W[1] == r
    assert np.all(np.diff(y) > 0)


def test_thresholds_and_scaled_widths():
    t = table_mp.load_table()
    W = t["W"]
    q = [t["r"] / W[0]] + [W[i + 1] / W[i] for i in range(1, 127)] + [0.0]
    for i in range(128):
        assert abs(t["k53"][i] * 2.0 ** -53 - q[i]) < 4e-16
        assert abs(t["k24"][i] * 2.0 ** -24 - q[i]) < 2.0 ** -24 + 4e-16
        assert t["w53"][i] == W[i] * 2.0 ** -53
        assert np.float32(t["w24f"][i]) == np.float32(W[i])
    assert t["k53"][127] == 0 and t["k24"][127] == 0


def test_acceptance_and_majorant_cover():
    c = _consts()["gaussian_integral"]
    t = table_mp.load_table()
    half = float(c["value"])
    assert abs(half - math.sqrt(math.pi / 2)) < 1e-15
    assert 128 * t["v"] >= half
    acc = half / (128 * t["v"])
    assert abs(acc - 0.9877447619598371) < 1e-12
    # fast/wedge/tail split of one attempt
    p_fast = sum(k * 2.0 ** -53 for k in t["k53"]) / 128
    p_tail = (1 - t["k53"][0] * 2.0 ** -53) / 128
    assert abs(p_fast - 0.9723986) < 1e-6 and abs(p_tail - 0.00060736) < 1e-7


def test_table_entries_are_correctly_rounded_at_higher_precision():
    """Recomputing at 80 digits rounds to the same FP64 entries."""
    with mp.workdps(80):
        old = table_mp.DPS
        table_mp.DPS = 80
        try:
            t80, _ = table_mp.build_table("B")
        finally:
            table_mp.DPS = old
    s = table_mp.load_table()
    for key in ("r", "W", "y", "dy", "k53", "k24", "w24f"):
        assert s[key] == t80[key], key
