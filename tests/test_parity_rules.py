"""The comparison rules of tests/parity.py, on the CPU with crafted values:
what each rule accepts and what it counts as a failure.  In particular the
bar for mutated values, x = clamp(RN(x0 + RN(sigma z))): a slow-path z that
differs from the oracle's by 2 ulp may move a small x by many ulps of x,
but never by more than the derived bound."""
import numpy as np
import pytest

from parity import compare, compare_mutated, ulp_distance


def _next(x, k=1):
    x = np.float64(x)
    for _ in range(abs(k)):
        x = np.nextafter(x, np.inf if k > 0 else -np.inf)
    return x


def test_ulp_distance_counts_steps_and_signs():
    assert ulp_distance(np.array([1.0]), np.array([_next(1.0, 3)]))[0] == 3
    # the two zeros are one point for the distance; bit equality tells them apart
    assert ulp_distance(np.array([-0.0]), np.array([0.0]))[0] == 0
    assert ulp_distance(np.array([-_next(0.0)]), np.array([_next(0.0)]))[0] == 2
    assert ulp_distance(np.array([np.float32(1.0)]), np.array([np.float32(1.0)]))[0] == 0
    with pytest.raises(AssertionError):
        compare(np.array([-0.0]), np.array([0.0]), np.array([0], dtype=np.uint8))


def test_fast_path_must_be_bit_exact():
    want = np.array([0.5, 1.5])
    got = np.array([0.5, _next(1.5)])
    with pytest.raises(AssertionError):
        compare(got, want, np.array([0, 0], dtype=np.uint8))
    # the same 1-ulp difference on a wedge variate (class 1) is within the bar
    compare(got, want, np.array([0, 1], dtype=np.uint8))


def test_slow_path_beyond_two_ulp_is_a_disagreement():
    want = np.array([0.75] * 4)
    got = want.copy()
    got[2] = _next(0.75, 3)
    with pytest.raises(AssertionError):
        compare(got, want, np.array([1, 1, 1, 1], dtype=np.uint8))


def test_mutated_value_bound_follows_the_variate():
    sigma = 0.3
    z_o = 1.2917713377304255           # a wedge variate of the oracle
    z_g = _next(z_o, 2)                # the device's, 2 ulp away
    x0 = -sigma * z_o + 1e-3           # x nearly cancels
    x_o = np.float64(x0) + np.float64(sigma * z_o)
    x_g = np.float64(x0) + np.float64(sigma * z_g)
    assert ulp_distance(np.array([x_g]), np.array([x_o]))[0] > 2    # many ulps of x
    cls = np.array([1], dtype=np.uint8)
    rep = compare_mutated(np.array([x_g]), np.array([x_o]), cls, lambda idx: np.array([z_o]),
                          sigma)
    assert rep["differ"] == 1 and rep["disagreements"] == 0
    # a larger move than 2 ulp of z can cause is a disagreement
    x_bad = np.float64(x0) + np.float64(sigma * _next(z_o, 40))
    with pytest.raises(AssertionError):
        compare_mutated(np.array([x_bad]), np.array([x_o]), cls, lambda idx: np.array([z_o]), sigma)


def test_mutated_fast_path_and_copies_stay_bit_exact():
    want = np.array([0.25, -1.0])
    got = np.array([0.25, _next(-1.0)])
    with pytest.raises(AssertionError):
        compare_mutated(got, want, np.array([0, 0], dtype=np.uint8), lambda idx: np.zeros(len(idx)),
                        0.1)
