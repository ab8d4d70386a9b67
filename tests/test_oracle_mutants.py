"""Planted mistakes: each plausible error in the ziggurat logic, planted in a
copy of the pure-Python oracle on the CPU, must fail one of the pins above
(the brute-force law on tiny tables)."""
import math

from oracle import table_mp, twin


def _law_error(T, bits=12):
    edges = sorted({0.0, 0.5, 1.0, 1.5, 2.0, 2.5, T.r, 40.0})
    acc, per_bin, tail_acc, total = twin.enumerate_attempt_mass(T, bits, bits, edges)
    bin_err = max(abs(per_bin[k] / acc - (twin.half_normal_cdf(edges[k + 1]) -
                                          twin.half_normal_cdf(edges[k])))
                  for k in range(len(edges) - 1))
    return bin_err, abs(tail_acc / acc - math.erfc(T.r / math.sqrt(2)))


# brute-force discretisation error of the correct logic is below 2^-bits
BOUND = 2.0 ** -12


def test_correct_oracle_passes():
    T = twin.TwinTable(8, 12, exact=table_mp.exact_layers("B", 8))
    e_bin, e_tail = _law_error(T)
    assert e_bin < BOUND and e_tail < BOUND


def test_wedge_with_wrong_height_index_fails():
    T = twin.TwinTable(8, 12, exact=table_mp.exact_layers("B", 8))
    T.y = T.y[1:] + [1.0]          # uses y_i where y_{i-1} belongs
    assert _law_error(T)[0] > BOUND


def test_wrong_base_area_reading_fails():
    """Table of reading A (integral tail area) under the majorant tail test."""
    T = twin.TwinTable(8, 12, exact=table_mp.exact_layers("A", 8))
    assert max(_law_error(T)) > BOUND


def test_dropped_wedge_term_fails():
    T = twin.TwinTable(8, 12, exact=table_mp.exact_layers("B", 8))
    T.dy = [0.0] + [2 * d for d in T.dy[1:]]   # wrong wedge height scale
    assert _law_error(T)[0] > BOUND


def test_wrong_fast_threshold_fails():
    T = twin.TwinTable(8, 12, exact=table_mp.exact_layers("B", 8))
    T.k = [min(k + 200, 4096) for k in T.k]    # inner box too wide
    assert _law_error(T)[0] > BOUND


def test_wrong_tail_start_fails():
    T = twin.TwinTable(8, 12, exact=table_mp.exact_layers("B", 8))
    T.r = T.r * 0.9                             # tail sampled from the wrong origin
    assert max(_law_error(T)) > BOUND
