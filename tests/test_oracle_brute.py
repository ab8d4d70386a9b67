"""Brute-force enumeration of the ziggurat's accept/reject logic on tiny tables
(4 and 8 layers, a few bits of j and of each extra uniform), and the boundary
words of the real 128-layer table.

With every first word and every extra uniform enumerated, the exact per-attempt
acceptance and the exact output mass per bin are known; they must converge to
sqrt(pi/2)/(N v) and to the half-normal bin probabilities at the rate of the
discretisation (halving per extra bit), which a dropped term, a wrong index or
a wrong sign in the logic would not do.
"""
import math

import pytest

from oracle import table_mp, twin


def _errors(n, bits, L):
    T = twin.TwinTable(n, bits, exact=L)
    edges = sorted({0.0, 0.5, 1.0, 1.5, 2.0, 2.5, T.r, 40.0})
    acc, per_bin, tail_acc, total = twin.enumerate_attempt_mass(T, bits, bits, edges)
    exp_acc = math.sqrt(math.pi / 2) / (n * float(L["v"]))
    bin_err = max(abs(per_bin[k] / acc - (twin.half_normal_cdf(edges[k + 1]) -
                                          twin.half_normal_cdf(edges[k])))
                  for k in range(len(edges) - 1))
    tail_err = tail_acc / acc - math.erfc(T.r / math.sqrt(2))
    return acc / total - exp_acc, bin_err, tail_err


@pytest.mark.parametrize("n", [4, 8])
def test_tiny_tables_converge_to_exact_law(n):
    L = table_mp.exact_layers("B", n)
    prev = None
    for bits in (10, 12, 14):
        e_acc, e_bin, e_tail = _errors(n, bits, L)
        bound = 2.0 ** -bits       # measured: <= 0.8 2^-bits for every quantity
        assert abs(e_acc) < bound and e_bin < bound and abs(e_tail) < bound, (bits, e_acc, e_bin, e_tail)
        if prev is not None:
            # discretisation error shrinks ~4x per two extra bits
            assert abs(e_acc) < 0.5 * abs(prev[0])
        prev = (e_acc, e_bin, e_tail)


def test_real_table_boundary_words(orc):
    """j = k_i - 1 is fast, j = k_i is slow, for all 128 layers and both signs;
    j = 0 and j = 2^53 - 1 as well; the candidate is (double)j * w53[i]."""
    t = orc.table_dict()
    J = (1 << 53) - 1
    T = twin.TwinTable(128, 53, exact=None) if False else None
    for i in range(128):
        k = t["k53"][i]
        for neg in (0, 1):
            for j in {max(k - 1, 0), k, min(k + 1, J), 0, J}:
                W = (i << 57) | (neg << 56) | (j << 3) | 0b101
                cls, x = orc.decide_word(W)
                want = 0 if j < k else (2 if i == 0 else 1)
                assert cls == want, (i, neg, j)
                xv = float(j) * t["w53"][i]
                assert x == (-xv if neg else xv)
                assert math.copysign(1.0, x) == (-1.0 if neg else 1.0)
                # twin decode of the same word
                ti, tneg, tj = twin.REAL.decode(W)
                assert (ti, tneg, tj) == (i, neg, j)
