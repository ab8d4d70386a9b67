"""Brute-force enumeration of the oracle's own accept/reject code on small
tables (4 and 8 layers, a few bits of j and of each extra uniform), and the
crafted-word pins of its decode, fast test, consumption order and extremes.

The enumeration runs every first word and every extra uniform through the
decision functions that the oracle's fills call (the C `orc_attempt`, the
Python twin's `attempt`).  The exact per-attempt acceptance and the exact
output mass per bin of |x| then converge to sqrt(pi/2)/(N v) and to the
half-normal probabilities at the rate of the discretisation (halving per extra
bit), which a dropped term, a wrong index or a wrong sign would not do.  The
pins themselves are in tests/oracle_pins.py; test_oracle_mutants.py plants
mistakes in copies of the oracle and checks that each one fails a pin.
"""
import math

import pytest

import oracle_pins
from oracle import table_mp, twin


@pytest.fixture(scope="module")
def layers():
    return {n: table_mp.exact_layers("B", n) for n in (4, 8)}


def c_enum(orc, L=None):
    def enum(T, n, bits, edges):
        return orc.enum_attempt(orc.small_table(T), n, bits, bits, edges, L=L)
    return enum


def twin_enum(mod):
    def enum(T, n, bits, edges):
        return mod.enumerate_attempt_mass(T, bits, bits, edges)
    return enum


@pytest.mark.parametrize("n", [4, 8])
def test_c_oracle_attempt_converges_to_exact_law(orc, layers, n):
    """The C oracle's orc_attempt, enumerated at 10, 12 and 13 bits."""
    prev = None
    for bits in (10, 12, 13):
        e = oracle_pins.law_errors(c_enum(orc), n, bits, layers[n], twin)
        assert max(abs(v) for v in e) < 2.0 ** -bits, (bits, e)
        if prev is not None and bits == 12:
            # the discretisation error shrinks about 4x per two extra bits
            assert abs(e[0]) < 0.5 * abs(prev[0])
        prev = e


def test_twin_attempt_converges_to_exact_law(layers):
    """The Python twin's attempt, enumerated through Python loops."""
    for n, bits in ((4, 8), (4, 10), (8, 8)):
        e = oracle_pins.law_errors(twin_enum(twin), n, bits, layers[n], twin)
        assert max(abs(v) for v in e) < 2.0 ** -bits, (n, bits, e)


def test_c_and_twin_enumerations_count_alike(orc, layers):
    """Both oracles make the same decision for every enumerated attempt:
    identical integer weights."""
    for n, bits in ((4, 9), (8, 8)):
        T = twin.TwinTable(n, bits, exact=layers[n])
        edges = sorted({0.0, 0.5, 1.0, 1.5, 2.0, 2.5, T.r, 40.0})
        assert orc.enum_attempt(orc.small_table(T), n, bits, bits, edges) == \
            twin.enumerate_attempt_mass(T, bits, bits, edges)


def c_battery(orc, layers, L=None):
    def variate(tape):
        x, cls, reads = orc.zig_f64_tape(tape, L=L)
        return x, reads
    return oracle_pins.run_battery(orc.table_dict(), variate,
                                   lambda W: orc.decide_word(W, L=L), c_enum(orc, L), twin,
                                   [(8, 12, layers[8]), (4, 10, layers[4])])


def twin_battery(mod, T128, layers):
    def variate(tape):
        reads = []

        def w(d):
            reads.append(d)
            return tape[d] if d < len(tape) else 0
        v, path, att = mod.variate(T128, mod.REAL, w)
        return v, reads
    return oracle_pins.run_battery(table_mp.load_table(), variate, None, twin_enum(mod), twin,
                                   [(4, 8, layers[4])])


@pytest.fixture(scope="module")
def twin128():
    return twin.TwinTable(128, 53, exact=table_mp.exact_layers("B", 128))


def test_c_oracle_pins(orc, layers):
    res = c_battery(orc, layers)
    assert all(v is None for v in res.values()), res


def test_twin_pins(layers, twin128):
    res = twin_battery(twin, twin128, layers)
    assert all(v is None for v in res.values()), res


def test_real_table_boundary_words(orc):
    """j = k_i - 1 is fast, j = k_i is slow, for all 128 layers and both signs;
    j = 0 and j = 2^53 - 1 as well; the candidate is (double)j * w53[i]."""
    t = orc.table_dict()
    J = (1 << 53) - 1
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
                ti, tneg, tj = twin.REAL.decode(W)
                assert (ti, tneg, tj) == (i, neg, j)
