"""Planted mistakes.  Each plausible error in the ziggurat's accept/reject
code is planted in a copy of the oracle's own source on the CPU (the C oracle
recompiled, the Python twin re-executed), and the copy must fail at least one
pin of tests/oracle_pins.py: the exact law on small tables, the boundary
words, the consumption order, the extreme tail or the strict wedge tie.
Table mistakes (wrong heights, the other base-area reading, a wrong threshold
or tail origin) run the unchanged code on a wrong table.
"""
import importlib.util
import os
import subprocess
import types

import pytest

import oracle_pins
from oracle import coracle, table_mp, twin
from test_oracle_brute import c_battery, c_enum, twin_battery

ORACLE_DIR = os.path.dirname(coracle.__file__)

# (name, text in the oracle's source, planted replacement)
C_MUTANTS = [
    ("wedge height y[i] for y[i-1]",
     "double y = T->y[i - 1] + u53(W1) * T->dy[i];", "double y = T->y[i] + u53(W1) * T->dy[i];"),
    ("wedge step dy[i-1] for dy[i]",
     "double y = T->y[i - 1] + u53(W1) * T->dy[i];", "double y = T->y[i - 1] + u53(W1) * T->dy[i - 1];"),
    ("wedge <= for <",
     "return y < exp(-0.5 * (x * x));", "return y <= exp(-0.5 * (x * x));"),
    ("wedge density without the square",
     "return y < exp(-0.5 * (x * x));", "return y < exp(-0.5 * x);"),
    ("tail restart at d+2", "return i == 0 ? 3u : 2u;", "return i == 0 ? 2u : 2u;"),
    ("wedge restart at d+1", "return i == 0 ? 3u : 2u;", "return i == 0 ? 3u : 1u;"),
    ("U for U+ in the tail logarithm",
     "double a = -log(u53p(W1)) / T->r;", "double a = -log(u53(W1)) / T->r;"),
    ("tail rate times r", "double a = -log(u53p(W1)) / T->r;", "double a = -log(u53p(W1)) * T->r;"),
    ("tail test on the candidate",
     "return u53(W2) < exp(-0.5 * (a * a));", "return u53(W2) < exp(-0.5 * (xt * xt));"),
    ("tail without the origin r", "double xt = T->r + a;", "double xt = a;"),
    ("fast test <= for <", "return j < T->k53[i];", "return j <= T->k53[i];"),
    ("sign from bit 55", "*neg = (int)((W >> 56) & 1);", "*neg = (int)((W >> 55) & 1);"),
    ("layer from the top 6 bits", "*i = (int)(W >> 57);", "*i = (int)(W >> 58);"),
    ("j from bits 4..56", "*j = (W >> 3) & ((1ULL << 53) - 1);", "*j = (W >> 4) & ((1ULL << 53) - 1);"),
    ("uniform from 52 bits",
     "static double u53(uint64_t W) { return (double)(W >> 11) * 0x1p-53; }",
     "static double u53(uint64_t W) { return (double)(W >> 12) * 0x1p-53; }"),
]

TWIN_MUTANTS = [
    ("wedge height y[i] for y[i-1]",
     "y = T.y[i - 1] + u_of(draw1) * T.dy[i]", "y = T.y[i] + u_of(draw1) * T.dy[i]"),
    ("wedge <= for <", "if y < math.exp(-0.5 * (x * x)):", "if y <= math.exp(-0.5 * (x * x)):"),
    ("tail restart at d+2", "d += 3 if i == 0 else 2", "d += 2 if i == 0 else 2"),
    ("wedge restart at d+1", "d += 3 if i == 0 else 2", "d += 3 if i == 0 else 1"),
    ("U for U+ in the tail logarithm",
     "a = -math.log(up_of(draw1)) / T.r", "a = -math.log(u_of(draw1)) / T.r"),
    ("fast test <= for <", "if j < T.k[i]:", "if j <= T.k[i]:"),
    ("sign from the wrong bit", "neg = (W >> (self.bits - self.lbits - 1)) & 1",
     "neg = (W >> (self.bits - self.lbits - 2)) & 1"),
    ("tail test on the candidate",
     "if u_of(draw2) < math.exp(-0.5 * (a * a)):", "if u_of(draw2) < math.exp(-0.5 * (xt * xt)):"),
]


@pytest.fixture(scope="module")
def layers():
    return {n: table_mp.exact_layers("B", n) for n in (4, 8)}


@pytest.fixture(scope="module")
def twin128():
    return twin.TwinTable(128, 53, exact=table_mp.exact_layers("B", 128))


def _failed(res):
    return sorted(k for k, v in res.items() if v is not None)


def test_unplanted_oracles_pass(orc, layers, twin128):
    assert _failed(c_battery(orc, layers)) == []
    assert _failed(twin_battery(twin, twin128, layers)) == []


@pytest.mark.parametrize("name,old,new", C_MUTANTS, ids=[m[0] for m in C_MUTANTS])
def test_c_oracle_mutant_fails_a_pin(orc, layers, tmp_path, name, old, new):
    with open(coracle.SRC) as fh:
        src = fh.read()
    assert src.count(old) == 1, f"target of '{name}' not found once in the oracle"
    path = tmp_path / "zg_oracle_mutant.c"
    path.write_text(src.replace(old, new))
    so = str(tmp_path / "libzg_oracle_mutant.so")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-pthread", str(path), "-o", so, "-lm"], check=True)
    L = coracle.load_variant(so)
    failed = _failed(c_battery(orc, layers, L))
    assert failed, f"planted mistake '{name}' passed every pin"


def _twin_variant(old, new):
    """The twin with every occurrence of `old` replaced."""
    spec = importlib.util.find_spec("oracle.twin")
    with open(spec.origin) as fh:
        src = fh.read()
    assert src.count(old) >= 1, f"target '{old}' not found in the twin"
    mod = types.ModuleType("oracle.twin_mutant")
    mod.__package__ = "oracle"
    mod.__file__ = os.path.join(ORACLE_DIR, "twin_mutant.py")
    exec(compile(src.replace(old, new), mod.__file__, "exec"), mod.__dict__)
    return mod


@pytest.mark.parametrize("name,old,new", TWIN_MUTANTS, ids=[m[0] for m in TWIN_MUTANTS])
def test_twin_mutant_fails_a_pin(layers, twin128, name, old, new):
    mod = _twin_variant(old, new)
    T = mod.TwinTable(128, 53, exact=twin128.exact)
    failed = _failed(twin_battery(mod, T, layers))
    assert failed, f"planted mistake '{name}' passed every pin"


# ----------------------------------------------------------- table mistakes

def _law_fails(orc, T, bits=12):
    e = oracle_pins.law_errors(lambda T_, n, b, edges: orc.enum_attempt(
        orc.small_table(T), T.n, b, b, edges), T.n, bits, T.exact, twin)
    return max(abs(v) for v in e) >= 2.0 ** -bits


def test_correct_table_passes(orc, layers):
    assert not _law_fails(orc, twin.TwinTable(8, 12, exact=layers[8]))


def test_table_heights_shifted_fail(orc, layers):
    T = twin.TwinTable(8, 12, exact=layers[8])
    T.y = T.y[1:] + [1.0]          # y_i where y_{i-1} belongs
    assert _law_fails(orc, T)


def test_wrong_base_area_reading_fails(orc):
    """Table of reading A (integral tail area) under the majorant tail test."""
    T = twin.TwinTable(8, 12, exact=table_mp.exact_layers("A", 8))
    assert _law_fails(orc, T)


def test_wrong_wedge_scale_fails(orc, layers):
    T = twin.TwinTable(8, 12, exact=layers[8])
    T.dy = [0.0] + [2 * d for d in T.dy[1:]]
    assert _law_fails(orc, T)


def test_wrong_fast_threshold_fails(orc, layers):
    T = twin.TwinTable(8, 12, exact=layers[8])
    T.k = [min(k + 200, 4096) for k in T.k]    # inner box too wide
    assert _law_fails(orc, T)


def test_wrong_tail_start_fails(orc, layers):
    T = twin.TwinTable(8, 12, exact=layers[8])
    T.r = T.r * 0.9                             # tail sampled from the wrong origin
    assert _law_fails(orc, T)
