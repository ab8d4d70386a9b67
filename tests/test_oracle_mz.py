"""Pins of the modified ziggurat in the oracle: McFarland's method, the
comparator that Sections 1 and 3 measure against the original ziggurat, and
whose reliance on the low-order bits of 64-bit words Section 3 discusses.

- The table (oracle/table_mz.py, 60 digits) is pinned by what fixes it from
  outside its construction:
  - the half-normal's total mass sqrt(pi/2);
  - the tail mass in closed form (erfc);
  - each overhang's geometry (the curve under or over its chord, corner to
    corner);
  - the layer count (no further layer fits);
  - the distribution the alias table induces.
- The oracle's three steps (first word, region, attempt) are pinned by:
  - exhaustive enumeration of tiny formats against the normal law, within a
    bound derived from the grids;
  - crafted words (consumption order, both sides of an alias threshold, the
    sign, the draw budget);
  - statistics at the real format;
  - planted mistakes, which must fail.
- Java's nextLong composition is pinned by the JDK outputs in
  tests/golden/java_random_pins.json.
- Last, the property Section 3 turns on. Fed by java.util.Random's LCG, the
  modified ziggurat's layer choice repeats with period 2^23 in the variate
  index. The original ziggurat's does not.
"""
import json
import math
import os
import subprocess

import mpmath
import numpy as np
import pytest
from mpmath import mp, mpf
from scipy import special

from oracle import coracle, stats, table_mz

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TWO63 = 1 << 63
M64 = (1 << 64) - 1
Z_MAX = 5.0


@pytest.fixture(scope="module")
def tab():
    return table_mz.load()


@pytest.fixture(scope="module")
def tiny():
    """Tiny formats (buckets, word bits, uniform bits) and their C tables."""
    out = {}
    for fmt in ((8, 22, 12), (16, 22, 10)):
        t = table_mz.build(*fmt)
        out[fmt] = (t, coracle.mz_struct(t))
    return out


# ------------------------------------------------------------------ table

def test_stored_table_is_the_script_output(tab):
    assert table_mz.build() == tab


def test_real_format_shape(tab):
    assert (tab["n_buckets"], tab["n_layers"], tab["bits"], tab["ubits"]) == (256, 253, 64, 53)
    assert tab["kind"][0] == 0
    assert tab["kind"].count(3) == 1


def test_masses_add_up_to_the_half_normal(tab):
    """L layers of mass A plus the L + 1 regions make sqrt(pi/2): the layers
    (root finding) and the regions (quadrature) are computed apart."""
    with mp.workdps(60):
        A = mpf(tab["A"])
        T = mpmath.sqrt(mpmath.pi / 2)
        assert abs(A * tab["n_buckets"] - T) < mpf(10) ** -50
        tot = A * tab["n_layers"] + mpmath.fsum(mpf(a) for a in tab["masses"])
        assert abs(tot - T) < mpf(10) ** -40


def test_tail_mass_closed_form(tab):
    with mp.workdps(60):
        X0 = mpf(tab["X"][0])
        want = mpmath.sqrt(mpmath.pi / 2) * mpmath.erfc(X0 / mpmath.sqrt(2))
        assert abs(mpf(tab["masses"][0]) - want) < mpf(10) ** -45
        # layer 0 is the box under f(X0) out to X0 with the bucket's mass
        assert abs(X0 * mpmath.exp(-X0 * X0 / 2) - mpf(tab["A"])) < mpf(10) ** -45


def test_no_further_layer_fits(tab):
    """In float64, independently of the construction: the last layer holds
    mass A, and no box [0, x] x [Y_{L-1}, f(x)] reaches A."""
    X = np.array([float(v) for v in tab["X"]])
    Y = np.array([float(v) for v in tab["Y"]])
    A = float(tab["A"])
    L = tab["n_layers"]
    assert abs(X[L - 1] * (Y[L - 1] - Y[L - 2]) - A) < 1e-12
    x = np.linspace(0, X[L - 1], 200001)[1:]
    assert np.max(x * (np.exp(-x * x / 2) - Y[L - 1])) < A
    # the layers decrease in x and increase in y
    assert np.all(np.diff(X) < 0) and np.all(np.diff(Y) > 0) and Y[-1] < 1


def test_overhang_geometry(tab):
    """Every overhang box runs from its bottom-right corner (s = 0, t = 0) on
    the curve to its top-left corner (s = 1, t = 1) on the curve, and the
    curve lies under the chord where the kind says convex, over it where it
    says concave (f'' = (x^2 - 1) f changes sign at 1)."""
    L = tab["n_layers"]
    f = lambda x: np.exp(-x * x / 2)
    for k in range(1, L + 1):
        ox, odx, oy, ody = tab["ox"][k], tab["odx"][k], tab["oy"][k], tab["ody"][k]
        assert abs(f(ox) - oy) < 1e-15 and abs(f(ox - odx) - (oy + ody)) < 1e-13
        s = np.linspace(0, 1, 1001)[1:-1]
        t_curve = (f(ox - s * odx) - oy) / ody
        under = np.all(t_curve <= s + 1e-12)
        over = np.all(t_curve >= s - 1e-12)
        kind = tab["kind"][k]
        if kind == 1:
            assert under, k
        elif kind == 2:
            assert over, k
        else:
            assert ox - odx < 1 < ox and not under and not over, k


def test_alias_table_reproduces_the_region_masses(tab):
    """The region picked by (bucket j, threshold, alias) has, over uniform j
    and a uniform 63-bit u, probability m_k / (N 2^63), within 2^-60 of
    a_k / sum a."""
    N, L = tab["n_buckets"], tab["n_layers"]
    thr = [int(t) for t in tab["thr"]]
    alias = tab["alias"]
    got = [0] * (L + 1)
    for j in range(N):
        assert 0 <= thr[j] <= TWO63
        if j <= L:
            got[j] += thr[j]
        else:
            assert thr[j] == 0
        if thr[j] < TWO63:
            assert 0 <= alias[j] <= L
            got[alias[j]] += TWO63 - thr[j]
    assert sum(got) == N * TWO63
    with mp.workdps(40):
        a = [mpf(v) for v in tab["masses"]]
        tot = mpmath.fsum(a)
        for k in range(L + 1):
            assert abs(mpf(got[k]) / (N * TWO63) - a[k] / tot) < mpf(2) ** -60, k


def test_stored_doubles_are_the_correctly_rounded_values(tab):
    with mp.workdps(60):
        L = tab["n_layers"]
        for i in range(L):
            assert tab["xs"][i] == float(mpf(tab["X"][i]) * mpf(2) ** -63)
        assert tab["x0"] == float(mpf(tab["X"][0]))


# ------------------------------------------------------- exhaustive law

POS = [0, .25, .5, .75, 1, 1.25, 1.5, 2, 2.5, 3, 4, 1e9]
EDGES = np.array([-p for p in POS[::-1][:-1]] + POS)   # signed bin edges


def enum_law(T, t, L=None):
    """The law of one variate over EDGES from exhaustive enumeration of every
    first word, every second-word bucket and every pair of attempt uniforms
    through the oracle's steps, and the bound on its distance from the normal
    law that the finite grids allow:
    - layer grid: each layer is a lattice of spacing N X_i 2^-(B-1); one
      point per bin edge is off, 2 L 2^-B per bin in all;
    - alias grid: the integer masses and the threshold compare on a lattice of
      step N give each region's probability within 2 N 2^-(B-1);
    - attempt grid: in region r the G x G pairs resolve the acceptance area
      and the magnitude's bins within 4/G of the box; divided by the
      acceptance fraction, times the region's probability."""
    lb, cnt, acc, tot = coracle.mz_enum(T, EDGES, L)
    N, B, G = t["n_buckets"], t["bits"], 1 << t["ubits"]
    nl = t["n_layers"]
    W = float(1 << B)
    nb = EDGES.size - 1
    h = nb // 2
    p = lb.astype(np.float64) / W
    bound = 2 * nl / W + (nl + 1) * 2 * N / (W / 2) * (N - nl) / N
    dead = False   # a region that is picked but never accepts
    for r in range(nl + 1):
        if tot[r] == 0:
            dead = dead or cnt[r].sum() > 0
            continue
        cond = acc[r][h:].astype(np.float64) / float(tot[r])
        pr = cnt[r].astype(np.float64) / (W * N)
        p[h:] += pr[0] * cond
        p[:h] += pr[1] * cond[::-1]
        bound += pr.sum() * 4.0 / (G * (float(tot[r]) / G / G))
    want = np.diff(0.5 * special.erfc(-EDGES / math.sqrt(2)))
    err = np.abs(p - want)
    return (err + np.inf if dead else err), bound


@pytest.mark.parametrize("fmt", [(8, 22, 12), (16, 22, 10)])
def test_exhaustive_law_within_grid_bound(tiny, fmt):
    t, T = tiny[fmt]
    err, bound = enum_law(T, t)
    assert bound < 1e-3, bound
    assert err.max() <= bound, (err.max(), bound)


# --------------------------------------------------------- crafted words

A_ALL = ((1 << 53) - 1) << 11   # attempt word: the largest uniform
W_FIRST_SLOW = 253              # a first-word bucket beyond the layers


def _first_word(u, neg=False):
    """A first word with the 63 low bits u (its low byte is the bucket)."""
    return (u | (TWO63 if neg else 0)) & M64


def _u_with_bucket(target, bucket=W_FIRST_SLOW, below=True):
    """The largest u < target (below) or the smallest u >= target whose low
    byte is `bucket`."""
    base = target & ~255
    if below:
        u = base + bucket
        return u if u < target else u - 256
    u = base + bucket
    return u if u >= target else u + 256


def _region_of(tab, x):
    """Regions whose magnitude range holds |x| (overhang k: [X_k, X_{k-1}],
    tail: beyond X_0)."""
    a = abs(x)
    out = {k for k in range(1, tab["n_layers"] + 1)
           if tab["ox"][k] - tab["odx"][k] <= a <= tab["ox"][k]}
    if a >= tab["x0"]:
        out.add(0)
    return out


def test_fast_path_reads_one_word(orc, tab):
    for i in (0, 1, 100, 252):
        for hi in (0x123456789abcd, (1 << 55) - 1):
            W1 = _first_word((hi << 8) | i, neg=bool(hi & 1))
            x, cls, reads = orc.mz_tape([W1])
            sv = W1 - (1 << 64) if W1 >> 63 else W1
            assert cls == 0 and reads == [0]
            assert x == tab["xs"][i] * float(sv)


def test_alias_threshold_both_sides(orc, tab):
    """A split bucket j: u just below its threshold takes region j, u at or
    above it takes alias[j]; the variate lands in that region's range, with
    the first word's sign, after reading words 0, 1, 2, 3."""
    T = orc.mz_table()
    L = orc.lib()
    thr = [int(v) for v in tab["thr"]]
    split = [j for j in range(tab["n_layers"] + 1)
             if 256 < thr[j] < TWO63 - 256 and tab["alias"][j] != j]
    assert len(split) > 10
    for j in split[:: max(1, len(split) // 12)]:
        for below, want in ((True, j), (False, tab["alias"][j])):
            u = _u_with_bucket(thr[j], below=below)
            assert (u < thr[j]) == below
            assert L.orc_mz_region(coracle.ctypes.byref(T), _first_word(u), j) == want
            for neg in (False, True):
                x, cls, reads = orc.mz_tape([_first_word(u, neg), j, A_ALL, 0])
                assert reads == [0, 1, 2, 3]
                assert (x < 0) == neg
                assert cls & 3 == (2 if want == 0 else 1) and cls >> 2 == 0
                assert want in _region_of(tab, x), (j, want, x)


def _u_for_region(tab, k):
    """(u, second-word bucket) that pick region k."""
    thr = [int(v) for v in tab["thr"]]
    if thr[k] > 256:
        return _u_with_bucket(thr[k], below=True), k
    j = next(j for j in range(tab["n_buckets"])
             if tab["alias"][j] == k and thr[j] < TWO63 - 256)
    return _u_with_bucket(thr[j], below=False), j


def test_tail_pairs_in_order_and_restart(orc, tab):
    """Tail: each attempt reads a pair of words; a = 0 gives E1 = 53 ln 2, far
    beyond what E2 can reach, so it is rejected; the next pair, (largest, 0),
    gives E1 = 0, E2 = 53 ln 2 and accepts X_0 exactly."""
    u, j = _u_for_region(tab, 0)
    tape = [_first_word(u, neg=True), j, 0, 0, 0, 0, A_ALL, 0]
    x, cls, reads = orc.mz_tape(tape)
    assert reads == list(range(8))
    assert cls == (2 | (2 << 2))
    assert x == -tab["x0"]


def test_overhang_accepts_near_its_inner_corner(orc, tab):
    """s = 1 - 2^-53 and t = 0 lie under the curve in every overhang."""
    for k in (1, 2, 50, 200, 203, 204, 205, 230, 253):
        u, j = _u_for_region(tab, k)
        x, cls, reads = orc.mz_tape([_first_word(u), j, A_ALL, 0])
        assert reads == [0, 1, 2, 3] and cls == 1
        want = tab["ox"][k] - (float((1 << 53) - 1) * 2.0 ** -53) * tab["odx"][k]
        assert x == want, k


def test_overhang_rejects_above_the_curve_then_retries(orc, tab):
    """Convex overhang: (a, b) = (m, m - 1) sits on the chord, above the
    curve, and is rejected. Concave: (0, largest) is the box's top-right
    corner, above the curve. Each takes the next pair."""
    mid = (1 << 52) << 11
    for k, pair in ((5, (mid, mid - (1 << 11))), (240, (0, A_ALL))):
        assert tab["kind"][k] == (1 if k == 5 else 2)
        u, j = _u_for_region(tab, k)
        x, cls, reads = orc.mz_tape([_first_word(u), j, pair[0], pair[1], A_ALL, 0])
        assert reads == list(range(6)) and cls == (1 | (1 << 2)), k
        assert k in _region_of(tab, x)


def test_draw_budget(orc, tab):
    """A variate that needs more draws than the budget is the canonical NaN
    with outcome 3, after the attempts that fit."""
    u, j = _u_for_region(tab, 0)
    x, cls, reads = orc.mz_tape([_first_word(u), j] + [0] * 20, dmax=6)
    assert math.isnan(x) and cls == (3 | (2 << 2)) and reads == list(range(6))
    x, cls, _ = orc.mz_tape([_first_word(u), j], dmax=1)
    assert math.isnan(x) and cls == 3


# --------------------------------------------------------------- words

def test_next_long_matches_the_jdk(orc):
    """nextLong = (next(32) << 32) + next(32): the first nextLong of
    Random(42) is built from the JDK's first two nextInt values of the same
    seed (next(32) is nextInt)."""
    pins = json.load(open(os.path.join(GOLDEN, "java_random_pins.json")))
    assert pins["nextInt"]["seed"] == 42
    i0, i1 = pins["nextInt"]["values"]
    assert orc.long_word(orc.LCG48, 42, 0, 0, 0) == ((i0 << 32) + i1) & M64
    # later calls: steps 2m+1 and 2m+2 of the documented recurrence
    a, c, mask = 0x5DEECE66D, 0xB, (1 << 48) - 1
    S = (42 ^ a) & mask
    for m in range(6):
        S = (a * S + c) & mask
        hi = S >> 16
        S = (a * S + c) & mask
        lo = S >> 16
        hi = hi - (1 << 32) if hi >> 31 else hi
        lo = lo - (1 << 32) if lo >> 31 else lo
        assert orc.long_word(orc.LCG48, 42, 0, m, 0) == ((hi << 32) + lo) & M64, m


def test_keyed_fill_equals_the_tape_of_its_words(orc):
    """The keyed fill gives, element by element, what the step interpreter
    gives on that variate's own words (draw d = nextLong of (s, v, d))."""
    for kind in (orc.SM64, orc.LCG48):
        x, cls, errs = orc.fill_streams_mz(kind, 99, 3, 2, 1000, 3000)
        assert errs == 0
        for e in list(range(0, 6000, 97)) + list(np.nonzero(cls)[0][:40]):
            s, v = 3 + e // 3000, 1000 + e % 3000
            tape = [orc.long_word(kind, 99, s, v, d) for d in range(24)]
            y, c, _ = orc.mz_tape(tape)
            assert (y == x[e] or (math.isnan(y) and math.isnan(x[e]))) and c == cls[e], e


# ----------------------------------------------------------- statistics

def test_statistics_1e7_sm64(orc, tab):
    x, cls, errs = orc.fill_mz(orc.SM64, 42, 0, 0, 10**7)
    assert errs == 0
    n = x.size
    z = stats.moment_zscores(x)
    assert all(abs(v) < Z_MAX for v in z.values()), z
    assert stats.ks_statistic(x) < stats.ks_critical(n, 0.001)
    tz, k, e = stats.tail_count_z(x, tab["x0"])
    assert abs(tz) < Z_MAX, (k, e)
    # path frequencies: the layers take L/N of the first words; the tail
    # region its share of the rest
    N, L = tab["n_buckets"], tab["n_layers"]
    path = cls & 3
    for pth, p in ((0, L / N),
                   (2, (N - L) / N * float(mpf(tab["masses"][0]) /
                                           mpmath.fsum(mpf(a) for a in tab["masses"])))):
        got = np.count_nonzero(path == pth)
        assert abs(got - n * p) < Z_MAX * math.sqrt(n * p * (1 - p)), (pth, got, n * p)
    # conditional law beyond X_0
    t = np.abs(x[np.abs(x) > tab["x0"]])
    assert stats.ks_statistic(t, stats.tail_conditional_cdf(tab["x0"])) < \
        stats.ks_critical(t.size, 0.001)


def test_statistics_1e6_lcg(orc, tab):
    x, cls, errs = orc.fill_mz(orc.LCG48, 123456789, 0, 0, 10**6)
    assert errs == 0
    z = stats.moment_zscores(x)
    assert all(abs(v) < Z_MAX for v in z.values()), z
    assert stats.ks_statistic(x) < stats.ks_critical(x.size, 0.001)


# ------------------------------------------------ Section 3: low-order bits

def test_lcg_low_bits_repeat_every_2_23_variates(orc):
    """Section 3: the modified ziggurat picks its layer from the low-order
    bits of nextLong.  With java.util.Random those are bits 16..23 of an LCG
    state modulo 2^48, whose low 24 bits repeat every 2^24 steps: two steps
    per variate make the layer choice of variate v the same as that of
    v + 2^23, for every v.  The original ziggurat takes its layer from the
    top of its 53-bit word, which shows no such period; nor does SplitMix64."""
    P = 1 << 23
    rng = np.random.Generator(np.random.PCG64(3))
    vs = [int(v) for v in rng.integers(0, 1 << 38, 2000)]
    same = lambda f: np.mean([f(v) == f(v + P) for v in vs])
    mz_lcg = lambda v: orc.long_word(orc.LCG48, 7, 0, v, 0) & 255
    assert same(mz_lcg) == 1.0
    # the original ziggurat's layer from the same generator: chance agreement
    orig_lcg = lambda v: orc.word(orc.LCG48, 7, 0, v, 0) >> 57
    assert same(orig_lcg) < 0.05
    mz_sm64 = lambda v: orc.long_word(orc.SM64, 7, 0, v, 0) & 255
    assert same(mz_sm64) < 0.05
    # the variates themselves: every fast-path decision repeats
    a, ca, _ = orc.fill_mz(orc.LCG48, 7, 0, 5_000_000, 4096)
    b, cb, _ = orc.fill_mz(orc.LCG48, 7, 0, 5_000_000 + P, 4096)
    assert np.array_equal(ca == 0, cb == 0)


# -------------------------------------------------------- planted mistakes

C_MUTANTS = [
    ("convex point above the chord",
     "if (T->kind[k] == 1 && b > a) {", "if (T->kind[k] == 1 && b < a) {"),
    ("concave early accept on the wrong side",
     "if (T->kind[k] == 2 && ti <= si) return 1;", "if (T->kind[k] == 2 && ti >= si) return 1;"),
    ("overhang measured from the left edge",
     "*x = T->ox[k] - ((double)si * g) * T->odx[k];",
     "*x = T->ox[k] - T->odx[k] + ((double)si * g) * T->odx[k];"),
    ("alias taken below the threshold",
     "return u < T->thr[j] ? j : T->alias[j];", "return u >= T->thr[j] ? j : T->alias[j];"),
    ("region bucket from the first word",
     "int j = (int)(W2 & (uint64_t)(T->n_buckets - 1));",
     "int j = (int)(W1 & (uint64_t)(T->n_buckets - 1));"),
    ("tail test without the square",
     "return 0.5 * (t * t) < e2;", "return 0.5 * t < e2;"),
    ("tail step times X0", "double t = e1 / T->x0;", "double t = e1 * T->x0;"),
    ("slow path drops the sign",
     "*cls = outcome(k == 0 ? 2 : 1, attempts);\n      return neg ? -x : x;",
     "*cls = outcome(k == 0 ? 2 : 1, attempts);\n      return x;"),
    ("overhang density without the square",
     "return y < exp(-0.5 * (*x * *x));", "return y < exp(-0.5 * *x);"),
    ("overhang height from the top",
     "double y = T->oy[k] + ((double)ti * g) * T->ody[k];",
     "double y = T->oy[k] + T->ody[k] - ((double)ti * g) * T->ody[k];"),
    ("layer bucket from the top byte",
     "int i = (int)(W1 & (uint64_t)(T->n_buckets - 1));",
     "int i = (int)((W1 >> (T->bits - 8)) & (uint64_t)(T->n_buckets - 1));"),
]


def mz_battery(L, tiny, tab):
    """Names of the pins a build of the oracle fails."""
    failed = []
    for fmt, (t, T) in tiny.items():
        try:
            err, bound = enum_law(T, t, L)
        except ValueError:
            err, bound = np.array([np.inf]), 0.0
        if not err.max() <= bound:
            failed.append(f"law {fmt}")
    u, j = _u_for_region(tab, 0)
    x, cls, _ = coracle.mz_tape([_first_word(u, neg=True), j, 0, 0, 0, 0, A_ALL, 0], L=L)
    if not (x == -tab["x0"] and cls == (2 | (2 << 2))):
        failed.append("tail tape")
    return failed


def test_unplanted_mz_oracle_passes(tiny, tab):
    assert mz_battery(coracle.lib(), tiny, tab) == []


@pytest.mark.parametrize("name,old,new", C_MUTANTS, ids=[m[0] for m in C_MUTANTS])
def test_mz_mutant_fails_a_pin(tiny, tab, tmp_path, name, old, new):
    with open(coracle.SRC) as fh:
        src = fh.read()
    assert src.count(old) == 1, f"target of '{name}' not found once in the oracle"
    path = tmp_path / "zg_oracle_mz_mutant.c"
    path.write_text(src.replace(old, new))
    so = str(tmp_path / "libzg_oracle_mz_mutant.so")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-pthread", str(path), "-o", so, "-lm"], check=True)
    L = coracle.load_variant(so)
    assert mz_battery(L, tiny, tab), f"planted mistake '{name}' passed every pin"
