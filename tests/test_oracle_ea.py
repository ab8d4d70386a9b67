"""Pins of the oracle's EA generation step (orc_ea_step): the fused consumer
of Section 1's prior work, an evolutionary algorithm whose Gaussian mutation
the ziggurat sped up.  The paper names the workload but not its EA; the
reading (tournament selection with replacement, a per-gene mutation rate as a
53-bit threshold, x += sigma z, clamping to [lo, hi]) is stated in the
oracle's header.

The pins:
- the selection law: with fitness increasing in the index, the winner of k
  draws with replacement is the least of k uniform indices, so
  P(i) = ((pop - i)^k - (pop - i - 1)^k) / pop^k (chi-square, k = 1, 2, 4);
- NaN fitness wins only when every draw of the tournament has one
  (half the population NaN: P = 2^-k);
- the draws themselves: each tournament recomputed from its words (which
  words, the index mapping, ties kept by the earlier draw, NaN), with
  tied, NaN and constant fitness;
- the mutation rate: each gene mutates with probability floor(rate 2^53)
  2^-53 (binomial); rate 0 copies the winners' rows bit for bit, rate 1
  mutates every gene;
- each mutated gene is clamp(parent + sigma z) with z the oracle's own
  ziggurat variate of its key (stream + 2, index (gen pop + c) genes + g);
- the keys: another generation or stream draws afresh, the same one repeats;
- planted mistakes in the C source fail one of the above.
"""
import os
import subprocess

import numpy as np
import pytest
from scipy import stats as sst

from oracle import coracle

Z_MAX = 5.0


def _chi2_p(counts, probs):
    exp = probs * counts.sum()
    keep = exp >= 5
    chi = (((counts - exp) ** 2) / np.where(exp > 0, exp, 1))[keep].sum()
    return sst.chi2.sf(chi, keep.sum() - 1)


def _winner_counts(orc, pop, k, gens, fitness, L=None, genes=1):
    cnt = np.zeros(pop, dtype=np.int64)
    P = np.zeros((pop, genes))
    for g in range(gens):
        _, W, _, _ = orc.ea_step(P, fitness, k, 5, 100, g, 0.0, 0.0, -1.0, 1.0, L=L)
        if W.max() >= pop:
            raise IndexError(f"winner {W.max()} outside the population")
        cnt += np.bincount(W, minlength=pop)
    return cnt


@pytest.mark.parametrize("k", [1, 2, 4])
def test_tournament_law(orc, k):
    pop, gens = 64, 1500
    cnt = _winner_counts(orc, pop, k, gens, np.arange(pop, dtype=np.float64))
    i = np.arange(pop, dtype=np.float64)
    probs = ((pop - i) ** k - (pop - i - 1) ** k) / float(pop) ** k
    assert abs(probs.sum() - 1) < 1e-12
    assert _chi2_p(cnt, probs) > 1e-6, cnt[:8]


@pytest.mark.parametrize("k", [1, 2, 3])
def test_nan_fitness_wins_only_when_every_draw_is_nan(orc, k):
    pop, gens = 64, 1000
    f = np.arange(pop, dtype=np.float64)
    f[::2] = np.nan
    cnt = _winner_counts(orc, pop, k, gens, f)
    n = cnt.sum()
    nan_wins = cnt[::2].sum()
    p = 0.5 ** k
    assert abs(nan_wins - n * p) < Z_MAX * np.sqrt(n * p * (1 - p)), (nan_wins, n * p)


def test_rate_zero_copies_and_rate_one_mutates_all(orc):
    rng = np.random.Generator(np.random.PCG64(3))
    P = rng.uniform(-2, 2, (200, 37))
    F = (P ** 2).sum(1)
    C0, W0, cls0, e0 = orc.ea_step(P, F, 3, 11, 7, 2, 0.0, 0.5, -5.0, 5.0)
    assert e0 == 0 and np.all(cls0 == 255)
    assert C0.tobytes() == P[W0].tobytes()
    C1, W1, cls1, e1 = orc.ea_step(P, F, 3, 11, 7, 2, 1.0, 0.5, -5.0, 5.0)
    assert np.array_equal(W0, W1) and np.all(cls1 != 255)


def test_mutation_rate_is_binomial(orc):
    rng = np.random.Generator(np.random.PCG64(4))
    P = rng.uniform(-1, 1, (2000, 100))
    F = rng.uniform(0, 1, 2000)
    for rate in (0.01, 0.1, 0.5):
        _, _, cls, _ = orc.ea_step(P, F, 2, 9, 1, 0, rate, 0.1, -5, 5)
        n = cls.size
        p = coracle.ea_rate53(rate) * 2.0 ** -53
        got = np.count_nonzero(cls != 255)
        assert abs(got - n * p) < Z_MAX * np.sqrt(n * p * (1 - p)), (rate, got, n * p)


def test_mutated_genes_are_clamped_parent_plus_sigma_z(orc):
    rng = np.random.Generator(np.random.PCG64(5))
    pop, genes, gen, stream, seed = 50, 40, 3, 20, 123
    P = rng.uniform(-3, 3, (pop, genes))
    F = rng.uniform(0, 1, pop)
    sigma, lo, hi = 1.5, -3.5, 3.5
    C, W, cls, _ = orc.ea_step(P, F, 2, seed, stream, gen, 0.3, sigma, lo, hi)
    clamped = 0
    for c in range(pop):
        for g in range(genes):
            x = P[W[c], g]
            if cls[c, g] == 255:
                assert C[c, g] == x
                continue
            w = (gen * pop + c) * genes + g
            z, zc, _ = orc.fill_f64(orc.SM64, seed, stream + 2, w, 1, nthreads=1)
            assert zc[0] == cls[c, g]
            y = x + sigma * z[0]
            want = lo if y < lo else (hi if y > hi else y)
            clamped += want != y
            assert C[c, g] == want, (c, g)
    assert clamped > 0   # the bounds were exercised
    assert np.all((C >= lo) & (C <= hi))


def test_keys(orc):
    rng = np.random.Generator(np.random.PCG64(6))
    P = rng.uniform(-1, 1, (300, 8))
    F = rng.uniform(0, 1, 300)
    a = orc.ea_step(P, F, 2, 1, 40, 0, 0.2, 0.1, -5, 5)
    b = orc.ea_step(P, F, 2, 1, 40, 0, 0.2, 0.1, -5, 5)
    c = orc.ea_step(P, F, 2, 1, 40, 1, 0.2, 0.1, -5, 5)
    d = orc.ea_step(P, F, 2, 1, 43, 0, 0.2, 0.1, -5, 5)
    assert a[0].tobytes() == b[0].tobytes() and np.array_equal(a[1], b[1])
    for other in (c, d):
        assert np.mean(a[1] == other[1]) < 0.1
        assert np.mean(a[2] == other[2]) < 0.95


def _python_winners(orc, F, k, seed, stream, gen):
    """The tournament recomputed from its words: draw t of child c is
    (W(seed, stream, gen pop + c, t) pop) >> 64; the first draw of least
    fitness wins, a number replacing a NaN best."""
    pop = F.size
    out = []
    for c in range(pop):
        u = gen * pop + c
        best = None
        for t in range(k):
            i = (orc.word(orc.SM64, seed, stream, u, t) * pop) >> 64
            if best is None:
                best = i
            else:
                fi, fb = F[i], F[best]
                if fi < fb or (np.isnan(fb) and not np.isnan(fi)):
                    best = i
        out.append(best)
    return np.array(out)


def _fitness_patterns(pop):
    f_ties = np.floor(np.arange(pop) / 4.0)          # groups of equal fitness
    f_nan = np.arange(pop, dtype=np.float64)
    f_nan[::3] = np.nan
    return [f_ties, f_nan, np.zeros(pop)]


def test_winners_follow_the_draws(orc):
    """Which words a tournament reads, how a word becomes an index, ties
    (the earlier draw keeps the win) and NaN, against the tournament
    recomputed from the words."""
    pop = 97
    P = np.zeros((pop, 1))
    for F in _fitness_patterns(pop):
        for k, gen in ((1, 0), (2, 5), (5, 1)):
            _, W, _, _ = orc.ea_step(P, F, k, 77, 9, gen, 0.0, 0.0, -1, 1)
            assert np.array_equal(W, _python_winners(orc, F, k, 77, 9, gen)), (k, gen)


C_MUTANTS = [
    ("winner is the largest fitness", "if (fi < fb || (isnan(fb) && !isnan(fi))) best = i;",
     "if (fi > fb || (isnan(fb) && !isnan(fi))) best = i;"),
    ("ties go to the later draw", "if (fi < fb || (isnan(fb) && !isnan(fi))) best = i;",
     "if (fi <= fb || (isnan(fb) && !isnan(fi))) best = i;"),
    ("NaN never replaced", "if (fi < fb || (isnan(fb) && !isnan(fi))) best = i;",
     "if (fi < fb) best = i;"),
    ("first draw skipped", "for (uint32_t t = 1; t < J->k; ++t) {",
     "for (uint32_t t = 2; t < J->k + 1; ++t) {"),
    ("index from the low bits", "return (uint32_t)(((unsigned __int128)W * pop) >> 64);",
     "return (uint32_t)(W % pop + (W >> 63));"),
    ("rate test on the wrong side",
     "if ((orc_sm64_word(J->seed, J->stream + 1, w, 0) >> 11) < J->rate53) {",
     "if ((orc_sm64_word(J->seed, J->stream + 1, w, 0) >> 11) >= J->rate53) {"),
    ("z from the rate's stream",
     "const double z = orc_zig_f64(J->T, ORC_SM64, J->seed, J->stream + 2, w, J->dmax, &cl);",
     "const double z = orc_zig_f64(J->T, ORC_SM64, J->seed, J->stream + 1, w, J->dmax, &cl);"),
    ("no clamp", "x = x < J->lo ? J->lo : (x > J->hi ? J->hi : x);", "(void)0;"),
]


def _battery(orc, L):
    failed = []
    try:
        return _battery_pins(orc, L, failed)
    except (ValueError, IndexError) as e:   # e.g. a winner index out of range
        return failed + [f"error: {e}"]


def _battery_pins(orc, L, failed):
    pop = 32
    cnt = _winner_counts(orc, pop, 2, 400, np.arange(pop, dtype=np.float64), L=L)
    i = np.arange(pop, dtype=np.float64)
    if not _chi2_p(cnt, ((pop - i) ** 2 - (pop - i - 1) ** 2) / pop ** 2) > 1e-6:
        failed.append("law")
    f = np.arange(pop, dtype=np.float64)
    f[::2] = np.nan
    c2 = _winner_counts(orc, pop, 2, 400, f, L=L)
    n = c2.sum()
    if not abs(c2[::2].sum() - n / 4) < Z_MAX * np.sqrt(n * 0.25 * 0.75):
        failed.append("nan")
    Pz = np.zeros((41, 1))
    for F in _fitness_patterns(41):
        _, Wz, _, _ = orc.ea_step(Pz, F, 3, 77, 9, 2, 0.0, 0.0, -1, 1, L=L)
        if not np.array_equal(Wz, _python_winners(orc, F, 3, 77, 9, 2)):
            failed.append("draws")
            break
    rng = np.random.Generator(np.random.PCG64(5))
    P = rng.uniform(-3, 3, (20, 30))
    F = rng.uniform(0, 1, 20)
    C, W, cls, _ = orc.ea_step(P, F, 2, 123, 20, 3, 0.3, 1.5, -3.5, 3.5, L=L)
    _, _, cls_p, _ = orc.ea_step(P, F, 2, 123, 20, 3, 0.1, 1.5, -3.5, 3.5, L=L)
    if abs(np.count_nonzero(cls_p != 255) / cls_p.size - 0.1) > 0.05:
        failed.append("rate")
    for c in range(20):
        for g in range(30):
            if cls[c, g] == 255:
                continue
            w = (3 * 20 + c) * 30 + g
            z, _, _ = orc.fill_f64(orc.SM64, 123, 22, w, 1, nthreads=1)
            y = P[W[c], g] + 1.5 * z[0]
            if C[c, g] != min(max(y, -3.5), 3.5):
                failed.append("value")
                break
        if "value" in failed:
            break
    return failed


def test_unplanted_ea_oracle_passes(orc):
    assert _battery(orc, coracle.lib()) == []


@pytest.mark.parametrize("name,old,new", C_MUTANTS, ids=[m[0] for m in C_MUTANTS])
def test_ea_mutant_fails_a_pin(orc, tmp_path, name, old, new):
    src = open(coracle.SRC).read()
    assert src.count(old) == 1, f"target of '{name}' not found once"
    path = tmp_path / "zg_oracle_ea_mutant.c"
    path.write_text(src.replace(old, new))
    so = str(tmp_path / "libzg_oracle_ea_mutant.so")
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-pthread", str(path), "-o", so, "-lm"], check=True)
    L = coracle.load_variant(so)
    assert _battery(orc, L), f"planted mistake '{name}' passed every pin"
