"""Comparison rules between the HIP path and the oracle.

- Fast-path variates (accepted by the integer test of a first word, on any
  attempt) must be bit-identical, signed zeros included.
- Variates accepted after a wedge or tail test must be within 2 ulp: the wedge
  value is exact by construction, the tail value goes through log, whose device
  and host implementations may differ by an ulp.
- A variate whose value differs beyond that is an accept-decision disagreement
  (exp/log on either side landed on the other side of a threshold); the count
  must be at most 1e-9 per variate.
- Polar method: its accept test (s >= 1 or s == 0) involves no transcendental
  and is exact on both sides; every value goes through log (1 ulp apart at
  most between the two libraries), a correctly rounded division and square
  root, and a multiply, so every value must be within 4 ulp.
- Mutated values x = clamp(RN(x0 + RN(sigma z))): a fast-path z is bit-exact,
  so x is too; a wedge or tail z within 2 ulp of the oracle's moves x by at
  most 2 |sigma| ulp(z) (the variates' difference, scaled) + 2 ulp(sigma z)
  (the product's roundings on both sides) + 2 ulp(x) (the sum's), which is
  many ulps of x when x is much smaller than sigma z.  The clamp only brings
  values together.
"""
import numpy as np

ULP_SLOW = 2
ULP_POLAR = 4
DISAGREE_RATE = 1e-9


def ulp_distance(a, b):
    """|a - b| in units in the last place, by ordered integer mapping."""
    a = np.asarray(a)
    b = np.asarray(b)
    if a.dtype == np.float64:
        ia = a.view(np.int64)
        ib = b.view(np.int64)
        big = np.int64(-0x8000000000000000)
    else:
        ia = a.view(np.int32).astype(np.int64)
        ib = b.view(np.int32).astype(np.int64)
        big = np.int64(-0x80000000)
    oa = np.where(ia < 0, big - ia, ia)
    ob = np.where(ib < 0, big - ib, ib)
    # same sign: the int64 difference is exact; opposite signs: far apart
    same = (oa >= 0) == (ob >= 0)
    diff = np.abs(np.where(same, oa - ob, 0)).astype(np.float64)
    far = np.abs(oa.astype(np.float64)) + np.abs(ob.astype(np.float64))
    return np.where(same, diff, far)


def compare_polar(gpu, orc_vals, label=""):
    gpu = np.asarray(gpu)
    orc_vals = np.asarray(orc_vals)
    nan_both = np.isnan(gpu) & np.isnan(orc_vals)
    d = ulp_distance(gpu, orc_vals)
    bad = np.flatnonzero(~nan_both & ~(d <= ULP_POLAR))
    rep = dict(n=gpu.size, exact=int(np.count_nonzero(d == 0)), ulp_max=float(d[~nan_both].max()) if np.any(~nan_both) else 0.0)
    assert bad.size == 0, (label, "polar beyond 4 ulp", rep, [(int(i), gpu[i], orc_vals[i]) for i in bad[:5]])
    return rep


def compare(gpu, orc_vals, orc_cls, label="", polar=False):
    """Applies the rules; returns a report dict and asserts the bar."""
    if polar:
        return compare_polar(gpu, orc_vals, label)
    gpu = np.asarray(gpu)
    orc_vals = np.asarray(orc_vals)
    n = gpu.size
    assert orc_vals.size == n
    same_bits = gpu.view(np.uint8).reshape(n, -1).tobytes() == orc_vals.view(np.uint8).reshape(n, -1).tobytes()
    if same_bits:
        return dict(n=n, exact=n, slow_ulp_max=0, disagreements=0)
    eq = gpu.view(np.uint64 if gpu.dtype == np.float64 else np.uint32) == \
        orc_vals.view(np.uint64 if gpu.dtype == np.float64 else np.uint32)
    path = orc_cls & 3
    fast = path == 0
    # fast path (on any attempt): bit exact
    bad_fast = np.flatnonzero(fast & ~eq)
    slow = ~fast & (path != 3)
    d = ulp_distance(gpu, orc_vals)
    nan_both = np.isnan(gpu) & np.isnan(orc_vals)
    within = (d <= ULP_SLOW) | nan_both
    disagree = np.flatnonzero(slow & ~within)
    budget = np.flatnonzero((path == 3) & ~nan_both)
    rep = dict(n=n, exact=int(eq.sum()), slow_ulp_max=float(d[slow & within].max()) if np.any(slow & within) else 0.0,
               disagreements=int(disagree.size), bad_fast=bad_fast[:10].tolist(),
               budget_mismatch=budget[:10].tolist())
    assert bad_fast.size == 0, (label, "fast-path mismatch", rep,
                                [(int(i), gpu[i], orc_vals[i]) for i in bad_fast[:5]])
    assert budget.size == 0, (label, "budget NaN mismatch", rep)
    assert disagree.size <= DISAGREE_RATE * n, (label, "decision disagreements", rep,
                                                 [(int(i), gpu[i], orc_vals[i], int(orc_cls[i])) for i in disagree[:5]])
    return rep


def compare_mutated(gpu, orc_vals, orc_cls, z_of, sigma, label=""):
    """The rules for mutated values (see the module notes); z_of(indices)
    gives the oracle's variates z of the given elements (called only for the
    few slow-path elements whose values differ)."""
    gpu = np.asarray(gpu, dtype=np.float64)
    orc_vals = np.asarray(orc_vals, dtype=np.float64)
    n = gpu.size
    assert orc_vals.size == n
    eq = gpu.view(np.uint64) == orc_vals.view(np.uint64)
    path = orc_cls & 3
    fast = path == 0
    bad_fast = np.flatnonzero(fast & ~eq)
    assert bad_fast.size == 0, (label, "fast-path mismatch",
                                [(int(i), gpu[i], orc_vals[i]) for i in bad_fast[:5]])
    nan_both = np.isnan(gpu) & np.isnan(orc_vals)
    budget = np.flatnonzero((path == 3) & ~nan_both)
    assert budget.size == 0, (label, "budget NaN mismatch", budget[:10].tolist())
    diff = np.flatnonzero((path != 0) & (path != 3) & ~eq & ~nan_both)
    if diff.size == 0:
        return dict(n=n, exact=int(eq.sum()), differ=0, disagreements=0)
    z = np.asarray(z_of(diff), dtype=np.float64)
    # each rounding may fall on either side of a binade edge: 2 ulp per rounding
    bound = (2.0 * abs(sigma) * np.spacing(np.abs(z)) + 2.0 * np.spacing(np.abs(sigma * z)) +
             2.0 * np.spacing(np.abs(orc_vals[diff])))
    within = np.abs(gpu[diff] - orc_vals[diff]) <= bound
    disagree = diff[~within]
    rep = dict(n=n, exact=int(eq.sum()), differ=int(diff.size), disagreements=int(disagree.size),
               worst_over_bound=float((np.abs(gpu[diff] - orc_vals[diff]) / bound).max()))
    assert disagree.size <= DISAGREE_RATE * n, (label, "decision disagreements", rep,
                                                 [(int(i), gpu[i], orc_vals[i], int(orc_cls[i]))
                                                  for i in disagree[:5]])
    return rep


def mutation_z(orc, kind, seed, s, first):
    """z_of for a mutation keyed (kind, seed, stream s, first index): element
    i was moved by the oracle's FP64 ziggurat variate first + i."""
    def z_of(idx):
        return np.array([orc.fill_f64(kind, seed, s, first + int(i), 1)[0][0] for i in idx])
    return z_of
