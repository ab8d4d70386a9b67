"""Pins of the oracle's own accept/reject code, as batteries that a test runs
on the oracle and on copies of it with a mistake planted (tests/test_oracle_
mutants.py).  Each pin returns None when it holds, else a message.

What fixes each pin, independently of the oracle:
- law: on a small table (8 layers, 12 bits of j and of each extra uniform),
  every first word and every extra uniform is enumerated through the
  oracle's own attempt function.  The exact acceptance per attempt must then
  be sqrt(pi/2)/(N v), the accepted mass per bin of |x| the half-normal
  probabilities, and the accepted base-strip mass erfc(r/sqrt 2), each to
  within the grid's discretisation (below 2^-bits).  This is the law of the
  original ziggurat (Sections 1-2: an exact sampler of the normal density).
- boundary: the fast test is the integer j < k_i with k_i = floor(q_i 2^53)
  (the inner box of the layer), for all 128 layers and both signs; the sign
  bit set means negative and -0.0 is produced for j = 0.
- consumption: rejection sampling needs fresh uniforms for each attempt, so
  no word may be read twice within one variate; a wedge attempt reads 2
  words, a base-strip attempt 3, and the next attempt starts at the next
  unread word (crafted word tapes).
- extreme tail: U+ lies in (0, 1], so the smallest word gives the largest
  output, finite: r + 53 ln 2 / r.
- strict wedge: where y equals exp(-x^2/2) exactly the attempt is rejected
  (the strict comparison; the two comparisons differ on measure zero, so no
  law can tell them apart, and the crafted word pins the reading).
"""
import math

import mpmath

J53 = (1 << 53) - 1


def word(i, neg, j, low=0b101):
    """First word of an attempt with layer i, sign, and j (bits 3..55)."""
    return (i << 57) | (neg << 56) | (j << 3) | low


def uword(m):
    """Word whose U = m 2^-53 (and U+ = (m + 1) 2^-53)."""
    return m << 11


def law_errors(enum, n, bits, L, twin):
    """Errors of an exhaustive one-attempt enumeration against the exact law;
    enum(T, n, bits, edges) returns (acc, per_bin, tail_acc, total)."""
    T = twin.TwinTable(n, bits, exact=L)
    edges = sorted({0.0, 0.5, 1.0, 1.5, 2.0, 2.5, T.r, 40.0})
    acc, per_bin, tail_acc, total = enum(T, n, bits, edges)
    exp_acc = math.sqrt(math.pi / 2) / (n * float(L["v"]))
    bin_err = max(abs(per_bin[k] / acc - (twin.half_normal_cdf(edges[k + 1]) -
                                          twin.half_normal_cdf(edges[k])))
                  for k in range(len(edges) - 1))
    tail_err = tail_acc / acc - math.erfc(T.r / math.sqrt(2))
    return acc / total - exp_acc, bin_err, tail_err


def _law_pin(enum, n, bits, L, twin):
    try:
        e = law_errors(enum, n, bits, L, twin)
    except AssertionError as ex:
        return f"enumeration check failed: {ex}"
    if max(abs(v) for v in e) >= 2.0 ** -bits:
        return f"law errors {e} at {n} layers, {bits} bits"
    return None


def _equal_wedge_case(t, i, j):
    """(x, m) with y_{i-1} + (m 2^-53) dy_i == exp(-x^2/2) exactly, x = j w53_i,
    or None.  y(m) is non-decreasing in m and steps far below an ulp of y, so
    every double between y_{i-1} and y_i is hit by some m."""
    x = float(j) * t["w53"][i]
    e = math.exp(-0.5 * (x * x))
    lo, hi = 0, J53

    def y(m):
        return t["y"][i - 1] + (m * 2.0 ** -53) * t["dy"][i]

    if not (y(lo) <= e <= y(hi)):
        return None
    while lo < hi:
        mid = (lo + hi) // 2
        if y(mid) < e:
            lo = mid + 1
        else:
            hi = mid
    return (x, lo) if y(lo) == e else None


def run_battery(t, variate, decide, enum, twin, laws):
    """t: the real table (dict with r, W, y, dy, w53, k53); variate(tape)
    returns (value, draw indices read) for one FP64 variate from crafted
    words; decide(W) returns (class 0/1/2, signed first-word candidate), or
    is None; enum as in law_errors; laws: (layers, bits, exact layers) of the
    small tables to enumerate.  Returns {pin: None or message}."""
    res = {}
    for n, bits, L in laws:
        res[f"law{n}_{bits}"] = _guard(lambda: _law_pin(enum, n, bits, L, twin))
    res["boundary"] = _guard(lambda: _boundary(t, variate, decide))
    res["consumption"] = _guard(lambda: _consumption(t, variate))
    res["extreme_tail"] = _guard(lambda: _extreme_tail(t, variate))
    res["strict_wedge"] = _guard(lambda: _strict_wedge(t, variate))
    return res


def _guard(fn):
    try:
        return fn()
    except Exception as ex:  # a planted mistake may raise instead of returning
        return f"raised {type(ex).__name__}: {ex}"


FAST_TAIL = word(20, 0, 1000)


def _boundary(t, variate, decide):
    """Boundary words and signs."""
    msg = None
    fast_tail = FAST_TAIL
    for i in range(128):
        k = t["k53"][i]
        for neg in (0, 1):
            for j in sorted({max(k - 1, 0), k, min(k + 1, J53), 0, J53}):
                W = word(i, neg, j)
                want_fast = j < k
                if decide is not None:
                    c, x = decide(W)
                    xv = float(j) * t["w53"][i]
                    want_c = 0 if want_fast else (2 if i == 0 else 1)
                    if c != want_c or math.copysign(1.0, x) != (-1.0 if neg else 1.0) or abs(x) != xv:
                        msg = msg or f"decide({i},{neg},{j}) = {c},{x}"
                if want_fast:
                    v, reads = variate([W, uword(0), uword(0), fast_tail])
                    xv = float(j) * t["w53"][i]
                    if reads != [0] or v != (-xv if neg else xv) or \
                            math.copysign(1.0, v) != (-1.0 if neg else 1.0):
                        msg = msg or f"fast word ({i},{neg},{j}) gave {v} reading {reads}"
    return msg


def _consumption(t, variate):
    """Consumption order on crafted tapes."""
    fast_tail = FAST_TAIL
    msg = None
    x_fast = 1000 * t["w53"][20]
    cases = {
        # wedge rejected (x near the layer's outer edge, U near 1), then a fast word
        "wedge_reject": ([word(10, 0, J53), uword(J53), fast_tail], [0, 1, 2], x_fast),
        # base strip rejected (U2 near 1), then a fast word
        "tail_reject": ([word(0, 1, J53), uword(1 << 52), uword(J53), fast_tail], [0, 1, 2, 3],
                        x_fast),
        # wedge accepted at once (x at the inner box edge, U = 0)
        "wedge_accept": ([word(10, 1, t["k53"][10]), uword(0), fast_tail], [0, 1],
                         -(t["k53"][10] * t["w53"][10])),
    }
    for name, (tape, want_reads, want_v) in cases.items():
        v, reads = variate(tape)
        if len(set(reads)) != len(reads):
            msg = msg or f"{name}: a word read twice {reads}"
        elif reads != want_reads or v != want_v:
            msg = msg or f"{name}: value {v} reading {reads}, want {want_v} reading {want_reads}"
    # base strip accepted: r - log(U+)/r with U+ = 1/2 + 2^-53, U2 = 0
    v, reads = variate([word(0, 0, J53), uword(1 << 52), uword(0), fast_tail])
    with mpmath.workdps(40):
        want = mpmath.mpf(t["r"]) - mpmath.log(mpmath.mpf(0.5) + mpmath.mpf(2) ** -53) / t["r"]
    if reads != [0, 1, 2] or abs(v - float(want)) > 4 * math.ulp(float(want)):
        msg = msg or f"tail_accept: value {v} reading {reads}, want {float(want)}"
    return msg


def _extreme_tail(t, variate):
    """The largest output: U+ = 2^-53, U2 = 0."""
    fast_tail = FAST_TAIL
    v, reads = variate([word(0, 0, J53), uword(0), uword(0), fast_tail])
    with mpmath.workdps(40):
        want = float(mpmath.mpf(t["r"]) + 53 * mpmath.log(2) / t["r"])
    return None if (reads == [0, 1, 2] and math.isfinite(v) and
                    abs(v - want) <= 4 * math.ulp(want)) else \
        f"smallest U+ gave {v} reading {reads}, want {want}"


def _strict_wedge(t, variate):
    """Strict wedge comparison at an exact tie."""
    fast_tail = FAST_TAIL
    x_fast = 1000 * t["w53"][20]
    msg = None
    found = 0
    for i, j in ((127, 1 << 52), (127, 3 << 51), (64, J53), (30, J53 - 12345), (100, J53 >> 1)):
        if j < t["k53"][i]:
            continue
        case = _equal_wedge_case(t, i, j)
        if case is None:
            continue
        found += 1
        x, m = case
        v, reads = variate([word(i, 0, j), uword(m), fast_tail])
        if reads != [0, 1, 2] or v != x_fast:
            msg = msg or f"tie at layer {i}: accepted ({v}, reading {reads})"
    if found == 0:
        msg = "no exact tie found"
    return msg
