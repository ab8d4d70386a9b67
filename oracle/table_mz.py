"""Oracle, part 1b: the table of McFarland's modified ziggurat in 60-digit
arithmetic.

TEST INFRASTRUCTURE ONLY.  The product library builds its own table; this
module shares no code with it.  It defines, as plainly as possible, the table
bits both sides must reproduce exactly (every real entry is the correctly
rounded value of its exact quantity; the alias table is exact integer
arithmetic on correctly rounded integer masses).

The method (McFarland 2016, the comparator of Sections 1 and 3, Java 17's
nextGaussian for SplittableRandom and the newer generators), as read here:

  f(x) = exp(-x^2/2) on x >= 0 (the sign is drawn separately), total mass
  T = sqrt(pi/2).  N = 256 equal-probability buckets of mass A = T/256.
  Layers fully under the curve, built from the bottom: layer 0 is the box
  [0, X_0] x [0, Y_0] with X_0 f(X_0) = A (X_0 > 1) and Y_0 = f(X_0); layer i
  is [0, X_i] x [Y_{i-1}, Y_i] with X_i (f(X_i) - Y_{i-1}) = A, X_i < X_{i-1},
  Y_i = f(X_i); as many layers as fit (L = 253 for N = 256).  The rest of the
  mass, (N - L) A, is in L + 1 regions: the tail R_0 = {x > X_0, y < f(x)}
  and, for 1 <= k <= L, the overhang R_k = {Y_{k-1} < y < Y_k,
  X_k < x < f^{-1}(y)} of strip k (with X_L = 0 and Y_L = 1 the top cap).
  Region masses a_0 = int_{X_0}^inf f, a_k = int_{X_k}^{X_{k-1}} (f - Y_{k-1}).
  An alias table of N buckets picks the region with probability a_k / sum a.

Stored entries (doubles are round-to-nearest of the exact values):
  xs[i]  = X_i 2^-63 (i < L): the fast-path multiplier of a signed 64-bit word
  x0     = X_0 (tail start), inv_x0 = 1/X_0
  ox[k]  = X_{k-1} (right edge of overhang k's box, k >= 1), odx[k] = X_{k-1} - X_k
  oy[k]  = Y_{k-1} (bottom), ody[k] = Y_k - Y_{k-1}
  kind[k]: 1 convex (X_k >= 1), 2 concave (X_{k-1} <= 1), 3 inflection, 0 tail
  thr[j], alias[j] (j < N): bucket j keeps its own region j (none for j > L)
  while a 63-bit uniform is below thr[j], else takes region alias[j].

Alias construction (exact, in integers; the library follows the same steps):
  masses m_k = round(a_k / sum a * N 2^63) for k <= L, corrected so that they
  sum to N 2^63 exactly (the rounding excess is taken from or given to the
  largest m, in index order among ties); buckets j > L have mass 0.  Buckets
  below 2^63 are "small", above are "large" (2^63 exactly: done, threshold
  2^63).  Repeatedly pair the lowest-index small j with the lowest-index large
  l: thr[j] = m_j, alias[j] = l, m_l -= 2^63 - m_j; l becomes small, done or
  stays large.  Leftover buckets get threshold 2^63 (they never alias).

Run as a script to (re)write oracle/table_mz256.json.
"""
from fractions import Fraction
import json
import os

import mpmath
from mpmath import mp, mpf

N_BUCKETS = 256
DPS = 60
TWO63 = 1 << 63


def f(x):
    return mpmath.exp(-x * x / 2)


def finv(y):
    return mpmath.sqrt(-2 * mpmath.log(y))


def _root(g, lo, hi, iters=240):
    """Bisection on [lo, hi] for a sign change of g (g(lo) > 0 > g(hi))."""
    lo, hi = mpf(lo), mpf(hi)
    for _ in range(iters):
        mid = (lo + hi) / 2
        if g(mid) > 0:
            lo = mid
        else:
            hi = mid
    return (lo + hi) / 2


def layers(n=N_BUCKETS):
    """X_i, Y_i of the layers that fit, and the bucket mass A."""
    with mp.workdps(DPS):
        T = mpmath.sqrt(mpmath.pi / 2)
        A = T / n
        # layer 0: x f(x) = A with x > 1 (x f(x) falls from e^-1/2 at x = 1)
        X = [_root(lambda x: x * f(x) - A, 1, 40)]
        Y = [f(X[0])]
        while True:
            prev = Y[-1]
            g = lambda x, prev=prev: x * (f(x) - prev) - A
            # g(X_{i-1}) = -A; the layer fits iff g rises above 0 on (0, X_{i-1}):
            # its maximum is found on a grid, then the root right of it
            grid = [X[-1] * k / 512 for k in range(1, 512)]
            vals = [g(x) for x in grid]
            k = max(range(len(vals)), key=lambda t: vals[t])
            if vals[k] <= 0:
                break
            X.append(_root(g, grid[k], X[-1]))
            Y.append(f(X[-1]))
        return X, Y, A, T


def regions(X, Y):
    """Masses of the tail and of the overhangs 1..L (L = len(X); the last is
    the cap under y = 1)."""
    with mp.workdps(DPS):
        L = len(X)
        Xe = list(X) + [mpf(0)]
        Ye = list(Y) + [mpf(1)]
        a = [mpmath.quad(f, [X[0], mpmath.inf])]
        for k in range(1, L + 1):
            a.append(mpmath.quad(lambda x, yl=Ye[k - 1]: f(x) - yl, [Xe[k], Xe[k - 1]]))
        return a, Xe, Ye


def alias_table(a, n=N_BUCKETS, unit=TWO63):
    """Integer masses (sum n unit) and the alias table of the regions'
    masses; thresholds are in units of 1/unit (unit = 2^(B-1) for B-bit
    words)."""
    with mp.workdps(DPS):
        tot = mpmath.fsum(a)
        scale = n * unit
        m = [int(mpmath.nint(ak / tot * scale)) for ak in a]
    excess = sum(m) - scale
    big = max(range(len(m)), key=lambda k: (m[k], -k))
    m[big] -= excess
    m += [0] * (n - len(m))
    thr = [unit] * n
    alias = list(range(n))
    small = [j for j in range(n) if m[j] < unit]
    large = [j for j in range(n) if m[j] > unit]
    while small and large:
        j = small.pop(0)
        l = large[0]
        thr[j] = m[j]
        alias[j] = l
        m[l] -= unit - m[j]
        if m[l] < unit:
            large.pop(0)
            small.append(l)
            small.sort()
        elif m[l] == unit:
            large.pop(0)
    return thr, alias


def rn64(x):
    """Round-to-nearest double of a high-precision value."""
    with mp.workdps(DPS):
        return float(mpf(x))


def build(n=N_BUCKETS, bits=64, ubits=53):
    """The table of n buckets for words of `bits` bits (slow-path uniforms of
    ubits bits): the real format is (256, 64, 53); tiny formats serve the
    exhaustive enumeration."""
    X, Y, A, T = layers(n)
    L = len(X)
    a, Xe, Ye = regions(X, Y)
    thr, alias = alias_table(a, n, 1 << (bits - 1))
    with mp.workdps(DPS):
        tab = {
            "n_buckets": n, "n_layers": L, "bits": bits, "ubits": ubits,
            "A": str(A), "X": [str(x) for x in X], "Y": [str(y) for y in Y],
            "masses": [str(v) for v in a],
            "xs": [rn64(x * mpf(2) ** -(bits - 1)) for x in X],
            "x0": rn64(X[0]), "inv_x0": rn64(1 / X[0]),
            "ox": [0.0] + [rn64(Xe[k - 1]) for k in range(1, L + 1)],
            "odx": [0.0] + [rn64(Xe[k - 1] - Xe[k]) for k in range(1, L + 1)],
            "oy": [0.0] + [rn64(Ye[k - 1]) for k in range(1, L + 1)],
            "ody": [0.0] + [rn64(Ye[k] - Ye[k - 1]) for k in range(1, L + 1)],
            "kind": [0] + [1 if Xe[k] >= 1 else (2 if Xe[k - 1] <= 1 else 3)
                           for k in range(1, L + 1)],
            "thr": [str(t) for t in thr], "alias": alias,
        }
    return tab


PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "table_mz256.json")


def load(path=PATH):
    with open(path) as fh:
        return json.load(fh)


if __name__ == "__main__":
    t = build()
    with open(PATH, "w") as fh:
        json.dump(t, fh, indent=0)
    print(PATH, t["n_layers"], "layers; x0 =", t["X"][0][:22])
