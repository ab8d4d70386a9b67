"""Oracle, part 1: the 128-layer ziggurat table in 60-digit arithmetic.

TEST INFRASTRUCTURE ONLY. The product library builds its own table; this module
shares no code with it.  Its purpose is to define, as plainly as possible, the
FP64/FP32 table bits that both sides must reproduce exactly: every stored entry
is the correctly rounded value of the exact mathematical quantity.

What is computed (the original ziggurat the paper ports from GSL, Section 1 and
Section 2 "Ziggurat": Marsaglia-Tsang 2000 / Leong 2005):

  f(x) = exp(-x^2/2), N = 128 equal-area layers.
  Reading B (chosen): the base layer is the box [0,r]x[0,f(r)] plus the mass of
  the exponential majorant f(r)*exp(-r(x-r)) beyond r, so
        v = r f(r) + f(r)/r.
  Reading A (kept only to pin the machinery against the constants Marsaglia and
  Tsang print for their 128-layer normal): v = r f(r) + int_r^inf f.
  b_0 = r,   b_i = f^{-1}( f(b_{i-1}) + v/b_{i-1} ),  i = 1..N-2,
  and r is the root of the closure condition  f(b_{N-2}) + v/b_{N-2} = 1
  (the top layer [0,b_{N-2}] x [f(b_{N-2}), 1] then also has area v).
  Layer widths: W_0 = v/f(r) (virtual box of area v), W_i = b_{i-1} (i >= 1).
  Fast-accept fraction q_0 = r/W_0, q_i = b_i/W_i, q_{N-1} = 0.
  Heights y_i = f(b_i) (y_{N-1} = 1), dy_i = y_i - y_{i-1}.
  Integer thresholds k53_i = floor(q_i 2^53), k24_i = floor(q_i 2^24).
  Scaled widths w53_i = RN64(W_i) 2^-53, w24_i = RN32(W_i) 2^-24.

Run as a script to (re)write oracle/table_b128.json, the stored oracle table.
"""
from fractions import Fraction
import json
import os

import mpmath
from mpmath import mp, mpf

N_LAYERS = 128
DPS = 60


def f(x):
    return mpmath.exp(-x * x / 2)


def finv(y):
    return mpmath.sqrt(-2 * mpmath.log(y))


def base_area(r, reading):
    """Area v of every layer as a function of r (reading 'B' or 'A')."""
    fr = f(r)
    if reading == "B":
        return r * fr + fr / r
    if reading == "A":
        # int_r^inf exp(-x^2/2) dx = sqrt(pi/2) erfc(r/sqrt 2)
        return r * fr + mpmath.sqrt(mpmath.pi / 2) * mpmath.erfc(r / mpmath.sqrt(2))
    raise ValueError(reading)


def closure(r, reading, n=N_LAYERS):
    """Closure residual g(r) = f(b_{n-2}) + v/b_{n-2} - 1 (decreasing in r).

    Returns +1 if the stack of layers already reaches the top before layer
    n-2 (r too small), which keeps bisection monotone.
    """
    v = base_area(r, reading)
    b = r
    for _ in range(1, n - 1):
        t = f(b) + v / b
        if t >= 1:
            return mpf(1)
        b = finv(t)
    return f(b) + v / b - 1


def solve_r(reading="B", n=N_LAYERS, lo=0.5, hi=5.0, iters=230):
    """Bisection for the closure root; 230 halvings of [0.5, 5] exceed 60 digits."""
    with mp.workdps(DPS):
        lo, hi = mpf(lo), mpf(hi)
        assert closure(lo, reading, n) > 0 and closure(hi, reading, n) < 0
        for _ in range(iters):
            mid = (lo + hi) / 2
            if closure(mid, reading, n) > 0:
                lo = mid
            else:
                hi = mid
        return (lo + hi) / 2


def exact_layers(reading="B", n=N_LAYERS):
    """All layer quantities as 60-digit mpf values (lists of length n)."""
    with mp.workdps(DPS):
        r = solve_r(reading, n)
        v = base_area(r, reading)
        b = [r]
        for _ in range(1, n - 1):
            b.append(finv(f(b[-1]) + v / b[-1]))
        b.append(mpf(0))                       # b_{n-1} = 0: top layer
        W = [v / f(r)] + [b[i - 1] for i in range(1, n)]
        q = [b[i] / W[i] for i in range(n)]    # q_{n-1} = 0
        y = [f(b[i]) for i in range(n - 1)] + [mpf(1)]
        dy = [mpf(0)] + [y[i] - y[i - 1] for i in range(1, n)]
        return dict(r=r, v=v, b=b, W=W, q=q, y=y, dy=dy)


def to_fraction(x):
    """Exact rational value of an mpf."""
    sign, man, exp, _ = x._mpf_
    val = Fraction(man) * (Fraction(2) ** exp)
    return -val if sign else val


def round_binary(x, mant_bits):
    """Correctly rounded (nearest, ties to even) binary float with mant_bits
    significant bits, returned as an exact Fraction (no overflow handling: the
    table values are all normal numbers)."""
    fr = to_fraction(x) if not isinstance(x, Fraction) else x
    if fr == 0:
        return Fraction(0)
    neg = fr < 0
    a = -fr if neg else fr
    e = 0
    while a >= 2:
        a /= 2
        e += 1
    while a < 1:
        a *= 2
        e -= 1
    scaled = a * (1 << (mant_bits - 1))
    m = scaled.numerator // scaled.denominator
    rem = scaled - m
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and m % 2 == 1):
        m += 1
    val = Fraction(m, 1 << (mant_bits - 1)) * (Fraction(2) ** e)
    return -val if neg else val


def rn64(x):
    return float(round_binary(x, 53))


def rn32_as_float(x):
    """RN32(x), returned as the (exactly representable) Python float."""
    return float(round_binary(x, 24))


def floor_scaled(x, bits):
    fr = to_fraction(x) * (1 << bits)
    return fr.numerator // fr.denominator


def build_table(reading="B", n=N_LAYERS):
    """The stored oracle table: correctly rounded FP64 (and FP32) entries."""
    L = exact_layers(reading, n)
    t = {
        "reading": reading,
        "n": n,
        "r": rn64(L["r"]),
        "v": rn64(L["v"]),
        "W": [rn64(w) for w in L["W"]],
        "y": [rn64(y) for y in L["y"]],
        "dy": [rn64(d) for d in L["dy"]],
        "k53": [floor_scaled(q, 53) for q in L["q"]],
        "k24": [floor_scaled(q, 24) for q in L["q"]],
        "w24f": [rn32_as_float(w) for w in L["W"]],
    }
    t["w53"] = [w * 2.0 ** -53 for w in t["W"]]
    t["w24"] = [w * 2.0 ** -24 for w in t["w24f"]]
    t["w24d"] = [w * 2.0 ** -24 for w in t["W"]]
    return t, L


TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "table_b128.json")


def _hex_table(t):
    out = {}
    for key, val in t.items():
        if isinstance(val, list) and val and isinstance(val[0], float):
            out[key] = [x.hex() for x in val]
        elif isinstance(val, float):
            out[key] = val.hex()
        else:
            out[key] = val
    return out


def load_table(path=TABLE_PATH):
    """Stored oracle table with floats decoded from their hex form."""
    with open(path) as fh:
        raw = json.load(fh)
    t = {}
    for key, val in raw.items():
        if isinstance(val, list) and val and isinstance(val[0], str):
            t[key] = [float.fromhex(x) for x in val]
        elif isinstance(val, str) and key not in ("reading",):
            t[key] = float.fromhex(val)
        else:
            t[key] = val
    return t


def main():
    t, L = build_table("B")
    with mp.workdps(30):
        meta = {"r_60": mpmath.nstr(L["r"], 40), "v_60": mpmath.nstr(L["v"], 40)}
    doc = _hex_table(t)
    doc["exact"] = meta
    with open(TABLE_PATH, "w") as fh:
        json.dump(doc, fh, indent=0)
    print("wrote", TABLE_PATH, "r =", meta["r_60"])


if __name__ == "__main__":
    main()
