"""Pure-Python twin of the oracle's ziggurat, parametrised by layer count and
word format, for brute-force enumeration on tiny tables.

TEST INFRASTRUCTURE ONLY.  Python floats are IEEE binary64 and math.exp/log
are the platform libm, so with the real format (128 layers, 64-bit words) the
twin must reproduce the C oracle bit for bit; with tiny formats (4 or 8
layers, a few bits of j and U) every first word and every extra uniform can be
enumerated, which pins the accept/reject logic to the geometry exactly.

Algorithm (original ziggurat after Marsaglia-Tsang / Leong, as ported from GSL
in Section 1 and Section 2 "Ziggurat"), one attempt for a first word:
  layer i, sign, integer j (J bits) from the word; x = j * (W_i 2^-J).
  fast accept iff j < k_i = floor(q_i 2^J);
  wedge (i >= 1): y = y_{i-1} + U dy_i, accept iff y < exp(-x^2/2);
  tail  (i == 0): a = -log(U1+)/r, x = r + a, accept iff U2 < exp(-a^2/2);
  any rejection restarts the whole attempt with fresh words.
"""
import math
from dataclasses import dataclass

from . import table_mp


@dataclass(frozen=True)
class WordFormat:
    """Bit layout of one uniform word: layer index in the top lbits, then one
    sign bit; j = (W >> jshift) & (2^jbits - 1); U = (W >> ushift) 2^-ubits."""
    bits: int
    lbits: int
    jbits: int
    jshift: int
    ubits: int
    ushift: int

    def decode(self, W):
        i = W >> (self.bits - self.lbits)
        neg = (W >> (self.bits - self.lbits - 1)) & 1
        j = (W >> self.jshift) & ((1 << self.jbits) - 1)
        return i, neg, j

    def u(self, W):
        return (W >> self.ushift) * 2.0 ** -self.ubits

    def u_plus(self, W):
        return ((W >> self.ushift) + 1) * 2.0 ** -self.ubits


REAL = WordFormat(bits=64, lbits=7, jbits=53, jshift=3, ubits=53, ushift=11)


class TwinTable:
    """Float table for n layers at a j-width of jbits, from the exact layers."""

    def __init__(self, n, jbits, reading="B", exact=None):
        L = exact if exact is not None else table_mp.exact_layers(reading, n)
        self.n = n
        self.exact = L
        self.r = table_mp.rn64(L["r"])
        self.v = table_mp.rn64(L["v"])
        self.W = [table_mp.rn64(w) for w in L["W"]]
        self.y = [table_mp.rn64(y) for y in L["y"]]
        self.dy = [table_mp.rn64(d) for d in L["dy"]]
        self.k = [table_mp.floor_scaled(q, jbits) for q in L["q"]]
        self.w = [w * 2.0 ** -jbits for w in self.W]


def attempt(T, i, j, draw1=None, draw2=None, u_of=None, up_of=None):
    """One attempt given the decoded first word (layer i, integer j) and the
    extra words it may consume.  Returns (outcome, x) with outcome one of
    'fast', 'wedge_acc', 'wedge_rej', 'tail_acc', 'tail_rej'."""
    x = j * T.w[i]
    if j < T.k[i]:
        return "fast", x
    if i == 0:
        a = -math.log(up_of(draw1)) / T.r
        xt = T.r + a
        if u_of(draw2) < math.exp(-0.5 * (a * a)):
            return "tail_acc", xt
        return "tail_rej", xt
    y = T.y[i - 1] + u_of(draw1) * T.dy[i]
    if y < math.exp(-0.5 * (x * x)):
        return "wedge_acc", x
    return "wedge_rej", x


def variate(T, fmt, word, dmax=256):
    """Full sampler for one variate: word(d) returns the d-th word of this
    variate.  Returns (value, path, attempts); value is NaN if the draw budget
    would be exceeded."""
    d = 0
    attempts = 0
    while True:
        if d >= dmax:
            return math.nan, 3, attempts + 1
        W = word(d)
        i, neg, j = fmt.decode(W)
        attempts += 1
        if j < T.k[i]:
            x = j * T.w[i]
            return (-x if neg else x), 0, attempts
        need = d + 2 if i == 0 else d + 1
        if need >= dmax:
            return math.nan, 3, attempts
        out, x = attempt(T, i, j, word(d + 1), word(d + 2) if i == 0 else None,
                         fmt.u, fmt.u_plus)
        if out.endswith("_acc"):
            return (-x if neg else x), (2 if i == 0 else 1), attempts
        d += 3 if i == 0 else 2


def half_normal_cdf(x):
    """P(|Z| <= x) for a standard normal Z."""
    return math.erf(x / math.sqrt(2.0))


def enumerate_attempt_mass(T, jbits, ubits, edges, attempt_fn=None):
    """Exhaustive enumeration of one attempt over every first word (layer i,
    j of jbits bits) and every extra uniform on a grid of G = 2^ubits points,
    each decision made by `attempt` itself (or by attempt_fn, same signature).

    The grid uniforms are U = m/G and U+ = (m+1)/G.  Every outcome has
    probability weight / (n 2^jbits G^2), with integer weights: a first word
    weighs G^2, a wedge uniform G, a base-strip pair 1.  Returns (accepted
    weight, accepted weight per bin of |x| between consecutive `edges`,
    accepted base-strip weight, total weight).  The sign bit only mirrors the
    output and is left out.  The base-strip decisions do not involve j: they
    are enumerated for the first slow j of layer 0, checked equal for the last
    one, and weighted by the number of slow j."""
    fn = attempt_fn or attempt
    n = T.n
    G = 1 << ubits
    J = 1 << jbits
    nb = len(edges) - 1
    per_bin = [0] * nb
    acc = 0
    tail_acc = 0
    us = [m / G for m in range(G)]
    ups = [(m + 1) / G for m in range(G)]

    def put(x, w):
        for b in range(nb):
            if edges[b] <= x < edges[b + 1]:
                per_bin[b] += w
                return

    def u_of(u):
        return u

    for i in range(n):
        slow = []
        for j in range(J):
            out, x = fn(T, i, j, 0.5, 0.5, u_of, u_of)
            if out == "fast":
                acc += G * G
                put(x, G * G)
                continue
            slow.append(j)
            if i == 0:
                continue
            for u in us:
                out, x = fn(T, i, j, u, None, u_of, u_of)
                if out == "wedge_acc":
                    acc += G
                    put(x, G)
        if i == 0 and slow:
            for u1 in ups:
                for u2 in us:
                    out, x = fn(T, 0, slow[0], u1, u2, u_of, u_of)
                    out_b, x_b = fn(T, 0, slow[-1], u1, u2, u_of, u_of)
                    assert (out, x) == (out_b, x_b), "base-strip decision depends on j"
                    if out == "tail_acc":
                        acc += len(slow)
                        tail_acc += len(slow)
                        put(x, len(slow))
    total = n * J * G * G
    return acc, per_bin, tail_acc, total


def variate_f32(T24, T53, word, sm64_pair_word=None, v=0, dmax=256):
    """FP32-mode sampler (twin of the oracle's FP32 mode).  T24 is a TwinTable at
    jbits = 24 (k24 thresholds), T53 the FP64 table; word(d) gives the 64-bit
    word of draw d.  For the SplitMix64 kind the first attempt uses half of the
    pair word W(s, v>>1, 0): the high half for even v, the low half for odd v
    (pass sm64_pair_word); otherwise the attempt word is hi32(word(d)).
    Returns (float32 value as numpy.float32, path, attempts)."""
    import numpy as np
    d = 0
    attempts = 0
    while True:
        if d >= dmax:
            return np.float32(np.nan), 3, attempts + 1
        if d == 0 and sm64_pair_word is not None:
            u = (sm64_pair_word & 0xFFFFFFFF) if (v & 1) else (sm64_pair_word >> 32)
        else:
            u = word(d) >> 32
        i = u >> 25
        neg = (u >> 24) & 1
        j = u & 0xFFFFFF
        attempts += 1
        if j < T24.k[i]:
            w24 = np.float32(table_mp.rn32_as_float(T24.exact["W"][i])) * np.float32(2.0 ** -24)
            xf = np.float32(j) * w24
            return (-xf if neg else xf), 0, attempts
        x = j * (T53.W[i] * 2.0 ** -24)
        need = d + 2 if i == 0 else d + 1
        if need >= dmax:
            return np.float32(np.nan), 3, attempts
        out, xo = _slow(T53, i, x, word, d)
        if out:
            return np.float32(-xo if neg else xo), (2 if i == 0 else 1), attempts
        d += 3 if i == 0 else 2


def _slow(T, i, x, word, d):
    """Wedge or tail step for layer i with candidate x at draw d (64-bit words)."""
    if i == 0:
        a = -math.log(REAL.u_plus(word(d + 1))) / T.r
        xt = T.r + a
        return REAL.u(word(d + 2)) < math.exp(-0.5 * (a * a)), xt
    y = T.y[i - 1] + REAL.u(word(d + 1)) * T.dy[i]
    return y < math.exp(-0.5 * (x * x)), x


def polar_pair(word, dmax=256):
    """Polar method for one pair: attempt a uses words 2a and 2a+1 (U in
    [0,1) from the top 53 bits).  Returns (z1, z2, attempts) or NaNs when
    the draw budget is exhausted."""
    a = 0
    while True:
        if 2 * a + 1 >= dmax:
            return math.nan, math.nan, a + 1
        v1 = 2.0 * REAL.u(word(2 * a)) - 1.0
        v2 = 2.0 * REAL.u(word(2 * a + 1)) - 1.0
        s = v1 * v1 + v2 * v2
        if not (s >= 1.0 or s == 0.0):
            m = math.sqrt(-2.0 * math.log(s) / s)
            return v1 * m, v2 * m, a + 1
        a += 1


MASK64 = (1 << 64) - 1
MASK48 = (1 << 48) - 1
GAMMA = 0x9E3779B97F4A7C15


def sm64_word(seed, s, v, d):
    """SplitMix64 keyed word: mix64(seed + gamma (1 + s 2^48 + d 2^40 + v))."""
    z = (seed + GAMMA * (1 + (s << 48) + (d << 40) + v)) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def lcg_state(seed, k):
    """java.util.Random state after k steps, by summing the geometric series
    c (a^k - 1)/(a - 1) exactly in integers before reducing mod 2^48."""
    a, c = 0x5DEECE66D, 0xB
    s0 = (seed ^ a) & MASK48
    ak = pow(a, k, 1 << 48)
    # (a^k - 1)/(a - 1) mod 2^48, computed exactly mod (a-1) 2^48 then divided
    mod = (a - 1) << 48
    geo = ((pow(a, k, mod) - 1) % mod) // (a - 1)
    return (ak * s0 + c * geo) & MASK48


LCG_WINDOW = 2**31 - 101
LCG_STREAM = 2**39 - 20325


def lcg_word(seed, s, v, d):
    """Keyed Random.nextDouble word: m = s LCG_STREAM + d LCG_WINDOW + v uses
    LCG steps 2m+1 and 2m+2."""
    m = s * LCG_STREAM + d * LCG_WINDOW + v
    S1 = lcg_state(seed, 2 * m + 1)
    S2 = (0x5DEECE66D * S1 + 0xB) & MASK48
    return (((S1 >> 22) << 27) + (S2 >> 21)) << 11
