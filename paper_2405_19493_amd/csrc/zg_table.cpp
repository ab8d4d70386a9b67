// Host-side construction, in double-double arithmetic, of the 128-layer
// ziggurat table and of the modified ziggurat's 256-bucket table (layers
// found by bisection, region masses from the Maclaurin series of the
// integral of f, alias table in exact integers), and of the java.util.Random
// jump-ahead tables.
//
// Table (Section 1 / Section 2 "Ziggurat": the GSL-style original ziggurat of
// Marsaglia-Tsang and Leong, 128 equal-area layers): f(x) = exp(-x^2/2);
// v = r f(r) + f(r)/r; b_0 = r, b_i = f^-1(f(b_{i-1}) + v/b_{i-1}); r is the
// root of the closure f(b_126) + v/b_126 = 1.  Every entry handed to the
// kernels is the correctly rounded value of the exact quantity: the
// double-double evaluation carries about 100 bits, so rounding it to 53 (or
// 24) bits is exact except for values within 2^-100 of a rounding boundary.
//
// Compiled with -ffp-contract=off: the error-free transformations below
// depend on every product and sum being rounded separately.
#include <cmath>
#include <cstdint>
#include <cstring>
#include <deque>
#include <set>
#include <vector>

#include "zg_internal.h"

namespace zg {
namespace {

struct dd {
  double hi, lo;
};

inline dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  return {s, e};
}
inline dd fast_two_sum(double a, double b) {
  double s = a + b;
  return {s, b - (s - a)};
}
inline dd two_prod(double a, double b) {
  double p = a * b;
  return {p, std::fma(a, b, -p)};
}
inline dd mk(double a) { return {a, 0.0}; }
inline dd add(dd a, dd b) {
  dd s = two_sum(a.hi, b.hi);
  dd t = two_sum(a.lo, b.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}
inline dd neg(dd a) { return {-a.hi, -a.lo}; }
inline dd sub(dd a, dd b) { return add(a, neg(b)); }
inline dd mul(dd a, dd b) {
  dd p = two_prod(a.hi, b.hi);
  p.lo += a.hi * b.lo + a.lo * b.hi;
  return fast_two_sum(p.hi, p.lo);
}
inline dd mul_pow2(dd a, double p2) { return {a.hi * p2, a.lo * p2}; }
inline dd divide(dd a, dd b) {
  double q1 = a.hi / b.hi;
  dd r = sub(a, mul(b, mk(q1)));
  double q2 = r.hi / b.hi;
  r = sub(r, mul(b, mk(q2)));
  double q3 = r.hi / b.hi;
  return add(fast_two_sum(q1, q2), mk(q3));
}
inline bool lt(dd a, dd b) { return a.hi < b.hi || (a.hi == b.hi && a.lo < b.lo); }

// sqrt by one Newton correction of the double root: s = x + (a - x^2)/(2x).
dd dd_sqrt(dd a) {
  if (a.hi <= 0.0) return mk(0.0);
  double x = std::sqrt(a.hi);
  dd r = sub(a, mul(mk(x), mk(x)));
  return add(mk(x), mk(r.hi / (2.0 * x)));
}

// ln 2 to about 107 bits.
const dd LN2 = {0x1.62e42fefa39efp-1, 0x1.abc9e3b39803fp-56};

// exp: a = k ln2 + t, |t| <= ln2/2; t' = t/2^10; expm1(t') by its Taylor
// series; undo the scaling with e <- 2e + e^2 (keeps relative accuracy of
// expm1), then 1 + e and the power of two.
dd dd_exp(dd a) {
  double k = std::nearbyint(a.hi / LN2.hi);
  dd t = sub(a, mul(LN2, mk(k)));
  t = mul_pow2(t, 1.0 / 1024.0);
  dd term = t, sum = t;
  for (int n = 2; n <= 14; ++n) {
    term = divide(mul(term, t), mk((double)n));
    sum = add(sum, term);
    if (std::fabs(term.hi) < 1e-36) break;
  }
  for (int i = 0; i < 10; ++i) sum = add(mul_pow2(sum, 2.0), mul(sum, sum));
  dd e = add(sum, mk(1.0));
  int ki = (int)k;
  return {std::ldexp(e.hi, ki), std::ldexp(e.lo, ki)};
}

// log: two Newton steps y <- y + a exp(-y) - 1 from the double logarithm.
dd dd_log(dd a) {
  dd y = mk(std::log(a.hi));
  for (int it = 0; it < 2; ++it) y = add(y, sub(mul(a, dd_exp(neg(y))), mk(1.0)));
  return y;
}

dd f_of(dd x) { return dd_exp(mul_pow2(neg(mul(x, x)), 0.5)); }
dd finv(dd y) { return dd_sqrt(mul_pow2(neg(dd_log(y)), 2.0)); }

// v(r) = r f(r) + f(r)/r: the base box plus the exponential majorant's mass.
dd area_of(dd r) {
  dd fr = f_of(r);
  return add(mul(r, fr), divide(fr, r));
}

// Closure residual: > 0 when the layers reach the top too early (r too
// small), otherwise f(b_126) + v/b_126 - 1 (decreasing in r).
dd closure(dd r) {
  dd v = area_of(r);
  dd b = r;
  for (int i = 1; i < ZG_LAYERS - 1; ++i) {
    dd t = add(f_of(b), divide(v, b));
    if (!lt(t, mk(1.0))) return mk(1.0);
    b = finv(t);
  }
  return sub(add(f_of(b), divide(v, b)), mk(1.0));
}

// Correctly rounded double of a dd value: the normalising sum hi + lo is
// itself rounded to nearest (an exact tie is left to ties-to-even; the dd
// value is then within 2^-100 of the midpoint and no rounding is certain).
double rn64(dd x) { return fast_two_sum(x.hi, x.lo).hi; }

// Correctly rounded float of a dd value.
float rn32(dd x) {
  dd n = fast_two_sum(x.hi, x.lo);
  float f = (float)n.hi;   // round-to-nearest-even of hi
  float fu = std::nextafter(f, INFINITY), fd = std::nextafter(f, -INFINITY);
  double mu = ((double)f + (double)fu) * 0.5, md = ((double)f + (double)fd) * 0.5;
  if (n.hi == mu && n.lo > 0) return fu;
  if (n.hi == md && n.lo < 0) return fd;
  if (n.hi == mu && n.lo < 0) return f;
  if (n.hi == md && n.lo > 0) return f;
  return f;
}

// floor of a non-negative dd value (below 2^63).
uint64_t floor_u64(dd x) {
  dd n = fast_two_sum(x.hi, x.lo);
  double fl = std::floor(n.hi);
  if (fl == n.hi) {
    if (n.lo < 0) return (uint64_t)fl - 1;
    return (uint64_t)fl + (uint64_t)std::floor(n.lo);
  }
  return (uint64_t)fl;
}

// ------------------------------------------------ modified ziggurat table

// pi to about 107 bits.
const dd PI = {0x1.921fb54442d18p+1, 0x1.1a62633145c07p-53};

// F(x): the integral of f over [0, x], by its Maclaurin series
// sum_n (-x^2/2)^n x / (n! (2n + 1)).  Below x = 4 the largest term is about
// 2^9 times the sum, and the terms fall under 1e-40 before n = 90.
dd F_of(dd x) {
  const dd q = neg(mul_pow2(mul(x, x), 0.5));
  dd p = x;   // q^n x / n!
  dd sum = x;
  for (int n = 1; n < 160; ++n) {
    p = divide(mul(p, q), mk((double)n));
    const dd t = divide(p, mk((double)(2 * n + 1)));
    sum = add(sum, t);
    if (n > 16 && std::fabs(t.hi) < 1e-40) break;
  }
  return sum;
}

// x (f(x) - ylo) - A: the mass of the box [0, x] x [ylo, f(x)] less a bucket's.
dd box_excess(dd x, dd ylo, dd A) { return sub(mul(x, sub(f_of(x), ylo)), A); }

// The root of box_excess in [lo, hi], where it falls from above 0 to below.
dd box_root(dd lo, dd hi, dd ylo, dd A) {
  for (int it = 0; it < 120; ++it) {
    const dd mid = mul_pow2(add(lo, hi), 0.5);
    if (box_excess(mid, ylo, A).hi > 0)
      lo = mid;
    else
      hi = mid;
  }
  return mul_pow2(add(lo, hi), 0.5);
}

// Nearest integer of a non-negative dd value below 2^100.
unsigned __int128 nint_u128(dd x) {
  const dd n = fast_two_sum(x.hi, x.lo);
  const double fh = std::floor(n.hi);
  const double frac = (n.hi - fh) + n.lo;
  return (unsigned __int128)fh + (unsigned __int128)(__int128)std::floor(frac + 0.5);
}

}  // namespace

zg_status build_mz_table(zg_mz_table_view *t) {
  constexpr int N = ZG_MZ_BUCKETS;
  std::memset(t, 0, sizeof(*t));
  const dd T = dd_sqrt(mul_pow2(PI, 0.5));   // mass of f on x >= 0
  const dd A = mul_pow2(T, 1.0 / N);
  const dd one = mk(1.0);
  // layers from the bottom: layer 0 solves x f(x) = A right of x = 1
  dd X[N], Y[N];
  X[0] = box_root(one, mk(8.0), mk(0.0), A);
  Y[0] = f_of(X[0]);
  int L = 1;
  while (L < N) {
    const dd ylo = Y[L - 1];
    // the box over ylo is heaviest where f(x) (1 - x^2) = ylo, left of x = 1
    // (that slope falls on (0, 1)); no layer fits unless it beats A there
    const auto slope = [&](double x) { return std::exp(-0.5 * x * x) * (1.0 - x * x) - ylo.hi; };
    double a = 0.0, b = std::min(1.0, X[L - 1].hi);
    if (slope(b) >= 0) {
      a = b;
    } else {
      for (int it = 0; it < 200; ++it) {
        const double m = 0.5 * (a + b);
        if (slope(m) > 0)
          a = m;
        else
          b = m;
      }
    }
    if (!(box_excess(mk(a), ylo, A).hi > 0)) break;
    X[L] = box_root(mk(a), X[L - 1], ylo, A);
    Y[L] = f_of(X[L]);
    ++L;
  }
  if (L != ZG_MZ_LAYERS) return ZG_EINVAL;
  // region masses: the tail beyond X_0, and overhang k between X_k and
  // X_{k-1} above Y_{k-1} (X_L = 0: the cap)
  dd Xe[N + 1], Ye[N + 1], Fx[N + 1], a[N + 1];
  for (int k = 0; k < L; ++k) {
    Xe[k] = X[k];
    Ye[k] = Y[k];
    Fx[k] = F_of(X[k]);
  }
  Xe[L] = mk(0.0);
  Ye[L] = one;
  Fx[L] = mk(0.0);
  a[0] = sub(T, Fx[0]);
  dd S = a[0];
  for (int k = 1; k <= L; ++k) {
    a[k] = sub(sub(Fx[k - 1], Fx[k]), mul(Ye[k - 1], sub(Xe[k - 1], Xe[k])));
    S = add(S, a[k]);
  }
  // the layers and the regions make up the whole mass
  const dd close = sub(add(mul(A, mk((double)L)), S), T);
  if (!(std::fabs(close.hi) < 1e-28)) return ZG_EINVAL;
  // integer masses in units of 2^-63 of a bucket, summing to N buckets
  using u128 = unsigned __int128;
  const u128 UNIT = (u128)1 << 63, TOTAL = (u128)N << 63;
  u128 m[N] = {};
  u128 sum = 0;
  int big = 0;
  for (int k = 0; k <= L; ++k) {
    m[k] = nint_u128(mul_pow2(divide(a[k], S), 0x1p71));
    sum += m[k];
    if (m[k] > m[big]) big = k;
  }
  m[big] = m[big] + TOTAL - sum;
  const std::vector<u128> mass(m, m + N);
  // alias table: the lowest-index bucket below one unit takes the rest of
  // its unit from the lowest-index bucket above
  std::set<int> small;
  std::deque<int> large;
  for (int j = 0; j < N; ++j) {
    t->thr[j] = (uint64_t)UNIT;
    t->alias[j] = (uint8_t)j;
    if (m[j] < UNIT)
      small.insert(j);
    else if (m[j] > UNIT)
      large.push_back(j);
  }
  while (!small.empty() && !large.empty()) {
    const int j = *small.begin();
    small.erase(small.begin());
    const int l = large.front();
    t->thr[j] = (uint64_t)m[j];
    t->alias[j] = (uint8_t)l;
    m[l] -= UNIT - m[j];
    if (m[l] < UNIT) {
      large.pop_front();
      small.insert(l);
    } else if (m[l] == UNIT) {
      large.pop_front();
    }
  }
  // the table gives every region its integer mass back
  std::vector<u128> got(N, 0);
  for (int j = 0; j < N; ++j) {
    got[j] += t->thr[j];
    got[t->alias[j]] += UNIT - t->thr[j];
  }
  if (got != mass) return ZG_EINVAL;
  t->x0 = rn64(X[0]);
  for (int i = 0; i < L; ++i) t->xs[i] = rn64(X[i]) * 0x1p-63;
  for (int k = 1; k <= L; ++k) {
    t->ox[k] = rn64(Xe[k - 1]);
    t->odx[k] = rn64(sub(Xe[k - 1], Xe[k]));
    t->oy[k] = rn64(Ye[k - 1]);
    t->ody[k] = rn64(sub(Ye[k], Ye[k - 1]));
    t->kind[k] = !lt(Xe[k], one) ? 1 : (!lt(one, Xe[k - 1]) ? 2 : 3);
  }
  return ZG_OK;
}

zg_status build_table(zg_table_view *t) {
  // bisection for r on [0.5, 5]: 110 halvings reach double-double resolution
  dd lo = mk(0.5), hi = mk(5.0);
  for (int it = 0; it < 110; ++it) {
    dd mid = mul_pow2(add(lo, hi), 0.5);
    if (closure(mid).hi > 0)
      lo = mid;
    else
      hi = mid;
  }
  dd r = mul_pow2(add(lo, hi), 0.5);
  dd v = area_of(r);
  dd b[ZG_LAYERS];
  b[0] = r;
  for (int i = 1; i < ZG_LAYERS - 1; ++i) b[i] = finv(add(f_of(b[i - 1]), divide(v, b[i - 1])));
  b[ZG_LAYERS - 1] = mk(0.0);
  dd W[ZG_LAYERS], y[ZG_LAYERS], q[ZG_LAYERS];
  W[0] = divide(v, f_of(r));
  for (int i = 1; i < ZG_LAYERS; ++i) W[i] = b[i - 1];
  for (int i = 0; i < ZG_LAYERS; ++i) q[i] = divide(b[i], W[i]);
  for (int i = 0; i < ZG_LAYERS - 1; ++i) y[i] = f_of(b[i]);
  y[ZG_LAYERS - 1] = mk(1.0);

  std::memset(t, 0, sizeof(*t));
  t->r = rn64(r);
  t->v = rn64(v);
  for (int i = 0; i < ZG_LAYERS; ++i) {
    t->W[i] = rn64(W[i]);
    t->y[i] = rn64(y[i]);
    t->dy[i] = i == 0 ? 0.0 : rn64(sub(y[i], y[i - 1]));
    t->k53[i] = floor_u64(mul_pow2(q[i], 0x1p53));
    t->k24[i] = (uint32_t)floor_u64(mul_pow2(q[i], 0x1p24));
    t->w53[i] = t->W[i] * 0x1p-53;
    t->w24d[i] = t->W[i] * 0x1p-24;
    t->w24[i] = rn32(W[i]) * 0x1p-24f;
  }
  // sanity of the geometry: equal areas to 1e-12 in plain double arithmetic
  for (int i = 1; i < ZG_LAYERS; ++i) {
    double area = t->W[i] * t->dy[i];
    if (!(std::fabs(area - t->v) <= 1e-12 * t->v)) return ZG_EINVAL;
  }
  if (!(std::fabs(t->W[0] * t->y[0] - t->v) <= 1e-12 * t->v)) return ZG_EINVAL;
  return ZG_OK;
}

// ---------------------------------------------------------------- LCG tables

static inline Affine compose(Affine first, Affine second) {
  // apply `first`, then `second`: S -> A2 (A1 S + C1) + C2
  return {(second.A * first.A) & LCG_M48, (second.A * first.C + second.C) & LCG_M48};
}

Affine lcg_power(uint64_t k) {
  Affine result = {1, 0};
  Affine base = {LCG_A, LCG_C};
  while (k) {
    if (k & 1) result = compose(result, base);
    base = compose(base, base);
    k >>= 1;
  }
  return result;
}

void build_log_tables(LogTables *L) {
  for (int k = 0; k < LOG_N; ++k) {
    const int idx = k + LOG_I0;
    // the interval of m: the lower binade [1/2, 1) in steps of 2^-8, the
    // upper [1, 2) in steps of 2^-7
    long double lo, hi;
    if (idx < 128) {
      lo = 0.5L * (1 + idx / 128.0L);
      hi = 0.5L * (1 + (idx + 1) / 128.0L);
    } else {
      lo = 1 + (idx - 128) / 128.0L;
      hi = 1 + (idx - 127) / 128.0L;
    }
    long double ic = 1.0L;
    if (idx != 127 && idx != 128) {   // next to m = 1 the reduction is m - 1 itself
      int ex = 0;
      const long double f = std::frexp(1.0L / (0.5L * (lo + hi)), &ex);
      ic = std::ldexp(std::rint(std::ldexp(f, 7)), ex - 7);   // 7 significant bits
    }
    const long double lc = -std::log(ic);
    const double h = (double)(std::rint(std::ldexp(lc, 33)) / 8589934592.0L);
    L->e[k] = {(double)ic, h};
    L->lo[k] = (double)(lc - (long double)h);
  }
}

void build_lcg_tables(LcgTables *L) {
  // jump[b][x] = x * 256^b steps, built by repeated composition
  for (int b = 0; b < LCG_JUMP_BYTES; ++b) {
    Affine unit = lcg_power(1ull << (8 * b));
    Affine acc = {1, 0};
    for (int x = 0; x < 256; ++x) {
      L->jump[b][x] = acc;
      acc = compose(acc, unit);
    }
  }
  // window[d] = 2 d LCG_WINDOW steps (draw d of the same variate)
  Affine w1 = lcg_power(2 * ZG_LCG_WINDOW);
  Affine acc = {1, 0};
  for (int d = 0; d < 256; ++d) {
    L->window[d] = acc;
    acc = compose(acc, w1);
  }
}

}  // namespace zg

namespace zg {

zg_status build_dev_tables(const zg_table_view &tv, DevTables *h) {
  std::memset(h, 0, sizeof(*h));
  for (int i = 0; i < ZG_LAYERS; ++i) {
    h->fast64[i] = {tv.k53[i], tv.w53[i]};
    h->fast32[i] = {tv.k24[i], tv.w24[i]};
    h->y[i] = tv.y[i];
    h->dy[i] = tv.dy[i];
    h->w53[i] = tv.w53[i];
    h->w24d[i] = tv.w24d[i];
  }
  h->r = tv.r;
  zg_mz_table_view mzv;
  const zg_status st = build_mz_table(&mzv);
  if (st != ZG_OK) return st;
  MzTabs &M = h->mz;
  for (int i = 0; i < ZG_MZ_BUCKETS; ++i) {
    M.xs[i] = mzv.xs[i];
    M.bucket[i] = {mzv.thr[i], mzv.alias[i], 0};
  }
  for (int k = 0; k <= ZG_MZ_LAYERS; ++k) {
    M.region[k] = {mzv.ox[k], mzv.odx[k], mzv.oy[k], mzv.ody[k]};
    M.kind[k] = mzv.kind[k];
  }
  M.x0 = mzv.x0;
  build_lcg_tables(&h->lcg);
  build_log_tables(&h->logt);
  return ZG_OK;
}

}  // namespace zg

extern "C" zg_status zg_build_table(zg_table_view *out) {
  if (!out) return ZG_EINVAL;
  return zg::build_table(out);
}

extern "C" zg_status zg_build_mz_table(zg_mz_table_view *out) {
  if (!out) return ZG_EINVAL;
  return zg::build_mz_table(out);
}
