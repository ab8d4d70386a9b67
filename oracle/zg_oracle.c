/*
 * zg_oracle.c -- plain, slow, scalar CPU oracle for the ziggurat Gaussian path.
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the CPU
 * baseline of the benchmark.  It shares no code with the product library.
 * Build: gcc -O2 -ffp-contract=off (no FMA contraction), glibc libm.
 *
 * What it follows:
 *  - The original ziggurat that the paper ports from GSL (Section 1, Section 2
 *    "Ziggurat", after Marsaglia-Tsang 2000 and Leong 2005): 128 equal-area
 *    layers, a fast accept inside the inner box of a layer, a wedge test
 *    against exp(-x^2/2), and sampling beyond r for the base layer.  The table
 *    is an input (correctly rounded values computed in 60-digit arithmetic).
 *  - The polar method (Section 1; Section 2 "Java 17" for Random/TLR):
 *    v = 2U-1 pairs, reject s >= 1 or s == 0, multiplier sqrt(-2 ln s / s).
 *  - The uniform sources of Section 2: SplittableRandom (SplitMix64) and
 *    java.util.Random (48-bit LCG, a = 0x5DEECE66D, c = 0xB), each made
 *    index-addressable: word(seed, stream s, variate v, draw d).  The LCG
 *    windows are spaced by odd numbers of doubles (see orc_lcg_word).
 *  - Gaussian mutation (Section 1): x <- x + sigma * z.
 *
 * Readings where the paper is silent (each one is listed in the design notes):
 *  - base layer area v = r f(r) + f(r)/r (exponential majorant), a tail
 *    rejection restarts the whole attempt;
 *  - the tail draw a = -log(U1+)/r, x = r + a, accept iff U2 < exp(-a^2/2);
 *  - word decode: layer = W>>57, sign = bit 56, j = bits 3..55, U = (W>>11)2^-53,
 *    U+ = ((W>>11)+1) 2^-53;
 *  - fast accept is the integer test j < k53[i], x = (double)j * w53[i];
 *  - wedge: y = y[i-1] + U dy[i], accept iff y < exp(-0.5 (x x));
 *  - a wedge rejection restarts at draw d+2, a tail rejection at d+3; words
 *    with draw index >= dmax (256 by default) are never used: the variate
 *    becomes the canonical quiet NaN and the error count is raised.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <string.h>

#define ORC_SM64 1
#define ORC_LCG48 2

typedef struct {
  double r;
  double W[128];    /* layer widths, RN64 */
  double y[128];    /* f(b_i), y[127] = 1 */
  double dy[128];   /* y[i] - y[i-1] */
  double w53[128];  /* W[i] * 2^-53 */
  double w24d[128]; /* W[i] * 2^-24 (FP64, slow path of the FP32 mode) */
  float w24[128];   /* RN32(W[i]) * 2^-24 */
  uint64_t k53[128];
  uint32_t k24[128];
} orc_table;

/* ---------------------------------------------------------------- uniforms */

/* SplitMix64 finaliser (Steele, Lea, Flood 2014; SplittableRandom.mix64). */
static uint64_t orc_mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  return z ^ (z >> 31);
}

/* SplittableRandom(seed): the k-th nextLong (0-based) is mix64(seed + (k+1)gamma).
 * Index-keyed: counter = 1 + s 2^48 + d 2^40 + v  (s < 2^16, d < 2^8, v < 2^40). */
uint64_t orc_sm64_word(uint64_t seed, uint32_t s, uint64_t v, uint32_t d) {
  uint64_t ctr = 1 + ((uint64_t)s << 48) + ((uint64_t)d << 40) + v;
  return orc_mix64(seed + 0x9E3779B97F4A7C15ULL * ctr);
}

#define LCG_A 0x5DEECE66DULL
#define LCG_C 0xBULL
#define M48 ((1ULL << 48) - 1)

/* java.util.Random initial scramble. */
uint64_t orc_lcg_state0(uint64_t seed) { return (seed ^ LCG_A) & M48; }

/* One LCG step S <- a S + c (mod 2^48). */
uint64_t orc_lcg_step(uint64_t S) { return (LCG_A * S + LCG_C) & M48; }

/* The affine map of k steps, S -> A S + C, by repeated squaring of (a, c).
 * Composition of two maps (A1,C1) then (A2,C2) is (A2 A1, A2 C1 + C2). */
void orc_lcg_affine(uint64_t k, uint64_t *A_out, uint64_t *C_out) {
  uint64_t A = 1, C = 0;            /* identity */
  uint64_t a = LCG_A, c = LCG_C;    /* one step */
  while (k) {
    if (k & 1) {
      C = (a * C + c) & M48;
      A = (a * A) & M48;
    }
    c = (a * c + c) & M48;
    a = (a * a) & M48;
    k >>= 1;
  }
  *A_out = A;
  *C_out = C;
}

/* State after k steps from state0. */
uint64_t orc_lcg_state(uint64_t seed, uint64_t k) {
  uint64_t A, C;
  orc_lcg_affine(k, &A, &C);
  return (A * orc_lcg_state0(seed) + C) & M48;
}

/* Index-keyed nextDouble of Random(seed).  Double index
 *   m = s * LCG_STREAM + d * LCG_WINDOW + v,  s < 2^8, d < 2^8, v < LCG_WINDOW,
 * consumes LCG steps 2m+1 and 2m+2 exactly as nextDouble does (26 high bits,
 * then 27), giving M = hi26 2^27 + lo27; the 64-bit word is M << 11 so that
 * U = (W >> 11) 2^-53 is Random.nextDouble.  Stream 0, draw 0 is the sequential
 * stream.  Both spacings are odd numbers of doubles: a jump of 2K steps then
 * has multiplier a^(2K) = 1 mod 8 only, whose 2-D lattice is as fine as that of
 * consecutive doubles.  A power-of-two spacing 2^k would give a multiplier
 * = 1 mod 2^(k+3) and nearly identical words across windows or streams. */
#define LCG_WINDOW 2147483547ULL        /* 2^31 - 101 */
#define LCG_STREAM 549755793563ULL      /* 2^39 - 20325 >= 256 LCG_WINDOW */
uint64_t orc_lcg_word(uint64_t seed, uint32_t s, uint64_t v, uint32_t d) {
  uint64_t m = (uint64_t)s * LCG_STREAM + (uint64_t)d * LCG_WINDOW + v;
  uint64_t S1 = orc_lcg_state(seed, 2 * m + 1);
  uint64_t S2 = orc_lcg_step(S1);
  uint64_t M = ((S1 >> 22) << 27) + (S2 >> 21);
  return M << 11;
}

/* Sequential Random(seed).nextDouble() numerators M (53 bits), n of them:
 * the plain sequential generator, used to check the index-keyed words. */
void orc_lcg_seq_doubles(uint64_t seed, uint64_t n, uint64_t *out) {
  uint64_t S = orc_lcg_state0(seed);
  for (uint64_t m = 0; m < n; ++m) {
    S = orc_lcg_step(S);
    uint64_t hi = S >> 22;
    S = orc_lcg_step(S);
    uint64_t lo = S >> 21;
    out[m] = (hi << 27) + lo;
  }
}

/* Sequential Random(seed).nextInt() values (next(32) as signed 32-bit). */
void orc_lcg_seq_ints(uint64_t seed, uint64_t n, int32_t *out) {
  uint64_t S = orc_lcg_state0(seed);
  for (uint64_t m = 0; m < n; ++m) {
    S = orc_lcg_step(S);
    out[m] = (int32_t)(uint32_t)(S >> 16);
  }
}

uint64_t orc_word(int kind, uint64_t seed, uint32_t s, uint64_t v, uint32_t d) {
  return kind == ORC_LCG48 ? orc_lcg_word(seed, s, v, d) : orc_sm64_word(seed, s, v, d);
}

static double u53(uint64_t W) { return (double)(W >> 11) * 0x1p-53; }         /* [0,1) */
static double u53p(uint64_t W) { return (double)((W >> 11) + 1) * 0x1p-53; }  /* (0,1] */

static double nan64(void) {
  uint64_t b = 0x7FF8000000000000ULL;
  double x;
  memcpy(&x, &b, 8);
  return x;
}
static float nan32(void) {
  uint32_t b = 0x7FC00000u;
  float x;
  memcpy(&x, &b, 4);
  return x;
}

/* ------------------------------------------------------- ziggurat pieces */

/* Outcome codes: low 2 bits = path of the accepted attempt (0 fast, 1 wedge,
 * 2 tail, 3 budget exhausted); bits 2..7 = min(attempts - 1, 63). */
static uint8_t outcome(int path, int attempts) {
  int a = attempts - 1;
  if (a > 63) a = 63;
  return (uint8_t)(path | (a << 2));
}

/* Where the words of one variate come from: word d is W(kind, seed, s, v, d),
 * or tape[d] for kind 0 (crafted words for the tests).  When `reads` is set,
 * every draw index read is appended to it (at most nreads_max entries). */
typedef struct {
  int kind;
  uint64_t seed;
  uint32_t s;
  uint64_t v;
  const uint64_t *tape;
  uint32_t ntape;
  uint32_t *reads;
  uint32_t nreads, nreads_max;
} orc_src;

static uint64_t orc_long_word_(int kind, uint64_t seed, uint32_t s, uint64_t v, uint32_t d);

/* kind > 0: the original ziggurat's words; kind < 0: nextLong words of the
 * source -kind (the modified ziggurat); 0: the tape. */
static uint64_t src_word(orc_src *S, uint32_t d) {
  if (S->reads && S->nreads < S->nreads_max) S->reads[S->nreads] = d;
  if (S->reads) S->nreads++;
  if (S->kind == 0) return d < S->ntape ? S->tape[d] : 0;
  if (S->kind < 0) return orc_long_word_(-S->kind, S->seed, S->s, S->v, d);
  return orc_word(S->kind, S->seed, S->s, S->v, d);
}

/* The three steps of one attempt of the original ziggurat.  They are the only
 * place where the oracle decides anything; every driver below (keyed FP64,
 * FP32, mutation, sequential consumption, crafted words, tiny tables) calls
 * them, so the tests that enumerate them pin every driver.
 *
 * 1. Decode of the first word: layer = top 7 bits, sign = bit 56, j = bits 3..55. */
static void decode64(uint64_t W, int *i, int *neg, uint64_t *j) {
  *i = (int)(W >> 57);
  *neg = (int)((W >> 56) & 1);
  *j = (W >> 3) & ((1ULL << 53) - 1);
}

/* 2. Fast test inside the layer's inner box: accept iff j < k53[i]; the
 * candidate x = j * w53[i] is the point under the layer, used by the wedge. */
static int fast_test(const orc_table *T, int i, uint64_t j, double *x) {
  *x = (double)j * T->w53[i];
  return j < T->k53[i];
}

/* 3. Slow part of an attempt whose first word failed the fast test, given the
 * attempt's next words.  Base layer (i = 0), the exponential majorant beyond
 * r: a = -log(U+ of W1)/r, candidate r + a, accept iff U of W2 < exp(-a^2/2).
 * Other layers, the wedge: y = y[i-1] + U dy[i] with U from W1, accept the
 * candidate x iff y < exp(-x^2/2).  Returns 1 and the accepted magnitude on
 * acceptance, 0 on rejection. */
static int slow_test(const orc_table *T, int i, double x, uint64_t W1, uint64_t W2, double *xo) {
  if (i == 0) {
    double a = -log(u53p(W1)) / T->r;
    double xt = T->r + a;
    *xo = xt;
    return u53(W2) < exp(-0.5 * (a * a));
  }
  double y = T->y[i - 1] + u53(W1) * T->dy[i];
  *xo = x;
  return y < exp(-0.5 * (x * x));
}

/* Words an attempt of layer i reads after its first word, and so the draw
 * offset of the next attempt after a rejection: 1 + 2 for the base layer,
 * 1 + 1 for a wedge.  Every word is read once. */
static uint32_t attempt_words(int i) { return i == 0 ? 3u : 2u; }

/* One FP64 standard normal from a word source, draws 0 .. dmax-1. */
static double zig_f64_src(const orc_table *T, orc_src *S, uint32_t dmax, uint8_t *cls) {
  uint32_t d = 0;
  int attempts = 0;
  for (;;) {
    if (d >= dmax) {
      *cls = outcome(3, attempts + 1);
      return nan64();
    }
    int i, neg;
    uint64_t j;
    double x;
    decode64(src_word(S, d), &i, &neg, &j);
    attempts++;
    if (fast_test(T, i, j, &x)) {
      *cls = outcome(0, attempts);
      return neg ? -x : x;
    }
    if (d + attempt_words(i) - 1 >= dmax) {
      *cls = outcome(3, attempts);
      return nan64();
    }
    uint64_t W1 = src_word(S, d + 1);
    uint64_t W2 = i == 0 ? src_word(S, d + 2) : 0;
    double xo;
    if (slow_test(T, i, x, W1, W2, &xo)) {
      *cls = outcome(i == 0 ? 2 : 1, attempts);
      return neg ? -xo : xo;
    }
    d += attempt_words(i);
  }
}

/* One FP64 standard normal for index v. */
double orc_zig_f64(const orc_table *T, int kind, uint64_t seed, uint32_t s, uint64_t v,
                   uint32_t dmax, uint8_t *cls) {
  orc_src S = {kind, seed, s, v, 0, 0, 0, 0, 0};
  return zig_f64_src(T, &S, dmax, cls);
}

/* One FP64 variate from crafted words tape[0..ntape) (word d = tape[d]; a
 * word past the tape reads as 0).  reads (optional, nreads_max entries)
 * receives the draw indices read, in order; returns their count in *nreads. */
double orc_zig_f64_tape(const orc_table *T, const uint64_t *tape, uint32_t ntape, uint32_t dmax,
                        uint8_t *cls, uint32_t *reads, uint32_t nreads_max, uint32_t *nreads) {
  orc_src S = {0, 0, 0, 0, tape, ntape, reads, 0, nreads_max};
  double x = zig_f64_src(T, &S, dmax, cls);
  if (nreads) *nreads = S.nreads;
  return x;
}

/* One attempt's class for a crafted first word (layer, sign, j decoded from W):
 * 0 fast, 1 wedge, 2 tail; *x is the first-word candidate (j * w53[i], signed). */
int orc_decide_word(const orc_table *T, uint64_t W, double *x) {
  int i, neg;
  uint64_t j;
  double xv;
  decode64(W, &i, &neg, &j);
  int fast = fast_test(T, i, j, &xv);
  *x = neg ? -xv : xv;
  if (fast) return 0;
  return i == 0 ? 2 : 1;
}

/* One attempt for a decoded first word (layer i, integer j) and the
 * attempt's next words W1, W2, with T possibly a small table (only layers
 * 0 .. n-1 used, k53 and w53 at any j width).  Returns 0 fast accept,
 * 1 wedge accept, 2 tail accept, 5 wedge reject, 6 tail reject; *x the
 * accepted or rejected magnitude.  For the exhaustive enumeration tests. */
int orc_attempt(const orc_table *T, int i, uint64_t j, uint64_t W1, uint64_t W2, double *x) {
  double xc;
  if (fast_test(T, i, j, &xc)) {
    *x = xc;
    return 0;
  }
  int acc = slow_test(T, i, xc, W1, W2, x);
  return (i == 0 ? 2 : 1) + (acc ? 0 : 4);
}

/* Exhaustive enumeration of one attempt on a table of n layers whose fast
 * thresholds and widths are at jbits bits (k53[i] = floor(q_i 2^jbits),
 * w53[i] = W_i 2^-jbits): every first word (layer i, j < 2^jbits; the sign
 * only mirrors the output) and every extra uniform on the grid of
 * G = 2^ubits points, U = m/G and U+ = (m+1)/G, each made into the word whose
 * top ubits carry it.  Each decision is made by orc_attempt.  Outcome weights
 * are integers: a first word weighs G^2, a wedge uniform G, a base-strip
 * pair 1, out of n 2^jbits G^2 in all.  acc_bin[b] receives the accepted
 * weight with edges[b] <= |x| < edges[b+1] (nedges edges); out[0] the
 * accepted weight, out[1] the accepted base-strip weight, out[2] the total.
 * The base-strip decisions do not involve j; they are enumerated for the
 * first slow j of layer 0 and checked equal for the last, then weighted by
 * the number of slow j.  Returns 0, or -1 if that check fails. */
int orc_enum_attempt(const orc_table *T, int n, int jbits, int ubits, const double *edges,
                     int nedges, uint64_t *acc_bin, uint64_t *out) {
  const uint64_t G = 1ULL << ubits;
  const uint64_t J = 1ULL << jbits;
  const int sh = 64 - ubits;
  uint64_t acc = 0, tail_acc = 0;
  for (int b = 0; b + 1 < nedges; ++b) acc_bin[b] = 0;
#define ORC_BIN(xv, wgt)                                              \
  do {                                                                \
    for (int b_ = 0; b_ + 1 < nedges; ++b_)                           \
      if ((xv) >= edges[b_] && (xv) < edges[b_ + 1]) {                \
        acc_bin[b_] += (wgt);                                         \
        break;                                                        \
      }                                                               \
  } while (0)
  for (int i = 0; i < n; ++i) {
    uint64_t nslow = 0, j_first_slow = J, j_last_slow = 0;
    for (uint64_t j = 0; j < J; ++j) {
      double x;
      if (orc_attempt(T, i, j, 0, 0, &x) == 0) {
        acc += G * G;
        ORC_BIN(x, G * G);
        continue;
      }
      nslow++;
      if (j_first_slow == J) j_first_slow = j;
      j_last_slow = j;
      if (i == 0) continue;
      for (uint64_t m = 0; m < G; ++m) {
        if (orc_attempt(T, i, j, m << sh, 0, &x) == 1) {
          acc += G;
          ORC_BIN(x, G);
        }
      }
    }
    if (i == 0 && nslow) {
      for (uint64_t m1 = 0; m1 < G; ++m1) {
        /* U+ = (m1 + 1)/G: the 53-bit field is (m1 + 1) 2^(53 - ubits) - 1 */
        uint64_t W1 = ((((m1 + 1) << (53 - ubits)) - 1) << 11);
        for (uint64_t m2 = 0; m2 < G; ++m2) {
          double xa, xb;
          int ra = orc_attempt(T, 0, j_first_slow, W1, m2 << sh, &xa);
          int rb = orc_attempt(T, 0, j_last_slow, W1, m2 << sh, &xb);
          if (ra != rb || (ra == 2 && xa != xb)) return -1;
          if (ra == 2) {
            acc += nslow;
            tail_acc += nslow;
            ORC_BIN(xa, nslow);
          }
        }
      }
    }
  }
#undef ORC_BIN
  out[0] = acc;
  out[1] = tail_acc;
  out[2] = (uint64_t)n * J * G * G;
  return 0;
}

/* FP32 output mode.  The attempt word is 32 bits: for the SplitMix64 kind the
 * first attempt of variates 2t and 2t+1 takes the high and low halves of
 * W(s, t, 0); every other attempt (and every LCG attempt) takes hi32(W(s,v,d)).
 * Decode: layer = u>>25, sign = bit 24, j = low 24 bits.  Fast path in FP32:
 * fl32(fl32(j) * w24[i]); wedge and tail in FP64 with x = j * w24d[i];
 * out = fl32(+-x).  *x64 receives the FP64 value of the same decision
 * (the fast path evaluated in FP64), for the error statement. */
float orc_zig_f32(const orc_table *T, int kind, uint64_t seed, uint32_t s, uint64_t v,
                  uint32_t dmax, uint8_t *cls, double *x64) {
  uint32_t d = 0;
  int attempts = 0;
  for (;;) {
    if (d >= dmax) {
      *cls = outcome(3, attempts + 1);
      *x64 = nan64();
      return nan32();
    }
    uint32_t u;
    if (d == 0 && kind == ORC_SM64) {
      uint64_t W = orc_sm64_word(seed, s, v >> 1, 0);
      u = (v & 1) ? (uint32_t)W : (uint32_t)(W >> 32);
    } else {
      u = (uint32_t)(orc_word(kind, seed, s, v, d) >> 32);
    }
    int i = (int)(u >> 25);
    int neg = (int)((u >> 24) & 1);
    uint32_t j = u & 0xFFFFFFu;
    attempts++;
    if (j < T->k24[i]) {
      float xf = (float)j * T->w24[i];
      double xd = (double)j * T->w24d[i];
      *cls = outcome(0, attempts);
      *x64 = neg ? -xd : xd;
      return neg ? -xf : xf;
    }
    double x = (double)j * T->w24d[i];
    if (d + attempt_words(i) - 1 >= dmax) {
      *cls = outcome(3, attempts);
      *x64 = nan64();
      return nan32();
    }
    uint64_t W1 = orc_word(kind, seed, s, v, d + 1);
    uint64_t W2 = i == 0 ? orc_word(kind, seed, s, v, d + 2) : 0;
    double xo;
    if (slow_test(T, i, x, W1, W2, &xo)) {
      double sx = neg ? -xo : xo;
      *cls = outcome(i == 0 ? 2 : 1, attempts);
      *x64 = sx;
      return (float)sx;
    }
    d += attempt_words(i);
  }
}

/* ------------------------------------------------------------------ polar */

/* One polar attempt from two uniforms in [0,1) (Knuth's polar method as in
 * java.util.Random.nextGaussian): returns 1 and the pair on acceptance. */
int orc_polar_core(double u1, double u2, double *o1, double *o2) {
  double v1 = 2.0 * u1 - 1.0;
  double v2 = 2.0 * u2 - 1.0;
  double s = v1 * v1 + v2 * v2;
  if (s >= 1.0 || s == 0.0) return 0;
  double m = sqrt(-2.0 * log(s) / s);
  *o1 = v1 * m;
  *o2 = v2 * m;
  return 1;
}

/* Pair p of stream s: attempt a uses draws 2a and 2a+1 of index p. */
static int polar_pair(int kind, uint64_t seed, uint32_t s, uint64_t p, uint32_t dmax,
                      double *o1, double *o2, int *attempts) {
  for (uint32_t a = 0;; ++a) {
    if (2 * a + 1 >= dmax) {
      *attempts = (int)a + 1;
      *o1 = *o2 = nan64();
      return 0;
    }
    double u1 = u53(orc_word(kind, seed, s, p, 2 * a));
    double u2 = u53(orc_word(kind, seed, s, p, 2 * a + 1));
    if (orc_polar_core(u1, u2, o1, o2)) {
      *attempts = (int)a + 1;
      return 1;
    }
  }
}

/* ---------------------------------------- McFarland's modified ziggurat */
/*
 * The comparator of Sections 1 and 3 (McFarland 2016; Java 17's Gaussian for
 * SplittableRandom and the newer generators), as read here (the paper gives
 * none of its steps; oracle/table_mz.py states the table):
 *  - N equal-probability buckets (256), L layers (253) of mass T/N each, every
 *    layer [0, X_i] x [Y_{i-1}, Y_i] wholly under f; the other N - L buckets'
 *    mass lies in L + 1 regions (tail beyond X_0, an overhang right of each
 *    layer, the cap above the top layer), picked by an alias table.
 *  - First word W1 as a signed B-bit integer (B = 64).  Its low log2 N bits
 *    are the bucket: a layer i < L returns x = X_i 2^-(B-1) * W1 at once (sign
 *    and magnitude from W1 itself).  These are the low-order bits Section 3
 *    says the method needs to be good.
 *  - Otherwise the sign is W1's top bit, and the region is bucket j = the low
 *    bits of the second word W2, or its alias when W1's other B-1 bits are at
 *    or above the bucket's threshold.
 *  - Region 0, the tail: pairs of words d, d+1 give E1 = -log U1+, E2 =
 *    -log U2+ and a = E1 / X_0; accept X_0 + a iff a^2/2 < E2 (Marsaglia's
 *    tail method); else the next pair.
 *  - Overhang k: pairs of words give integers a, b (top ubits bits); in the
 *    box [X_k, X_{k-1}] x [Y_{k-1}, Y_k], s = distance from the right edge,
 *    t = height above the bottom, both in units of the box, so the curve runs
 *    from (0, 0) to (1, 1) and the chord is t = s.  Convex strips (X_k >= 1:
 *    the curve lies under the chord) take (s, t) = (max, min) of (a, b), a
 *    uniform point under the chord; concave strips (X_{k-1} <= 1: the curve
 *    lies over the chord) accept at once when t <= s; otherwise (and for the
 *    strip holding x = 1) accept x = X_{k-1} - s dx iff
 *    Y_{k-1} + t dy < exp(-x^2/2); else the next pair, same region.
 *  - Words: the SplitMix64 word, or for java.util.Random its nextLong
 *    ((next(32) << 32) + next(32), the LCG steps 2m+1 and 2m+2 of the keyed
 *    double index m).  Draws 0 and 1 are W1 and W2, pairs from draw 2; the
 *    draw budget and the NaN are the original ziggurat's.
 */
typedef struct {
  int n_buckets;          /* N, a power of two <= 256 */
  int n_layers;           /* L < N */
  int bits;               /* B: bits of a word (64 in the real format) */
  int ubits;              /* bits of a slow-path uniform (53 in the real format) */
  double xs[256];         /* X_i 2^-(B-1), i < L */
  double x0;              /* X_0 */
  double ox[257], odx[257], oy[257], ody[257];   /* overhang k >= 1: X_{k-1}, X_{k-1} - X_k, Y_{k-1}, Y_k - Y_{k-1} */
  int kind[257];          /* 0 tail, 1 convex, 2 concave, 3 the strip holding x = 1 */
  uint64_t thr[256];      /* in units of 2^-(B-1) */
  int alias[256];
} orc_mz_table;

/* nextLong of Random(seed) at the keyed double index of (s, v, d): the same
 * two LCG steps as orc_lcg_word, combined as (int)(S1 >> 16) << 32 plus the
 * sign-extended (int)(S2 >> 16). */
uint64_t orc_lcg_long(uint64_t seed, uint32_t s, uint64_t v, uint32_t d) {
  uint64_t m = (uint64_t)s * LCG_STREAM + (uint64_t)d * LCG_WINDOW + v;
  uint64_t S1 = orc_lcg_state(seed, 2 * m + 1);
  uint64_t S2 = orc_lcg_step(S1);
  int32_t hi = (int32_t)(uint32_t)(S1 >> 16), lo = (int32_t)(uint32_t)(S2 >> 16);
  return ((uint64_t)(int64_t)hi << 32) + (uint64_t)(int64_t)lo;
}

/* The word of draw d for the modified ziggurat: nextLong of each source. */
uint64_t orc_long_word(int kind, uint64_t seed, uint32_t s, uint64_t v, uint32_t d) {
  return kind == ORC_LCG48 ? orc_lcg_long(seed, s, v, d) : orc_sm64_word(seed, s, v, d);
}
static uint64_t orc_long_word_(int kind, uint64_t seed, uint32_t s, uint64_t v, uint32_t d) {
  return orc_long_word(kind, seed, s, v, d);
}

static uint64_t mz_mask(int bits) { return bits >= 64 ? ~0ULL : ((1ULL << bits) - 1); }
static int64_t mz_signed(const orc_mz_table *T, uint64_t W) {
  return (int64_t)(W << (64 - T->bits)) >> (64 - T->bits);
}

/* Step 1: the first word.  Returns 1 and the signed x when its bucket is a
 * layer; otherwise 0, the sign in *neg. */
static int mz_first(const orc_mz_table *T, uint64_t W1, double *x, int *neg) {
  int i = (int)(W1 & (uint64_t)(T->n_buckets - 1));
  int64_t sv = mz_signed(T, W1);
  *neg = sv < 0;
  if (i < T->n_layers) {
    *x = T->xs[i] * (double)sv;
    return 1;
  }
  return 0;
}

/* Step 2: the region of a slow variate from W1's other bits and W2's bucket. */
static int mz_region(const orc_mz_table *T, uint64_t W1, uint64_t W2) {
  uint64_t u = W1 & mz_mask(T->bits - 1);
  int j = (int)(W2 & (uint64_t)(T->n_buckets - 1));
  return u < T->thr[j] ? j : T->alias[j];
}

/* Step 3: one attempt in region k with the pair of words (Wa, Wb); returns 1
 * and the magnitude on acceptance. */
static int mz_attempt(const orc_mz_table *T, int k, uint64_t Wa, uint64_t Wb, double *x) {
  const int sh = T->bits - T->ubits;
  const double g = ldexp(1.0, -T->ubits);
  uint64_t a = (Wa & mz_mask(T->bits)) >> sh, b = (Wb & mz_mask(T->bits)) >> sh;
  if (k == 0) {
    double e1 = -log((double)(a + 1) * g), e2 = -log((double)(b + 1) * g);
    double t = e1 / T->x0;
    *x = T->x0 + t;
    return 0.5 * (t * t) < e2;
  }
  uint64_t si = a, ti = b;
  if (T->kind[k] == 1 && b > a) {
    si = b;
    ti = a;
  }
  *x = T->ox[k] - ((double)si * g) * T->odx[k];
  if (T->kind[k] == 2 && ti <= si) return 1;
  double y = T->oy[k] + ((double)ti * g) * T->ody[k];
  return y < exp(-0.5 * (*x * *x));
}

/* One FP64 standard normal from a word source.  Outcome path: 0 layer,
 * 1 overhang, 2 tail, 3 budget. */
static double mz_f64_src(const orc_mz_table *T, orc_src *S, uint32_t dmax, uint8_t *cls) {
  double x;
  int neg;
  if (dmax < 1) {
    *cls = outcome(3, 1);
    return nan64();
  }
  const uint64_t W1 = src_word(S, 0);
  if (mz_first(T, W1, &x, &neg)) {
    *cls = outcome(0, 1);
    return x;
  }
  if (dmax < 2) {
    *cls = outcome(3, 1);
    return nan64();
  }
  int k = mz_region(T, W1, src_word(S, 1));
  int attempts = 1;
  for (uint32_t d = 2;; d += 2, ++attempts) {
    if (d + 1 >= dmax) {
      *cls = outcome(3, attempts);
      return nan64();
    }
    const uint64_t Wa = src_word(S, d);
    const uint64_t Wb = src_word(S, d + 1);
    if (mz_attempt(T, k, Wa, Wb, &x)) {
      *cls = outcome(k == 0 ? 2 : 1, attempts);
      return neg ? -x : x;
    }
  }
}

double orc_mz_f64(const orc_mz_table *T, int kind, uint64_t seed, uint32_t s, uint64_t v,
                  uint32_t dmax, uint8_t *cls) {
  orc_src S = {-kind, seed, s, v, 0, 0, 0, 0, 0};
  return mz_f64_src(T, &S, dmax, cls);
}

/* One variate from crafted words (word d = tape[d], 0 past the tape). */
double orc_mz_f64_tape(const orc_mz_table *T, const uint64_t *tape, uint32_t ntape,
                       uint32_t dmax, uint8_t *cls, uint32_t *reads, uint32_t nreads_max,
                       uint32_t *nreads) {
  orc_src S = {0, 0, 0, 0, tape, ntape, reads, 0, nreads_max};
  double x = mz_f64_src(T, &S, dmax, cls);
  if (nreads) *nreads = S.nreads;
  return x;
}

/* The steps one at a time, for crafted words and enumeration. */
int orc_mz_first(const orc_mz_table *T, uint64_t W1, double *x, int *neg) {
  return mz_first(T, W1, x, neg);
}
int orc_mz_region(const orc_mz_table *T, uint64_t W1, uint64_t W2) {
  return mz_region(T, W1, W2);
}
int orc_mz_attempt(const orc_mz_table *T, int k, uint64_t Wa, uint64_t Wb, double *x) {
  return mz_attempt(T, k, Wa, Wb, x);
}

/* Exhaustive enumeration of a tiny format (B bits) through the three steps
 * above.  The law of one variate: every first word (weight 1 of 2^B) either
 * returns a layer's signed x (binned by signed value into layer_bins), or is
 * slow with a sign; with each of the N buckets of the second word it picks a
 * region: cnt[2 r + neg] counts those (first word, bucket) pairs.  Within a
 * region, the accepted attempts over all 2^ubits x 2^ubits pairs of (a, b)
 * give the conditional law of the magnitude (acc[r][bin] over the bins of
 * the positive edges, acc_tot[r]).  Words carry a in their top ubits bits.
 * edges: nb + 1 increasing bin edges (signed for layer_bins; the bins with
 * edges >= 0 serve the magnitudes).  layer_bins[nb], cnt[2 (L+1)],
 * acc[(L+1) nb], acc_tot[L+1].  Returns 0, -1 if the format is too large,
 * -2 if a region index falls outside 0..L. */
int orc_mz_enum(const orc_mz_table *T, const double *edges, int nb, uint64_t *layer_bins,
                uint64_t *cnt, uint64_t *acc, uint64_t *acc_tot) {
  if (T->bits > 24 || T->ubits > 12 || T->ubits > T->bits) return -1;
  const uint64_t nw = 1ULL << T->bits;
  const int N = T->n_buckets, L = T->n_layers;
  memset(layer_bins, 0, sizeof(uint64_t) * nb);
  memset(cnt, 0, sizeof(uint64_t) * 2 * (L + 1));
  memset(acc, 0, sizeof(uint64_t) * (L + 1) * nb);
  memset(acc_tot, 0, sizeof(uint64_t) * (L + 1));
  for (uint64_t W1 = 0; W1 < nw; ++W1) {
    double x;
    int neg;
    if (mz_first(T, W1, &x, &neg)) {
      for (int b = 0; b < nb; ++b)
        if (x >= edges[b] && x < edges[b + 1]) {
          layer_bins[b]++;
          break;
        }
      continue;
    }
    for (int j = 0; j < N; ++j) {
      const int r = mz_region(T, W1, (uint64_t)j);
      if (r < 0 || r > L) return -2;
      cnt[2 * r + neg]++;
    }
  }
  const uint64_t G = 1ULL << T->ubits;
  const int sh = T->bits - T->ubits;
  for (int r = 0; r <= L; ++r) {
    if (!cnt[2 * r] && !cnt[2 * r + 1]) continue;
    for (uint64_t a = 0; a < G; ++a)
      for (uint64_t b = 0; b < G; ++b) {
        double x;
        if (!mz_attempt(T, r, a << sh, b << sh, &x)) continue;
        acc_tot[r]++;
        for (int k = 0; k < nb; ++k)
          if (x >= edges[k] && x < edges[k + 1]) {
            acc[(uint64_t)r * nb + k]++;
            break;
          }
      }
  }
  return 0;
}

/* ------------------------------------------------------------ bulk fills */

typedef struct {
  const orc_table *T;
  int op; /* 0 zig f64, 1 zig f32, 2 polar f64, 3 mutate f64, 4 modified ziggurat f64 */
  int kind;
  uint64_t seed;
  uint32_t s;
  uint64_t first;
  uint64_t lo, hi;
  uint32_t dmax;
  double sigma;
  void *out;
  double *out64;
  uint8_t *cls;
  uint64_t errors;
  uint64_t n_per;   /* > 0: element k is variate first + k % n_per of stream s + k / n_per */
  const orc_mz_table *M;   /* op 4 */
} orc_job;

static void *run_job(void *arg) {
  orc_job *J = (orc_job *)arg;
  uint64_t errs = 0;
  for (uint64_t k = J->lo; k < J->hi; ++k) {
    uint64_t v = J->first + (J->n_per ? k % J->n_per : k);
    uint32_t s = J->n_per ? J->s + (uint32_t)(k / J->n_per) : J->s;
    uint8_t c = 0;
    if (J->op == 0) {
      ((double *)J->out)[k] = orc_zig_f64(J->T, J->kind, J->seed, s, v, J->dmax, &c);
    } else if (J->op == 1) {
      double x64;
      ((float *)J->out)[k] = orc_zig_f32(J->T, J->kind, J->seed, s, v, J->dmax, &c, &x64);
      if (J->out64) J->out64[k] = x64;
    } else if (J->op == 2) {
      double o1, o2;
      int att;
      int ok = polar_pair(J->kind, J->seed, s, v >> 1, J->dmax, &o1, &o2, &att);
      ((double *)J->out)[k] = (v & 1) ? o2 : o1;
      c = (uint8_t)(ok ? ((att - 1 > 63 ? 63 : att - 1) << 2) : (3 | ((att - 1 > 63 ? 63 : att - 1) << 2)));
    } else if (J->op == 4) {
      ((double *)J->out)[k] = orc_mz_f64(J->M, J->kind, J->seed, s, v, J->dmax, &c);
    } else {
      double z = orc_zig_f64(J->T, J->kind, J->seed, s, v, J->dmax, &c);
      double *x = (double *)J->out;
      x[k] = x[k] + J->sigma * z;
    }
    if ((c & 3) == 3) errs++;
    if (J->cls) J->cls[k] = c;
  }
  J->errors = errs;
  return 0;
}

/* Runs an op over [0, n) split into nthreads contiguous chunks; returns the
 * number of variates that exhausted the draw budget. */
static uint64_t run_split(orc_job proto, uint64_t n, int nthreads) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 256) nthreads = 256;
  if ((uint64_t)nthreads > n) nthreads = n ? (int)n : 1;
  pthread_t th[256];
  orc_job jobs[256];
  for (int t = 0; t < nthreads; ++t) {
    jobs[t] = proto;
    jobs[t].lo = n * (uint64_t)t / (uint64_t)nthreads;
    jobs[t].hi = n * (uint64_t)(t + 1) / (uint64_t)nthreads;
  }
  if (nthreads == 1) {
    run_job(&jobs[0]);
    return jobs[0].errors;
  }
  for (int t = 0; t < nthreads; ++t) pthread_create(&th[t], 0, run_job, &jobs[t]);
  uint64_t errs = 0;
  for (int t = 0; t < nthreads; ++t) {
    pthread_join(th[t], 0);
    errs += jobs[t].errors;
  }
  return errs;
}

uint64_t orc_fill_f64(const orc_table *T, int kind, uint64_t seed, uint32_t s, uint64_t first,
                      uint64_t n, uint32_t dmax, double *out, uint8_t *cls, int nthreads) {
  orc_job j = {T, 0, kind, seed, s, first, 0, 0, dmax, 0.0, out, 0, cls, 0};
  return run_split(j, n, nthreads);
}

/* Streams s0 .. s0 + n_streams - 1, variates first .. first + n_per - 1 of
 * each, stream-major in out (the multi-stream layout), split over nthreads. */
uint64_t orc_fill_streams_f64(const orc_table *T, int kind, uint64_t seed, uint32_t s0,
                              uint32_t n_streams, uint64_t first, uint64_t n_per, uint32_t dmax,
                              double *out, uint8_t *cls, int nthreads) {
  orc_job j = {T, 0, kind, seed, s0, first, 0, 0, dmax, 0.0, out, 0, cls, 0, n_per};
  return run_split(j, (uint64_t)n_streams * n_per, nthreads);
}

/* The same for the FP32 mode (out: float, out64: the FP64 value of the same
 * decision) and for the polar method. */
uint64_t orc_fill_streams_f32(const orc_table *T, int kind, uint64_t seed, uint32_t s0,
                              uint32_t n_streams, uint64_t first, uint64_t n_per, uint32_t dmax,
                              float *out, double *out64, uint8_t *cls, int nthreads) {
  orc_job j = {T, 1, kind, seed, s0, first, 0, 0, dmax, 0.0, out, out64, cls, 0, n_per};
  return run_split(j, (uint64_t)n_streams * n_per, nthreads);
}

uint64_t orc_fill_streams_polar(int kind, uint64_t seed, uint32_t s0, uint32_t n_streams,
                                uint64_t first, uint64_t n_per, uint32_t dmax, double *out,
                                uint8_t *cls, int nthreads) {
  orc_job j = {0, 2, kind, seed, s0, first, 0, 0, dmax, 0.0, out, 0, cls, 0, n_per};
  return run_split(j, (uint64_t)n_streams * n_per, nthreads);
}

/* The modified ziggurat: variates first .. first + n_per - 1 of streams
 * s0 .. s0 + n_streams - 1, stream-major (n_streams = 1: one stream). */
uint64_t orc_fill_streams_mz(const orc_mz_table *M, int kind, uint64_t seed, uint32_t s0,
                             uint32_t n_streams, uint64_t first, uint64_t n_per, uint32_t dmax,
                             double *out, uint8_t *cls, int nthreads) {
  orc_job j = {0, 4, kind, seed, s0, first, 0, 0, dmax, 0.0, out, 0, cls, 0, n_per, M};
  return run_split(j, (uint64_t)n_streams * n_per, nthreads);
}

uint64_t orc_fill_f32(const orc_table *T, int kind, uint64_t seed, uint32_t s, uint64_t first,
                      uint64_t n, uint32_t dmax, float *out, double *out64, uint8_t *cls,
                      int nthreads) {
  orc_job j = {T, 1, kind, seed, s, first, 0, 0, dmax, 0.0, out, out64, cls, 0};
  return run_split(j, n, nthreads);
}

uint64_t orc_fill_polar(int kind, uint64_t seed, uint32_t s, uint64_t first, uint64_t n,
                        uint32_t dmax, double *out, uint8_t *cls, int nthreads) {
  orc_job j = {0, 2, kind, seed, s, first, 0, 0, dmax, 0.0, out, 0, cls, 0};
  return run_split(j, n, nthreads);
}

uint64_t orc_mutate(const orc_table *T, int kind, uint64_t seed, uint32_t s, uint64_t first,
                    uint64_t n, uint32_t dmax, double sigma, double *x, uint8_t *cls,
                    int nthreads) {
  orc_job j = {T, 3, kind, seed, s, first, 0, 0, dmax, sigma, x, 0, cls, 0};
  return run_split(j, n, nthreads);
}

/* ------------------------------------------------ one EA generation step */
/*
 * The fused consumer of Section 1's prior work (an evolutionary algorithm
 * that ran 20-25% faster with the ziggurat), as read here: one generation
 * of a population of `pop` genomes of `genes` doubles, minimising fitness.
 *  - Child c (0 <= c < pop) of generation `gen` has the key u = gen pop + c.
 *    Its parent wins a tournament of `k` draws with replacement: draw t
 *    picks index floor(W(seed, stream, u, t) pop / 2^64), and the winner is
 *    the first draw of least fitness: a later draw replaces the current best
 *    when its fitness is strictly smaller, or when the best's is NaN and its
 *    own is not (a NaN fitness wins only when every draw has one).
 *  - Gene g of child c (key w = u genes + g) copies the winner's gene g; it
 *    mutates iff (W(seed, stream + 1, w, 0) >> 11) < rate53, a 53-bit
 *    threshold (the host rounds rate 2^53 down), by x += sigma z with z the
 *    FP64 ziggurat variate w of stream stream + 2 (SplitMix64, the oracle's
 *    own orc_zig_f64); then x is clamped to [lo, hi] (a NaN stays NaN).
 * Outputs: children (pop x genes), winners (pop), cls per gene (255 for a
 * copy, else the ziggurat's outcome code).  Returns the budget failures.
 */
typedef struct {
  const orc_table *T;
  const double *parents, *fitness;
  double *children;
  uint32_t *winners;
  uint8_t *cls;
  uint64_t seed, gen, rate53;
  uint32_t pop, genes, k, stream, dmax;
  double sigma, lo, hi;
  uint32_t c0, c1;
  uint64_t errors;
} orc_ea_job;

static uint32_t ea_draw(uint64_t W, uint32_t pop) {
  return (uint32_t)(((unsigned __int128)W * pop) >> 64);
}

static void *run_ea(void *arg) {
  orc_ea_job *J = (orc_ea_job *)arg;
  for (uint32_t c = J->c0; c < J->c1; ++c) {
    const uint64_t u = J->gen * J->pop + c;
    uint32_t best = ea_draw(orc_sm64_word(J->seed, J->stream, u, 0), J->pop);
    for (uint32_t t = 1; t < J->k; ++t) {
      const uint32_t i = ea_draw(orc_sm64_word(J->seed, J->stream, u, t), J->pop);
      const double fi = J->fitness[i], fb = J->fitness[best];
      if (fi < fb || (isnan(fb) && !isnan(fi))) best = i;
    }
    if (J->winners) J->winners[c] = best;
    for (uint32_t g = 0; g < J->genes; ++g) {
      const uint64_t w = u * J->genes + g;
      double x = J->parents[(uint64_t)best * J->genes + g];
      uint8_t cl = 255;
      if ((orc_sm64_word(J->seed, J->stream + 1, w, 0) >> 11) < J->rate53) {
        const double z = orc_zig_f64(J->T, ORC_SM64, J->seed, J->stream + 2, w, J->dmax, &cl);
        if ((cl & 3) == 3) J->errors++;
        x = x + J->sigma * z;
        x = x < J->lo ? J->lo : (x > J->hi ? J->hi : x);
      }
      J->children[(uint64_t)c * J->genes + g] = x;
      if (J->cls) J->cls[(uint64_t)c * J->genes + g] = cl;
    }
  }
  return 0;
}

uint64_t orc_ea_step(const orc_table *T, const double *parents, const double *fitness,
                     double *children, uint32_t *winners, uint8_t *cls, uint32_t pop,
                     uint32_t genes, uint32_t k, uint64_t seed, uint32_t stream, uint64_t gen,
                     uint64_t rate53, double sigma, double lo, double hi, uint32_t dmax,
                     int nthreads) {
  if (nthreads < 1) nthreads = 1;
  if (nthreads > 64) nthreads = 64;
  pthread_t th[64];
  orc_ea_job jobs[64];
  for (int t = 0; t < nthreads; ++t) {
    orc_ea_job j = {T, parents, fitness, children, winners, cls, seed, gen, rate53,
                    pop, genes, k, stream, dmax, sigma, lo, hi,
                    (uint32_t)((uint64_t)pop * t / nthreads),
                    (uint32_t)((uint64_t)pop * (t + 1) / nthreads), 0};
    jobs[t] = j;
    pthread_create(&th[t], 0, run_ea, &jobs[t]);
  }
  uint64_t errs = 0;
  for (int t = 0; t < nthreads; ++t) {
    pthread_join(th[t], 0);
    errs += jobs[t].errors;
  }
  return errs;
}

/* Raw words W(seed, s, first + k, d) for k < n. */
void orc_words(int kind, uint64_t seed, uint32_t s, uint32_t d, uint64_t first, uint64_t n,
               uint64_t *out) {
  for (uint64_t k = 0; k < n; ++k) out[k] = orc_word(kind, seed, s, first + k, d);
}

/* ------------------------------------------------- sequential consumption */

/* The paper's nextGaussian(random) (Section 2, Listing 2) takes its uniforms
 * from one generator object, in call order.  Here that generator is stream s
 * of (seed, kind) read from position `first`: its word at position p is
 * W(seed, s, p, 0), which for stream 0 is SplittableRandom(seed).nextLong()
 * number p (SplitMix64) or the numerator of Random(seed).nextDouble() number p
 * shifted left by 11 (LCG).  kind 0 reads a caller-given list instead, word p
 * being list[p], for crafted streams.  Positions >= limit are unavailable. */
typedef struct {
  int kind;
  uint64_t seed;
  uint32_t s;
  const uint64_t *list;
  uint64_t limit;
  uint64_t pos;
} orc_gen;

static int gen_next(orc_gen *g, uint64_t *W) {
  if (g->pos >= g->limit) return 0;
  *W = g->kind == 0 ? g->list[g->pos] : orc_word(g->kind, g->seed, g->s, g->pos, 0);
  g->pos++;
  return 1;
}

/* One FP64 variate taken from the generator: each attempt reads one word;
 * a wedge test reads one more (U), the base strip two more (U1+, then U2);
 * after a rejection the next attempt reads the next unread word.  The
 * arithmetic of each attempt is that of orc_zig_f64.  Returns 0 (value NaN)
 * when the generator runs out first. */
static int seq_variate(const orc_table *T, orc_gen *g, double *out, uint8_t *cls) {
  for (int att = 1;; ++att) {
    uint64_t W, W1, W2 = 0;
    if (!gen_next(g, &W)) {
      *cls = outcome(3, att);
      break;
    }
    int i, neg;
    uint64_t j;
    double x, xo;
    decode64(W, &i, &neg, &j);
    if (fast_test(T, i, j, &x)) {
      *cls = outcome(0, att);
      *out = neg ? -x : x;
      return 1;
    }
    if (!gen_next(g, &W1) || (i == 0 && !gen_next(g, &W2))) {
      *cls = outcome(3, att);
      break;
    }
    if (slow_test(T, i, x, W1, W2, &xo)) {
      *cls = outcome(i == 0 ? 2 : 1, att);
      *out = neg ? -xo : xo;
      return 1;
    }
  }
  *out = nan64();
  return 0;
}

/* n variates of sequential consumption starting at position `first`.
 * starts (optional) receives each variate's first position; *next the
 * position after the last word read.  Returns the number of variates the
 * generator could not complete (each NaN). */
uint64_t orc_seq_f64(const orc_table *T, int kind, uint64_t seed, uint32_t s, uint64_t first,
                     uint64_t n, const uint64_t *list, uint64_t limit, double *out,
                     uint8_t *cls, uint64_t *starts, uint64_t *next) {
  orc_gen g = {kind, seed, s, list, limit, first};
  uint64_t fails = 0;
  for (uint64_t k = 0; k < n; ++k) {
    uint8_t c = 0;
    if (starts) starts[k] = g.pos;
    if (!seq_variate(T, &g, &out[k], &c)) fails++;
    if (cls) cls[k] = c;
  }
  *next = g.pos;
  return fails;
}
