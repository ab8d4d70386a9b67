// Device code of libzg for gfx950 (CDNA4, wave64).
//
// Hot path (Section 1 / Section 2 "Ziggurat": the original 128-layer
// ziggurat of Marsaglia-Tsang and Leong, as in GSL):
//   keyed uniform word -> decode (layer, sign, j) -> fast accept j < k[i]
//   with x = j w[i] (one multiply and one compare per lane) -> coalesced
//   128-bit stores.  Elements that fail the fast test (about 2.8% of them)
//   are appended to one LDS queue per workgroup; the queue is drained 64
//   entries at a time, each lane taking one queued variate through its
//   wedge test (the few left undecided, and the base-strip tails, are
//   finished later in full rounds of their own), so the rare slow path does
//   not diverge the fast one.
//   Every variate is a pure function of its index, so the launch shape, the
//   queue order and the batch layout never change the bits.
//
// Also here: the polar method (Section 1; Java's nextGaussian), the uniform
// word export, the per-word decision probe, and the batch kernels (counter
// reservation, one specialised kernel per work class, completion words).
//
// Build with -ffp-contract=off: the fast-path product and the wedge
// y = y[i-1] + U dy[i] must be rounded exactly as written.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>

#include "zg_internal.h"

namespace zg {

#define DEV __device__ __forceinline__

constexpr uint64_t MASK53 = (1ull << 53) - 1;
constexpr int QCAP = 1088;             // polar queue entries per wave (>= 63 + 2 per lane of a step)

// ------------------------------------------------------------ uniform words

DEV uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

DEV uint64_t sm64_word(uint64_t seed, uint32_t s, uint64_t v, uint32_t d) {
  return mix64(seed + GAMMA * (1ull + ((uint64_t)s << 48) + ((uint64_t)d << 40) + v));
}

DEV uint64_t aff(Affine f, uint64_t S) { return (f.A * S + f.C) & LCG_M48; }

DEV Affine aff_cat(Affine first, Affine second) {
  return {(second.A * first.A) & LCG_M48, (second.A * first.C + second.C) & LCG_M48};
}

DEV uint64_t lcg_state0(uint64_t seed) { return (seed ^ LCG_A) & LCG_M48; }

// Advance a state by k < 2^48 steps with the byte tables (the maps commute).
DEV uint64_t lcg_jump(const LcgTables *L, uint64_t S, uint64_t k) {
#pragma unroll
  for (int b = 0; b < LCG_JUMP_BYTES; ++b) {
    uint32_t x = (uint32_t)(k >> (8 * b)) & 255u;
    if (x) S = aff(L->jump[b][x], S);
  }
  return S;
}

DEV uint64_t lcg_index(uint32_t s, uint64_t v, uint32_t d) {
  return (uint64_t)s * ZG_LCG_STREAM_SPACING + (uint64_t)d * ZG_LCG_WINDOW + v;
}

// The word of the nextDouble whose first LCG state (step 2m+1) is S1.
DEV uint64_t lcg_word_from(uint64_t S1) {
  uint64_t S2 = (LCG_A * S1 + LCG_C) & LCG_M48;
  return (((S1 >> 22) << 27) + (S2 >> 21)) << 11;
}

// java.util.Random's nextLong whose first LCG state (step 2m+1) is S1:
// (next(32) << 32) + next(32), the second int sign-extended.
DEV uint64_t lcg_long_from(uint64_t S1) {
  const uint64_t S2 = (LCG_A * S1 + LCG_C) & LCG_M48;
  const int64_t hi = (int32_t)(uint32_t)(S1 >> 16), lo = (int32_t)(uint32_t)(S2 >> 16);
  return ((uint64_t)hi << 32) + (uint64_t)lo;
}

// The 53-bit integer j = bits 3..55 of a word (whi:wlo), as its two halves
// (bit-field extracts, so that the conversion below stays two 32-bit ones).
DEV uint32_t j_hi(uint32_t whi) { return __builtin_amdgcn_ubfe(whi, 3, 21); }
DEV uint32_t j_lo(uint32_t whi, uint32_t wlo) { return __builtin_amdgcn_alignbit(whi, wlo, 3); }

// Exact conversion of an integer below 2^53 given as hi * 2^32 + lo: the sum
// is representable, so the fused multiply-add rounds nothing.
DEV double to_f64(uint32_t hi, uint32_t lo) {
  return fma((double)hi, 4294967296.0, (double)lo);
}

DEV double u53(uint64_t W) { return (double)(W >> 11) * 0x1p-53; }
DEV double u53p(uint64_t W) { return (double)((W >> 11) + 1) * 0x1p-53; }

DEV double nan64() { return __longlong_as_double(0x7FF8000000000000ll); }

DEV double flip(double x, uint64_t neg) {
  return __longlong_as_double(__double_as_longlong(x) ^ (long long)(neg << 63));
}

// ------------------------------------------------------- slow path (FP64)

// Word of draw d for variate v of stream s, specialised on the kind.
template <int KIND>
DEV uint64_t wordk(const DevTables *T, uint64_t seed, uint32_t s, uint64_t v, uint32_t d) {
  if (KIND == ZG_JAVA_LCG48)
    return lcg_word_from(lcg_jump(&T->lcg, lcg_state0(seed), 2 * lcg_index(s, v, d) + 1));
  return sm64_word(seed, s, v, d);
}

// The modified ziggurat's long of draw d: the SplitMix64 word itself, or
// nextLong of the LCG at the keyed index of (s, v, d).
template <int KIND>
DEV uint64_t longk(const DevTables *T, uint64_t seed, uint32_t s, uint64_t v, uint32_t d) {
  if (KIND == ZG_JAVA_LCG48)
    return lcg_long_from(lcg_jump(&T->lcg, lcg_state0(seed), 2 * lcg_index(s, v, d) + 1));
  return sm64_word(seed, s, v, d);
}

// The 32-bit attempt word of FP32 mode.
template <int KIND>
DEV uint32_t word32(const DevTables *T, uint64_t seed, uint32_t s, uint64_t v, uint32_t d) {
  if (d == 0 && KIND == ZG_SPLITMIX64) {
    uint64_t W = sm64_word(seed, s, v >> 1, 0);
    return (v & 1) ? (uint32_t)W : (uint32_t)(W >> 32);
  }
  return (uint32_t)(wordk<KIND>(T, seed, s, v, d) >> 32);
}

struct PolarStep {
  int status;
  double z1, z2;
  uint32_t next_d;
};

// 2 U - 1 for U = (W >> 11) 2^-53, exactly: the 53-bit integer in two halves,
// each step exact (every value is a multiple of 2^-52 of magnitude <= 1).
DEV double sym53(uint64_t W) {
  const uint32_t hi = (uint32_t)(W >> 43), lo = (uint32_t)(W >> 11);
  return fma((double)hi, 0x1p-20, fma((double)lo, 0x1p-52, -1.0));
}

// Natural logarithm of x in [2^-1022, 1) (the polar method's s):
// x = 2^e m with m in [sqrt(1/2), sqrt(2)); the table entry of m's interval
// gives invc ~ 1/c and -log(invc) = hi + lo, so that
// log x = e ln2 + (hi + lo) + log(1 + r), r = m invc - 1 (exact: invc has 7
// significant bits), |r| < 2^-6.7, and log(1 + r) = r + r^2 Q(r) with
// Q = sum_{k=2..9} (-1)^(k+1) r^(k-2) / k (the first omitted term is below
// 2^-60 of r).  e ln2_hi + hi is exact (both are multiples of 2^-33); r is
// added to it by an error-free two-sum, and the small terms last.  Within
// 0.51 ulp of the true logarithm on (0, 1) (checked against an
// extended-precision logarithm on 3e7 points).
DEV double log_unit(double x, const LogTables &L) {
  int e;
  double m = frexp(x, &e);   // m in [1/2, 1)
  if (m < 0x1.6a09e667f3bcdp-1) {
    m *= 2.0;
    --e;
  }
  const int k = (int)((__double2hiint(m) >> 13) & 0xFF) - LOG_I0;   // low exponent bit, top 7 mantissa bits
  const LogEnt t = L.e[k];
  const double r = fma(m, t.invc, -1.0);
  double Q = 1.0 / 9.0;
  Q = fma(Q, r, -1.0 / 8.0);
  Q = fma(Q, r, 1.0 / 7.0);
  Q = fma(Q, r, -1.0 / 6.0);
  Q = fma(Q, r, 1.0 / 5.0);
  Q = fma(Q, r, -1.0 / 4.0);
  Q = fma(Q, r, 1.0 / 3.0);
  Q = fma(Q, r, -0.5);
  const double de = (double)e;
  const double big = fma(de, 0x1.62e42ffp-1, t.hi);   // e ln2_hi + hi, exact
  const double s1 = big + r;
  const double bb = s1 - big;
  const double err = (big - (s1 - bb)) + (r - bb);    // s1 + err = big + r
  const double small = fma(r * r, Q, err) + fma(de, -0x1.718432a1b0e26p-35, L.lo[k]);   // e ln2_lo
  return s1 + small;
}

// The log table of the polar kernels in LDS (whole block; then a barrier).
DEV void load_log_table(const DevTables *T, LogTables &L) {
  const double *src = (const double *)&T->logt;
  double *dst = (double *)&L;
  for (uint32_t i = threadIdx.x; i < sizeof(LogTables) / sizeof(double); i += blockDim.x)
    dst[i] = src[i];
}

// Polar attempt from the words of draws d and d+1 (Knuth; Random.nextGaussian).
DEV PolarStep polar_from_words(uint64_t W1, uint64_t W2, uint32_t d, const LogTables &L) {
  const double v1 = sym53(W1);
  const double v2 = sym53(W2);
  const double ss = v1 * v1 + v2 * v2;
  if (ss >= 1.0 || ss == 0.0) return {0, 0.0, 0.0, d + 2};
  const double m = sqrt(-2.0 * log_unit(ss, L) / ss);
  return {1, v1 * m, v2 * m, d};
}

template <int KIND>
DEV PolarStep polar_attempt(const DevTables *T, const LogTables &L, uint64_t seed, uint32_t s,
                            uint64_t p, uint32_t d, uint32_t dmax) {
  if (d + 1 >= dmax) return {-1, 0.0, 0.0, d};
  return polar_from_words(wordk<KIND>(T, seed, s, p, d), wordk<KIND>(T, seed, s, p, d + 1), d, L);
}

// --------------------------------------------------------- wave utilities

DEV uint32_t lane_id() { return __lane_id(); }

DEV uint32_t prefix_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

DEV uint32_t uni(uint32_t x) { return __builtin_amdgcn_readfirstlane(x); }
DEV uint64_t uni64(uint64_t x) {
  return ((uint64_t)uni((uint32_t)(x >> 32)) << 32) | uni((uint32_t)x);
}

// Queue entry (32 bits): element offset from the tile base (21 bits), draw d
// of the next attempt (8 bits), flags (3 bits; F_PAIR: polar entry covering
// both elements of a pair).
constexpr uint32_t OFF_MASK = (1u << 21) - 1;
constexpr uint32_t F_PAIR = 1u;
DEV uint32_t qent(uint32_t off, uint32_t d, uint32_t fl) { return off | (d << 21) | (fl << 29); }

// Appends up to two entries per lane (a, then b).  Wave-uniform control flow
// only: the queue count qn is the same in every lane.
DEV void qpush2(uint32_t *q, uint32_t &qn, bool pa, uint32_t ea, bool pb, uint32_t eb) {
  const uint64_t ma = __builtin_amdgcn_ballot_w64(pa), mb = __builtin_amdgcn_ballot_w64(pb);
  if ((ma | mb) != 0) {
    const uint32_t base = qn + prefix_below(ma) + prefix_below(mb);
    if (pa) q[base] = ea;
    if (pb) q[base + (pa ? 1u : 0u)] = eb;
    qn = uni(qn + (uint32_t)__popcll(ma) + (uint32_t)__popcll(mb));
    __builtin_amdgcn_wave_barrier();
  }
}

// Element e of a job -> (stream, variate index).  Rare paths only (drain):
// the quotient from the reciprocal is within one of the true one (e < 2^40),
// and one correction step fixes it.
DEV void split(const Job &J, uint64_t e, uint32_t &s, uint64_t &v) {
  if (J.n_streams == 1) {
    s = J.s0;
    v = J.first + e;
    return;
  }
  uint64_t k = (uint64_t)((double)e * J.inv_n_per);
  int64_t r = (int64_t)(e - k * J.n_per);
  if (r < 0) {
    k -= 1;
    r += (int64_t)J.n_per;
  } else if ((uint64_t)r >= J.n_per) {
    k += 1;
    r -= (int64_t)J.n_per;
  }
  s = J.s0 + (uint32_t)k;
  v = J.first + (uint64_t)r;
}

DEV void raise_flag(uint32_t *flags, uint32_t bit) { atomicOr(flags, bit); }

// ------------------------------------------------------------ polar path
//
// Each wave owns an LDS queue of 32-bit entries (element offset from the
// tile base, draw index, flags): pairs whose first attempt was rejected, and
// elements whose pair straddles a stream boundary or the tile edge.  The
// queue is drained 64 entries per round, one attempt per lane per round.

// LDS bytes of the log table at the start of a polar kernel's LDS.
constexpr size_t POLAR_LOG_BYTES = (sizeof(LogTables) + 15) / 16 * 16;

// Context of the polar path.
struct PolarCtx {
  const DevTables *T;
  uint32_t dmax;
  uint32_t *flags;
  const LogTables *L;   // in LDS
};

struct Queue {
  uint32_t *q;    // QCAP entries
  uint32_t qn;    // wave-uniform count
};

// Queue length at which a polar tile drains (down to POLAR_DRAIN - 1
// entries): one full round of 64, soon after the placeholders were stored.
constexpr uint32_t POLAR_DRAIN = 64;

// Polar drain: one attempt per round, rejected pairs requeued.
template <int KIND>
DEV void drain_polar(const Job &J, const PolarCtx &C, Queue &Q, uint32_t keep, uint64_t e_base) {
  const uint32_t lane = lane_id();
  // a rejected pair's placeholder was stored by another lane: order it first
  if (Q.qn > keep) __threadfence_block();
  while (Q.qn > keep) {
    const uint32_t m = Q.qn < 64 ? Q.qn : 64;
    const bool has = lane < m;
    const uint32_t ent = has ? Q.q[Q.qn - m + lane] : 0u;
    Q.qn = uni(Q.qn - m);
    __builtin_amdgcn_wave_barrier();
    bool pend = false;
    uint32_t requeue = 0;
    if (has) {
      const uint32_t off = ent & OFF_MASK;
      const uint32_t d = (ent >> 21) & 255u;
      const uint32_t fl = ent >> 29;
      const uint64_t e = e_base + off;
      uint32_t s;
      uint64_t v;
      split(J, e, s, v);
      PolarStep st = polar_attempt<KIND>(C.T, *C.L, J.seed, s, v >> 1, d, C.dmax);
      if (st.status == 0) {
        pend = true;
        requeue = qent(off, st.next_d, fl);
      } else {
        if (st.status < 0) {
          raise_flag(C.flags, ZG_FLAG_BUDGET);
          st.z1 = st.z2 = nan64();
        }
        double *out = (double *)J.out;
        if (fl & F_PAIR) {
          out[e] = st.z1;
          out[e + 1] = st.z2;
        } else {
          out[e] = (v & 1) ? st.z2 : st.z1;
        }
      }
    }
    qpush2(Q.q, Q.qn, pend, requeue, false, 0u);
  }
}

// --------------------------------------------------------- lane constants

struct LaneConst {
  uint64_t g[4];    // SplitMix64: gamma * offset of each word of the lane
  Affine a[4];      // LCG: jump from the chunk base state to each element
};

template <int OP, int KIND>
DEV LaneConst lane_constants(const DevTables *T) {
  LaneConst c;
  const uint32_t lane = lane_id();
  for (int t = 0; t < 4; ++t) {
    c.g[t] = 0;
    c.a[t] = {1, 0};
  }
  if (OP == OP_ZIG32) {
    // SplitMix64 pair words: word offsets 2*lane and 2*lane+1 (and +2)
    c.g[0] = GAMMA * (2ull * lane);
    c.g[1] = GAMMA * (2ull * lane + 1);
    c.g[2] = GAMMA * (2ull * lane + 2);
    if (KIND == ZG_JAVA_LCG48) {
      // element offsets 4*lane + t -> 2 (4 lane + t) steps
      for (int t = 0; t < 4; ++t) {
        uint32_t k = 2u * (4u * lane + t);
        c.a[t] = aff_cat(T->lcg.jump[0][k & 255u], T->lcg.jump[1][k >> 8]);
      }
    }
  } else if (OP == OP_POLAR) {
    c.g[0] = GAMMA * (uint64_t)lane;   // pair offset
    if (KIND == ZG_JAVA_LCG48) c.a[0] = T->lcg.jump[0][2u * lane];
  } else {
    c.g[0] = GAMMA * (2ull * lane);
    c.g[1] = GAMMA * (2ull * lane + 1);
    if (KIND == ZG_JAVA_LCG48) {
      c.a[0] = T->lcg.jump[0][4u * lane];
      c.a[1] = T->lcg.jump[0][4u * lane + 2];
    }
  }
  return c;
}

// ------------------------------------------------------------- tile work

// FP64 fast path of one element: returns the signed candidate and whether the
// integer test accepted it (tab: the signed table, indexed by the top byte).
DEV double fast64(const Fast64 *tab, uint64_t W, bool &fast) {
  const uint32_t whi = (uint32_t)(W >> 32), wlo = (uint32_t)W;
  const Fast64 f = tab[whi >> 24];
  const uint32_t jh = j_hi(whi), jl = j_lo(whi, wlo);
  fast = (((uint64_t)jh << 32) | jl) < f.k;
  return to_f64(jh, jl) * f.w;
}

// Modified ziggurat, fast path of one element: bucket i = the low byte of
// the long; a layer (i < ZG_MZ_LAYERS) gives x = X_i 2^-63 times the long as
// a signed integer (tab[i].w holds X_i 2^-63, 0 past the layers, so a slow
// element's placeholder is 0).
DEV double fast_mz(const Fast64 *tab, uint64_t W, bool &fast) {
  const uint32_t i = (uint32_t)W & 255u;
  fast = i < ZG_MZ_LAYERS;
  return tab[i].w * (double)(int64_t)W;
}

// One polar step: a pair per lane (2 elements).
template <int KIND>
DEV void polar_step(const Job &J, const PolarCtx &C, const LaneConst &LC, Queue &Q, uint64_t ec,
                    uint64_t e_end, uint32_t s, uint64_t vc, bool clean, uint32_t o0) {
  constexpr bool LCG = KIND == ZG_JAVA_LCG48;
  const uint32_t lane = lane_id();
  const uint64_t e0 = ec + 2ull * lane;
  const bool ok0 = e0 < e_end, ok1 = e0 + 1 < e_end;
  const bool paired = clean && (vc & 1) == 0 && ok1;   // vc parity is wave-uniform
  bool push_a, push_b = false;
  uint32_t ent_a, ent_b = 0;
  if (paired) {
    // pair p = vc/2 + lane, attempt 0: draws 0 and 1
    uint64_t W1, W2;
    if (LCG) {
      uint64_t Sc = lcg_jump(&C.T->lcg, lcg_state0(J.seed), 2 * lcg_index(s, vc >> 1, 0) + 1);
      uint64_t S1 = aff(LC.a[0], Sc);
      W1 = lcg_word_from(S1);
      W2 = lcg_word_from(aff(C.T->lcg.window[1], S1));
    } else {
      const uint64_t zc = J.seed + GAMMA * (1ull + ((uint64_t)s << 48) + (vc >> 1));
      const uint64_t z = zc + LC.g[0];
      W1 = mix64(z);
      W2 = mix64(z + (GAMMA << 40));
    }
    const PolarStep st = polar_from_words(W1, W2, 0, *C.L);
    const bool acc = st.status == 1 && C.dmax >= 2;
    *(double2 *)((double *)J.out + e0) = make_double2(st.z1, st.z2);   // placeholder if rejected
    push_a = !acc;
    ent_a = qent(o0, st.status == 1 ? 0u : 2u, F_PAIR);
  } else {
    push_a = ok0;
    ent_a = qent(o0, 0, 0);
    push_b = ok1;
    ent_b = qent(o0 + 1, 0, 0);
  }
  qpush2(Q.q, Q.qn, push_a, ent_a, push_b, ent_b);
}

// Polar method over elements [e_begin, e_end) of job J with one wave, then
// a full drain.  e_begin is 16-byte aligned in the output; elements [0, head)
// of the job (before the aligned body) are queued first when `with_head`.
// Every lane takes one pair per step; a pair is attempted at once when it
// lies inside one stream and inside the tile, otherwise its elements are
// queued one by one (each keyed by itself).
template <int KIND>
DEV void polar_tile(const Job &J, const PolarCtx &C, const LaneConst &LC, uint32_t *lds,
                    uint64_t e_begin, uint64_t e_end, uint32_t head, bool with_head) {
  constexpr uint32_t STEP = 128;   // elements per step (a pair per lane)
  const uint32_t lane = lane_id();
  e_begin = uni64(e_begin);
  e_end = uni64(e_end);
  // queue offsets are relative to e_base; the head elements precede e_begin
  const uint64_t e_base = with_head ? 0 : e_begin;
  Queue Q{lds, 0u};
  if (with_head && head) qpush2(Q.q, Q.qn, lane < head, qent(lane, 0, 0), false, 0u);
  const bool multi = J.n_streams != 1;
  uint64_t k = 0, r = e_begin;
  if (multi) {
    k = uni64(e_begin / J.n_per);
    r = uni64(e_begin - k * J.n_per);
  }
  uint32_t o0 = (uint32_t)(e_begin - e_base) + 2 * lane;
  for (uint64_t ec = e_begin; ec < e_end; ec += STEP) {
    const bool clean = !multi || r + STEP <= J.n_per;
    const uint32_t s = uni(J.s0 + (uint32_t)k);
    const uint64_t vc = uni64(J.first + r);
    polar_step<KIND>(J, C, LC, Q, ec, e_end, s, vc, clean, o0);
    o0 += STEP;
    if (Q.qn >= POLAR_DRAIN) drain_polar<KIND>(J, C, Q, POLAR_DRAIN - 1, e_base);
    r += STEP;
    if (multi)
      while (r >= J.n_per) {
        r -= J.n_per;
        ++k;
      }
  }
  drain_polar<KIND>(J, C, Q, 0, e_base);
}

// ------------------------------------------------ block-pooled ziggurat fill
//
// The plain ziggurat fills (FP64, FP32, mutation).  The waves of a workgroup
// stream its tile in groups of 4 steps of 256 elements, taken in turn from a
// shared counter; each step is stored at once with 128-bit stores (an
// element that failed the fast test gets a placeholder: the rejected
// candidate, or for mutation the old value).  The slow elements of all waves
// go into one LDS queue (offsets from the tile base).  After one workgroup
// barrier, which also orders every placeholder store before any patch, the
// waves drain the pooled queue 64 entries at a time, each lane taking one
// variate through its wedge test and, on rejection, the fast test of its
// next attempt, and storing the value when that decides it.  The 3-4% left
// undecided, and the base-strip attempts (the tail, with its logarithm), go
// to a retry queue that later rounds finish with the whole attempt loop:
// whole rounds of 64 at the start of the workgroup's next tile, the rest at
// the end of the kernel (the batch kernels, whose consecutive tiles belong to
// different jobs, finish them with each tile).  Pooling keeps the drain
// rounds nearly full: a tile of
// 16 x 2048 elements has about 900 slow elements, one wave's share about 57.
//
// Queue overflow (more slow elements than the queue holds, which hash words
// practically never produce): an element that finds the queue full is
// resolved at once by its own lane, which stored its placeholder.

constexpr uint32_t BSTEP = 256;    // elements per wave step
constexpr uint32_t BGROUP = 4;     // steps per queue flush of the batch kernels (plain
                                   // fills take it from their launch shape, 1..8)
constexpr uint32_t BQ = 2048;      // block queue capacity (entries)

// Tables of the fast and slow paths, in LDS.  The fast-path tables are
// indexed by the word's top byte, layer and sign: entry 2i + s holds k[i] and
// the width w[i] with the sign s applied (fl(j (-w)) = -fl(j w) exactly, -0.0
// for j = 0), so the fast path needs no sign step; the slow paths read entry
// 2i and apply the sign themselves.
struct LdsTabs {
  Fast64 f64[2 * ZG_LAYERS];
  Fast32 f32[2 * ZG_LAYERS];
  double2 yd[ZG_LAYERS];     // (y[i-1], dy[i]) of the wedge test, i >= 1
  double w24d[ZG_LAYERS];    // FP32 mode: w24 as a double
};

constexpr uint32_t RQ = 512;       // retry queue capacity (entries)
constexpr uint32_t ENT_D = 48;     // retry entry: element | first draw << ENT_D
constexpr uint64_t ENT_E = (1ull << ENT_D) - 1;

struct BlockLds {
  LdsTabs t;
  uint32_t cnt;
  uint32_t next;             // next group of the workgroup tile to stream
  uint32_t rcnt;             // retry queue count
  uint32_t rbeg, rtake;      // retries taken at the start of a tile: [rbeg, + rtake)
  uint32_t q[BQ];            // element offsets from the block base
  uint64_t rq[RQ];           // variates left undecided by a first drain step
};

// Loads the tables an op needs (whole block; no barrier).
template <int OP>
DEV void load_tabs(const DevTables *T, LdsTabs &L) {
  if (OP == OP_MZ64) {
    // modified ziggurat: the bucket multipliers in the FP64 fast-path slots
    for (uint32_t i = threadIdx.x; i < ZG_MZ_BUCKETS; i += blockDim.x)
      L.f64[i] = {0, T->mz.xs[i]};
    return;
  }
  for (uint32_t i = threadIdx.x; i < ZG_LAYERS; i += blockDim.x) {
    if (OP == OP_ZIG32) {
      const Fast32 f = T->fast32[i];
      L.f32[2 * i] = f;
      L.f32[2 * i + 1] = {f.k, -f.w};
      L.w24d[i] = T->w24d[i];
    } else {
      const Fast64 f = T->fast64[i];
      L.f64[2 * i] = f;
      L.f64[2 * i + 1] = {f.k, -f.w};
    }
    L.yd[i] = make_double2(i ? T->y[i - 1] : 0.0, T->dy[i]);
  }
}

// ------------------------------------------- modified ziggurat, slow path

// One attempt in region k with the longs (Wa, Wb): their top 53 bits a, b.
// Tail (k = 0): t = -log((a+1) 2^-53) / x0, x = x0 + t, accepted iff
// t^2/2 < -log((b+1) 2^-53).  Overhang k: (s, t) = (a, b), or (max, min)
// in a convex strip; x = X_{k-1} - s dx; accepted at once in a concave strip
// when t <= s, otherwise iff Y_{k-1} + t dy < exp(-x^2/2).
DEV bool mz_attempt(const MzTabs &M, uint32_t k, uint64_t Wa, uint64_t Wb, double &x) {
  constexpr double g = 0x1p-53;
  const uint64_t a = Wa >> 11, b = Wb >> 11;
  if (k == 0) {
    const double e1 = -log((double)(a + 1) * g), e2 = -log((double)(b + 1) * g);
    const double t = e1 / M.x0;
    x = M.x0 + t;
    return 0.5 * (t * t) < e2;
  }
  const uint32_t kind = M.kind[k];
  uint64_t si = a, ti = b;
  if (kind == 1 && b > a) {
    si = b;
    ti = a;
  }
  const MzRegion R = M.region[k];
  x = R.ox - ((double)si * g) * R.odx;
  if (kind == 2 && ti <= si) return true;
  const double y = R.oy + ((double)ti * g) * R.ody;
  return y < exp(-0.5 * (x * x));
}

// The modified ziggurat's variate v of stream s from draw d0 (0: from its
// first long; else the draw of the next attempt pair), at most max_att
// attempts.  Returns whether it is decided (value z: the signed variate, or
// the NaN when the draw budget runs out); otherwise dn is the draw to resume
// from.  The first long gives the bucket, sign and alias word; the second the
// region's bucket.
template <int KIND>
DEV bool mz_run(const Job &J, const DevTables *T, uint32_t dmax, uint32_t s, uint64_t v,
                uint32_t d0, uint32_t max_att, double &z, uint32_t &dn, bool &budget) {
  const MzTabs &M = T->mz;
  if (dmax < 1) {
    budget = true;
    z = nan64();
    return true;
  }
  const uint64_t W1 = longk<KIND>(T, J.seed, s, v, 0);
  const uint32_t i = (uint32_t)W1 & 255u;
  if (i < ZG_MZ_LAYERS) {
    z = M.xs[i] * (double)(int64_t)W1;
    return true;
  }
  if (dmax < 2) {
    budget = true;
    z = nan64();
    return true;
  }
  const uint64_t W2 = longk<KIND>(T, J.seed, s, v, 1);
  const uint32_t j = (uint32_t)W2 & 255u;
  const MzBucket B = M.bucket[j];
  const uint32_t k = (W1 & 0x7FFFFFFFFFFFFFFFull) < B.thr ? j : B.alias;
  const bool neg = (W1 >> 63) != 0;
  uint32_t d = d0 < 2 ? 2 : d0;
  for (uint32_t att = 0; att < max_att; ++att, d += 2) {
    if (d + 1 >= dmax) {
      budget = true;
      z = nan64();
      return true;
    }
    const uint64_t Wa = longk<KIND>(T, J.seed, s, v, d);
    const uint64_t Wb = longk<KIND>(T, J.seed, s, v, d + 1);
    double x;
    if (mz_attempt(M, k, Wa, Wb, x)) {
      z = neg ? -x : x;
      return true;
    }
  }
  dn = d;
  return false;
}

// The whole attempt sequence of one variate from draw 0 (the same steps, in
// the same order and precision, as attempt64 / attempt32): returns the signed
// FP64 value, or for FP32 mode the FP32 value widened exactly to double, or
// the canonical NaN when the draw budget runs out.
template <int OP, int KIND>
DEV double resolve(const Job &J, const LdsTabs &L, const DevTables *T, double r, uint32_t dmax,
                   uint32_t s, uint64_t v, bool &budget, uint32_t d = 0) {
  double z;
  if (OP == OP_MZ64) {
    uint32_t dn;
    mz_run<KIND>(J, T, dmax, s, v, d, 0xFFFFFFFFu, z, dn, budget);
    return z;
  }
  for (;;) {
    if (d >= dmax) {
      budget = true;
      z = nan64();
      break;
    }
    uint32_t i, neg;
    double x;
    if (OP == OP_ZIG32) {
      const uint32_t u = word32<KIND>(T, J.seed, s, v, d);
      i = u >> 25;
      neg = (u >> 24) & 1;
      const uint32_t j = u & 0xFFFFFFu;
      const Fast32 f = L.f32[2 * i];
      if (j < f.k) {
        const float xf = (float)j * f.w;
        z = (double)(neg ? -xf : xf);
        break;
      }
      x = (double)j * L.w24d[i];
    } else {
      const uint64_t W = wordk<KIND>(T, J.seed, s, v, d);
      i = (uint32_t)(W >> 57);
      neg = (uint32_t)(W >> 56) & 1;
      const uint32_t jh = j_hi((uint32_t)(W >> 32)), jl = j_lo((uint32_t)(W >> 32), (uint32_t)W);
      const uint64_t j = ((uint64_t)jh << 32) | jl;
      const Fast64 f = L.f64[2 * i];
      x = to_f64(jh, jl) * f.w;
      if (j < f.k) {
        z = neg ? -x : x;
        break;
      }
    }
    double thr, arg, xc;
    uint32_t dn;
    if (i == 0) {   // tail: x = r + a, a = -log(U1)/r, accept U2 < exp(-a^2/2)
      if (d + 2 >= dmax) {
        budget = true;
        z = nan64();
        break;
      }
      const double u1 = u53p(wordk<KIND>(T, J.seed, s, v, d + 1));
      thr = u53(wordk<KIND>(T, J.seed, s, v, d + 2));
      arg = -log(u1) / r;
      xc = r + arg;
      dn = d + 3;
    } else {        // wedge: accept y[i-1] + U dy[i] < exp(-x^2/2)
      if (d + 1 >= dmax) {
        budget = true;
        z = nan64();
        break;
      }
      const double u = u53(wordk<KIND>(T, J.seed, s, v, d + 1));
      const double2 yd = L.yd[i];
      thr = yd.x + u * yd.y;
      arg = x;
      xc = x;
      dn = d + 2;
    }
    if (thr < exp(-0.5 * (arg * arg))) {
      z = neg ? -xc : xc;
      break;
    }
    d = dn;
  }
  return z;
}

// Element of slot t (0..3) of a lane in a step starting at ec.
template <int OP>
DEV uint64_t slot_elem(uint64_t ec, uint32_t lane, uint32_t t) {
  if (OP == OP_ZIG32) return ec + 4ull * lane + t;
  return ec + (t >> 1) * 128ull + 2ull * lane + (t & 1);
}

// Fast path of one clean step into registers (x: FP64 values, or for mutation
// old + sigma z with the old value kept where the element is slow; xf: FP32
// values).  Elements at or beyond e_end are neither computed nor marked.
// Returns the lane's 4 slow bits.  For the LCG, Sc is the state of LCG step
// 2 lcg_index(s, vc, 0) + 1 (the first state of variate vc's word).
template <int OP, int KIND, bool FULL>
DEV uint32_t step_regs(const Job &J, const Fast64 *f64t, const Fast32 *f32t, const DevTables *T,
                       const LaneConst &LC, uint64_t ec, uint64_t e_end, uint32_t s, uint64_t vc,
                       uint64_t Sc, double *x, float *xf) {
  constexpr bool LCG = KIND == ZG_JAVA_LCG48;
  const uint32_t lane = lane_id();
  const uint64_t seed = J.seed;
  uint32_t b4 = 0;
  if (OP == OP_ZIG64 || OP == OP_MUTATE || OP == OP_MZ64) {
    constexpr uint32_t CH = 128;
    uint64_t W[4];
    if (LCG) {
      // the two LCG states of a variate make its nextDouble word, or for the
      // modified ziggurat its nextLong
      const auto lw = [](uint64_t S1) {
        return OP == OP_MZ64 ? lcg_long_from(S1) : lcg_word_from(S1);
      };
      W[0] = lw(aff(LC.a[0], Sc));
      W[1] = lw(aff(LC.a[1], Sc));
      Sc = aff(T->lcg.jump[1][1], Sc);   // 256 steps = the next 128-element chunk
      W[2] = lw(aff(LC.a[0], Sc));
      W[3] = lw(aff(LC.a[1], Sc));
    } else {
      const uint64_t zc = seed + GAMMA * (1ull + ((uint64_t)s << 48) + vc);
      W[0] = mix64(zc + LC.g[0]);
      W[1] = mix64(zc + LC.g[1]);
      W[2] = mix64(zc + GAMMA * (uint64_t)CH + LC.g[0]);
      W[3] = mix64(zc + GAMMA * (uint64_t)CH + LC.g[1]);
    }
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u) {
      const uint64_t ea = ec + u * CH + 2ull * lane;
      const bool ok0 = FULL || ea < e_end, ok1 = FULL || ea + 1 < e_end;
      bool fast0, fast1;
      double x0 = OP == OP_MZ64 ? fast_mz(f64t, W[2 * u], fast0) : fast64(f64t, W[2 * u], fast0);
      double x1 = OP == OP_MZ64 ? fast_mz(f64t, W[2 * u + 1], fast1)
                                : fast64(f64t, W[2 * u + 1], fast1);
      if (OP == OP_MUTATE) {
        const double *out = (const double *)J.out + ea;
        if (FULL || (ok0 && ok1)) {
          const double2 old = *(const double2 *)out;
          x0 = fast0 ? old.x + J.sigma * x0 : old.x;
          x1 = fast1 ? old.y + J.sigma * x1 : old.y;
        } else if (ok0) {
          const double old = out[0];
          x0 = fast0 ? old + J.sigma * x0 : old;
        }
      }
      x[2 * u] = x0;
      x[2 * u + 1] = x1;
      b4 |= ((ok0 && !fast0) ? 1u : 0u) << (2 * u);
      b4 |= ((ok1 && !fast1) ? 2u : 0u) << (2 * u);
    }
  } else {  // OP_ZIG32
    uint32_t uw[4];
    if (!LCG) {
      const uint64_t zc = seed + GAMMA * (1ull + ((uint64_t)s << 48) + (vc >> 1));
      const uint64_t Wa = mix64(zc + LC.g[0]), Wb = mix64(zc + LC.g[1]);
      if ((vc & 1) == 0) {
        uw[0] = (uint32_t)(Wa >> 32);
        uw[1] = (uint32_t)Wa;
        uw[2] = (uint32_t)(Wb >> 32);
        uw[3] = (uint32_t)Wb;
      } else {
        const uint64_t Wc = mix64(zc + LC.g[2]);
        uw[0] = (uint32_t)Wa;
        uw[1] = (uint32_t)(Wb >> 32);
        uw[2] = (uint32_t)Wb;
        uw[3] = (uint32_t)(Wc >> 32);
      }
    } else {
#pragma unroll
      for (int t = 0; t < 4; ++t) uw[t] = (uint32_t)(lcg_word_from(aff(LC.a[t], Sc)) >> 32);
    }
    const uint64_t e0 = ec + 4ull * lane;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const Fast32 f = f32t[uw[t] >> 24];
      const uint32_t j = uw[t] & 0xFFFFFFu;
      const bool ok = FULL || e0 + t < e_end;
      xf[t] = (float)j * f.w;
      b4 |= ((ok && !(j < f.k)) ? 1u : 0u) << t;
    }
  }
  return b4;
}

// Writes the lane's elements of a step from registers (masked at e_end).
template <int OP, bool FULL>
DEV void step_store(const Job &J, uint64_t ec, uint64_t e_end, const double *x, const float *xf) {
  const uint32_t lane = lane_id();
  if (OP == OP_ZIG32) {
    const uint64_t e0 = ec + 4ull * lane;
    float *out = (float *)J.out + e0;
    if (FULL || e0 + 3 < e_end) {
      *(float4 *)out = make_float4(xf[0], xf[1], xf[2], xf[3]);
    } else {
#pragma unroll
      for (int t = 0; t < 3; ++t)
        if (e0 + t < e_end) out[t] = xf[t];
    }
  } else {
#pragma unroll
    for (uint32_t u = 0; u < 2; ++u) {
      const uint64_t ea = ec + u * 128ull + 2ull * lane;
      double *out = (double *)J.out + ea;
      if (FULL || ea + 1 < e_end)
        *(double2 *)out = make_double2(x[2 * u], x[2 * u + 1]);
      else if (ea < e_end)
        out[0] = x[2 * u];
    }
  }
}

// Fast path of a step that straddles a stream boundary: every element is
// keyed by itself (stream and index from its element number).  Same outputs
// and slow bits as step_regs.
template <int OP, int KIND>
DEV uint32_t step_general(const Job &J, const Fast64 *f64t, const Fast32 *f32t,
                          const DevTables *T, uint64_t ec, uint64_t e_end, double *x, float *xf) {
  const uint32_t lane = lane_id();
  uint32_t b4 = 0;
#pragma unroll
  for (uint32_t t = 0; t < 4; ++t) {
    const uint64_t e = slot_elem<OP>(ec, lane, t);
    if (e < e_end) {
      uint32_t s;
      uint64_t v;
      split(J, e, s, v);
      bool fast;
      if (OP == OP_ZIG32) {
        const uint32_t u = word32<KIND>(T, J.seed, s, v, 0);
        const Fast32 f = f32t[u >> 24];
        const uint32_t j = u & 0xFFFFFFu;
        xf[t] = (float)j * f.w;
        fast = j < f.k;
      } else if (OP == OP_MZ64) {
        x[t] = fast_mz(f64t, longk<KIND>(T, J.seed, s, v, 0), fast);
      } else {
        x[t] = fast64(f64t, wordk<KIND>(T, J.seed, s, v, 0), fast);
        if (OP == OP_MUTATE) {
          const double old = ((const double *)J.out)[e];
          x[t] = fast ? old + J.sigma * x[t] : old;
        }
      }
      b4 |= (fast ? 0u : 1u) << t;
    }
  }
  return b4;
}

// Stores the resolved value z of element e (the placeholder is overwritten;
// for mutation the placeholder is the old value).
template <int OP>
DEV void patch_store(const Job &J, uint64_t e, double z) {
  if (OP == OP_ZIG32) {
    ((float *)J.out)[e] = (float)z;
  } else {
    double *out = (double *)J.out;
    if (OP == OP_MUTATE)
      out[e] = out[e] + J.sigma * z;
    else
      out[e] = z;
  }
}

// Resolves element e in its own lane and stores it over its placeholder
// (queue overflow only).
template <int OP, int KIND>
DEV void resolve_store(const Job &J, const LdsTabs &L, const DevTables *T, uint32_t dmax,
                       uint64_t e, uint32_t *flags) {
  uint32_t se;
  uint64_t ve;
  split(J, e, se, ve);
  bool budget = false;
  patch_store<OP>(J, e, resolve<OP, KIND>(J, L, T, T->r, dmax, se, ve, budget));
  if (budget) raise_flag(flags, ZG_FLAG_BUDGET);
}

// Attempt d of variate v of stream s: the layer i, the sign, and x (the
// attempt's abscissa); returns whether the attempt passes the fast test,
// and then z is its value (the same arithmetic as resolve).
template <int OP, int KIND>
DEV bool attempt_at(const Job &J, const LdsTabs &L, const DevTables *T, uint32_t s, uint64_t v,
                    uint32_t d, uint32_t &i, uint32_t &neg, double &x, double &z) {
  if (OP == OP_ZIG32) {
    const uint32_t u = word32<KIND>(T, J.seed, s, v, d);
    i = u >> 25;
    neg = (u >> 24) & 1;
    const uint32_t j = u & 0xFFFFFFu;
    const Fast32 f = L.f32[2 * i];
    const float xf = (float)j * f.w;
    z = (double)(neg ? -xf : xf);
    x = (double)j * L.w24d[i];
    return j < f.k;
  } else {
    const uint64_t W = wordk<KIND>(T, J.seed, s, v, d);
    i = (uint32_t)(W >> 57);
    neg = (uint32_t)(W >> 56) & 1;
    const uint32_t jh = j_hi((uint32_t)(W >> 32)), jl = j_lo((uint32_t)(W >> 32), (uint32_t)W);
    const Fast64 f = L.f64[2 * i];
    x = to_f64(jh, jl) * f.w;
    z = neg ? -x : x;
    return (((uint64_t)jh << 32) | jl) < f.k;
  }
}

// First drain step of slow element e: its attempt 0 in a wedge (and, on
// rejection, the fast test of attempt 2).  A variate still undecided after
// that, or whose attempt 0 falls in the base strip (the tail's logarithm),
// goes to the retry queue (capacity rqc <= RQ), where full rounds of 64
// finish such variates together; with the retry queue full the lane
// finishes it itself.  The steps, draws and arithmetic are those of resolve.
// The first drain step of variate v of stream s whose attempt 0 failed the
// fast test: that attempt's wedge test and, on rejection, the fast test of
// attempt 2.  Returns whether that decided the variate (value z); otherwise
// d is the draw to resume from (0 for a base-strip attempt, 2 after a wedge
// rejection).  The steps, draws and arithmetic are those of resolve.
template <int OP, int KIND>
DEV bool first_step(const Job &J, const LdsTabs &L, const DevTables *T, uint32_t dmax, uint32_t s,
                    uint64_t v, double &z, uint32_t &d, bool &budget) {
  // modified ziggurat: the region and its first attempt pair
  if (OP == OP_MZ64) return mz_run<KIND>(J, T, dmax, s, v, 0, 1, z, d, budget);
  uint32_t i, neg;
  double x;
  d = 0;
  bool done = attempt_at<OP, KIND>(J, L, T, s, v, 0, i, neg, x, z);
  if (d >= dmax) {
    budget = true;
    z = nan64();
    done = true;
  } else if (!done && i != 0) {
    if (d + 1 >= dmax) {
      budget = true;
      z = nan64();
      done = true;
    } else {
      const double u = u53(wordk<KIND>(T, J.seed, s, v, d + 1));
      const double2 yd = L.yd[i];
      if (yd.x + u * yd.y < exp(-0.5 * (x * x))) {
        z = neg ? -x : x;
        done = true;
      } else {
        d += 2;
        if (d >= dmax) {
          budget = true;
          z = nan64();
          done = true;
        } else {
          done = attempt_at<OP, KIND>(J, L, T, s, v, d, i, neg, x, z);
        }
      }
    }
  }
  return done;
}

template <int OP, int KIND>
DEV void drain_first(const Job &J, BlockLds &L, const DevTables *T, double r, uint32_t dmax,
                     uint32_t rqc, uint64_t e, bool &budget) {
  uint32_t s;
  uint64_t v;
  split(J, e, s, v);
  uint32_t d;
  double z;
  const bool done = first_step<OP, KIND>(J, L.t, T, dmax, s, v, z, d, budget);
  if (!done) {
    const uint32_t p = atomicAdd(&L.rcnt, 1u);
    if (p < rqc) {
      L.rq[p] = e | ((uint64_t)d << ENT_D);
      return;
    }
    z = resolve<OP, KIND>(J, L.t, T, r, dmax, s, v, budget, d);
  }
  patch_store<OP>(J, e, z);
}

// A round over retry entries [p0, p0 + n) (n <= 64), one per lane, each
// finished by resolve from its recorded draw.
template <int OP, int KIND>
DEV void retry_round(const Job &J, const BlockLds &L, const DevTables *T, double r, uint32_t dmax,
                     uint32_t p0, uint32_t n, bool &budget) {
  const uint32_t lane = lane_id();
  if (lane < n) {
    const uint64_t ent = L.rq[p0 + lane];
    const uint64_t e = ent & ENT_E;
    uint32_t s;
    uint64_t v;
    split(J, e, s, v);
    patch_store<OP>(J, e, resolve<OP, KIND>(J, L.t, T, r, dmax, s, v, budget,
                                            (uint32_t)(ent >> ENT_D)));
  }
}

// Finishes every entry of the retry queue (capacity rqc; whole workgroup,
// the caller brackets this with barriers).
template <int OP, int KIND>
DEV void retry_all(const Job &J, BlockLds &L, const DevTables *T, double r, uint32_t dmax,
                   uint32_t rqc, bool &budget) {
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t wave = uni(threadIdx.x >> 6);
  const uint32_t n = uni(L.rcnt < rqc ? L.rcnt : rqc);
  for (uint32_t b = wave * 64; b < n; b += nw * 64)
    retry_round<OP, KIND>(J, L, T, r, dmax, b, n - b < 64 ? n - b : 64, budget);
}

// The streaming pass over a workgroup tile [b0, b1): the waves take groups
// of gsteps steps (1..8; 256 elements each) in turn from a shared counter, so that
// they all run out of work together.  Per step: fast path and stores; per
// group, each lane with slow elements appends them to the workgroup queue
// (one LDS atomic per such lane; queue order is immaterial, every result is
// keyed by its element).  Elements that do not fit in the queue are resolved
// by their own lane at once, after its own store of the same address.
template <int OP, int KIND>
DEV void tile_pass(const Job &J, BlockLds &L, const DevTables *T, const LaneConst &LC,
                   uint64_t b0, uint64_t b1, uint32_t qcap, uint32_t dmax, uint32_t *flags,
                   uint32_t gsteps) {
  const uint32_t GE = gsteps * BSTEP;
  const uint32_t lane = lane_id();
  const bool multi = J.n_streams != 1;
  for (;;) {
    uint32_t g = 0;
    if (lane == 0) g = atomicAdd(&L.next, 1u);
    const uint32_t gofs = uni(g) * GE;   // the group's first element, from b0
    const uint64_t gs = b0 + gofs;
    if (gs >= b1) break;
    const uint64_t ge = gs + GE < b1 ? gs + GE : b1;
    uint32_t s = J.s0;
    uint64_t rr = gs;
    if (multi) {
      uint64_t v;
      split(J, gs, s, v);
      s = uni(s);
      rr = uni64(v - J.first);
    }
    uint32_t bits = 0, sub = 0;
    uint64_t Sc = 0;   // LCG: the first state of the step's word (wave-uniform)
    bool have = false;
    for (uint64_t ec = gs; ec < ge; ec += BSTEP, ++sub) {
      double x[4];
      float xf[4];
      uint32_t b4;
      const bool full = ec + BSTEP <= ge;
      if (!multi || rr + BSTEP <= J.n_per) {
        const uint64_t vc = J.first + rr;
        if (KIND == ZG_JAVA_LCG48 && !have) {
          Sc = lcg_jump(&T->lcg, lcg_state0(J.seed), 2 * lcg_index(s, vc, 0) + 1);
          have = true;
        }
        if (full)
          b4 = step_regs<OP, KIND, true>(J, L.t.f64, L.t.f32, T, LC, ec, ge, s, vc, Sc, x, xf);
        else
          b4 = step_regs<OP, KIND, false>(J, L.t.f64, L.t.f32, T, LC, ec, ge, s, vc, Sc, x, xf);
        if (KIND == ZG_JAVA_LCG48) Sc = aff(T->lcg.jump[1][2], Sc);   // 2 x 256 LCG steps on
      } else {
        b4 = step_general<OP, KIND>(J, L.t.f64, L.t.f32, T, ec, ge, x, xf);
        have = false;
      }
      if (full)
        step_store<OP, true>(J, ec, ge, x, xf);
      else
        step_store<OP, false>(J, ec, ge, x, xf);
      bits |= b4 << (4 * sub);
      rr += BSTEP;
      if (multi)
        while (rr >= J.n_per) {
          rr -= J.n_per;
          ++s;
          have = false;
        }
    }
    if (bits) {
      uint32_t p = atomicAdd(&L.cnt, (uint32_t)__builtin_popcount(bits));
      do {
        const uint32_t b = __builtin_ctz(bits);
        bits &= bits - 1;
        const uint32_t off = gofs + (b >> 2) * BSTEP + (uint32_t)slot_elem<OP>(0, lane, b & 3);
        if (p < qcap)
          L.q[p] = off;
        else
          resolve_store<OP, KIND>(J, L.t, T, dmax, b0 + off, flags);
        ++p;
      } while (bits);
    }
  }
}

// One workgroup tile [b0, b1) of job J: streaming pass, one barrier, pooled
// drain; `head` elements before b0 (the unaligned start of the job) are
// resolved too when non-zero.  The tables in L are loaded; the caller
// separates consecutive calls with a barrier (the queue count and the group
// counter are reset here, before the first barrier).
template <int OP, int KIND>
DEV void zig_block(const Job &J, BlockLds &L, const DevTables *__restrict__ T,
                   const LaneConst &LC, double r, uint32_t dmax, uint32_t *flags, uint64_t b0,
                   uint64_t b1, uint32_t head, uint32_t qcap, bool carry, bool &budget,
                   uint32_t gsteps) {
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t wave = uni(threadIdx.x >> 6);
  const uint32_t lane = lane_id();
  const uint32_t rqc = qcap < RQ ? qcap : RQ;   // a forced small queue caps both
  if (threadIdx.x == 0) {
    L.cnt = 0;
    L.next = 0;
    // retries carried from earlier tiles (same job): whole rounds, one per wave
    const uint32_t rc = carry ? (L.rcnt < rqc ? L.rcnt : rqc) : 0;
    uint32_t take = rc / 64 * 64;
    if (take > nw * 64) take = nw * 64;
    L.rtake = take;
    L.rbeg = rc - take;
    L.rcnt = rc - take;
  }
  __syncthreads();
  if (wave * 64 < uni(L.rtake))
    retry_round<OP, KIND>(J, L, T, r, dmax, uni(L.rbeg) + wave * 64, 64, budget);
  tile_pass<OP, KIND>(J, L, T, LC, b0, b1, qcap, dmax, flags, gsteps);
  __syncthreads();   // placeholders before patches; the queue is complete
  const uint32_t n = uni(L.cnt < qcap ? L.cnt : qcap);
  for (uint32_t cb = wave * 64; cb < n; cb += nw * 64) {
    const uint32_t p = cb + lane;
    if (p < n) drain_first<OP, KIND>(J, L, T, r, dmax, rqc, b0 + L.q[p], budget);
  }
  if (!carry) {
    __syncthreads();   // the retry queue is complete
    retry_all<OP, KIND>(J, L, T, r, dmax, rqc, budget);
  }
  // the elements before the first aligned one (wave 0)
  if (wave == 0 && lane < head) {
    uint32_t se;
    uint64_t ve;
    split(J, lane, se, ve);
    patch_store<OP>(J, lane, resolve<OP, KIND>(J, L.t, T, r, dmax, se, ve, budget));
  }
}

// Plain fills: workgroup tile t covers [head + t bt, + bt), bt = waves x tile;
// a workgroup takes tiles blockIdx.x, + gridDim.x, ... (one tile each when
// the grid has one workgroup per tile).
template <int OP, int KIND>
__global__ __launch_bounds__(1024) void k_zig(Job J, const DevTables *__restrict__ T,
                                              uint32_t dmax, uint32_t *flags, uint32_t tile,
                                              uint32_t head, uint32_t qcap, uint64_t ntiles,
                                              uint32_t gsteps) {
  __shared__ BlockLds L;
  load_tabs<OP>(T, L.t);
  const double r = T->r;
  const LaneConst LC = lane_constants<OP, KIND>(T);
  bool budget = false;
  if (threadIdx.x == 0) L.rcnt = 0;
  const uint64_t bt = (uint64_t)tile * (blockDim.x >> 6);
  for (uint64_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
    const uint64_t b0 = uni64(t * bt + head);
    const uint64_t b1 = uni64(b0 + bt < J.n_total ? b0 + bt : J.n_total);
    zig_block<OP, KIND>(J, L, T, LC, r, dmax, flags, b0, b1, t == 0 ? head : 0u, qcap, true,
                        budget, gsteps);
    __syncthreads();   // the next tile resets the queue
  }
  __syncthreads();
  retry_all<OP, KIND>(J, L, T, r, dmax, qcap < RQ ? qcap : RQ, budget);
  if (__builtin_amdgcn_ballot_w64(budget) != 0 && lane_id() == 0)
    raise_flag(flags, ZG_FLAG_BUDGET);
}

// ------------------------------------------- wave-specialised ziggurat fill
//
// The same values as k_zig, with the slow path taken off the streaming
// waves.  Workgroup w owns one contiguous range of the job.  Its first S
// waves stream the range in groups of 4 steps (1024 elements) taken from a
// shared counter: fast path, 128-bit stores with a placeholder where an
// element failed the fast test, and each such element published in an LDS
// ring right after its store.  The other waves (one per SIMD) take the
// ring's entries in rounds of 64, one per lane, resolve each variate in full
// (resolve: every attempt from draw 0) and store it over its placeholder.
// No streaming wave waits at a barrier, and a patch follows its placeholder
// closely, while the line is still in L2.  The ring entry is published after
// a workgroup-scope release and read before a workgroup-scope acquire, so
// each patch is ordered after its placeholder.
//
// Ring protocol: a writer reserves slots with an atomic on `tail` and waits
// until its slot is empty (0) before writing element + 1 into it; a drain
// wave claims [head, head + m) with a compare-and-swap on `head`, waits until
// each claimed slot is written, reads it and empties it.  The oldest
// unconsumed slot always has its writer able to proceed (its slot's previous
// occupant is older, hence consumed), so the ring never deadlocks.  The
// drain waves leave once every streaming wave has finished and the ring is
// empty; the elements before the first aligned one are resolved after a
// final barrier.

constexpr uint32_t WS_RING = 2048;   // ring slots (a power of two)

constexpr uint32_t WS_MAX_DRAIN = 8;
constexpr uint32_t WS_RQ = 128;     // retry entries per drain wave

struct WsLds {
  LdsTabs t;
  uint32_t next;    // next group of the workgroup's range to stream
  uint32_t tail;    // ring slots reserved
  uint32_t head;    // ring slots claimed by drain waves
  uint32_t done;    // streaming waves that have finished
  uint64_t ring[WS_RING];   // element + 1; 0 = empty
  uint64_t rq[WS_MAX_DRAIN][WS_RQ];   // each drain wave's undecided variates (element | draw << ENT_D)
};

DEV uint32_t lds_load(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Ring and retry entries of the batch kernel carry the request: ring entry
// (request << 40 | element) + 1, retry entry element | draw << 40 |
// request << 49 (elements < 2^40, draws <= ZG_MAX_DRAWS < 2^9, requests <
// ZG_MAX_BATCH = 2^15).  The plain kernel's entries are element + 1, and
// element | draw << ENT_D.
constexpr uint32_t WSB_E = 40;
constexpr uint64_t WSB_EMASK = (1ull << WSB_E) - 1;
constexpr uint32_t WSB_R = 49;
static_assert(ZG_MAX_BATCH <= (1u << (64 - WSB_R)) && ZG_MAX_DRAWS < (1u << (WSB_R - WSB_E)),
              "batch ring entry fields");

// Streams elements [gs, ge) of a job (one group: whole steps, and a ragged
// last one at a job's end) with 128-bit stores and placeholders, then
// publishes the lane's slow elements in the ring, each as tag | element.
template <int OP, int KIND>
DEV void ws_group(const Job &J, WsLds &L, const DevTables *T, const LaneConst &LC, uint64_t gs,
                  uint64_t ge, uint64_t tag) {
  const uint32_t lane = lane_id();
  const bool multi = J.n_streams != 1;
  uint32_t s = J.s0;
  uint64_t rr = gs;
  if (multi) {
    uint64_t v;
    split(J, gs, s, v);
    s = uni(s);
    rr = uni64(v - J.first);
  }
  uint32_t bits = 0, sub = 0;
  uint64_t Sc = 0;
  bool have = false;
  for (uint64_t ec = gs; ec < ge; ec += BSTEP, ++sub) {
    double x[4];
    float xf[4];
    uint32_t b4;
    if (ec + 2 * BSTEP <= ge && (!multi || rr + 2 * BSTEP <= J.n_per)) {
      // two whole steps of one stream: both steps' words are computed before
      // either step's stores, so their hash chains overlap
      const uint64_t vc = J.first + rr;
      if (KIND == ZG_JAVA_LCG48 && !have) {
        Sc = lcg_jump(&T->lcg, lcg_state0(J.seed), 2 * lcg_index(s, vc, 0) + 1);
        have = true;
      }
      double x2[4];
      float xf2[4];
      b4 = step_regs<OP, KIND, true>(J, L.t.f64, L.t.f32, T, LC, ec, ge, s, vc, Sc, x, xf);
      if (KIND == ZG_JAVA_LCG48) Sc = aff(T->lcg.jump[1][2], Sc);
      const uint32_t b4b = step_regs<OP, KIND, true>(J, L.t.f64, L.t.f32, T, LC, ec + BSTEP, ge, s,
                                                     vc + BSTEP, Sc, x2, xf2);
      if (KIND == ZG_JAVA_LCG48) Sc = aff(T->lcg.jump[1][2], Sc);
      step_store<OP, true>(J, ec, ge, x, xf);
      step_store<OP, true>(J, ec + BSTEP, ge, x2, xf2);
      bits |= (b4 | b4b << 4) << (4 * sub);
      ec += BSTEP;
      ++sub;
      rr += 2 * BSTEP;
      if (multi)
        while (rr >= J.n_per) {
          rr -= J.n_per;
          ++s;
          have = false;
        }
      continue;
    }
    const bool full = ec + BSTEP <= ge;
    if (!multi || rr + BSTEP <= J.n_per) {
      const uint64_t vc = J.first + rr;
      if (KIND == ZG_JAVA_LCG48 && !have) {
        Sc = lcg_jump(&T->lcg, lcg_state0(J.seed), 2 * lcg_index(s, vc, 0) + 1);
        have = true;
      }
      if (full)
        b4 = step_regs<OP, KIND, true>(J, L.t.f64, L.t.f32, T, LC, ec, ge, s, vc, Sc, x, xf);
      else
        b4 = step_regs<OP, KIND, false>(J, L.t.f64, L.t.f32, T, LC, ec, ge, s, vc, Sc, x, xf);
      if (KIND == ZG_JAVA_LCG48) Sc = aff(T->lcg.jump[1][2], Sc);
    } else {
      b4 = step_general<OP, KIND>(J, L.t.f64, L.t.f32, T, ec, ge, x, xf);
      have = false;
    }
    if (full)
      step_store<OP, true>(J, ec, ge, x, xf);
    else
      step_store<OP, false>(J, ec, ge, x, xf);
    bits |= b4 << (4 * sub);
    rr += BSTEP;
    if (multi)
      while (rr >= J.n_per) {
        rr -= J.n_per;
        ++s;
        have = false;
      }
  }
  if (bits) {
    // the placeholders before their ring entries
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    uint32_t p = atomicAdd(&L.tail, (uint32_t)__builtin_popcount(bits));
    do {
      const uint32_t b = __builtin_ctz(bits);
      const uint64_t e = gs + (b >> 2) * BSTEP + slot_elem<OP>(0, lane, b & 3);
      uint64_t *slot = &L.ring[p & (WS_RING - 1)];
      while (__hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP) != 0)
        __builtin_amdgcn_s_sleep(1);
      __hip_atomic_store(slot, (tag | e) + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      bits &= bits - 1;
      ++p;
    } while (bits);
  }
}

// Streaming role: the workgroup's groups in turn (group c of workgroup w is
// group c * gridDim.x + w of the body that starts at b0, so the workgroups
// write neighbouring groups at any time), each lane's slow elements published
// in the ring after the group's stores.
template <int OP, int KIND>
DEV void ws_stream(const Job &J, WsLds &L, const DevTables *T, const LaneConst &LC, uint64_t b0,
                   uint64_t b1, uint32_t gsteps) {
  const uint32_t lane = lane_id();
  const uint32_t GE = gsteps * BSTEP;
  for (;;) {
    uint32_t g = 0;
    if (lane == 0) g = atomicAdd(&L.next, 1u);
    const uint64_t gs = b0 + ((uint64_t)uni(g) * gridDim.x + blockIdx.x) * GE;
    if (gs >= b1) break;
    ws_group<OP, KIND>(J, L, T, LC, gs, gs + GE < b1 ? gs + GE : b1, 0);
  }
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
  if (lane == 0) atomicAdd(&L.done, 1u);
}

// A round over the last n (<= 64) entries of a drain wave's retry queue,
// one per lane, each finished by resolve from its recorded draw.
// BATCH: entries name their request, whose job the lane reads (R).
template <int OP, int KIND, bool BATCH>
DEV void ws_retry(const Job &J0, const DevRequest *R, const LdsTabs &L, const DevTables *T,
                  double r, uint32_t dmax, const uint64_t *rq, uint32_t base, uint32_t n,
                  bool &budget) {
  const uint32_t lane = lane_id();
  if (lane < n) {
    const uint64_t ent = rq[base + lane];
    const uint64_t e = BATCH ? ent & WSB_EMASK : ent & ENT_E;
    const uint32_t d = BATCH ? (uint32_t)(ent >> WSB_E) & ((1u << (WSB_R - WSB_E)) - 1)
                             : (uint32_t)(ent >> ENT_D);
    const Job J = BATCH ? R[ent >> WSB_R].job : J0;
    uint32_t s;
    uint64_t v;
    split(J, e, s, v);
    patch_store<OP>(J, e, resolve<OP, KIND>(J, L, T, r, dmax, s, v, budget, d));
  }
}

// Drain role: rounds of up to 64 ring entries until every streaming wave has
// finished and the ring is empty.  While streaming goes on, only full rounds
// are claimed.  Each entry gets its first drain step; the few it leaves
// undecided (and the base-strip attempts) go to the wave's own retry queue,
// which is finished 64 at a time, the rest at the end.
template <int OP, int KIND, bool BATCH>
DEV void ws_drain(const Job &J0, const DevRequest *R, WsLds &L, const DevTables *T, double r,
                  uint32_t dmax, uint32_t n_stream, uint32_t slot_id, bool &budget) {
  const uint32_t lane = lane_id();
  uint64_t *rq = L.rq[slot_id];
  uint32_t rn = 0;   // wave-uniform
  for (;;) {
    const uint32_t fin = uni(lds_load(&L.done));
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
    const uint32_t h = uni(lds_load(&L.head));
    const uint32_t tl = uni(lds_load(&L.tail));
    const uint32_t avail = tl - h;
    if (avail == 0 && fin == n_stream) break;
    if (avail < 64 && fin != n_stream) {
      __builtin_amdgcn_s_sleep(2);
      continue;
    }
    const uint32_t m = avail < 64 ? avail : 64;
    uint32_t got = 0;
    if (lane == 0) got = atomicCAS(&L.head, h, h + m) == h ? 1u : 0u;
    if (uni(got) == 0) continue;
    bool und = false;
    uint64_t rent = 0;
    if (lane < m) {
      uint64_t *slot = &L.ring[(h + lane) & (WS_RING - 1)];
      uint64_t ent;
      while ((ent = __hip_atomic_load(slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) == 0)
        __builtin_amdgcn_s_sleep(1);
      __hip_atomic_store(slot, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
      const uint64_t x = ent - 1;
      const uint64_t e = BATCH ? x & WSB_EMASK : x;
      const Job J = BATCH ? R[x >> WSB_E].job : J0;
      uint32_t s;
      uint64_t v;
      split(J, e, s, v);
      double z;
      uint32_t d;
      if (first_step<OP, KIND>(J, L.t, T, dmax, s, v, z, d, budget)) {
        patch_store<OP>(J, e, z);
      } else {
        und = true;
        rent = BATCH ? e | ((uint64_t)d << WSB_E) | ((x >> WSB_E) << WSB_R)
                     : e | ((uint64_t)d << ENT_D);
      }
    }
    // undecided: to this wave's retry queue (rn < 64 before, so it fits)
    const uint64_t mk = __builtin_amdgcn_ballot_w64(und);
    if (mk) {
      if (und) rq[rn + prefix_below(mk)] = rent;
      rn = uni(rn + (uint32_t)__popcll(mk));
      __builtin_amdgcn_wave_barrier();
    }
    if (rn >= 64) {
      rn -= 64;
      ws_retry<OP, KIND, BATCH>(J0, R, L.t, T, r, dmax, rq, rn, 64, budget);
      __builtin_amdgcn_wave_barrier();
    }
  }
  while (rn) {
    const uint32_t m = rn < 64 ? rn : 64;
    rn -= m;
    ws_retry<OP, KIND, BATCH>(J0, R, L.t, T, r, dmax, rq, rn, m, budget);
    __builtin_amdgcn_wave_barrier();
  }
}

// Plain fills, wave-specialised: a persistent grid; workgroup w streams the
// groups w, w + gridDim.x, ... of the body [head, n_total) with its first
// (waves - n_drain) waves while its last n_drain waves resolve the slow
// elements.
template <int OP, int KIND>
__global__ __launch_bounds__(1024) void k_zigws(Job J, const DevTables *__restrict__ T,
                                                uint32_t dmax, uint32_t *flags, uint32_t head,
                                                uint32_t n_drain, uint32_t gsteps) {
  __shared__ WsLds L;
  load_tabs<OP>(T, L.t);
  for (uint32_t i = threadIdx.x; i < WS_RING; i += blockDim.x) L.ring[i] = 0;
  if (threadIdx.x == 0) {
    L.next = 0;
    L.tail = 0;
    L.head = 0;
    L.done = 0;
  }
  __syncthreads();
  const double r = T->r;
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t n_stream = nw - n_drain;
  const uint32_t wave = uni(threadIdx.x >> 6);
  const uint32_t lane = lane_id();
  bool budget = false;
  if (wave < n_stream) {
    const LaneConst LC = lane_constants<OP, KIND>(T);
    ws_stream<OP, KIND>(J, L, T, LC, head, J.n_total, gsteps);
  } else {
    // The drain waves share each SIMD with streaming waves.  At equal issue
    // priority their long dependent chains (hashes, exp, log) fall behind
    // the slow elements the streaming waves publish, the ring fills and the
    // streaming waves wait on it; one step of priority keeps the drain ahead
    // (the streaming waves still fill the store pipe).
    __builtin_amdgcn_s_setprio(1);
    ws_drain<OP, KIND, false>(J, nullptr, L, T, r, dmax, n_stream, wave - n_stream, budget);
  }
  __syncthreads();
  // the elements before the first aligned one
  if (blockIdx.x == 0 && wave == 0 && lane < head) {
    uint32_t se;
    uint64_t ve;
    split(J, lane, se, ve);
    patch_store<OP>(J, lane, resolve<OP, KIND>(J, L.t, T, r, dmax, se, ve, budget));
  }
  if (__builtin_amdgcn_ballot_w64(budget) != 0 && lane == 0) raise_flag(flags, ZG_FLAG_BUDGET);
}

// ------------------------------------------------- one EA generation step
//
// One wave per child at a time (children: the global wave index, then every
// wave count further).  The tournament's draws run in lanes 0..63; the
// winner is taken in draw order (the first draw of least fitness, a number
// beating a NaN), the fitness of each draw read by a scalar load (per-lane
// loads, for tournaments of more than 64 draws).  The child's genes then go
// in groups of EA_U chunks of 64, one gene per lane per chunk:
// - the winner's 64 EA_U genes loaded, all loads issued before any is used
//   (EA_U x 512 bytes in flight per wave);
// - each gene's mutation decided from its own word, whose key is a
//   wave-uniform part plus a per-lane constant (an add per gene, not a
//   multiply); the mutating genes listed in LDS;
// - the list's variates drawn 64 at a time, one gene per lane (ziggurat fast
//   path and, rarely, the slow path), back into LDS: the variate's code runs
//   once per 64 mutating genes, not once per chunk for its few mutating
//   lanes (5% of the genes at the usual rates);
// - each chunk stored once: the winner's gene, or it plus sigma times its
//   variate, clamped.  Whole cache lines are written at once; a line
//   written in two parts (the unmutated genes, later the mutated ones) can
//   leave L2 in between and cost HBM a second, partial write.

DEV double readlane_f64(double x, uint32_t q) {
  const long long b = __double_as_longlong(x);
  const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)b, (int)q);
  const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), (int)q);
  return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

constexpr uint32_t EA_WAVES = 8;    // waves per workgroup
constexpr uint32_t EA_BPC = 4;      // workgroups per compute unit in the grid

// U: gene chunks of 64 per group (2, 4 or 8, from the genome's length)
template <uint32_t U>
struct EaLds {
  LdsTabs t;
  double z[EA_WAVES][64 * U];     // their variates
  uint32_t g[EA_WAVES][64 * U];   // the group's mutating genes
};

// The draws of one tournament chunk (draws t0 + lane): winner index, fitness.
DEV void ea_draws(const EaJob &E, uint64_t u, uint32_t t0, uint32_t &idx, double &f) {
  const uint32_t t = t0 + lane_id();
  idx = 0;
  f = 0.0;
  if (t < E.tournament) {
    idx = (uint32_t)__umul64hi(sm64_word(E.seed, E.stream, u, t), (uint64_t)E.pop);
    f = E.fitness[idx];
  }
}

// A fitness value read with a wave-uniform index, through the constant
// address space: a scalar load, waited for on its own counter, so that the
// fold does not wait for the wave's outstanding gene stores.
DEV double fitness_uniform(const double *f, uint32_t i) {
  return ((const __attribute__((address_space(4))) double *)f)[i];
}

// Folds tournament draws 0 .. k - 1 of child key u (k <= 64): the winners'
// indices from the lanes, their fitness by scalar loads.
DEV void ea_fold_short(const EaJob &E, uint64_t u, uint32_t &best) {
  const uint32_t t = lane_id();
  const uint32_t idx =
      t < E.tournament
          ? (uint32_t)__umul64hi(sm64_word(E.seed, E.stream, u, t), (uint64_t)E.pop)
          : 0u;
  double fbest = 0.0;
  for (uint32_t q = 0; q < E.tournament; ++q) {
    const uint32_t iq = (uint32_t)__builtin_amdgcn_readlane((int)idx, (int)q);
    const double fq = fitness_uniform(E.fitness, iq);
    if (q == 0 || fq < fbest || (isnan(fbest) && !isnan(fq))) {
      best = iq;
      fbest = fq;
    }
  }
}

// Folds the draws t0 .. t0 + m - 1 (lanes 0 .. m - 1) into (best, fbest).
DEV void ea_fold(uint32_t idx, double f, uint32_t m, bool first, uint32_t &best, double &fbest) {
  for (uint32_t q = 0; q < m; ++q) {
    const uint32_t iq = (uint32_t)__builtin_amdgcn_readlane((int)idx, (int)q);
    const double fq = readlane_f64(f, q);
    if ((first && q == 0) || fq < fbest || (isnan(fbest) && !isnan(fq))) {
      best = iq;
      fbest = fq;
    }
  }
}

template <int KIND, uint32_t EA_U>
__global__ __launch_bounds__(64 * EA_WAVES) void k_ea(EaJob E, const DevTables *__restrict__ T,
                                                     uint32_t dmax, uint32_t *flags) {
  __shared__ EaLds<EA_U> L;
  load_tabs<OP_ZIG64>(T, L.t);
  __syncthreads();
  const double r = T->r;
  const uint32_t lane = lane_id();
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t wave = uni(threadIdx.x >> 6);
  uint32_t *ql = L.g[wave];
  double *qz = L.z[wave];
  const uint64_t tw = (uint64_t)gridDim.x * nw;
  Job Jz{};   // the variates' key: the seed (stream and index per gene)
  Jz.seed = E.seed;
  Jz.kind = KIND;
  Jz.op = OP_ZIG64;
  bool budget = false;
  // the mutation word of gene w is mix64(seed + GAMMA (1 + (stream + 1) 2^48 + w)):
  // a wave-uniform part per chunk plus GAMMA lane (mod 2^64).  The per-lane
  // term is opaque to the compiler, which would otherwise fold the sum back
  // into a multiply per gene.
  uint64_t klane = GAMMA * (uint64_t)lane;
  asm volatile("" : "+v"(klane));

  for (uint64_t c = (uint64_t)blockIdx.x * nw + wave; c < E.pop; c += tw) {
    const uint64_t u = E.generation * E.pop + c;
    uint32_t best = 0;
    if (E.tournament <= 64) {
      ea_fold_short(E, u, best);
    } else {
      double fbest = 0.0;
      for (uint32_t t0 = 0; t0 < E.tournament; t0 += 64) {
        uint32_t idx;
        double f;
        ea_draws(E, u, t0, idx, f);
        const uint32_t m = E.tournament - t0 < 64 ? E.tournament - t0 : 64;
        ea_fold(idx, f, m, t0 == 0, best, fbest);
      }
    }
    if (lane == 0 && E.winners) E.winners[c] = best;
    const double *prow = E.parents + (uint64_t)best * E.genes;
    double *crow = E.children + c * E.genes;
    const uint64_t w0 = u * E.genes;
    // key of gene g0 of this chunk group in lane 0; advanced per group
    uint64_t kg = E.seed + GAMMA * (1ull + ((uint64_t)(E.stream + 1) << 48) + w0);
    for (uint32_t g0 = 0; g0 < E.genes; g0 += 64 * EA_U, kg += GAMMA * (64ull * EA_U)) {
      // unconditional loads (a lane past the row's end reads its last gene)
      double xv[EA_U];
#pragma unroll
      for (uint32_t k = 0; k < EA_U; ++k) {
        const uint32_t g = g0 + 64 * k + lane;
        xv[k] = prow[g < E.genes ? g : E.genes - 1];
      }
      // the decisions; the mutating genes listed, chunk by chunk
      uint32_t qn = 0;          // list length (wave-uniform)
      uint32_t at[EA_U];        // a mutating lane's list position
      uint32_t mutk = 0;        // bit k: this lane's gene of chunk k mutates
#pragma unroll
      for (uint32_t k = 0; k < EA_U; ++k) {
        const uint32_t g = g0 + 64 * k + lane;
        const uint64_t key = kg + GAMMA * (64ull * k) + klane;
        const bool mut = g < E.genes && (mix64(key) >> 11) < E.rate53;
        const uint64_t bm = __builtin_amdgcn_ballot_w64(mut);
        at[k] = qn + prefix_below(bm);
        if (mut) {
          ql[at[k]] = g;
          mutk |= 1u << k;
        }
        qn = uni(qn + (uint32_t)__popcll(bm));
      }
      __builtin_amdgcn_wave_barrier();
      // the variates, 64 genes at a time, one per lane
      for (uint32_t b = 0; b < qn; b += 64) {
        if (b + lane < qn) {
          const uint32_t g = ql[b + lane];
          qz[b + lane] =
              resolve<OP_ZIG64, KIND>(Jz, L.t, T, r, dmax, E.stream + 2, w0 + g, budget);
        }
      }
      __builtin_amdgcn_wave_barrier();
      // each chunk stored once, whole lines: the winner's gene, or it plus
      // sigma times its variate, clamped
#pragma unroll
      for (uint32_t k = 0; k < EA_U; ++k) {
        const uint32_t g = g0 + 64 * k + lane;
        // the value is needed here, on every path: the wait for its load is
        // then the exact count, not a full drain at the next group's loads
        asm volatile("" ::"v"(xv[k]));
        double x = xv[k];
        if (mutk & (1u << k)) {
          x = x + E.sigma * qz[at[k]];
          x = x < E.lo ? E.lo : (x > E.hi ? E.hi : x);
        }
        if (g < E.genes) crow[g] = x;
      }
      __builtin_amdgcn_wave_barrier();
    }
  }
  if (__builtin_amdgcn_ballot_w64(budget) != 0 && lane == 0) raise_flag(flags, ZG_FLAG_BUDGET);
}

// ---------------------------------------------------------------- kernels

// Polar method: one tile per wave; tile t covers [head + t tile, + tile).
template <int KIND>
__global__ __launch_bounds__(1024) void k_polar(Job J, const DevTables *__restrict__ T,
                                                uint32_t dmax, uint32_t *flags, uint32_t tile,
                                                uint32_t head) {
  extern __shared__ __align__(16) unsigned char s_polar[];   // log table, then waves x QCAP
  LogTables &Lt = *(LogTables *)s_polar;
  uint32_t *s_q = (uint32_t *)(s_polar + POLAR_LOG_BYTES);
  load_log_table(T, Lt);
  __syncthreads();
  const uint32_t wave = uni(threadIdx.x >> 6);
  const uint64_t gw = (uint64_t)blockIdx.x * (blockDim.x >> 6) + wave;
  const uint64_t b = head + gw * tile;
  const PolarCtx C{T, dmax, flags, &Lt};
  if (b < J.n_total || (gw == 0 && head)) {
    const LaneConst LC = lane_constants<OP_POLAR, KIND>(T);
    const uint64_t e_end = b + tile < J.n_total ? b + tile : J.n_total;
    const uint64_t e_begin = b < e_end ? b : e_end;
    polar_tile<KIND>(J, C, LC, s_q + wave * QCAP, e_begin, e_end, head, gw == 0);
  }
}

__global__ __launch_bounds__(256) void k_words(uint64_t *out, uint64_t n, const DevTables *T,
                                               uint32_t kind, uint64_t seed, uint32_t s,
                                               uint32_t d, uint64_t first) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  if (kind == ZG_JAVA_LCG48) {
    // per-thread jump-ahead to the first index, then a constant stride map
    if (i >= n) return;
    const uint64_t S0 = lcg_state0(seed);
    uint64_t S1 = lcg_jump(&T->lcg, S0, 2 * lcg_index(s, first + i, d) + 1);
    Affine step = {1, 0};
    {
      // 2*stride steps, composed from the byte tables once per thread
      uint64_t k = 2 * stride;
      for (int b = 0; b < LCG_JUMP_BYTES; ++b) {
        uint32_t x = (uint32_t)(k >> (8 * b)) & 255u;
        if (x) step = aff_cat(step, T->lcg.jump[b][x]);
      }
    }
    for (; i < n; i += stride) {
      out[i] = lcg_word_from(S1);
      S1 = aff(step, S1);
    }
  } else {
    for (; i < n; i += stride) out[i] = sm64_word(seed, s, first + i, d);
  }
}

__global__ __launch_bounds__(256) void k_decide(const uint64_t *words, uint64_t n,
                                                const DevTables *T, uint8_t *cls, double *x) {
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t W = words[i];
  uint32_t li = (uint32_t)(W >> 57);
  uint64_t j = (W >> 3) & MASK53;
  Fast64 f = T->fast64[li];
  x[i] = flip((double)j * f.w, (W >> 56) & 1);
  cls[i] = j < f.k ? 0 : (li == 0 ? 2 : 1);
}

// Resolves counter-keyed requests in submission order: every request reads
// its handle's counter as it stood before the batch, adds its offset among the
// batch's earlier requests of that handle, then the last request of each
// handle advances the counter.  One workgroup, two phases.
__global__ __launch_bounds__(1024) void k_reserve(DevRequest *R, const BatchHeader *H,
                                                  uint64_t *counters, uint32_t *flags) {
  const uint32_t nreq = H->nreq;
  for (uint32_t i = threadIdx.x; i < nreq; i += blockDim.x) {
    DevRequest &r = R[i];
    if (r.handle >= 0) {
      uint64_t first = counters[r.handle] + r.off;
      r.job.first = first;
      if (first + r.job.n_total > r.limit || first + r.job.n_total < first) {
        r.status = ZG_FLAG_RANGE;
        atomicOr(flags, ZG_FLAG_RANGE);
      }
    }
  }
  __syncthreads();
  for (uint32_t i = threadIdx.x; i < nreq; i += blockDim.x) {
    const DevRequest &r = R[i];
    if (r.handle >= 0 && r.last_of_handle) counters[r.handle] = r.job.first + r.job.n_total;
    // ordered before the completion word by the batch kernel's system fence
    if (r.first_host) *r.first_host = r.job.first;
  }
}

// Publishes the completion word of every request of a batch.  It runs after
// the class kernels (a graph dependency), so all their stores are released
// by the kernel boundary; the first indices were written by the reserve
// kernel before them.
__global__ __launch_bounds__(256) void k_complete(const DevRequest *R, const BatchHeader *H) {
  const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= H->nreq) return;
  const DevRequest &rq = R[i];
  if (!rq.done_flag) return;
  __threadfence_system();
  const uint32_t val = rq.done_value | (rq.status ? 0x80000000u : 0u);
  __hip_atomic_store(rq.done_flag, val, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

// Batch work of one ziggurat class: a persistent grid takes the class's items
// (workgroup tiles of its requests) in turn and runs each as the plain fill
// runs one workgroup tile.
template <int OP, int KIND>
__global__ __launch_bounds__(1024) void k_bzig(DevRequest *R, const BatchHeader *H,
                                               const DevTables *__restrict__ T,
                                               uint32_t *flags) {
  constexpr int C = batch_class(OP, KIND);
  const uint32_t cnt = H->cls_cnt[C];
  if (blockIdx.x >= cnt) return;
  __shared__ BlockLds L;
  load_tabs<OP>(T, L.t);
  const uint64_t *items = (const uint64_t *)((const char *)H + H->items_off);
  const uint32_t off = H->cls_off[C];
  const uint32_t dmax = H->dmax;
  const uint32_t nw = blockDim.x >> 6;
  const double r = T->r;
  const LaneConst LC = lane_constants<OP, KIND>(T);
  bool budget = false;
  for (uint32_t k = blockIdx.x; k < cnt; k += gridDim.x) {
    const uint64_t it = items[off + k];
    const DevRequest &rq = R[(uint32_t)(it >> 32)];
    const uint32_t j = (uint32_t)it;
    if (rq.status == 0) {
      const Job J = rq.job;
      const uint64_t bt = (uint64_t)rq.tile * nw;
      const uint64_t b0 = uni64(rq.head + j * bt);
      const uint64_t b1 = uni64(b0 + bt < J.n_total ? b0 + bt : J.n_total);
      zig_block<OP, KIND>(J, L, T, LC, r, dmax, flags, b0, b1, j == 0 ? rq.head : 0u, BQ, false,
                          budget, BGROUP);
    }
    __syncthreads();   // the next tile resets the queue
  }
  if (__builtin_amdgcn_ballot_w64(budget) != 0 && lane_id() == 0)
    raise_flag(flags, ZG_FLAG_BUDGET);
}

// Batch work of one ziggurat class, wave-specialised: a persistent grid, each
// workgroup's first (waves - ws_drain) waves take (item, group) units from an
// LDS counter (item i of workgroup w is the class's item w + i gridDim.x, a
// request tile of tile x waves elements, cut into groups of ws_gsteps steps)
// and stream them as the plain wave-specialised fill does, publishing slow
// elements with their request; the last ws_drain waves resolve and patch
// them, reading each entry's job from its request.  A request's elements
// before its first aligned one are resolved by the wave that streams its
// first group.
template <int OP, int KIND>
__global__ __launch_bounds__(1024) void k_bzigws(DevRequest *R, const BatchHeader *H,
                                                 const DevTables *__restrict__ T,
                                                 uint32_t *flags) {
  constexpr int C = batch_class(OP, KIND);
  const uint32_t cnt = H->cls_cnt[C];
  if (blockIdx.x >= cnt) return;
  __shared__ WsLds L;
  load_tabs<OP>(T, L.t);
  for (uint32_t i = threadIdx.x; i < WS_RING; i += blockDim.x) L.ring[i] = 0;
  if (threadIdx.x == 0) {
    L.next = 0;
    L.tail = 0;
    L.head = 0;
    L.done = 0;
  }
  __syncthreads();
  const double r = T->r;
  const uint32_t dmax = H->dmax;
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t n_stream = nw - H->ws_drain;
  const uint32_t wave = uni(threadIdx.x >> 6);
  const uint32_t lane = lane_id();
  bool budget = false;
  if (wave < n_stream) {
    const LaneConst LC = lane_constants<OP, KIND>(T);
    const uint64_t *items = (const uint64_t *)((const char *)H + H->items_off);
    const uint32_t off = H->cls_off[C];
    const uint32_t G = H->cls_groups[C];
    const uint64_t GE = (uint64_t)H->ws_gsteps * BSTEP;
    for (;;) {
      uint32_t u = 0;
      if (lane == 0) u = atomicAdd(&L.next, 1u);
      u = uni(u);
      const uint32_t i = u / G, g = u - i * G;
      const uint64_t k = blockIdx.x + (uint64_t)i * gridDim.x;
      if (k >= cnt) break;
      const uint64_t it = items[off + k];
      const uint32_t ri = uni((uint32_t)(it >> 32)), j = uni((uint32_t)it);
      const DevRequest &rq = R[ri];
      // the item's remaining groups are empty from here (a skipped request,
      // or past the tile's end): the counter moves on to the next item
      const uint32_t next_item = (i + 1) * G;
      if (rq.status != 0) {
        if (lane == 0) atomicMax(&L.next, next_item);
        continue;
      }
      const Job J = rq.job;
      const uint64_t t0 = rq.head + (uint64_t)j * rq.tile * nw;
      const uint64_t t1 = t0 + (uint64_t)rq.tile * nw < J.n_total ? t0 + (uint64_t)rq.tile * nw
                                                                  : J.n_total;
      if (j == 0 && g == 0 && lane < rq.head) {
        uint32_t se;
        uint64_t ve;
        split(J, lane, se, ve);
        patch_store<OP>(J, lane, resolve<OP, KIND>(J, L.t, T, r, dmax, se, ve, budget));
      }
      const uint64_t gs = t0 + g * GE;
      if (gs >= t1) {
        if (lane == 0) atomicMax(&L.next, next_item);
        continue;
      }
      ws_group<OP, KIND>(J, L, T, LC, gs, gs + GE < t1 ? gs + GE : t1, (uint64_t)ri << WSB_E);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
    if (lane == 0) atomicAdd(&L.done, 1u);
  } else {
    // drain waves ahead of the ring, as in the plain wave-specialised fill
    __builtin_amdgcn_s_setprio(1);
    const Job none{};
    ws_drain<OP, KIND, true>(none, R, L, T, r, dmax, n_stream, wave - n_stream, budget);
  }
  if (__builtin_amdgcn_ballot_w64(budget) != 0 && lane == 0) raise_flag(flags, ZG_FLAG_BUDGET);
}

// Batch work of the polar class: every wave of a workgroup tile runs the
// per-wave polar path over its part.
template <int KIND>
__global__ __launch_bounds__(1024) void k_bpolar(DevRequest *R, const BatchHeader *H,
                                                 const DevTables *__restrict__ T,
                                                 uint32_t *flags) {
  constexpr int C = batch_class(OP_POLAR, KIND);
  const uint32_t cnt = H->cls_cnt[C];
  if (blockIdx.x >= cnt) return;
  extern __shared__ __align__(16) unsigned char s_polar[];   // log table, then waves x QCAP
  LogTables &Lt = *(LogTables *)s_polar;
  uint32_t *s_q = (uint32_t *)(s_polar + POLAR_LOG_BYTES);
  load_log_table(T, Lt);
  __syncthreads();
  const uint64_t *items = (const uint64_t *)((const char *)H + H->items_off);
  const uint32_t off = H->cls_off[C];
  const uint32_t nw = blockDim.x >> 6;
  const uint32_t wave = uni(threadIdx.x >> 6);
  const PolarCtx Cx{T, H->dmax, flags, &Lt};
  const LaneConst LC = lane_constants<OP_POLAR, KIND>(T);
  for (uint32_t k = blockIdx.x; k < cnt; k += gridDim.x) {
    const uint64_t it = items[off + k];
    const DevRequest &rq = R[(uint32_t)(it >> 32)];
    const uint32_t j = (uint32_t)it;
    if (rq.status == 0) {
      const Job J = rq.job;
      const uint64_t b = rq.head + ((uint64_t)j * nw + wave) * rq.tile;
      const uint64_t e_end = b + rq.tile < J.n_total ? b + rq.tile : J.n_total;
      const uint64_t e_begin = b < e_end ? b : e_end;
      const bool with_head = j == 0 && wave == 0;
      if (e_begin < e_end || (with_head && rq.head))
        polar_tile<KIND>(J, Cx, LC, s_q + wave * QCAP, e_begin, e_end, rq.head, with_head);
    }
  }
}

// ------------------------------------------------ sequential consumption
//
// The variates that successive nextGaussian(random) calls produce when every
// call takes its words from one generator in order (Section 2, Listing 2).
// Word p of the generator (position p) is W(seed, s, p, 0): for stream 0 the
// SplittableRandom / Random sequence itself.  An attempt at position p reads
// word p; a wedge test also reads word p+1 and the base strip words p+1 and
// p+2; whatever the outcome, the next attempt starts at the next unread
// position.  So the attempt starts form a chain p -> p + adv(p), adv in
// {1, 2, 3} a function of word p alone, and variate k is the value of the
// k-th accepting attempt on the chain from the first position.
//
// Since adv <= 3, the chain enters a chunk of positions at one of its first
// three.  Pass 1 evaluates every attempt of its chunk (one wave, a window of
// 64 positions per step, one per lane) and walks the chunk from each of the
// three entries with scalar bit scans over the window's ballots, recording
// the exit offset and the accepted count of each: the chunk's three-state
// map.  Pass 2 (one workgroup) composes the workgroups' maps in order and
// gives each workgroup its entry and its first output index.  Pass 3
// composes within the workgroup, walks each chunk again from its true entry
// and stores the accepted values at their ranks.  Pass 4, one lane, goes on
// from the end of the scanned positions only if they held fewer than n
// accepting attempts (the scan covers the expected count with a wide margin).

// A lane's generator at position P = window base + lane: SplitMix64 keeps the
// pre-mix counter word, the LCG the state of step 2 m + 1 of P's double.
struct SeqLane {
  uint64_t z;
  uint64_t S1;
};

template <int KIND>
DEV SeqLane seq_lane_at(const SeqJob &J, const DevTables *T, uint64_t P) {
  SeqLane g;
  if (KIND == ZG_JAVA_LCG48) {
    g.z = 0;
    g.S1 = lcg_jump(&T->lcg, lcg_state0(J.seed), 2 * lcg_index(J.s, P, 0) + 1);
  } else {
    g.z = J.seed + GAMMA * (1ull + ((uint64_t)J.s << 48) + P);
    g.S1 = 0;
  }
  return g;
}

// The same for every lane of a window based at Pb (uniform): one jump per
// window, then the lane's offset.
template <int KIND>
DEV SeqLane seq_window(const SeqJob &J, const DevTables *T, uint64_t Pb, uint32_t lane) {
  SeqLane g;
  if (KIND == ZG_JAVA_LCG48) {
    const uint64_t Sb = lcg_jump(&T->lcg, lcg_state0(J.seed), 2 * lcg_index(J.s, Pb, 0) + 1);
    g.z = 0;
    g.S1 = aff(T->lcg.jump[0][2 * lane], Sb);
  } else {
    g.z = J.seed + GAMMA * (1ull + ((uint64_t)J.s << 48) + Pb) + GAMMA * (uint64_t)lane;
    g.S1 = 0;
  }
  return g;
}

// Moves a lane's generator 64 positions on (the next window).
template <int KIND>
DEV void seq_advance(SeqLane &g, const DevTables *T) {
  if (KIND == ZG_JAVA_LCG48)
    g.S1 = aff(T->lcg.jump[0][128], g.S1);
  else
    g.z += GAMMA * 64ull;
}

// Word k positions after the lane's own (k = 0, 1, 2).
template <int KIND>
DEV uint64_t seq_word(const SeqLane &g, const DevTables *T, uint32_t k) {
  if (KIND == ZG_JAVA_LCG48)
    return lcg_word_from(k ? aff(T->lcg.jump[0][2 * k], g.S1) : g.S1);
  return mix64(g.z + GAMMA * (uint64_t)k);
}

struct SeqAtt {
  uint32_t adv;   // positions this attempt reads: 1 fast, 2 wedge, 3 base strip
  bool acc;
  double z;       // the signed value when accepted
};

// The attempt at the lane's position, with the arithmetic of resolve.
template <int KIND>
DEV SeqAtt seq_attempt(const LdsTabs &L, const DevTables *T, double r, const SeqLane &g) {
  const uint64_t W = seq_word<KIND>(g, T, 0);
  const uint32_t whi = (uint32_t)(W >> 32), wlo = (uint32_t)W;
  const uint32_t i = whi >> 25;
  const uint32_t neg = (whi >> 24) & 1u;
  const Fast64 f = L.f64[2 * i];
  const uint32_t jh = j_hi(whi), jl = j_lo(whi, wlo);
  const double x = to_f64(jh, jl) * f.w;
  SeqAtt a;
  a.adv = 1;
  a.acc = true;
  double xc = x;
  if ((((uint64_t)jh << 32) | jl) >= f.k) {
    const double u = u53(seq_word<KIND>(g, T, 1));
    double thr, arg;
    if (i == 0) {   // tail: x = r + a, a = -log(U1+)/r, accept U2 < exp(-a^2/2)
      const double u1 = u53p(seq_word<KIND>(g, T, 1));
      thr = u53(seq_word<KIND>(g, T, 2));
      arg = -log(u1) / r;
      xc = r + arg;
      a.adv = 3;
    } else {        // wedge: accept y[i-1] + U dy[i] < exp(-x^2/2)
      const double2 yd = L.yd[i];
      thr = yd.x + u * yd.y;
      arg = x;
      a.adv = 2;
    }
    a.acc = thr < exp(-0.5 * (arg * arg));
  }
  a.z = neg ? -xc : xc;
  return a;
}

// The chain through one window: from offset cur (0..2, wave-uniform) it
// takes every position up to the next slow attempt q, then jumps to q + adv(q).
// Returns the mask of chain positions in the window and leaves cur at the
// chain's offset in the next window.  slow, m3: ballots of adv >= 2, adv == 3.
DEV uint64_t seq_walk(uint32_t &cur, uint64_t slow, uint64_t m3) {
  uint64_t on = 0;
  uint32_t c = cur;
  while (c < 64) {
    const uint64_t rem = slow & (~0ull << c);
    if (rem == 0) {
      on |= ~0ull << c;
      c = 64;
      break;
    }
    const uint32_t q = (uint32_t)__builtin_ctzll(rem);
    on |= (~0ull << c) & ((2ull << q) - 1);   // positions c..q
    c = q + 2 + (uint32_t)((m3 >> q) & 1ull);
  }
  cur = c - 64;
  return on;
}

DEV uint32_t seq_exit(uint32_t exits, uint32_t e) { return (exits >> (2 * e)) & 3u; }

// Element e (0..2) of a 3-entry array by selects (no indexed private memory).
template <typename V>
DEV V pick3(const V *a, uint32_t e) { return e == 0 ? a[0] : (e == 1 ? a[1] : a[2]); }

// Pass 1: the three-state map of every chunk, and of every workgroup.
template <int KIND>
__global__ __launch_bounds__(1024) void k_seq_maps(SeqJob J, const DevTables *__restrict__ T,
                                                   SeqMap *maps, SeqMap *wg_maps) {
  __shared__ LdsTabs L;
  __shared__ SeqMap wm[SEQ_WAVES];
  load_tabs<OP_ZIG64>(T, L);
  __syncthreads();
  const uint32_t wave = uni(threadIdx.x >> 6), lane = lane_id();
  const double r = T->r;
  const uint64_t c = (uint64_t)blockIdx.x * SEQ_WAVES + wave;
  SeqLane g = seq_window<KIND>(J, T, J.first + c * SEQ_CHUNK, lane);
  uint32_t cur0 = 0, cur1 = 1, cur2 = 2, n0 = 0, n1 = 0, n2 = 0;
  for (uint32_t w = 0; w < SEQ_WINDOWS; ++w) {
    const SeqAtt a = seq_attempt<KIND>(L, T, r, g);
    const uint64_t slow = __builtin_amdgcn_ballot_w64(a.adv != 1);
    const uint64_t m3 = __builtin_amdgcn_ballot_w64(a.adv == 3);
    const uint64_t macc = __builtin_amdgcn_ballot_w64(a.acc);
    n0 += (uint32_t)__builtin_popcountll(seq_walk(cur0, slow, m3) & macc);
    n1 += (uint32_t)__builtin_popcountll(seq_walk(cur1, slow, m3) & macc);
    n2 += (uint32_t)__builtin_popcountll(seq_walk(cur2, slow, m3) & macc);
    seq_advance<KIND>(g, T);
  }
  if (lane == 0) {
    SeqMap m;
    m.cnt[0] = n0;
    m.cnt[1] = n1;
    m.cnt[2] = n2;
    m.exits = cur0 | (cur1 << 2) | (cur2 << 4);
    maps[c] = m;
    wm[wave] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    SeqMap acc;
    for (uint32_t e = 0; e < 3; ++e) {
      uint32_t x = e, n = 0;
      for (uint32_t w = 0; w < SEQ_WAVES; ++w) {
        n += wm[w].cnt[x];
        x = seq_exit(wm[w].exits, x);
      }
      acc.cnt[e] = n;
      acc.exits = e ? acc.exits | (x << (2 * e)) : x;
    }
    wg_maps[blockIdx.x] = acc;
  }
}

// A map with 64-bit counts, for the scan over workgroups.
struct SeqMap64 {
  uint64_t cnt[3];
  uint32_t ex[3];
  uint32_t pad;
};

DEV SeqMap64 seq_identity() {
  SeqMap64 m;
#pragma unroll
  for (uint32_t e = 0; e < 3; ++e) {
    m.cnt[e] = 0;
    m.ex[e] = e;
  }
  m.pad = 0;
  return m;
}

// a, then b
DEV SeqMap64 seq_cat(const SeqMap64 &a, const SeqMap64 &b) {
  SeqMap64 m;
#pragma unroll
  for (uint32_t e = 0; e < 3; ++e) {
    const uint32_t x = a.ex[e];
    m.cnt[e] = a.cnt[e] + pick3(b.cnt, x);
    m.ex[e] = pick3(b.ex, x);
  }
  m.pad = 0;
  return m;
}

DEV SeqMap64 seq_widen(const SeqMap &w) {
  SeqMap64 m;
#pragma unroll
  for (uint32_t e = 0; e < 3; ++e) {
    m.cnt[e] = w.cnt[e];
    m.ex[e] = seq_exit(w.exits, e);
  }
  m.pad = 0;
  return m;
}

// Pass 2 (one workgroup of 1024 threads): each thread composes a run of
// workgroup maps, the runs are scanned in order, and each thread hands out
// the entries of its run from the chain's start (offset 0, variate 0).
__global__ __launch_bounds__(1024) void k_seq_scan(const SeqMap *wg_maps, uint32_t n_wg,
                                                   SeqEntry *wg_entry, SeqHdr *hdr) {
  __shared__ SeqMap64 sm[1024];
  const uint32_t t = threadIdx.x, nt = blockDim.x;
  const uint32_t per = (n_wg + nt - 1) / nt;
  const uint32_t b = t * per < n_wg ? t * per : n_wg;
  const uint32_t e_ = b + per < n_wg ? b + per : n_wg;
  SeqMap64 m = seq_identity();
  for (uint32_t k = b; k < e_; ++k) m = seq_cat(m, seq_widen(wg_maps[k]));
  sm[t] = m;
  __syncthreads();
  for (uint32_t d = 1; d < nt; d <<= 1) {
    SeqMap64 v = sm[t];
    if (t >= d) v = seq_cat(sm[t - d], v);
    __syncthreads();
    sm[t] = v;
    __syncthreads();
  }
  uint32_t ent = t ? sm[t - 1].ex[0] : 0u;
  uint64_t base = t ? sm[t - 1].cnt[0] : 0ull;
  for (uint32_t k = b; k < e_; ++k) {
    SeqEntry E;
    E.base = base;
    E.e = ent;
    E.pad = 0;
    wg_entry[k] = E;
    const SeqMap w = wg_maps[k];
    base += pick3(w.cnt, ent);
    ent = seq_exit(w.exits, ent);
  }
  if (t == nt - 1) {
    SeqHdr H;
    H.total = sm[t].cnt[0];
    H.exit = sm[t].ex[0];
    H.pad = 0;
    *hdr = H;
  }
}

// Pass 3: the values, at their ranks along the chain.
template <int KIND>
__global__ __launch_bounds__(1024) void k_seq_write(SeqJob J, const DevTables *__restrict__ T,
                                                    const SeqMap *maps, const SeqEntry *wg_entry) {
  __shared__ LdsTabs L;
  __shared__ uint64_t wbase[SEQ_WAVES];
  __shared__ uint32_t went[SEQ_WAVES];
  load_tabs<OP_ZIG64>(T, L);
  if (threadIdx.x == 0) {
    const SeqEntry E = wg_entry[blockIdx.x];
    uint64_t base = E.base;
    uint32_t e = E.e;
    for (uint32_t w = 0; w < SEQ_WAVES; ++w) {
      wbase[w] = base;
      went[w] = e;
      const SeqMap m = maps[(uint64_t)blockIdx.x * SEQ_WAVES + w];
      base += pick3(m.cnt, e);
      e = seq_exit(m.exits, e);
    }
  }
  __syncthreads();
  const uint32_t wave = uni(threadIdx.x >> 6), lane = lane_id();
  uint64_t base = uni64(wbase[wave]);
  uint32_t cur = uni(went[wave]);
  if (base >= J.n) return;
  const double r = T->r;
  const uint64_t c = (uint64_t)blockIdx.x * SEQ_WAVES + wave;
  uint64_t Pb = J.first + c * SEQ_CHUNK;
  SeqLane g = seq_window<KIND>(J, T, Pb, lane);
  const uint64_t below = (1ull << lane) - 1ull;
  for (uint32_t w = 0; w < SEQ_WINDOWS; ++w) {
    const SeqAtt a = seq_attempt<KIND>(L, T, r, g);
    const uint64_t slow = __builtin_amdgcn_ballot_w64(a.adv != 1);
    const uint64_t m3 = __builtin_amdgcn_ballot_w64(a.adv == 3);
    const uint64_t macc = __builtin_amdgcn_ballot_w64(a.acc);
    const uint64_t accm = seq_walk(cur, slow, m3) & macc;
    if ((accm >> lane) & 1ull) {
      const uint64_t k = base + (uint64_t)__builtin_popcountll(accm & below);
      if (k < J.n) {
        J.out[k] = a.z;
        if (k == J.n - 1 && J.next_word) *J.next_word = Pb + lane + a.adv;
      }
    }
    base += (uint64_t)__builtin_popcountll(accm);
    if (base >= J.n) break;
    Pb += 64;
    seq_advance<KIND>(g, T);
  }
}

// Pass 4 (one lane): only when the scanned positions held fewer than n
// accepting attempts, the rest one attempt at a time from where the chain
// left them; bounded by the index window and SEQ_FINISH_CAP attempts (then
// the remaining variates are NaN and a flag is raised).
template <int KIND>
__global__ __launch_bounds__(64) void k_seq_finish(SeqJob J, const DevTables *__restrict__ T,
                                                   const SeqHdr *hdr, uint32_t *flags) {
  __shared__ LdsTabs L;
  load_tabs<OP_ZIG64>(T, L);
  __syncthreads();
  if (threadIdx.x != 0) return;
  const SeqHdr H = *hdr;
  if (H.total >= J.n) return;
  const double r = T->r;
  uint64_t p = J.first + J.n_pos + H.exit;
  uint64_t k = H.total;
  uint64_t steps = 0;
  while (k < J.n) {
    if (p + 3 > J.limit) {
      raise_flag(flags, ZG_FLAG_RANGE);
      break;
    }
    if (steps >= SEQ_FINISH_CAP) {
      raise_flag(flags, ZG_FLAG_BUDGET);
      break;
    }
    const SeqLane g = seq_lane_at<KIND>(J, T, p);
    const SeqAtt a = seq_attempt<KIND>(L, T, r, g);
    if (a.acc) J.out[k++] = a.z;
    p += a.adv;
    ++steps;
  }
  for (; k < J.n; ++k) J.out[k] = nan64();
  if (J.next_word) *J.next_word = p;
}

// ------------------------------------------------------------ host launch

template <int OP, int KIND>
static hipError_t launch_fill_op(const Job &J, const DevTables *T, uint32_t dmax, uint32_t *flags,
                                 uint32_t tile, uint32_t waves, uint32_t head, uint32_t qcap,
                                 uint32_t resident, uint32_t n_drain, uint32_t gsteps,
                                 hipStream_t stream) {
  uint64_t body = J.n_total > head ? J.n_total - head : 0;
  if (gsteps < 1 || gsteps > 8) gsteps = BGROUP;
  if constexpr (OP != OP_POLAR) {
    if (n_drain > 0) {
      // wave-specialised: a persistent grid of `resident` workgroups of
      // `waves` waves per CU (at least one, capped by occupancy), at least one
      // streaming wave each; the workgroups take whole groups in turn
      int dev = 0, cus = 256;
      (void)hipGetDevice(&dev);
      (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
      const uint32_t nw = waves < 2 ? 2u : (waves > 16 ? 16u : waves);
      if (n_drain > WS_MAX_DRAIN) n_drain = WS_MAX_DRAIN;
      if (n_drain > nw - 1) n_drain = nw - 1;
      int occ = 0;
      uint32_t per_cu = resident ? resident : 1u;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)k_zigws<OP, KIND>,
                                                       (int)(64 * nw), 0) == hipSuccess &&
          occ > 0 && (uint32_t)occ < per_cu)
        per_cu = (uint32_t)occ;
      const uint64_t ge = (uint64_t)gsteps * BSTEP;
      const uint64_t groups = (body + ge - 1) / ge;
      const uint64_t cap = (uint64_t)cus * per_cu;
      uint64_t blocks = groups < cap ? (groups ? groups : 1) : cap;
      hipLaunchKernelGGL((k_zigws<OP, KIND>), dim3((uint32_t)blocks), dim3(64 * nw), 0, stream, J,
                         T, dmax, flags, head, n_drain, gsteps);
      return hipGetLastError();
    }
    int dev = 0, cus = 256;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    // small jobs: shorter tiles, so that every CU gets at least two workgroup
    // tiles; whole steps per wave
    const uint64_t fit = body / ((uint64_t)waves * (uint64_t)cus * 2);
    if (fit < tile) tile = (uint32_t)(fit < BSTEP ? BSTEP : fit);
    tile = (tile + BSTEP - 1) / BSTEP * BSTEP;
    const uint64_t bt = (uint64_t)tile * waves;
    uint64_t ntiles = (body + bt - 1) / bt;
    if (ntiles == 0) ntiles = 1;   // head-only jobs still need block 0
    uint64_t blocks = ntiles;
    if (resident) {
      // persistent: at most `resident` workgroups per CU, capped by occupancy
      int occ = 0;
      if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, (const void *)k_zig<OP, KIND>,
                                                        (int)(64 * waves), 0) != hipSuccess ||
          occ < 1)
        occ = 1;
      const uint64_t cap = (uint64_t)cus * (resident < (uint32_t)occ ? resident : (uint32_t)occ);
      if (blocks > cap) blocks = cap;
    }
    const uint32_t qc = qcap == 0 || qcap > BQ ? BQ : qcap;
    hipLaunchKernelGGL((k_zig<OP, KIND>), dim3((uint32_t)blocks), dim3(64 * waves), 0, stream, J,
                       T, dmax, flags, tile, head, qc, ntiles, gsteps);
  } else {
    (void)resident;
    (void)qcap;
    uint64_t tiles = (body + tile - 1) / tile;
    if (tiles == 0) tiles = 1;   // head-only jobs still need wave 0
    uint64_t blocks = (tiles + waves - 1) / waves;
    hipLaunchKernelGGL((k_polar<KIND>), dim3((uint32_t)blocks), dim3(64 * waves),
                       POLAR_LOG_BYTES + (size_t)waves * QCAP * sizeof(uint32_t), stream, J, T, dmax,
                       flags, tile,
                       head);
  }
  return hipGetLastError();
}

template <int OP>
static hipError_t launch_kind(const Job &J, const DevTables *T, uint32_t dmax, uint32_t *flags,
                              uint32_t tile, uint32_t waves, uint32_t head, uint32_t qcap,
                              uint32_t resident, uint32_t n_drain, uint32_t gsteps,
                              hipStream_t stream) {
  if (J.kind == ZG_JAVA_LCG48)
    return launch_fill_op<OP, ZG_JAVA_LCG48>(J, T, dmax, flags, tile, waves, head, qcap, resident,
                                             n_drain, gsteps, stream);
  return launch_fill_op<OP, ZG_SPLITMIX64>(J, T, dmax, flags, tile, waves, head, qcap, resident,
                                           n_drain, gsteps, stream);
}

hipError_t launch_fill(const Job &J, const DevTables *T, uint32_t dmax, uint32_t *flags,
                       uint32_t tile, uint32_t waves, uint32_t head, uint32_t qcap,
                       uint32_t resident, uint32_t n_drain, uint32_t gsteps,
                       hipStream_t stream) {
  switch (J.op) {
    case OP_ZIG64:
      return launch_kind<OP_ZIG64>(J, T, dmax, flags, tile, waves, head, qcap, resident, n_drain,
                                   gsteps, stream);
    case OP_ZIG32:
      return launch_kind<OP_ZIG32>(J, T, dmax, flags, tile, waves, head, qcap, resident, n_drain,
                                   gsteps, stream);
    case OP_POLAR:
      return launch_kind<OP_POLAR>(J, T, dmax, flags, tile, waves, head, qcap, resident, n_drain,
                                   gsteps, stream);
    case OP_MZ64:
      return launch_kind<OP_MZ64>(J, T, dmax, flags, tile, waves, head, qcap, resident, n_drain,
                                  gsteps, stream);
    default:
      return launch_kind<OP_MUTATE>(J, T, dmax, flags, tile, waves, head, qcap, resident, n_drain,
                                    gsteps, stream);
  }
}

hipError_t launch_ea(const EaJob &E, const DevTables *T, uint32_t dmax, uint32_t *flags,
                     hipStream_t stream) {
  int dev = 0, cus = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  // EA_WAVES-wave workgroups, one child per wave at a time, at most EA_BPC
  // per CU; groups of 512 genes, or of 256 or 128 for short genomes
  const uint64_t want = ((uint64_t)E.pop + EA_WAVES - 1) / EA_WAVES;
  const uint64_t cap = (uint64_t)EA_BPC * (uint64_t)cus;
  const uint32_t blocks = (uint32_t)(want < cap ? want : cap);
  if (E.genes > 256)
    hipLaunchKernelGGL((k_ea<ZG_SPLITMIX64, 8>), dim3(blocks), dim3(64 * EA_WAVES), 0, stream, E,
                       T, dmax, flags);
  else if (E.genes > 128)
    hipLaunchKernelGGL((k_ea<ZG_SPLITMIX64, 4>), dim3(blocks), dim3(64 * EA_WAVES), 0, stream, E,
                       T, dmax, flags);
  else
    hipLaunchKernelGGL((k_ea<ZG_SPLITMIX64, 2>), dim3(blocks), dim3(64 * EA_WAVES), 0, stream, E,
                       T, dmax, flags);
  return hipGetLastError();
}

hipError_t launch_words(uint64_t *out, uint64_t n, const DevTables *T, uint32_t kind,
                        uint64_t seed, uint32_t s, uint32_t d, uint64_t first,
                        hipStream_t stream) {
  uint64_t threads = n < (1ull << 22) ? n : (1ull << 22);
  uint32_t blocks = (uint32_t)((threads + 255) / 256);
  hipLaunchKernelGGL(k_words, dim3(blocks), dim3(256), 0, stream, out, n, T, kind, seed, s, d,
                     first);
  return hipGetLastError();
}

hipError_t launch_decide(const uint64_t *words, uint64_t n, const DevTables *T, uint8_t *cls,
                         double *x, hipStream_t stream) {
  uint32_t blocks = (uint32_t)((n + 255) / 256);
  hipLaunchKernelGGL(k_decide, dim3(blocks), dim3(256), 0, stream, words, n, T, cls, x);
  return hipGetLastError();
}

const void *kernel_reserve() { return (const void *)k_reserve; }
const void *kernel_complete() { return (const void *)k_complete; }

const void *kernel_batch_class(int cls, bool ws) {
  switch (cls) {
    case batch_class(OP_ZIG64, ZG_SPLITMIX64):
      return ws ? (const void *)k_bzigws<OP_ZIG64, ZG_SPLITMIX64>
                : (const void *)k_bzig<OP_ZIG64, ZG_SPLITMIX64>;
    case batch_class(OP_ZIG64, ZG_JAVA_LCG48):
      return ws ? (const void *)k_bzigws<OP_ZIG64, ZG_JAVA_LCG48>
                : (const void *)k_bzig<OP_ZIG64, ZG_JAVA_LCG48>;
    case batch_class(OP_ZIG32, ZG_SPLITMIX64):
      return ws ? (const void *)k_bzigws<OP_ZIG32, ZG_SPLITMIX64>
                : (const void *)k_bzig<OP_ZIG32, ZG_SPLITMIX64>;
    case batch_class(OP_ZIG32, ZG_JAVA_LCG48):
      return ws ? (const void *)k_bzigws<OP_ZIG32, ZG_JAVA_LCG48>
                : (const void *)k_bzig<OP_ZIG32, ZG_JAVA_LCG48>;
    case batch_class(OP_MUTATE, ZG_SPLITMIX64):
      return ws ? (const void *)k_bzigws<OP_MUTATE, ZG_SPLITMIX64>
                : (const void *)k_bzig<OP_MUTATE, ZG_SPLITMIX64>;
    case batch_class(OP_MUTATE, ZG_JAVA_LCG48):
      return ws ? (const void *)k_bzigws<OP_MUTATE, ZG_JAVA_LCG48>
                : (const void *)k_bzig<OP_MUTATE, ZG_JAVA_LCG48>;
    case batch_class(OP_POLAR, ZG_SPLITMIX64): return (const void *)k_bpolar<ZG_SPLITMIX64>;
    default: return (const void *)k_bpolar<ZG_JAVA_LCG48>;
  }
}

template <int OP, int KIND>
static hipError_t launch_bz(bool ws, dim3 g, dim3 b, DevRequest *R, const BatchHeader *H,
                            const DevTables *T, uint32_t *flags, hipStream_t stream) {
  if (ws)
    hipLaunchKernelGGL((k_bzigws<OP, KIND>), g, b, 0, stream, R, H, T, flags);
  else
    hipLaunchKernelGGL((k_bzig<OP, KIND>), g, b, 0, stream, R, H, T, flags);
  return hipGetLastError();
}

hipError_t launch_batch_class(int cls, bool ws, uint32_t grid, uint32_t waves, DevRequest *R,
                              const BatchHeader *H, const DevTables *T, uint32_t *flags,
                              hipStream_t stream) {
  const dim3 g(grid), b(64 * waves);
  switch (cls) {
    case batch_class(OP_ZIG64, ZG_SPLITMIX64):
      return launch_bz<OP_ZIG64, ZG_SPLITMIX64>(ws, g, b, R, H, T, flags, stream);
    case batch_class(OP_ZIG64, ZG_JAVA_LCG48):
      return launch_bz<OP_ZIG64, ZG_JAVA_LCG48>(ws, g, b, R, H, T, flags, stream);
    case batch_class(OP_ZIG32, ZG_SPLITMIX64):
      return launch_bz<OP_ZIG32, ZG_SPLITMIX64>(ws, g, b, R, H, T, flags, stream);
    case batch_class(OP_ZIG32, ZG_JAVA_LCG48):
      return launch_bz<OP_ZIG32, ZG_JAVA_LCG48>(ws, g, b, R, H, T, flags, stream);
    case batch_class(OP_MUTATE, ZG_SPLITMIX64):
      return launch_bz<OP_MUTATE, ZG_SPLITMIX64>(ws, g, b, R, H, T, flags, stream);
    case batch_class(OP_MUTATE, ZG_JAVA_LCG48):
      return launch_bz<OP_MUTATE, ZG_JAVA_LCG48>(ws, g, b, R, H, T, flags, stream);
    case batch_class(OP_POLAR, ZG_SPLITMIX64):
      hipLaunchKernelGGL(k_bpolar<ZG_SPLITMIX64>, g, b, batch_class_lds_bytes(cls, waves), stream,
                         R, H, T, flags);
      return hipGetLastError();
    default:
      hipLaunchKernelGGL(k_bpolar<ZG_JAVA_LCG48>, g, b, batch_class_lds_bytes(cls, waves), stream,
                         R, H, T, flags);
      return hipGetLastError();
  }
}

// Device-resident workspace of the sequential fill that allocates nothing
// (zg_fill_sequential_noalloc): each GPU the library runs on holds one copy
// until the process ends.  Host code never passes this name to a kernel (on
// the host it is a stand-in, not a device address): it uses the address that
// seq_scratch_ptr resolved for the device.
static __device__ __align__(256) unsigned char scratch[SEQ_SCRATCH_BYTES];

namespace {
constexpr int SCRATCH_MAX_DEVICES = 64;
std::mutex scratch_mu;
void *scratch_dev[SCRATCH_MAX_DEVICES] = {};
}  // namespace

hipError_t seq_scratch_ptr(int dev, void **out) {
  if (dev < 0 || dev >= SCRATCH_MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_dev[dev]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != dev) return hipErrorInvalidDevice;   // the caller makes dev current
    void *ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    scratch_dev[dev] = ptr;
  }
  *out = scratch_dev[dev];
  return hipSuccess;
}

static uint64_t seq_align(uint64_t b) { return (b + 255) / 256 * 256; }

// Positions scanned for n variates, in whole workgroup spans: the expected
// 1.041 n words, plus 0.9% of n and 16 sqrt(n) + 64 (the words that n
// variates read have a standard deviation of about 0.26 sqrt(n)).  The
// workspace holds the chunk maps, the workgroup maps, the workgroup entries
// and the scan result, each 256-byte aligned.
SeqPlan seq_plan(uint64_t n, uint64_t cap_wg) {
  SeqPlan P{};
  const uint64_t want = n + n / 20 + 16 * (uint64_t)std::sqrt((double)n) + 64;
  P.n_pos = (want + SEQ_SPAN - 1) / SEQ_SPAN * SEQ_SPAN;
  P.n_wg = P.n_pos / SEQ_SPAN;
  P.wg_cap = P.n_wg;
  P.off_wg_maps = seq_align(P.wg_cap * SEQ_WAVES * sizeof(SeqMap));
  P.off_entry = P.off_wg_maps + seq_align(P.wg_cap * sizeof(SeqMap));
  P.off_hdr = P.off_entry + seq_align(P.wg_cap * sizeof(SeqEntry));
  P.bytes = P.off_hdr + seq_align(sizeof(SeqHdr));
  if (cap_wg && cap_wg < P.n_wg) {
    P.n_wg = cap_wg;
    P.n_pos = cap_wg * SEQ_SPAN;
  }
  return P;
}

// Whether every buffer of the plan lies inside a workspace of `bytes`.
static bool seq_plan_fits(const SeqPlan &P, uint64_t bytes) {
  return P.n_pos == P.n_wg * SEQ_SPAN && P.n_wg <= P.wg_cap &&
         P.off_wg_maps >= P.wg_cap * SEQ_WAVES * sizeof(SeqMap) &&
         P.off_entry >= P.off_wg_maps + P.wg_cap * sizeof(SeqMap) &&
         P.off_hdr >= P.off_entry + P.wg_cap * sizeof(SeqEntry) &&
         P.bytes >= P.off_hdr + sizeof(SeqHdr) && bytes >= P.bytes && P.n_wg < (1ull << 31);
}

template <int KIND>
static hipError_t launch_seq_kind(const SeqJob &J, const SeqPlan &P, const DevTables *T,
                                  void *work, uint32_t *flags, hipStream_t stream) {
  char *p = (char *)work;
  SeqMap *maps = (SeqMap *)p;
  SeqMap *wg_maps = (SeqMap *)(p + P.off_wg_maps);
  SeqEntry *wg_entry = (SeqEntry *)(p + P.off_entry);
  SeqHdr *hdr = (SeqHdr *)(p + P.off_hdr);
  const dim3 blk(64 * SEQ_WAVES);
  if (P.n_wg)
    hipLaunchKernelGGL((k_seq_maps<KIND>), dim3((uint32_t)P.n_wg), blk, 0, stream, J, T, maps,
                       wg_maps);
  hipLaunchKernelGGL(k_seq_scan, dim3(1), dim3(1024), 0, stream, (const SeqMap *)wg_maps,
                     (uint32_t)P.n_wg, wg_entry, hdr);
  if (P.n_wg)
    hipLaunchKernelGGL((k_seq_write<KIND>), dim3((uint32_t)P.n_wg), blk, 0, stream, J, T,
                       (const SeqMap *)maps, (const SeqEntry *)wg_entry);
  hipLaunchKernelGGL((k_seq_finish<KIND>), dim3(1), dim3(64), 0, stream, J, T,
                     (const SeqHdr *)hdr, flags);
  return hipGetLastError();
}

hipError_t launch_seq(const SeqJob &J, const SeqPlan &P, const DevTables *T, void *work,
                      uint64_t work_bytes, uint32_t *flags, hipStream_t stream) {
  if (!work || J.n_pos != P.n_pos || !seq_plan_fits(P, work_bytes)) return hipErrorInvalidValue;
  if (J.kind == ZG_JAVA_LCG48)
    return launch_seq_kind<ZG_JAVA_LCG48>(J, P, T, work, flags, stream);
  return launch_seq_kind<ZG_SPLITMIX64>(J, P, T, work, flags, stream);
}

size_t batch_class_lds_bytes(int cls, uint32_t waves) {
  return cls >= batch_class(OP_POLAR, ZG_SPLITMIX64)
             ? POLAR_LOG_BYTES + (size_t)waves * QCAP * sizeof(uint32_t)
             : 0;
}

}  // namespace zg
