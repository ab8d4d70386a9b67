/*
 * zg.h -- C ABI of libzg, an MI355X (gfx950) generator of standard Gaussian
 * variates by the original ziggurat algorithm.
 *
 * The method is the one the paper studies (Section 1 and Section 2,
 * "Ziggurat"): the 128-layer equal-area ziggurat of Marsaglia-Tsang 2000 /
 * Leong 2005 as implemented in GSL, which the paper ports to Java.  The
 * paper's problem is drawing one normal variate from a given generator
 * object (Listing 2, nextGaussian(random)); here a generator is the tuple
 * (kind, seed, stream id, counter), and the bulk call fills n normals.
 *
 * Conventions for every entry point:
 *  - Every call returns a zg_status (ZG_OK == 0, errors < 0).  No exception
 *    crosses the ABI and the library never aborts the process.
 *  - Device pointers (named d_*) are caller-owned device memory (for example
 *    from the torch allocator); they must stay valid until the work queued on
 *    the given HIP stream has completed.  Host pointers are read during the
 *    call only, unless stated otherwise.
 *  - hip_stream is a hipStream_t passed as void*; NULL is the null stream.
 *    Generation calls are asynchronous on that stream.
 *  - n == 0 is a no-op that returns ZG_OK.
 *  - Output is always the standard normal N(0,1); sigma appears only in
 *    zg_mutate.
 *  - Variates are index-keyed: variate v of stream s is a pure function of
 *    (kind, seed, s, v), whatever the launch geometry, batch or call split.
 *  - The plain generation calls (zg_fill, zg_fill_streams, zg_mutate,
 *    zg_ea_step) allocate nothing and issue no memset: a caller may capture
 *    them in a HIP graph on hip_stream and replay it.
 *
 * Uniform sources (Section 2 measures both classes):
 *  - ZG_SPLITMIX64: the generator of SplittableRandom.  Word of draw d of
 *    variate v in stream s: mix64(seed + gamma (1 + s 2^48 + d 2^40 + v)),
 *    gamma = 0x9E3779B97F4A7C15.  Limits: s < 2^16, v < 2^40, d < 2^8.
 *    Stream 0, draw 0 is SplittableRandom(seed).nextLong() in order.
 *  - ZG_JAVA_LCG48: java.util.Random (a = 0x5DEECE66D, c = 0xB, m = 2^48,
 *    seed scrambled by xor with a).  Double index
 *    m = s (2^39 - 20325) + d (2^31 - 101) + v consumes LCG steps 2m+1 and
 *    2m+2 as nextDouble does; the word is the 53-bit double numerator << 11.
 *    Limits: s < 2^8, v < 2^31 - 101, d < 2^8.  Stream 0, draw 0 is
 *    Random(seed).nextDouble() in order.
 *
 * Decoding of a 64-bit word W: layer i = W >> 57, sign = bit 56 (set means
 * negative), j = bits 3..55, U = (W >> 11) 2^-53 in [0,1),
 * U+ = ((W >> 11) + 1) 2^-53 in (0,1].
 */
#ifndef ZG_H
#define ZG_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t zg_status;
#define ZG_OK 0
#define ZG_EINVAL (-1)   /* bad argument: null pointer, unknown enum, misalignment, limit */
#define ZG_ERANGE (-2)   /* first_index + n beyond the stream's index window */
#define ZG_ENOMEM (-3)   /* device or host allocation failed */
#define ZG_EHIP (-4)     /* a HIP runtime call failed; zg_last_error() has the text */
#define ZG_EBUSY (-5)    /* admission refused (slots or memory cap), resource in use */
#define ZG_ENOENT (-6)   /* unknown handle or ticket */
#define ZG_ESTATE (-7)   /* object in the wrong state (server stopped, ...) */

typedef enum { ZG_SPLITMIX64 = 1, ZG_JAVA_LCG48 = 2 } zg_kind;
typedef enum { ZG_ZIGGURAT = 0, ZG_POLAR = 1, ZG_MCFARLAND = 2 } zg_method;
typedef enum { ZG_F64 = 0, ZG_F32 = 1 } zg_dtype;

#define ZG_LAYERS 128
#define ZG_MAX_DRAWS 256u
#define ZG_SM64_MAX_STREAMS 65536u
#define ZG_SM64_WINDOW (1ull << 40)
#define ZG_LCG_MAX_STREAMS 256u
#define ZG_LCG_WINDOW 2147483547ull
#define ZG_LCG_STREAM_SPACING 549755793563ull

/* Sticky device error flags, read with zg_error_flags. */
#define ZG_FLAG_BUDGET 1u   /* a variate needed more than the draw budget: NaN written */
#define ZG_FLAG_RANGE 2u    /* a counter-keyed request ran past its index window: skipped */

typedef struct zg_ctx zg_ctx;

/* ------------------------------------------------------------------ table */

/* The layer table (Section 2 "Ziggurat": the GSL-style 128-layer table).
 * f(x) = exp(-x^2/2); r solves the closure of 128 equal areas
 * v = r f(r) + f(r)/r (base box plus the exponential majorant beyond r).
 * W[0] = v/f(r), W[i] = b_{i-1}; y[i] = f(b_i) (y[127] = 1);
 * dy[i] = y[i] - y[i-1]; k53[i] = floor(b_i/W[i] 2^53); k24 likewise with
 * 2^24; w53[i] = W[i] 2^-53; w24d[i] = W[i] 2^-24; w24[i] = RN32(W[i]) 2^-24.
 * Every floating entry is the correctly rounded value of the exact quantity;
 * the library computes it in double-double arithmetic. */
typedef struct zg_table_view {
  double r;
  double v;
  double W[ZG_LAYERS];
  double y[ZG_LAYERS];
  double dy[ZG_LAYERS];
  double w53[ZG_LAYERS];
  double w24d[ZG_LAYERS];
  float w24[ZG_LAYERS];
  uint64_t k53[ZG_LAYERS];
  uint32_t k24[ZG_LAYERS];
} zg_table_view;

/* Builds the table on the host (no device needed).  out: caller-owned. */
zg_status zg_build_table(zg_table_view *out);

/* The modified ziggurat's table (McFarland's method: the comparator that
 * Sections 1 and 3 measure, whose need for good low-order bits Section 3
 * discusses; the paper gives none of its steps, so this is the published
 * method as read here).  f(x) = exp(-x^2/2) on x >= 0, total mass
 * sqrt(pi/2); 256 buckets of mass A = sqrt(pi/2)/256.  Layers lie wholly
 * under f, built from the bottom: X_0 f(X_0) = A with X_0 > 1, then
 * X_i (f(X_i) - Y_{i-1}) = A with Y_i = f(X_i), as many as fit
 * (ZG_MZ_LAYERS).  The rest of the mass lies in ZG_MZ_LAYERS + 1 regions:
 * region 0 is the tail beyond X_0; region k >= 1 is the overhang
 * {Y_{k-1} < y < f(x), X_k < x < X_{k-1}} (X_L = 0 and Y_L = 1: the cap).
 *  xs[i] = X_i 2^-63 (i < ZG_MZ_LAYERS, 0 beyond); x0 = X_0;
 *  ox[k] = X_{k-1}, odx[k] = X_{k-1} - X_k, oy[k] = Y_{k-1},
 *  ody[k] = Y_k - Y_{k-1} (k >= 1; entry 0 unused);
 *  kind[k]: 0 tail, 1 convex (X_k >= 1), 2 concave (X_{k-1} <= 1), 3 the
 *  strip holding x = 1;
 *  thr[j], alias[j]: bucket j gives region j while the 63 low bits of the
 *  first word are below thr[j] (units of 2^-63), else region alias[j].
 * Region masses a_k are rounded to integers m_k = round(a_k / sum a 2^71),
 * the excess taken from the largest (lowest index among equals); the alias
 * table pairs the lowest-index bucket below 2^63 with the lowest-index one
 * above, until none is left.  Every floating entry is the correctly rounded
 * value of the exact quantity (double-double here). */
#define ZG_MZ_BUCKETS 256
#define ZG_MZ_LAYERS 253
typedef struct zg_mz_table_view {
  double x0;
  double xs[ZG_MZ_BUCKETS];
  double ox[ZG_MZ_LAYERS + 1], odx[ZG_MZ_LAYERS + 1], oy[ZG_MZ_LAYERS + 1],
      ody[ZG_MZ_LAYERS + 1];
  uint64_t thr[ZG_MZ_BUCKETS];
  uint8_t kind[ZG_MZ_LAYERS + 1];
  uint8_t alias[ZG_MZ_BUCKETS];
} zg_mz_table_view;

/* Builds the modified ziggurat's table on the host (no device needed).
 * out: caller-owned.  ZG_EINVAL if the construction does not give
 * ZG_MZ_LAYERS layers or fails its own checks (masses adding up to
 * sqrt(pi/2), the alias table reproducing the masses). */
zg_status zg_build_mz_table(zg_mz_table_view *out);

/* ---------------------------------------------------------------- context */

/* Creates a context on HIP device hip_device: builds the table, uploads it
 * and the LCG jump tables, allocates the device counter table.  *out is owned
 * by the caller and released with zg_destroy. */
zg_status zg_create(int hip_device, zg_ctx **out);

/* Synchronises the device, frees everything the context owns.  Caller
 * buffers are untouched.  NULL is accepted. */
zg_status zg_destroy(zg_ctx *ctx);

/* Copies the context's table (the exact bits the kernels use) to *out. */
zg_status zg_table(const zg_ctx *ctx, zg_table_view *out);

/* ------------------------------------------------------------- generation */

/* Fills d_out[0..n) with variates first_index .. first_index+n-1 of stream
 * `stream` (Section 2: one generator per PRNG instance; bulk instead of one
 * call per variate).  d_out holds doubles (ZG_F64) or floats (ZG_F32) and
 * must be aligned to the element size.
 *  ZG_ZIGGURAT: per attempt, word W(d): fast accept iff j < k53[i] with
 *    x = (double)j * w53[i]; otherwise the wedge (i >= 1: U from W(d+1),
 *    y = y[i-1] + U dy[i], accept iff y < exp(-0.5 x x); rejection restarts at
 *    d+2) or the tail (i == 0: a = -log(U+ of W(d+1))/r, x = r + a, accept iff
 *    U of W(d+2) < exp(-0.5 a a); rejection restarts at d+3).
 *    ZG_F32: the attempt word is 32 bits: with ZG_SPLITMIX64 the first attempt
 *    of variates 2t and 2t+1 takes the high and low halves of W(s,t,0), all
 *    other attempts take hi32(W(s,v,d)); layer = u >> 25, sign = bit 24,
 *    j = low 24 bits; fast path fl32(fl32(j) w24[i]); wedge and tail in FP64
 *    with x = j w24d[i], output rounded to FP32.
 *  ZG_POLAR (ZG_F64 only): Knuth's polar method as in Random.nextGaussian;
 *    pair p = v >> 1, attempt a uses W(p, 2a) and W(p, 2a+1):
 *    v1 = 2U-1, v2 = 2U-1, s = v1 v1 + v2 v2, reject s >= 1 or s == 0,
 *    m = sqrt(-2 log(s) / s); variate 2p is v1 m, variate 2p+1 is v2 m.
 *  ZG_MCFARLAND (ZG_F64 only): the modified ziggurat (zg_mz_table_view).
 *    Words are 64-bit longs L(d): the SplitMix64 word, or for ZG_JAVA_LCG48
 *    nextLong = (next(32) << 32) + next(32) of LCG steps 2m+1, 2m+2 of the
 *    keyed index m of (s, v, d).  L(0) read as a signed integer picks bucket
 *    i = its low 8 bits; i < ZG_MZ_LAYERS gives x = xs[i] * (double)L(0).
 *    Otherwise the sign is L(0)'s top bit and the region is j = the low 8
 *    bits of L(1), or alias[j] when the 63 low bits of L(0) are >= thr[j].
 *    Attempts take pairs (L(d), L(d+1)), d = 2, 4, ..., as 53-bit integers
 *    a, b (top bits) and g = 2^-53.  Tail: t = -log((a+1) g) / x0,
 *    x = x0 + t, accept iff 0.5 t t < -log((b+1) g).  Overhang k: (s, t) =
 *    (a, b), or (max, min) of them where kind[k] == 1; x = ox[k] - (s g)
 *    odx[k]; accept at once where kind[k] == 2 and t <= s; otherwise accept
 *    iff oy[k] + (t g) ody[k] < exp(-0.5 x x).  A rejection takes the next
 *    pair in the same region; a pair needing d + 1 >= 256 gives the NaN.
 * A variate that would need a word with d >= 256 becomes a quiet NaN and
 * raises ZG_FLAG_BUDGET (probability below 1e-200).
 * Errors: ZG_EINVAL (null, enum, alignment, stream limit, polar or
 * McFarland with F32),
 * ZG_ERANGE (first_index + n past the window), ZG_EHIP. */
zg_status zg_fill(zg_ctx *ctx, void *d_out, uint64_t n, zg_dtype dtype, zg_method method,
                  zg_kind kind, uint64_t seed, uint32_t stream, uint64_t first_index,
                  void *hip_stream);

/* Multi-stream fill in one launch: d_out[k n_per_stream + i] = variate
 * first_index + i of stream stream0 + k, for k < n_streams, i < n_per_stream
 * (independent PRNG instances, as ThreadLocalRandom gives one per thread in
 * Section 2).  Same rules and errors as zg_fill. */
zg_status zg_fill_streams(zg_ctx *ctx, void *d_out, uint64_t n_per_stream, uint32_t n_streams,
                          zg_dtype dtype, zg_method method, zg_kind kind, uint64_t seed,
                          uint32_t stream0, uint64_t first_index, void *hip_stream);

/* Raw uniform words: d_out[i] = W(seed, stream, first_index + i, draw).
 * For ZG_JAVA_LCG48 at stream 0, draw 0 these are Random(seed).nextDouble()
 * numerators << 11.  d_out: n uint64 in device memory, 8-byte aligned. */
zg_status zg_uniform_words(zg_ctx *ctx, uint64_t *d_out, uint64_t n, zg_kind kind, uint64_t seed,
                           uint32_t stream, uint32_t draw, uint64_t first_index, void *hip_stream);

/* Gaussian mutation (Section 1: the EA's Gaussian mutation that motivated the
 * ziggurat): d_x[i] = d_x[i] + sigma * z_i in place, z_i = ziggurat FP64 variate
 * first_index + i of (kind, seed, stream); the product is rounded before the
 * sum.  d_x: n doubles, 8-byte aligned. */
zg_status zg_mutate(zg_ctx *ctx, double *d_x, uint64_t n, double sigma, zg_kind kind,
                    uint64_t seed, uint32_t stream, uint64_t first_index, void *hip_stream);

/* One generation of an evolutionary algorithm, fused (Section 1: the EA whose
 * Gaussian mutation motivated the ziggurat; the paper does not describe the
 * EA, so this is the read here).  A population of `pop` genomes of `genes`
 * doubles (row-major) with their fitness (minimised) gives the next one:
 *  - child c (key u = generation pop + c) copies the winner of a tournament
 *    of `tournament` draws with replacement, draw t picking parent
 *    floor(W(seed, stream, u, t) pop / 2^64) (SplitMix64 words); the first
 *    draw of least fitness wins, a number beating a NaN;
 *  - gene g (key w = u genes + g) mutates iff (W(seed, stream + 1, w, 0) >> 11)
 *    < floor(rate 2^53), by x = x + sigma z (the product rounded first) with
 *    z the FP64 ziggurat variate w of stream stream + 2; a mutated gene is
 *    then clamped to [lo, hi] (a NaN stays NaN).
 * d_children must not overlap d_parents.  d_winners (pop uint32, may be NULL)
 * receives each child's parent.  All device pointers 8-byte aligned (4 for
 * d_winners).  Asynchronous.  Errors: ZG_EINVAL (null, alignment, overlap,
 * pop or genes 0, tournament outside 1..256, rate outside [0, 1], lo > hi,
 * stream + 2 >= ZG_SM64_MAX_STREAMS), ZG_ERANGE ((generation + 1) pop genes
 * past ZG_SM64_WINDOW), ZG_EHIP. */
typedef struct zg_ea_params {
  uint64_t seed;
  uint64_t generation;
  uint32_t stream;       /* streams stream, stream + 1, stream + 2 */
  uint32_t tournament;   /* draws per tournament */
  double rate;           /* per-gene mutation probability */
  double sigma;
  double lo, hi;         /* bounds of a mutated gene */
} zg_ea_params;
zg_status zg_ea_step(zg_ctx *ctx, const double *d_parents, const double *d_fitness,
                     double *d_children, uint32_t *d_winners, uint32_t pop, uint32_t genes,
                     const zg_ea_params *params, void *hip_stream);

/* Sequential consumption (Section 2, Listing 2: nextGaussian(random) takes
 * its uniforms from one generator object, in call order): d_out[k] is the
 * k-th of n successive FP64 ziggurat variates that all read one generator in
 * order.  The generator is stream `stream` of (seed, kind) from word position
 * first_word; its word at position p is W(seed, stream, p, 0), so stream 0 is
 * SplittableRandom(seed).nextLong() (ZG_SPLITMIX64) or the numerators of
 * Random(seed).nextDouble() (ZG_JAVA_LCG48) in call order.  An attempt reads
 * one word, a wedge test one more, the base strip two more; after a rejection
 * the next attempt reads the next unread word.  Each attempt's arithmetic is
 * zg_fill's, with no draw budget.
 * d_next_word (device, 8-byte aligned, or NULL) receives the position after
 * the last word read: passed back as first_word it continues the generator.
 * d_work: device workspace (16-byte aligned) of work_bytes >=
 * zg_sequential_workspace(n) bytes, owned by the caller and in use until the
 * call's work on hip_stream has completed (the library allocates nothing).
 * d_out: n doubles, 8-byte aligned.  n = 0 does nothing.  Asynchronous.
 * n is limited to ZG_SEQ_MAX_N (10^6), the largest size checked on the device.
 * Errors: ZG_EINVAL (null, enum, alignment, stream limit, n > ZG_SEQ_MAX_N,
 * no or too small workspace), ZG_ERANGE (the scanned positions, about 1.05 n + 16 sqrt(n) from
 * first_word, would pass the stream's window: ZG_SM64_WINDOW or
 * ZG_LCG_WINDOW words), ZG_ENOMEM, ZG_EHIP.  Should the variates need words
 * past the window after all, the rest are NaN and ZG_FLAG_RANGE is raised. */
zg_status zg_fill_sequential(zg_ctx *ctx, double *d_out, uint64_t n, zg_kind kind, uint64_t seed,
                             uint32_t stream, uint64_t first_word, uint64_t *d_next_word,
                             void *d_work, uint64_t work_bytes, void *hip_stream);

#define ZG_SEQ_MAX_N 1000000ull

/* Workspace bytes zg_fill_sequential needs for n variates (0 for n = 0). */
zg_status zg_sequential_workspace(uint64_t n, uint64_t *bytes);

/* zg_fill_sequential without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): the workspace is a device-resident
 * array of the library, 8 MiB per GPU, held until the process ends; this
 * call allocates nothing.  Same arguments, bits and errors as
 * zg_fill_sequential, plus ZG_EINVAL for n above ZG_SEQ_NOALLOC_MAX_N (the
 * workspace of larger n would not fit; ZG_SEQ_MAX_N applies as well) and
 * ZG_ESTATE if the context could not resolve the array's address.  Every
 * call on one GPU shares that array: calls whose work overlaps on one GPU
 * (other streams, other contexts or threads) race and may write wrong
 * values; order them on one stream or by events.  No part of the array needs
 * clearing between calls (each call writes what it reads). */
zg_status zg_fill_sequential_noalloc(zg_ctx *ctx, double *d_out, uint64_t n, zg_kind kind,
                                     uint64_t seed, uint32_t stream, uint64_t first_word,
                                     uint64_t *d_next_word, void *hip_stream);
#define ZG_SEQ_NOALLOC_MAX_N 268435456ull

/* Test hook: one ziggurat attempt per crafted word.  d_class[i] = 0 (fast),
 * 1 (wedge), 2 (tail); d_x[i] = the signed first-word candidate
 * (double)j * w53[i].  All pointers are device memory. */
zg_status zg_decide_words(zg_ctx *ctx, const uint64_t *d_words, uint64_t n, uint8_t *d_class,
                          double *d_x, void *hip_stream);

/* Synchronises the device and reads the sticky ZG_FLAG_* bits; clears them
 * when clear != 0. */
zg_status zg_error_flags(zg_ctx *ctx, uint32_t *flags, int clear);

/* Test knobs.  ZG_KNOB_DMAX: draw budget (1..256, default 256), so that a
 * test can force budget exhaustion from the host.  ZG_KNOB_SEQ_SPANS: caps
 * the positions the parallel pass of zg_fill_sequential scans at value x
 * 16384 (0 = automatic, the default; at most 1024), so that a test can make
 * its one-lane finish produce the rest. */
#define ZG_KNOB_DMAX 1
#define ZG_KNOB_SEQ_SPANS 2
zg_status zg_set_test_knob(zg_ctx *ctx, int knob, int64_t value);

/* ------------------------------------------------ device-resident counters */

/* A handle names one device counter slot bound to (seed, stream, kind) and
 * to one output mode (dtype, method); counter = the next unused variate
 * index.  Fills through a handle reserve their index range on the device, in
 * the order they are enqueued, so the bits never depend on timing.
 * The mode is fixed because the variate index maps to uniform words
 * differently per mode (an FP32 variate pair shares one draw-0 word, a polar
 * pair reads the draw-0 and draw-1 words of one index): consecutive ranges of
 * one counter in different modes would read the same words again.  A
 * ZG_OP_MUTATE request consumes FP64 ziggurat variates and so goes through a
 * (ZG_F64, ZG_ZIGGURAT) handle.  Requests in another mode than the handle's
 * are refused with ZG_EINVAL by zg_stream_fill, zg_batch and
 * zg_server_submit.  zg_stream_open errors: ZG_EINVAL (null, enum, stream
 * limit, ZG_F32 with ZG_POLAR), ZG_EBUSY (every slot open), ZG_EHIP. */
typedef uint32_t zg_handle;
#define ZG_MAX_HANDLES 65536u
zg_status zg_stream_open(zg_ctx *ctx, uint64_t seed, uint32_t stream, zg_kind kind,
                         zg_dtype dtype, zg_method method, zg_handle *out);
zg_status zg_stream_close(zg_ctx *ctx, zg_handle h);
/* Reserves [counter, counter + n) and fills d_out with those variates;
 * dtype and method must be the handle's. */
zg_status zg_stream_fill(zg_ctx *ctx, zg_handle h, void *d_out, uint64_t n, zg_dtype dtype,
                         zg_method method, void *hip_stream);
/* Checkpoint / resume: read (after all queued work) or set the counter. */
zg_status zg_stream_get_counter(zg_ctx *ctx, zg_handle h, uint64_t *counter);
zg_status zg_stream_set_counter(zg_ctx *ctx, zg_handle h, uint64_t counter);

/* ------------------------------------------------------------------ batch */

#define ZG_OP_FILL 0
#define ZG_OP_MUTATE 1
#define ZG_NO_HANDLE (-1)
#define ZG_MAX_BATCH 32768u

/* One request of a batch.  op ZG_OP_FILL writes n variates to out (dtype,
 * method as zg_fill); ZG_OP_MUTATE applies zg_mutate to out (doubles, sigma).
 * handle >= 0 takes the first index from that device counter (and advances
 * it by n); otherwise first_index, seed, stream and kind are used as given.
 * A counter-keyed request whose range would pass its stream's index window
 * is skipped on the device (nothing written, ZG_FLAG_RANGE raised, its
 * completion word carries the skip bit), and its range stays reserved: the
 * counter still advances by n, so that the ranges of the batch's later
 * requests on that handle, planned on the host, stay as planned.  The handle
 * is then past its window until zg_stream_set_counter moves it back. */
typedef struct zg_request {
  void *out;
  uint64_t n;
  uint64_t seed;
  uint64_t first_index;
  double sigma;
  uint32_t stream;
  int32_t handle;
  uint8_t dtype;
  uint8_t method;
  uint8_t kind;
  uint8_t op;
  uint32_t reserved;
} zg_request;

/* Runs nreq uneven requests as one launch: the descriptors and the work
 * items (one per workgroup tile, grouped by op x uniform kind) are uploaded
 * in one copy, a reservation kernel resolves the counter-keyed first indices
 * in submission order, one persistent kernel per work class with work runs
 * the tiles, and a completion kernel publishes the completion words.  Large
 * batches launch as a hipGraph; batches of a few requests launch the same
 * kernels directly.  Same bits as the per-request calls.  first_out (host,
 * optional): receives each request's first index once the work has completed
 * (the call then synchronises the stream).  Errors as zg_fill for any
 * request; nothing is launched if any request is invalid.  Async on
 * hip_stream otherwise. */
zg_status zg_batch(zg_ctx *ctx, const zg_request *reqs, uint32_t nreq, uint64_t *first_out,
                   void *hip_stream);

/* The per-request form of a request array: each request (no handles) runs as
 * its own plain launch (zg_fill or zg_mutate), in order on hip_stream, from
 * one C loop.  Same bits as zg_batch; the baseline a batch is measured
 * against.  Every request is checked first (errors as zg_fill, ZG_EINVAL for
 * a handle); nothing is launched if any is invalid. */
zg_status zg_fill_each(zg_ctx *ctx, const zg_request *reqs, uint32_t nreq, void *hip_stream);

/* ----------------------------------------------------------------- tuning */

/* Launch shape of the generation kernels: tile, the elements per wave of a
 * workgroup tile (f64 units; multiple of 128; a workgroup tile is tile x
 * waves elements, which the waves of the plain fills take in groups of
 * group_steps steps of 256 elements), waves per workgroup (1..16),
 * batch_blocks_per_cu: for the batch kernels the persistent workgroups per CU
 * (1..8), for the plain fills 0 (one workgroup per tile) or the most
 * persistent workgroups per CU (capped by occupancy), queue_cap: the
 * workgroup's slow-path queue capacity of the plain ziggurat fills (0 = the
 * built-in maximum of 2048; smaller values, which also cap the retry queue
 * below its 512 entries, only serve to exercise the overflow paths),
 * drain_waves: 0 runs the plain ziggurat fills (FP64, FP32, mutation) with
 * the block-pooled kernel (streaming, one barrier, a drain of the pooled
 * slow elements, per workgroup tile), 1..8 with the wave-specialised kernel
 * (persistent workgroups of waves_per_block waves, batch_blocks_per_cu of
 * them per CU at most (at least one, capped by occupancy), drain_waves of
 * whose waves, at most waves_per_block - 1, resolve the slow elements the
 * others publish in an LDS ring; tile and queue_cap then do not apply; for
 * the batch class, drain_waves selects the wave-specialised class kernels
 * with the same meaning), and group_steps: the
 * 256-element steps a wave streams between queue appends (1, 2, 4 or 8; the
 * plain ziggurat fills and the wave-specialised batch class kernels).  Any
 * shape gives the same bits. */
typedef struct zg_tune {
  uint32_t tile;
  uint32_t waves_per_block;
  uint32_t batch_blocks_per_cu;
  uint32_t queue_cap;
  uint32_t drain_waves;
  uint32_t group_steps;
} zg_tune;
#define ZG_TUNE_FILL_F64 0
#define ZG_TUNE_FILL_F32 1
#define ZG_TUNE_POLAR 2
#define ZG_TUNE_MUTATE 3
#define ZG_TUNE_BATCH 4
#define ZG_TUNE_FILL_MZ 5   /* the modified ziggurat's plain fills */
#define ZG_TUNE_CLASSES 6
zg_status zg_get_tune(const zg_ctx *ctx, int cls, zg_tune *out);
zg_status zg_set_tune(zg_ctx *ctx, int cls, const zg_tune *in);
/* Times each candidate shape for each class on a scratch buffer of `bytes`
 * (0 = 1 GiB) and keeps the fastest; writes/reads a JSON cache at cache_path
 * (NULL: no cache).  When use_cache != 0 and the cache has an entry for this
 * device, nothing is timed.  The modified ziggurat's class keeps its current
 * shape (it is not timed). */
zg_status zg_autotune(zg_ctx *ctx, const char *cache_path, uint64_t bytes, int use_cache);

/* ---------------------------------------------------------------- serving */

typedef struct zg_server zg_server;
typedef struct zg_server_config {
  uint64_t mem_cap_bytes;     /* output arena size; admission keeps in-flight bytes below it */
  uint32_t max_inflight;      /* request slots in flight (admission) */
  uint32_t max_batch;         /* requests per batch launch (<= ZG_MAX_BATCH) */
  uint32_t batch_window_us;   /* how long the batcher waits to fill a batch */
  uint32_t n_streams;         /* HIP streams with batches in flight (1 or 2) */
  uint32_t mode;              /* ZG_SERVE_BATCHED or ZG_SERVE_PER_REQUEST */
  uint32_t reserved;
} zg_server_config;
#define ZG_SERVE_BATCHED 0
#define ZG_SERVE_PER_REQUEST 1

typedef struct zg_server_request {
  uint64_t n;
  zg_handle handle;           /* counter slot: seed, stream, kind, next index */
  uint8_t dtype;
  uint8_t method;
  uint16_t reserved;
  double arrival_s;           /* caller's arrival time on the server clock (zg_server_now) */
} zg_server_request;

typedef struct zg_completion {
  int32_t status;             /* ZG_OK, or an error for this request */
  int32_t done;               /* 1 once complete */
  void *d_out;                /* arena pointer with the output; valid until zg_server_release */
  uint64_t first_index;       /* index range the request received */
  double arrival_s, admit_s, complete_s;
} zg_completion;

typedef struct zg_server_stats {
  uint64_t submitted, completed, rejected, batches;
  uint64_t variates;
  uint64_t inflight_bytes, peak_inflight_bytes;
  double p50_latency_s, p99_latency_s, max_latency_s;
  double first_arrival_s, last_complete_s;
} zg_server_stats;

/* Starts a server (batcher and completion threads, its HIP streams, a device
 * arena of mem_cap_bytes and host-mapped completion records).  ZG_EINVAL for
 * a zero cap or slot count, max_batch above ZG_MAX_BATCH, n_streams outside
 * 1..2 or an unknown mode.  Batches on different streams that reserve from
 * the same handle are ordered by events, so every handle's ranges follow
 * submission order. */
zg_status zg_server_create(zg_ctx *ctx, const zg_server_config *cfg, zg_server **out);
/* Enqueues a request; returns a ticket.  Thread-safe.  ZG_EINVAL for a
 * request larger than the memory cap. */
zg_status zg_server_submit(zg_server *srv, const zg_server_request *req, uint64_t *ticket);
/* Non-blocking status of a ticket. */
zg_status zg_server_poll(zg_server *srv, uint64_t ticket, zg_completion *out);
/* Blocks until the ticket completes or timeout_s passes (ZG_EBUSY). */
zg_status zg_server_wait(zg_server *srv, uint64_t ticket, double timeout_s, zg_completion *out);
/* Gives the request's output memory back to the arena and forgets the ticket. */
zg_status zg_server_release(zg_server *srv, uint64_t ticket);
/* Blocks until every submitted request has completed. */
zg_status zg_server_drain(zg_server *srv);
zg_status zg_server_stats_get(zg_server *srv, zg_server_stats *out);
/* Seconds on the server's monotonic clock. */
double zg_server_now(const zg_server *srv);
/* Open-loop replay of a request trace (load generation for the serving
 * benchmark): submits reqs[k] when reqs[k].arrival_s seconds have passed
 * since the call, from the calling thread, so submission itself adds no
 * queueing; releases each output as soon as it completes (the arena then
 * bounds only the bytes in flight); returns once all have completed, or
 * ZG_EBUSY when timeout_s passes first (requests still running then are
 * released by the server when they complete).  first_out (host, optional, n
 * entries) receives each request's first index.  Returns the first request
 * error seen, if any (the other requests still run). */
zg_status zg_server_replay(zg_server *srv, const zg_server_request *reqs, uint32_t n,
                           uint64_t *first_out, double timeout_s);
/* Stops the threads (after draining), frees the arena and the streams. */
zg_status zg_server_destroy(zg_server *srv);

/* ----------------------------------------------------------------- errors */

const char *zg_strerror(zg_status st);
/* Text of the last HIP failure seen by this context (empty if none). */
const char *zg_last_error(const zg_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* ZG_H */
