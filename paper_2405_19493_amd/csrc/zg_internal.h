// Internal declarations shared by the host and device sources of libzg.
#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

#include "../../include/zg.h"

namespace zg {

constexpr uint64_t GAMMA = 0x9E3779B97F4A7C15ull;
constexpr uint64_t LCG_A = 0x5DEECE66Dull;
constexpr uint64_t LCG_C = 0xBull;
constexpr uint64_t LCG_M48 = (1ull << 48) - 1;
constexpr int LCG_JUMP_BYTES = 6;

// S -> (A S + C) mod 2^48: `k` LCG steps.
struct Affine {
  uint64_t A, C;
};

struct LcgTables {
  Affine jump[LCG_JUMP_BYTES][256];   // x * 256^b steps
  Affine window[256];                 // 2 d ZG_LCG_WINDOW steps
};

// Fast-path table entries, packed so one LDS read serves one lane.
struct Fast64 {
  uint64_t k;   // k53
  double w;     // w53
};
struct Fast32 {
  uint32_t k;   // k24
  float w;      // w24
};

// The modified ziggurat's slow-path tables (zg_mz_table_view): one region's
// box, and one bucket's threshold and alias, each read as one unit.
struct MzRegion {
  double ox, odx, oy, ody;
};
struct MzBucket {
  uint64_t thr;
  uint32_t alias;
  uint32_t pad;
};
struct MzTabs {
  double xs[ZG_MZ_BUCKETS];
  MzRegion region[ZG_MZ_LAYERS + 1];
  MzBucket bucket[ZG_MZ_BUCKETS];
  uint32_t kind[ZG_MZ_LAYERS + 3];
  double x0;
};

// Everything the kernels read, in one device allocation per context.
// Logarithm table of the polar method: for m in [sqrt(1/2), sqrt(2)) split
// at the top 7 mantissa bits of its binade (index LOG_I0 + k), invc[k] is a
// 7-bit approximation of 1/m (exactly 1 next to m = 1), so that m invc - 1 is
// exact, and -log(invc) = hi + lo with hi a multiple of 2^-33.
constexpr int LOG_N = 129;
constexpr int LOG_I0 = 53;
struct LogEnt {
  double invc;
  double hi;
};
struct LogTables {
  LogEnt e[LOG_N];
  double lo[LOG_N];
};

struct DevTables {
  Fast64 fast64[ZG_LAYERS];
  Fast32 fast32[ZG_LAYERS];
  double y[ZG_LAYERS];
  double dy[ZG_LAYERS];
  double w53[ZG_LAYERS];
  double w24d[ZG_LAYERS];
  double r;
  double pad[7];
  LcgTables lcg;
  LogTables logt;
  MzTabs mz;
};

// Operation selector shared by the plain and batch kernels.
enum Op : uint32_t { OP_ZIG64 = 0, OP_ZIG32 = 1, OP_POLAR = 2, OP_MUTATE = 3, OP_MZ64 = 4 };

// One generation job over elements [0, n_streams * n_per) of an output:
// element e is variate first + (e mod n_per) of stream s0 + e / n_per.
struct Job {
  void *out;
  uint64_t n_per;
  uint64_t n_total;
  uint64_t first;
  uint64_t seed;
  double sigma;
  double inv_n_per;   // RN(1 / n_per): element -> stream split on rare paths
  uint32_t s0;
  uint32_t n_streams;
  uint32_t kind;
  uint32_t op;
};

// A batch request as the device sees it (host fills all but `first`,
// which the reserve kernel resolves from the counters when handle >= 0).
// The request is split into workgroup tiles of `tile` elements per wave; its
// completion word is written once the whole batch has run.
struct DevRequest {
  Job job;
  uint64_t off;          // counter offset of this request among earlier
                         // requests of the same handle in the batch
  int32_t handle;
  uint32_t last_of_handle;   // 1: advance the counter by off + n after the batch
  uint64_t limit;        // index window of the kind (first + n must stay <= limit)
  uint32_t *done_flag;   // host-visible completion word (may be null)
  uint64_t *first_host;  // host-visible copy of the resolved first index (may be null)
  uint32_t done_value;
  uint32_t tiles;        // workgroup tiles of this request
  uint32_t status;       // 0 ok, ZG_FLAG_RANGE when skipped
  uint32_t pad;
  uint32_t tile;         // elements per wave of a workgroup tile
  uint32_t head;         // elements before the first 16-byte aligned one
};

// Work classes of a batch: op (ZIG64, ZIG32, MUTATE, POLAR) x uniform kind
// (SplitMix64, LCG48); each runs in its own specialised kernel.
constexpr int BATCH_CLASSES = 8;
__host__ __device__ constexpr int batch_class(uint32_t op, uint32_t kind) {
  return 2 * (op == OP_ZIG64 ? 0 : op == OP_ZIG32 ? 1 : op == OP_MUTATE ? 2 : 3) +
         (kind == ZG_JAVA_LCG48 ? 1 : 0);
}

// Batch header, uploaded with the requests and the work items (one 64-bit
// item per workgroup tile: request index << 32 | tile index, grouped by class).
struct BatchHeader {
  uint32_t nreq;
  uint32_t dmax;
  uint32_t n_items;
  uint32_t items_off;   // byte offset of the items from the header
  uint32_t cls_off[BATCH_CLASSES];
  uint32_t cls_cnt[BATCH_CLASSES];
  // wave-specialised class kernels (ws_drain > 0): drain waves per
  // workgroup, steps per streaming group, and groups per item of each class
  uint32_t ws_drain;
  uint32_t ws_gsteps;
  uint32_t cls_groups[BATCH_CLASSES];
  uint64_t pad[1];
};

// Sequential consumption (one generator read in order): the parallel pass
// scans positions in chunks of SEQ_CHUNK (one wave each), SEQ_WAVES chunks per
// workgroup.
constexpr uint32_t SEQ_WINDOWS = 16;                   // windows of 64 positions per chunk
constexpr uint32_t SEQ_CHUNK = 64 * SEQ_WINDOWS;       // positions per chunk
constexpr uint32_t SEQ_WAVES = 16;                     // chunks (waves) per workgroup
constexpr uint64_t SEQ_SPAN = (uint64_t)SEQ_CHUNK * SEQ_WAVES;   // positions per workgroup
constexpr uint64_t SEQ_FINISH_CAP = 1ull << 22;        // attempts of the sequential finish
constexpr uint64_t SEQ_MAX_WG = 1024;                  // largest plan accepted (workgroups)

// Three-state map of a chunk (or of a workgroup's chunks in order): entered
// at offset e (0..2) of its first position, the chain leaves it at offset
// exit(e) of the next chunk's first position, having accepted cnt[e] attempts.
struct SeqMap {
  uint32_t cnt[3];
  uint32_t exits;   // bits 2e..2e+1: exit(e)
};
// A workgroup's entry: the chain enters at offset e, and its first accepted
// attempt is variate `base`.
struct SeqEntry {
  uint64_t base;
  uint32_t e;
  uint32_t pad;
};
// Result of the scan over all workgroups: accepted attempts in the scanned
// positions, and the chain's entry offset past them.
struct SeqHdr {
  uint64_t total;
  uint32_t exit;
  uint32_t pad;
};
struct SeqJob {
  double *out;
  uint64_t n;           // variates wanted
  uint64_t seed;
  uint64_t first;       // word position of the first attempt
  uint64_t n_pos;       // positions of the parallel pass (whole SEQ_SPANs)
  uint64_t limit;       // word positions must stay below this (the index window)
  uint64_t *next_word;  // device (may be null): position after the last word read
  uint32_t s;           // stream
  uint32_t kind;
};

// Host entry points of the device code (zg_kernels.hip).
// resident: 0 = one workgroup per tile; k > 0 = a persistent grid of at most
// k workgroups per CU (capped by occupancy) looping over the tiles.
// n_drain > 0 (ziggurat ops): the wave-specialised kernel, one 16-wave
// workgroup per CU of which n_drain waves resolve the slow elements (tile,
// waves, qcap and resident do not apply).  gsteps: 256-element steps a wave
// streams between queue appends (1..8).
hipError_t launch_fill(const Job &J, const DevTables *T, uint32_t dmax, uint32_t *flags,
                       uint32_t tile, uint32_t waves, uint32_t head, uint32_t qcap,
                       uint32_t resident, uint32_t n_drain, uint32_t gsteps, hipStream_t stream);
// One EA generation (zg_ea_step); rate53 = floor(rate 2^53).
struct EaJob {
  const double *parents;
  const double *fitness;
  double *children;
  uint32_t *winners;
  uint64_t seed, generation, rate53;
  double sigma, lo, hi;
  uint32_t pop, genes, tournament, stream;
};
hipError_t launch_ea(const EaJob &E, const DevTables *T, uint32_t dmax, uint32_t *flags,
                     hipStream_t stream);
hipError_t launch_words(uint64_t *out, uint64_t n, const DevTables *T, uint32_t kind,
                        uint64_t seed, uint32_t s, uint32_t d, uint64_t first, hipStream_t stream);
hipError_t launch_decide(const uint64_t *words, uint64_t n, const DevTables *T, uint8_t *cls,
                         double *x, hipStream_t stream);
// The plan of a sequential fill of n variates: the positions its parallel
// passes scan, their workgroups, and where each buffer lies in the
// workspace.  seq_plan is the only place these are derived, for the size
// query, the entry points and the launch alike, so the workspace is always
// sized for the grid that writes it.
struct SeqPlan {
  uint64_t n_pos;     // positions scanned (whole SEQ_SPANs)
  uint64_t n_wg;      // workgroups of the map and write passes: n_pos / SEQ_SPAN
  uint64_t wg_cap;    // workgroups the buffers are sized for (>= n_wg)
  uint64_t off_wg_maps, off_entry, off_hdr;   // byte offsets (chunk maps at 0)
  uint64_t bytes;     // workspace bytes
};
// cap_wg > 0 scans at most cap_wg workgroups of positions (a test knob that
// leaves the rest to the one-lane finish); the buffers keep the sizes of the
// uncapped plan.
SeqPlan seq_plan(uint64_t n, uint64_t cap_wg = 0);
// The four passes of a sequential fill (maps, scan, write, finish) on one
// stream.  J.n_pos must be P.n_pos and `work` must hold P.bytes bytes; a plan
// that does not fit its buffers is refused (hipErrorInvalidValue) before
// anything is launched.
hipError_t launch_seq(const SeqJob &J, const SeqPlan &P, const DevTables *T, void *work,
                      uint64_t work_bytes, uint32_t *flags, hipStream_t stream);
// Bytes of the device-resident sequential workspace (one per GPU).
constexpr size_t SEQ_SCRATCH_BYTES = 8u << 20;
// Device address of that workspace on device `dev`, which must be current;
// resolved once per device (hipGetSymbolAddress) and kept.
hipError_t seq_scratch_ptr(int dev, void **out);
const void *kernel_reserve();
const void *kernel_complete();
// The kernel of a work class, and its dynamic LDS for `waves` waves.
// Class kernel of a batch: the wave-specialised one (ziggurat classes) when
// ws, else the block-pooled one.
const void *kernel_batch_class(int cls, bool ws);
hipError_t launch_batch_class(int cls, bool ws, uint32_t grid, uint32_t waves, DevRequest *R,
                              const BatchHeader *H, const DevTables *T, uint32_t *flags,
                              hipStream_t stream);
size_t batch_class_lds_bytes(int cls, uint32_t waves);

zg_status build_table(zg_table_view *t);
zg_status build_mz_table(zg_mz_table_view *t);
// Everything the kernels read, from the layer table tv: the fast-path and
// slow-path entries, the modified ziggurat's tables, the LCG jump tables and
// the polar log table.
zg_status build_dev_tables(const zg_table_view &tv, DevTables *h);
void build_lcg_tables(LcgTables *L);
void build_log_tables(LogTables *L);
Affine lcg_power(uint64_t k);

}  // namespace zg
