// The device source of libzg built for the host, with the shim in
// tests/host/shim, and run through its own launch functions.  Built with
// AddressSanitizer, so that any access outside its buffer stops it.
//   kernel_emu N KIND SEED STREAM FIRST OUTFILE
//     the sequential-consumption passes (launch_seq): writes the position
//     after the last word read, then the N values;
//   kernel_emu scan N_WG SEED
//     the scan pass alone over synthetic maps (see scan_only);
//   kernel_emu fill OP KIND SEED S0 NSTREAMS NPER FIRST HEAD NDRAIN GSTEPS OUTFILE [INFILE]
//     a plain fill (launch_fill) of NSTREAMS x NPER elements, OP 0 FP64,
//     1 FP32, 3 mutation (sigma 0.1, the initial doubles read from INFILE),
//     with the output HEAD elements past a 16-byte boundary, by the pooled
//     kernel (NDRAIN 0) or the wave-specialised one with NDRAIN drain waves,
//     GSTEPS steps per group; writes the values.
//   kernel_emu batch WS WAVES NDRAIN GSTEPS TILE GRID SPEC OUTFILE INFILE
//     one batch class kernel (launch_batch_class), wave-specialised (WS 1,
//     NDRAIN drain waves, GSTEPS steps per group) or block-pooled (WS 0),
//     WAVES waves per workgroup, TILE elements per wave (twice for FP32), a
//     grid of GRID workgroups, over the requests of SPEC (lines: op kind n
//     seed stream head; one class), each output HEAD elements before a 16-byte
//     boundary; mutation requests start from INFILE's doubles in request
//     order.  The header, requests and items are laid out as zg_batch lays
//     them out; writes every request's values in request order.
#include "hip/hip_runtime.h"

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <map>

thread_local uint3_ threadIdx;
uint3_ blockIdx, blockDim, gridDim;
std::vector<std::unique_ptr<EmuWave>> emu_waves;
std::unique_ptr<std::barrier<>> emu_block_bar;

namespace {
// One pool of nt threads per block size, reused for every block.
struct Pool {
  explicit Pool(uint32_t n) : nt(n), start(n + 1), done(n + 1) {
    for (uint32_t t = 0; t < nt; ++t)
      th.emplace_back([this, t]() {
        threadIdx = {t, 0, 0};
        for (;;) {
          start.arrive_and_wait();
          if (quit) return;
          (*body)();
          done.arrive_and_wait();
        }
      });
  }
  ~Pool() {
    quit = true;
    start.arrive_and_wait();
    for (auto &x : th) x.join();
  }
  uint32_t nt;
  std::barrier<> start, done;
  std::vector<std::thread> th;
  const std::function<void()> *body = nullptr;
  bool quit = false;
};
std::map<uint32_t, std::unique_ptr<Pool>> pools;
}  // namespace

void emu_run_grid(dim3 grid, dim3 block, const std::function<void()> &body) {
  const uint32_t nt = block.x;
  auto &pool = pools[nt];
  if (!pool) pool = std::make_unique<Pool>(nt);
  blockDim = {block.x, 1, 1};
  gridDim = {grid.x, 1, 1};
  pool->body = &body;
  for (uint32_t b = 0; b < grid.x; ++b) {
    blockIdx = {b, 0, 0};
    emu_block_bar = std::make_unique<std::barrier<>>(nt);
    emu_waves.clear();
    for (uint32_t w = 0; w < (nt + 63) / 64; ++w) {
      auto x = std::make_unique<EmuWave>();
      x->bar = std::make_unique<std::barrier<>>(nt - 64 * w < 64 ? nt - 64 * w : 64);
      emu_waves.push_back(std::move(x));
    }
    pool->start.arrive_and_wait();
    pool->done.arrive_and_wait();
  }
}

namespace zg {
alignas(16) unsigned char s_polar[1 << 17];
}

#include "zg_table.cpp"
#include "zg_kernels_emu.cpp"

using namespace zg;

// kernel_emu scan N_WG SEED: the scan pass alone over N_WG synthetic workgroup
// maps (random counts, random exits), against the maps composed in order one
// at a time.  Prints "scan ok" or the first difference.
static int scan_only(uint32_t n_wg, uint64_t seed) {
  std::vector<SeqMap> maps(n_wg);
  uint64_t x = seed * 0x9E3779B97F4A7C15ull + 1;
  auto next = [&x]() {
    x ^= x << 13;
    x ^= x >> 7;
    x ^= x << 17;
    return x;
  };
  for (auto &m : maps) {
    for (int e = 0; e < 3; ++e) m.cnt[e] = (uint32_t)(next() % 20000);
    m.exits = 0;
    for (int e = 0; e < 3; ++e) m.exits |= (uint32_t)(next() % 3) << (2 * e);
  }
  // buffers of exactly the sizes the pass may touch, so that ASan sees any
  // access outside them
  SeqMap *d_maps = (SeqMap *)malloc(sizeof(SeqMap) * n_wg);
  std::memcpy(d_maps, maps.data(), sizeof(SeqMap) * n_wg);
  SeqEntry *d_ent = (SeqEntry *)malloc(sizeof(SeqEntry) * n_wg);
  SeqHdr *d_hdr = (SeqHdr *)malloc(sizeof(SeqHdr));
  hipLaunchKernelGGL(k_seq_scan, dim3(1), dim3(1024), 0, nullptr, (const SeqMap *)d_maps, n_wg,
                     d_ent, d_hdr);
  uint64_t base = 0;
  uint32_t ent = 0;
  int bad = 0;
  for (uint32_t k = 0; k < n_wg && !bad; ++k) {
    if (d_ent[k].base != base || d_ent[k].e != ent) {
      std::fprintf(stderr, "workgroup %u: got (%llu, %u) want (%llu, %u)\n", k,
                   (unsigned long long)d_ent[k].base, d_ent[k].e, (unsigned long long)base, ent);
      bad = 1;
    }
    base += maps[k].cnt[ent];
    ent = (maps[k].exits >> (2 * ent)) & 3u;
  }
  if (!bad && (d_hdr->total != base || d_hdr->exit != ent)) {
    std::fprintf(stderr, "header: got (%llu, %u) want (%llu, %u)\n",
                 (unsigned long long)d_hdr->total, d_hdr->exit, (unsigned long long)base, ent);
    bad = 1;
  }
  free(d_maps);
  free(d_ent);
  free(d_hdr);
  pools.clear();
  if (!bad) std::printf("scan ok n_wg=%u total=%llu\n", n_wg, (unsigned long long)base);
  return bad;
}

static DevTables *host_tables() {
  zg_table_view tv;
  if (build_table(&tv) != ZG_OK) return nullptr;
  DevTables *T = new DevTables();
  if (build_dev_tables(tv, T) != ZG_OK) {
    delete T;
    return nullptr;
  }
  return T;
}

static int fill_only(char **a) {
  const uint32_t op = (uint32_t)atoi(a[0]), kind = (uint32_t)atoi(a[1]);
  const uint64_t seed = strtoull(a[2], 0, 10);
  const uint32_t s0 = (uint32_t)atoi(a[3]), ns = (uint32_t)atoi(a[4]);
  const uint64_t n_per = strtoull(a[5], 0, 10), first = strtoull(a[6], 0, 10);
  const uint32_t head = (uint32_t)atoi(a[7]), n_drain = (uint32_t)atoi(a[8]);
  const uint32_t gsteps = (uint32_t)atoi(a[9]);
  const char *outfile = a[10], *infile = a[11];
  const uint64_t n = (uint64_t)ns * n_per;
  const size_t esz = op == OP_ZIG32 ? 4 : 8;
  const uint32_t per16 = (uint32_t)(16 / esz);
  if (head >= per16 || n == 0) return 2;
  DevTables *T = host_tables();
  if (!T) return 2;
  // exactly n elements, starting `head` elements before a 16-byte boundary
  const size_t lead = (per16 - head) % per16;
  // malloc's blocks are 16-byte aligned here; the exact size lets
  // AddressSanitizer see any store past the last element
  char *base = (char *)malloc((n + lead) * esz);
  if (((uintptr_t)base) % 16) return 5;
  void *out = base + lead * esz;
  std::vector<char> keep(n * esz);
  if (op == OP_MUTATE) {
    FILE *f = fopen(infile, "rb");
    if (!f || fread(out, 8, n, f) != n) return 3;
    fclose(f);
  }
  uint32_t *flags = (uint32_t *)calloc(1, sizeof(uint32_t));
  Job J{out, n_per, n, first, seed, 0.1, 1.0 / (double)n_per, s0, ns, kind, op};
  const uint32_t h = op == OP_ZIG32 ? (uint32_t)((4 - (((uintptr_t)out >> 2) & 3)) & 3)
                                    : (uint32_t)(((uintptr_t)out >> 3) & 1);
  const uint32_t hd = (uint32_t)std::min<uint64_t>(h, n);
  std::fprintf(stderr, "fill op=%u n=%llu head=%u drain=%u\n", op, (unsigned long long)n, hd,
               n_drain);
  // the block-pooled kernel's shape: EMU_TILE, EMU_WAVES, EMU_RES (persistent
  // workgroups per compute unit) override 1024 x 16 x 2
  const char *et = getenv("EMU_TILE"), *ew = getenv("EMU_WAVES"), *er = getenv("EMU_RES");
  const uint32_t tile = et ? (uint32_t)atoi(et) : 1024, waves = ew ? (uint32_t)atoi(ew) : 16;
  const uint32_t res = er ? (uint32_t)atoi(er) : 2;
  if (launch_fill(J, T, ZG_MAX_DRAWS, flags, tile, waves, hd, 0, res, n_drain, gsteps, nullptr) !=
      hipSuccess)
    return 4;
  FILE *f = fopen(outfile, "wb");
  if (!f) return 3;
  fwrite(out, esz, n, f);
  fclose(f);
  std::fprintf(stderr, "flags=%u\n", *flags);
  free(base);
  free(flags);
  delete T;
  pools.clear();
  return 0;
}

static int batch_only(char **a) {
  const bool ws = atoi(a[0]) != 0;
  const uint32_t waves = (uint32_t)atoi(a[1]), n_drain = (uint32_t)atoi(a[2]);
  const uint32_t gsteps = (uint32_t)atoi(a[3]), tile = (uint32_t)atoi(a[4]);
  const uint32_t grid = (uint32_t)atoi(a[5]);
  FILE *sp = fopen(a[6], "r");
  if (!sp) return 3;
  struct Spec {
    uint32_t op, kind;
    uint64_t n, seed;
    uint32_t stream, head;
  };
  std::vector<Spec> sv;
  Spec x;
  while (fscanf(sp, "%u %u %llu %llu %u %u", &x.op, &x.kind, (unsigned long long *)&x.n,
                (unsigned long long *)&x.seed, &x.stream, &x.head) == 6)
    sv.push_back(x);
  fclose(sp);
  if (sv.empty()) return 2;
  const int c = batch_class(sv[0].op, sv[0].kind);
  FILE *in = sv[0].op == OP_MUTATE ? fopen(a[8], "rb") : nullptr;
  std::vector<char *> bases;
  std::vector<DevRequest> reqs;
  std::vector<uint64_t> items;
  for (size_t k = 0; k < sv.size(); ++k) {
    const Spec &q = sv[k];
    if (batch_class(q.op, q.kind) != c || q.n == 0) return 2;
    const size_t esz = q.op == OP_ZIG32 ? 4 : 8;
    const uint32_t per16 = (uint32_t)(16 / esz);
    if (q.head >= per16) return 2;
    const size_t lead = (per16 - q.head) % per16;
    char *base = (char *)malloc((q.n + lead) * esz);   // exact: ASan sees any overrun
    if (((uintptr_t)base) % 16) return 5;
    bases.push_back(base);
    void *out = base + lead * esz;
    if (q.op == OP_MUTATE && (!in || fread(out, 8, q.n, in) != q.n)) return 3;
    DevRequest d{};
    d.job = Job{out, q.n, q.n, 0, q.seed, 0.1, 1.0 / (double)q.n, q.stream, 1, q.kind, q.op};
    d.handle = ZG_NO_HANDLE;
    d.limit = q.kind == ZG_JAVA_LCG48 ? ZG_LCG_WINDOW : ZG_SM64_WINDOW;
    const uint32_t wave_tile = q.op == OP_ZIG32 ? 2 * tile : tile;
    d.tile = (wave_tile + 255) / 256 * 256;
    const uint32_t h = q.op == OP_ZIG32 ? (uint32_t)((4 - (((uintptr_t)out >> 2) & 3)) & 3)
                                        : (uint32_t)(((uintptr_t)out >> 3) & 1);
    d.head = (uint32_t)std::min<uint64_t>(h, q.n);
    const uint64_t per = (uint64_t)d.tile * waves;
    uint64_t tiles = (q.n - d.head + per - 1) / per;
    if (tiles == 0) tiles = 1;
    d.tiles = (uint32_t)tiles;
    for (uint32_t j = 0; j < d.tiles; ++j) items.push_back(((uint64_t)k << 32) | j);
    reqs.push_back(d);
  }
  if (in) fclose(in);
  // header, requests, items: one buffer, as a batch slot holds them
  const size_t items_off = sizeof(BatchHeader) + reqs.size() * sizeof(DevRequest);
  char *buf = (char *)calloc(1, items_off + items.size() * sizeof(uint64_t));
  BatchHeader *H = (BatchHeader *)buf;
  DevRequest *R = (DevRequest *)(buf + sizeof(BatchHeader));
  H->nreq = (uint32_t)reqs.size();
  H->dmax = ZG_MAX_DRAWS;
  H->n_items = (uint32_t)items.size();
  H->items_off = (uint32_t)items_off;
  H->cls_off[c] = 0;
  H->cls_cnt[c] = (uint32_t)items.size();
  H->ws_drain = ws ? n_drain : 0;
  H->ws_gsteps = gsteps;
  const uint64_t per = (uint64_t)reqs[0].tile * waves, ge = 256ull * gsteps;
  H->cls_groups[c] = (uint32_t)((per + ge - 1) / ge);
  std::memcpy(R, reqs.data(), reqs.size() * sizeof(DevRequest));
  std::memcpy(buf + items_off, items.data(), items.size() * sizeof(uint64_t));
  DevTables *T = host_tables();
  uint32_t *flags = (uint32_t *)calloc(1, sizeof(uint32_t));
  std::fprintf(stderr, "batch class=%d requests=%zu items=%zu ws=%d groups=%u\n", c, reqs.size(),
               items.size(), (int)ws, H->cls_groups[c]);
  if (launch_batch_class(c, ws, grid, waves, R, H, T, flags, nullptr) != hipSuccess) return 4;
  FILE *f = fopen(a[7], "wb");
  if (!f) return 3;
  for (size_t k = 0; k < reqs.size(); ++k)
    fwrite(reqs[k].job.out, sv[k].op == OP_ZIG32 ? 4 : 8, sv[k].n, f);
  fclose(f);
  std::fprintf(stderr, "flags=%u\n", *flags);
  for (char *b : bases) free(b);
  free(buf);
  free(flags);
  delete T;
  pools.clear();
  return 0;
}

// ea POP GENES K SEED STREAM GEN RATE SIGMA LO HI PARENTS FITNESS CHILDREN WINNERS:
// one EA generation (launch_ea) from float64 files, outputs to files.
static int ea_only(char **a) {
  EaJob E{};
  E.pop = (uint32_t)atoi(a[0]);
  E.genes = (uint32_t)atoi(a[1]);
  E.tournament = (uint32_t)atoi(a[2]);
  E.seed = strtoull(a[3], 0, 10);
  E.stream = (uint32_t)atoi(a[4]);
  E.generation = strtoull(a[5], 0, 10);
  E.rate53 = (uint64_t)(atof(a[6]) * 9007199254740992.0);
  E.sigma = atof(a[7]);
  E.lo = atof(a[8]);
  E.hi = atof(a[9]);
  const uint64_t cells = (uint64_t)E.pop * E.genes;
  double *P = (double *)malloc(cells * 8), *F = (double *)malloc((size_t)E.pop * 8);
  double *C = (double *)malloc(cells * 8);
  uint32_t *W = (uint32_t *)malloc((size_t)E.pop * 4);
  FILE *f = fopen(a[10], "rb");
  if (!f || fread(P, 8, cells, f) != cells) return 3;
  fclose(f);
  f = fopen(a[11], "rb");
  if (!f || fread(F, 8, E.pop, f) != E.pop) return 3;
  fclose(f);
  E.parents = P;
  E.fitness = F;
  E.children = C;
  E.winners = W;
  DevTables *T = host_tables();
  uint32_t *flags = (uint32_t *)calloc(1, sizeof(uint32_t));
  if (launch_ea(E, T, ZG_MAX_DRAWS, flags, nullptr) != hipSuccess) return 4;
  f = fopen(a[12], "wb");
  fwrite(C, 8, cells, f);
  fclose(f);
  f = fopen(a[13], "wb");
  fwrite(W, 4, E.pop, f);
  fclose(f);
  std::fprintf(stderr, "flags=%u\n", *flags);
  free(P);
  free(F);
  free(C);
  free(W);
  free(flags);
  delete T;
  pools.clear();
  return 0;
}

int main(int argc, char **argv) {
  if (argc >= 16 && std::strcmp(argv[1], "ea") == 0) return ea_only(argv + 2);
  if (argc >= 11 && std::strcmp(argv[1], "batch") == 0) return batch_only(argv + 2);
  if (argc == 4 && std::strcmp(argv[1], "scan") == 0)
    return scan_only((uint32_t)strtoul(argv[2], 0, 10), strtoull(argv[3], 0, 10));
  if (argc >= 13 && std::strcmp(argv[1], "fill") == 0) return fill_only(argv + 2);
  if (argc < 7) return 2;
  const uint64_t n = strtoull(argv[1], 0, 10);
  const uint32_t kind = (uint32_t)atoi(argv[2]);
  const uint64_t seed = strtoull(argv[3], 0, 10);
  const uint32_t s = (uint32_t)atoi(argv[4]);
  const uint64_t first = strtoull(argv[5], 0, 10);
  DevTables *T = host_tables();
  if (!T) return 2;
  // the plan of zg_fill_sequential (without its size caps), and a workspace
  // of exactly its size
  const SeqPlan P = seq_plan(n);
  const uint64_t limit = kind == ZG_JAVA_LCG48 ? ZG_LCG_WINDOW : ZG_SM64_WINDOW;
  double *out = (double *)malloc(n * sizeof(double));
  uint64_t *next = (uint64_t *)malloc(sizeof(uint64_t));
  uint32_t *flags = (uint32_t *)calloc(1, sizeof(uint32_t));
  void *work = malloc(P.bytes);
  std::fprintf(stderr, "n=%llu n_pos=%llu workgroups=%llu\n", (unsigned long long)n,
               (unsigned long long)P.n_pos, (unsigned long long)P.n_wg);
  SeqJob J{out, n, seed, first, P.n_pos, limit, next, s, kind};
  if (launch_seq(J, P, T, work, P.bytes, flags, nullptr) != hipSuccess) return 4;
  FILE *f = fopen(argv[6], "wb");
  if (!f) return 3;
  fwrite(next, 8, 1, f);
  fwrite(out, 8, n, f);
  fclose(f);
  free(out);
  free(next);
  free(flags);
  free(work);
  delete T;
  pools.clear();
  return 0;
}
