// Launch-shape autotuner: for each kernel class, times a small grid of shapes
// on a scratch buffer and keeps the fastest: for the plain ziggurat fills the
// block-pooled kernel at (tile, waves per block, persistent blocks per CU,
// steps per group) and the wave-specialised kernel at (drain waves, steps per
// group); for the polar kernel (tile, waves); for the batch kernels (tile,
// waves, persistent blocks per CU).  The output bits do not depend on the
// shape (variates are index-keyed), so tuning never changes results.  Results
// are cached in a small JSON file keyed by the device architecture and the
// HIP runtime version.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "zg_ctx.h"

using namespace zg;

namespace {

const char *CLASS_NAME[ZG_TUNE_CLASSES] = {"fill_f64", "fill_f32", "polar",
                                          "mutate",   "batch",    "fill_mz"};

bool read_cache(const char *path, const std::string &arch, zg_tune *out) {
  FILE *f = std::fopen(path, "r");
  if (!f) return false;
  std::string text;
  char buf[4096];
  size_t k;
  while ((k = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, k);
  std::fclose(f);
  std::string key = "\"" + arch + "\"";
  size_t pos = text.find(key);
  if (pos == std::string::npos) return false;
  for (int c = 0; c < ZG_TUNE_CLASSES; ++c) {
    std::string ck = std::string("\"") + CLASS_NAME[c] + "\"";
    size_t p = text.find(ck, pos);
    if (p == std::string::npos) return false;
    unsigned a, b, d, w, g;
    if (std::sscanf(text.c_str() + p + ck.size(), " : [ %u , %u , %u , %u , %u ]", &a, &b, &d,
                    &w, &g) != 5)
      return false;
    out[c] = {a, b, d, 0, w, g};
  }
  return true;
}

bool write_cache(const char *path, const std::string &arch, const zg_tune *t) {
  FILE *f = std::fopen(path, "w");
  if (!f) return false;
  std::fprintf(f, "{\n  \"%s\": {\n", arch.c_str());
  for (int c = 0; c < ZG_TUNE_CLASSES; ++c)
    std::fprintf(f, "    \"%s\": [%u, %u, %u, %u, %u]%s\n", CLASS_NAME[c], t[c].tile,
                 t[c].waves_per_block, t[c].batch_blocks_per_cu, t[c].drain_waves,
                 t[c].group_steps, c + 1 < ZG_TUNE_CLASSES ? "," : "");
  std::fprintf(f, "  }\n}\n");
  std::fclose(f);
  return true;
}

// Median time in ms of `reps` runs of fn on stream s.
template <class F>
float time_ms(F fn, hipStream_t s, hipEvent_t a, hipEvent_t b, int reps) {
  std::vector<float> t;
  for (int r = 0; r < reps + 1; ++r) {
    (void)hipEventRecord(a, s);
    fn();
    (void)hipEventRecord(b, s);
    (void)hipEventSynchronize(b);
    float ms = 0;
    (void)hipEventElapsedTime(&ms, a, b);
    if (r > 0) t.push_back(ms);   // first run warms up
  }
  std::sort(t.begin(), t.end());
  return t[t.size() / 2];
}

}  // namespace

extern "C" zg_status zg_autotune(zg_ctx *ctx, const char *cache_path, uint64_t bytes,
                                 int use_cache) {
  if (!ctx) return ZG_EINVAL;
  // cache key: the architecture and the HIP runtime (a new runtime may favour
  // other shapes)
  std::string arch = ctx->arch.empty() ? std::string("unknown") : ctx->arch;
  int rt = 0;
  if (hipRuntimeGetVersion(&rt) == hipSuccess) arch += " hip " + std::to_string(rt);
  if (use_cache && cache_path) {
    zg_tune t[ZG_TUNE_CLASSES];
    if (read_cache(cache_path, arch, t)) {
      for (int c = 0; c < ZG_TUNE_CLASSES; ++c) {
        zg_status st = zg_set_tune(ctx, c, &t[c]);
        if (st != ZG_OK) return st;
      }
      return ZG_OK;
    }
  }
  if (bytes == 0) bytes = 1ull << 30;
  bytes &= ~(uint64_t)255;
  if (bytes < (1u << 20)) return ZG_EINVAL;
  int prev = -1;
  (void)hipGetDevice(&prev);
  (void)hipSetDevice(ctx->device);
  void *buf = nullptr;
  hipStream_t s = nullptr;
  hipEvent_t a = nullptr, b = nullptr;
  hipError_t e = hipMalloc(&buf, bytes);
  if (e == hipSuccess) e = hipStreamCreateWithFlags(&s, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&a);
  if (e == hipSuccess) e = hipEventCreate(&b);
  zg_status st = e == hipSuccess ? ZG_OK : hip_fail(ctx, e, "autotune setup");
  // candidate shapes of the plain fills: block-pooled ones, then
  // wave-specialised ones (drain waves > 0; tile and waves do not apply)
  std::vector<zg_tune> cands;
  for (uint32_t tl : {1024u, 2048u, 4096u})
    for (uint32_t w : {8u, 16u})
      for (uint32_t res : {0u, 2u})
        for (uint32_t gs : {2u, 4u}) cands.push_back({tl, w, res, 0, 0, gs});
  for (uint32_t dw : {3u, 4u, 6u, 8u})
    for (uint32_t gs : {2u, 4u, 8u}) cands.push_back({1024, 16, 2, 0, dw, gs});
  // the plain-fill classes (the batch below; the modified ziggurat keeps its shape)
  for (int c = 0; c < ZG_TUNE_BATCH && st == ZG_OK; ++c) {
    zg_tune best = ctx->tune[c];
    float best_ms = 1e30f;
    for (const zg_tune &base : cands) {
      zg_tune cand = base;
      if (c == ZG_TUNE_POLAR && (cand.batch_blocks_per_cu || cand.drain_waves || cand.group_steps != 4))
        continue;   // the polar kernel is never persistent and has no groups
      if (c == ZG_TUNE_FILL_F32) cand.tile *= 2;
      st = zg_set_tune(ctx, c, &cand);
      if (st != ZG_OK) break;
      auto run = [&]() {
        uint64_t n8 = bytes / 8, n4 = bytes / 4;
        switch (c) {
          case ZG_TUNE_FILL_F64:
            zg_fill(ctx, buf, n8, ZG_F64, ZG_ZIGGURAT, ZG_SPLITMIX64, 1, 0, 0, s);
            break;
          case ZG_TUNE_FILL_F32:
            zg_fill(ctx, buf, n4, ZG_F32, ZG_ZIGGURAT, ZG_SPLITMIX64, 1, 0, 0, s);
            break;
          case ZG_TUNE_POLAR:
            zg_fill(ctx, buf, n8, ZG_F64, ZG_POLAR, ZG_SPLITMIX64, 1, 0, 0, s);
            break;
          default:
            zg_mutate(ctx, (double *)buf, n8 / 2, 0.0, ZG_SPLITMIX64, 1, 0, 0, s);
            break;
        }
      };
      if (c == ZG_TUNE_MUTATE) (void)hipMemsetAsync(buf, 0, bytes, s);
      float ms = time_ms(run, s, a, b, 5);
      if (ms < best_ms) {
        best_ms = ms;
        best = cand;
      }
    }
    if (st == ZG_OK) st = zg_set_tune(ctx, c, &best);
  }
  // batch: a synthetic uneven batch of fills over the scratch buffer
  if (st == ZG_OK) {
    std::vector<zg_request> reqs;
    uint64_t off = 0, n8 = bytes / 8;
    uint64_t size = 1;
    for (uint32_t i = 0; i < 4096 && off < n8; ++i) {
      zg_request r{};
      uint64_t n = std::min<uint64_t>(size, n8 - off);
      r.out = (char *)buf + off * 8;
      r.n = n;
      r.seed = i;
      r.stream = i % ZG_SM64_MAX_STREAMS;
      r.handle = ZG_NO_HANDLE;
      r.dtype = ZG_F64;
      r.method = ZG_ZIGGURAT;
      r.kind = ZG_SPLITMIX64;
      r.op = ZG_OP_FILL;
      reqs.push_back(r);
      off += (n + 31) & ~31ull;
      size = size * 3 % 1048573 + 1;
    }
    zg_tune best = ctx->tune[ZG_TUNE_BATCH];
    float best_ms = 1e30f;
    const uint32_t btiles[] = {1024, 2048, 4096};
    const uint32_t bpc[] = {1, 2, 4};
    // block-pooled (no drain waves) and wave-specialised (a quarter of the
    // waves drain) class kernels
    for (uint32_t tl : btiles)
      for (uint32_t w : {4u, 8u, 16u})
        for (uint32_t k : bpc)
          for (uint32_t dw : {0u, w / 4}) {
          if (w == 16 && dw == 0) continue;
          zg_tune cand = {tl, w, k, 0, dw, 4};
          st = zg_set_tune(ctx, ZG_TUNE_BATCH, &cand);
          if (st != ZG_OK) break;
          auto run = [&]() { zg_batch(ctx, reqs.data(), (uint32_t)reqs.size(), nullptr, s); };
          float ms = time_ms(run, s, a, b, 3);
          if (ms < best_ms) {
            best_ms = ms;
            best = cand;
          }
        }
    if (st == ZG_OK) st = zg_set_tune(ctx, ZG_TUNE_BATCH, &best);
  }
  if (s) (void)hipStreamSynchronize(s);
  if (a) (void)hipEventDestroy(a);
  if (b) (void)hipEventDestroy(b);
  if (s) (void)hipStreamDestroy(s);
  if (buf) (void)hipFree(buf);
  if (prev >= 0) (void)hipSetDevice(prev);
  if (st == ZG_OK && cache_path) write_cache(cache_path, arch, ctx->tune);
  return st;
}
