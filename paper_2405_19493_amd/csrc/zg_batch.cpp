// Batch planning, staging slots and the hipGraphs that launch a batch:
// {descriptor upload, counter reservation, persistent batch kernel}.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <thread>
#include <unordered_map>

#include "zg_ctx.h"

namespace zg {

namespace {
constexpr uint32_t SLOT_COUNT = 8;
// batches of at most this many requests are launched directly, not as a graph
constexpr size_t DIRECT_MAX = 8;

void destroy_graph(hipGraph_t &g, hipGraphExec_t &x) {
  if (x) (void)hipGraphExecDestroy(x);
  if (g) (void)hipGraphDestroy(g);
  g = nullptr;
  x = nullptr;
}
}  // namespace

// The ziggurat classes run wave-specialised when the shape has drain waves
// and at least one streaming wave.
static bool batch_ws(const zg_tune &bt) {
  return bt.drain_waves > 0 && bt.drain_waves < bt.waves_per_block;
}

static bool same_tune(const zg_tune &a, const zg_tune &b) {
  return a.tile == b.tile && a.waves_per_block == b.waves_per_block &&
         a.batch_blocks_per_cu == b.batch_blocks_per_cu && a.queue_cap == b.queue_cap &&
         a.drain_waves == b.drain_waves && a.group_steps == b.group_steps;
}

zg_status plan_batch(zg_ctx *ctx, const zg_request *reqs, uint32_t nreq,
                     uint32_t *const *done_flags, uint32_t done_value, BatchPlan *plan,
                     uint64_t *const *first_host) {
  plan->reqs.clear();
  plan->index.clear();
  plan->items.clear();
  plan->total_elems = 0;
  std::unordered_map<int32_t, size_t> last_of;   // handle -> planned index of its last request
  std::unordered_map<int32_t, uint64_t> off_of;  // handle -> running offset
  std::lock_guard<std::mutex> lk(ctx->mu);
  // the shape is read under the lock that zg_set_tune writes it under
  const zg_tune bt = ctx->tune[ZG_TUNE_BATCH];
  plan->bt = bt;
  for (uint32_t i = 0; i < nreq; ++i) {
    const zg_request &r = reqs[i];
    if (r.op != ZG_OP_FILL && r.op != ZG_OP_MUTATE) return ZG_EINVAL;
    uint64_t seed = r.seed;
    uint32_t stream = r.stream;
    uint32_t kind = r.kind;
    zg_dtype dt = r.op == ZG_OP_MUTATE ? ZG_F64 : (zg_dtype)r.dtype;
    zg_method me = r.op == ZG_OP_MUTATE ? ZG_ZIGGURAT : (zg_method)r.method;
    if (r.op == ZG_OP_MUTATE && (r.dtype != ZG_F64 || r.method != ZG_ZIGGURAT)) return ZG_EINVAL;
    if (me == ZG_MCFARLAND) return ZG_EINVAL;   // plain fills only
    if (r.handle >= 0) {
      if ((uint32_t)r.handle >= ZG_MAX_HANDLES || !ctx->handles[r.handle].open) return ZG_ENOENT;
      const HandleInfo &h = ctx->handles[r.handle];
      // a counter serves one mode: another mode would read its words again
      if (!handle_mode_ok(h, dt, me)) return ZG_EINVAL;
      seed = h.seed;
      stream = h.stream;
      kind = h.kind;
    } else if (r.handle != ZG_NO_HANDLE) {
      return ZG_EINVAL;
    }
    uint32_t op;
    // with a handle the first index is only known on the device: check the
    // shape here and the window there
    uint64_t first_chk = r.handle >= 0 ? 0 : r.first_index;
    zg_status st = check_gen(r.out, r.n, dt, me, (zg_kind)kind, stream, 1, first_chk, r.n, &op);
    if (st != ZG_OK) return st;
    if (r.op == ZG_OP_MUTATE) op = OP_MUTATE;
    if (r.n == 0) continue;
    DevRequest d{};
    d.job.out = r.out;
    d.job.n_per = r.n;
    d.job.n_total = r.n;
    d.job.first = r.first_index;
    d.job.seed = seed;
    d.job.sigma = r.sigma;
    d.job.inv_n_per = 1.0 / (double)r.n;
    d.job.s0 = stream;
    d.job.n_streams = 1;
    d.job.kind = kind;
    d.job.op = op;
    d.handle = r.handle;
    d.limit = window_of(kind);
    if (r.handle >= 0) {
      uint64_t &off = off_of[r.handle];
      d.off = off;
      off += r.n;
      last_of[r.handle] = plan->reqs.size();
    }
    // whole 256-element steps per wave; FP32 tiles hold twice the elements
    const uint32_t wave_tile = op == OP_ZIG32 ? 2 * bt.tile : bt.tile;
    d.tile = (wave_tile + 255) / 256 * 256;
    d.head = head_of(r.out, op, r.n);
    const uint64_t body = r.n - d.head;
    const uint64_t per = (uint64_t)d.tile * bt.waves_per_block;
    uint64_t tiles = (body + per - 1) / per;
    if (tiles == 0) tiles = 1;
    if (tiles > 0xFFFFFFFFull) return ZG_EINVAL;
    d.tiles = (uint32_t)tiles;
    d.done_flag = done_flags ? done_flags[i] : nullptr;
    d.first_host = first_host ? first_host[i] : nullptr;
    d.done_value = done_value;
    plan->total_elems += r.n;
    plan->reqs.push_back(d);
    plan->index.push_back(i);
  }
  for (auto &kv : last_of) plan->reqs[kv.second].last_of_handle = 1;
  // work items, grouped by class
  uint64_t total = 0;
  for (int c = 0; c < BATCH_CLASSES; ++c) plan->cls_cnt[c] = 0;
  for (const DevRequest &d : plan->reqs) {
    plan->cls_cnt[batch_class(d.job.op, d.job.kind)] += d.tiles;
    total += d.tiles;
  }
  if (total > 0xFFFFFFFFull) return ZG_EINVAL;
  uint32_t acc = 0;
  for (int c = 0; c < BATCH_CLASSES; ++c) {
    plan->cls_off[c] = acc;
    acc += plan->cls_cnt[c];
  }
  plan->items.resize(total);
  uint32_t fill[BATCH_CLASSES];
  for (int c = 0; c < BATCH_CLASSES; ++c) fill[c] = plan->cls_off[c];
  for (size_t k = 0; k < plan->reqs.size(); ++k) {
    const DevRequest &d = plan->reqs[k];
    uint32_t &f = fill[batch_class(d.job.op, d.job.kind)];
    for (uint32_t j = 0; j < d.tiles; ++j) plan->items[f++] = ((uint64_t)k << 32) | j;
  }
  return ZG_OK;
}

zg_status acquire_slot(zg_ctx *ctx, BatchSlot **out) {
  for (;;) {
    BatchSlot *pick = nullptr;
    {
      std::lock_guard<std::mutex> lk(ctx->mu);
      if (ctx->slots.empty()) ctx->slots.resize(SLOT_COUNT);
      // prefer a free slot whose previous launch has completed
      for (auto &s : ctx->slots)
        if (!s.busy && (!s.recorded || hipEventQuery(s.done) == hipSuccess)) {
          pick = &s;
          break;
        }
      if (!pick)
        for (auto &s : ctx->slots)
          if (!s.busy) {
            pick = &s;
            break;
          }
      if (pick) pick->busy = true;
    }
    if (pick) {
      if (pick->recorded) {
        hipError_t e = hipEventSynchronize(pick->done);
        if (e != hipSuccess) {
          release_slot(ctx, pick);
          return hip_fail(ctx, e, "slot wait");
        }
      }
      *out = pick;
      return ZG_OK;
    }
    std::this_thread::yield();
  }
}

void release_slot(zg_ctx *ctx, BatchSlot *slot) {
  std::lock_guard<std::mutex> lk(ctx->mu);
  slot->busy = false;
}

void BatchSlot::invalidate_graphs() {
  destroy_graph(g_full, x_full);
  destroy_graph(g_prep, x_prep);
  destroy_graph(g_run, x_run);
  cpy_full = cpy_prep = nullptr;
  for (int c = 0; c < BATCH_CLASSES; ++c) cls_full[c] = cls_run[c] = nullptr;
  mask_full = mask_run = 0xFFu;
}

void BatchSlot::release() {
  invalidate_graphs();
  if (done) (void)hipEventDestroy(done);
  if (h_buf) (void)hipHostFree(h_buf);
  if (d_buf) (void)hipFree(d_buf);
  done = nullptr;
  h_buf = d_buf = nullptr;
  cap = 0;
  recorded = false;
}

zg_status BatchSlot::ensure(zg_ctx *ctx, size_t nreq, size_t nitems) {
  if (!done) {
    hipError_t e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(ctx, e, "slot event");
  }
  if (nreq <= cap && nitems <= item_cap) return ZG_OK;
  size_t want = std::max<size_t>(nreq, 256);
  want = std::min<size_t>(std::max(want, nreq <= cap ? cap : cap * 2), ZG_MAX_BATCH);
  if (want < nreq) return ZG_EINVAL;
  size_t want_items = std::max<size_t>(std::max<size_t>(nitems, 4096),
                                       nitems <= item_cap ? item_cap : item_cap * 2);
  invalidate_graphs();
  if (h_buf) (void)hipHostFree(h_buf);
  if (d_buf) (void)hipFree(d_buf);
  h_buf = d_buf = nullptr;
  cap = item_cap = 0;
  size_t bytes = sizeof(BatchHeader) + want * sizeof(DevRequest) + want_items * sizeof(uint64_t);
  if (bytes > 0xFFFFFFFFull) return ZG_EINVAL;
  hipError_t e = hipHostMalloc(&h_buf, bytes, hipHostMallocDefault);
  if (e != hipSuccess) return hip_fail(ctx, e, "slot staging");
  e = hipMalloc(&d_buf, bytes);
  if (e != hipSuccess) return hip_fail(ctx, e, "slot device buffer");
  cap = want;
  item_cap = want_items;
  return ZG_OK;
}

zg_status BatchSlot::build_graphs(zg_ctx *ctx, const zg_tune &bt) {
  if (x_full && same_tune(graph_bt, bt)) return ZG_OK;
  invalidate_graphs();
  graph_bt = bt;
  const bool ws = batch_ws(bt);
  BatchHeader *dH = (BatchHeader *)d_buf;
  DevRequest *dR = d_reqs();
  DevTables *T = ctx->d_tables;
  uint32_t *flags = ctx->d_flags;
  uint64_t *counters = ctx->d_counters;
  size_t bytes = sizeof(BatchHeader) + sizeof(DevRequest);   // resized per launch

  void *reserve_args[] = {&dR, &dH, &counters, &flags};
  hipKernelNodeParams kr{};
  kr.func = (void *)kernel_reserve();
  kr.gridDim = dim3(1);
  kr.blockDim = dim3(1024);
  kr.sharedMemBytes = 0;
  kr.kernelParams = reserve_args;
  kr.extra = nullptr;

  void *class_args[] = {&dR, &dH, &T, &flags};
  hipKernelNodeParams kc[BATCH_CLASSES];
  for (int c = 0; c < BATCH_CLASSES; ++c) {
    kc[c] = hipKernelNodeParams{};
    kc[c].func = (void *)kernel_batch_class(c, ws);
    kc[c].gridDim = dim3((uint32_t)(ctx->num_cus * bt.batch_blocks_per_cu));
    kc[c].blockDim = dim3(64 * bt.waves_per_block);
    kc[c].sharedMemBytes = (unsigned)batch_class_lds_bytes(c, bt.waves_per_block);
    kc[c].kernelParams = class_args;
    kc[c].extra = nullptr;
  }

  void *complete_args[] = {&dR, &dH};
  hipKernelNodeParams kd{};
  kd.func = (void *)kernel_complete();
  kd.gridDim = dim3(ZG_MAX_BATCH / 256);
  kd.blockDim = dim3(256);
  kd.sharedMemBytes = 0;
  kd.kernelParams = complete_args;
  kd.extra = nullptr;

  // full = {copy -> reserve -> class kernels -> completion words};
  // prep = {copy -> reserve}; run = {class kernels -> completion words}
  hipError_t e;
  hipGraphNode_t nr, nd;
  e = hipGraphCreate(&g_full, 0);
  if (e == hipSuccess)
    e = hipGraphAddMemcpyNode1D(&cpy_full, g_full, nullptr, 0, d_buf, h_buf, bytes,
                                hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipGraphAddKernelNode(&nr, g_full, &cpy_full, 1, &kr);
  for (int c = 0; c < BATCH_CLASSES && e == hipSuccess; ++c)
    e = hipGraphAddKernelNode(&cls_full[c], g_full, &nr, 1, &kc[c]);
  if (e == hipSuccess) e = hipGraphAddKernelNode(&nd, g_full, cls_full, BATCH_CLASSES, &kd);
  if (e == hipSuccess) e = hipGraphInstantiate(&x_full, g_full, nullptr, nullptr, 0);
  if (e == hipSuccess) e = hipGraphCreate(&g_prep, 0);
  if (e == hipSuccess)
    e = hipGraphAddMemcpyNode1D(&cpy_prep, g_prep, nullptr, 0, d_buf, h_buf, bytes,
                                hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipGraphAddKernelNode(&nr, g_prep, &cpy_prep, 1, &kr);
  if (e == hipSuccess) e = hipGraphInstantiate(&x_prep, g_prep, nullptr, nullptr, 0);
  if (e == hipSuccess) e = hipGraphCreate(&g_run, 0);
  for (int c = 0; c < BATCH_CLASSES && e == hipSuccess; ++c)
    e = hipGraphAddKernelNode(&cls_run[c], g_run, nullptr, 0, &kc[c]);
  if (e == hipSuccess) e = hipGraphAddKernelNode(&nd, g_run, cls_run, BATCH_CLASSES, &kd);
  if (e == hipSuccess) e = hipGraphInstantiate(&x_run, g_run, nullptr, nullptr, 0);
  mask_full = mask_run = 0xFFu;
  if (e != hipSuccess) {
    invalidate_graphs();
    return hip_fail(ctx, e, "batch graph build");
  }
  return ZG_OK;
}

zg_status BatchSlot::launch(zg_ctx *ctx, const BatchPlan &plan, hipStream_t stream, bool full,
                            hipStream_t run_stream, hipEvent_t prep_done) {
  zg_status st = ensure(ctx, plan.reqs.size(), plan.items.size());
  if (st != ZG_OK) return st;
  // the kernels, the header and the plan's tiles all follow the plan's shape
  const zg_tune &bt = plan.bt;
  const bool ws = batch_ws(bt);
  st = build_graphs(ctx, bt);
  if (st != ZG_OK) return st;
  BatchHeader *H = (BatchHeader *)h_buf;
  std::memset(H, 0, sizeof(*H));
  H->nreq = (uint32_t)plan.reqs.size();
  H->dmax = ctx->dmax;
  H->n_items = (uint32_t)plan.items.size();
  H->items_off = (uint32_t)(sizeof(BatchHeader) + plan.reqs.size() * sizeof(DevRequest));
  H->ws_drain = ws ? bt.drain_waves : 0;
  H->ws_gsteps = bt.group_steps;
  for (int c = 0; c < BATCH_CLASSES; ++c) {
    H->cls_off[c] = plan.cls_off[c];
    H->cls_cnt[c] = plan.cls_cnt[c];
    // a class's request tiles hold tile x waves elements (twice the tile for
    // FP32, as plan_batch cuts them), in groups of group_steps steps
    const uint32_t wave_tile = c / 2 == 1 ? 2 * bt.tile : bt.tile;
    const uint64_t per = (uint64_t)((wave_tile + 255) / 256 * 256) * bt.waves_per_block;
    const uint64_t ge = 256ull * bt.group_steps;
    H->cls_groups[c] = (uint32_t)((per + ge - 1) / ge);
  }
  std::memcpy((char *)h_buf + sizeof(BatchHeader), plan.reqs.data(),
              plan.reqs.size() * sizeof(DevRequest));
  // the items follow the descriptors
  std::memcpy((char *)h_buf + H->items_off, plan.items.data(),
              plan.items.size() * sizeof(uint64_t));
  size_t bytes = H->items_off + plan.items.size() * sizeof(uint64_t);
  hipError_t e;
  if (full && plan.reqs.size() <= DIRECT_MAX) {
    // a few requests: plain launches of the classes with work, each grid
    // sized to its tiles (cheaper than updating and launching the graph)
    const uint32_t cap_blocks = (uint32_t)(ctx->num_cus * bt.batch_blocks_per_cu);
    BatchHeader *dH = (BatchHeader *)d_buf;
    DevRequest *dR = d_reqs();
    DevTables *T = ctx->d_tables;
    uint32_t *flags = ctx->d_flags;
    uint64_t *counters = ctx->d_counters;
    void *reserve_args[] = {&dR, &dH, &counters, &flags};
    void *complete_args[] = {&dR, &dH};
    e = hipMemcpyAsync(d_buf, h_buf, bytes, hipMemcpyHostToDevice, stream);
    if (e == hipSuccess)
      e = hipLaunchKernel(kernel_reserve(), dim3(1), dim3(1024), reserve_args, 0, stream);
    for (int c = 0; c < BATCH_CLASSES && e == hipSuccess; ++c) {
      if (!plan.cls_cnt[c]) continue;
      const uint32_t grid = plan.cls_cnt[c] < cap_blocks ? plan.cls_cnt[c] : cap_blocks;
      e = launch_batch_class(c, ws, grid, bt.waves_per_block, dR, dH, T, flags, stream);
    }
    if (e == hipSuccess)
      e = hipLaunchKernel(kernel_complete(), dim3(1), dim3(256), complete_args, 0, stream);
    if (e == hipSuccess) e = hipEventRecord(done, stream);
    if (e != hipSuccess) return hip_fail(ctx, e, "batch launch");
    recorded = true;
    return ZG_OK;
  }
  // only the classes with work run
  uint32_t mask = 0;
  for (int c = 0; c < BATCH_CLASSES; ++c)
    if (plan.cls_cnt[c]) mask |= 1u << c;
  hipGraphExec_t xg = full ? x_full : x_run;
  hipGraphNode_t *nodes = full ? cls_full : cls_run;
  uint32_t &cur = full ? mask_full : mask_run;
  e = hipSuccess;
  for (int c = 0; c < BATCH_CLASSES && e == hipSuccess; ++c)
    if (((cur ^ mask) >> c) & 1u) e = hipGraphNodeSetEnabled(xg, nodes[c], (mask >> c) & 1u);
  if (e != hipSuccess) return hip_fail(ctx, e, "batch class enable");
  cur = mask;
  if (full) {
    e = hipGraphExecMemcpyNodeSetParams1D(x_full, cpy_full, d_buf, h_buf, bytes,
                                          hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipGraphLaunch(x_full, stream);
    if (e == hipSuccess) e = hipEventRecord(done, stream);
  } else {
    e = hipGraphExecMemcpyNodeSetParams1D(x_prep, cpy_prep, d_buf, h_buf, bytes,
                                          hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipGraphLaunch(x_prep, stream);
    if (e == hipSuccess && prep_done) e = hipEventRecord(prep_done, stream);
    if (e == hipSuccess && prep_done) e = hipStreamWaitEvent(run_stream, prep_done, 0);
    if (e == hipSuccess) e = hipGraphLaunch(x_run, run_stream);
    if (e == hipSuccess) e = hipEventRecord(done, run_stream);
  }
  if (e != hipSuccess) return hip_fail(ctx, e, "batch launch");
  recorded = true;
  return ZG_OK;
}

}  // namespace zg
