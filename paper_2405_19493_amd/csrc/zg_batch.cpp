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

void destroy_graph(hipGraph_t &g, hipGraphExec_t &x) {
  if (x) (void)hipGraphExecDestroy(x);
  if (g) (void)hipGraphDestroy(g);
  g = nullptr;
  x = nullptr;
}
}  // namespace

zg_status plan_batch(zg_ctx *ctx, const zg_request *reqs, uint32_t nreq,
                     uint32_t *const *done_flags, uint32_t done_value, BatchPlan *plan,
                     uint64_t *const *first_host) {
  plan->reqs.clear();
  plan->index.clear();
  plan->total_tiles = 0;
  plan->total_elems = 0;
  const zg_tune bt = ctx->tune[ZG_TUNE_BATCH];
  std::unordered_map<int32_t, size_t> last_of;   // handle -> planned index of its last request
  std::unordered_map<int32_t, uint64_t> off_of;  // handle -> running offset
  std::lock_guard<std::mutex> lk(ctx->mu);
  for (uint32_t i = 0; i < nreq; ++i) {
    const zg_request &r = reqs[i];
    if (r.op != ZG_OP_FILL && r.op != ZG_OP_MUTATE) return ZG_EINVAL;
    uint64_t seed = r.seed;
    uint32_t stream = r.stream;
    uint32_t kind = r.kind;
    if (r.handle >= 0) {
      if ((uint32_t)r.handle >= ZG_MAX_HANDLES || !ctx->handles[r.handle].open) return ZG_ENOENT;
      const HandleInfo &h = ctx->handles[r.handle];
      seed = h.seed;
      stream = h.stream;
      kind = h.kind;
    } else if (r.handle != ZG_NO_HANDLE) {
      return ZG_EINVAL;
    }
    zg_dtype dt = r.op == ZG_OP_MUTATE ? ZG_F64 : (zg_dtype)r.dtype;
    zg_method me = r.op == ZG_OP_MUTATE ? ZG_ZIGGURAT : (zg_method)r.method;
    if (r.op == ZG_OP_MUTATE && (r.dtype != ZG_F64 || r.method != ZG_ZIGGURAT)) return ZG_EINVAL;
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
    d.tile = op == OP_ZIG32 ? 2 * bt.tile : bt.tile;
    d.head = head_of(r.out, op, r.n);
    uint64_t body = r.n - d.head;
    uint64_t tiles = (body + d.tile - 1) / d.tile;
    if (tiles == 0) tiles = 1;
    if (tiles > 0xFFFFFFFFull) return ZG_EINVAL;
    d.tiles = (uint32_t)tiles;
    d.remaining = (uint32_t)tiles;
    d.tile0 = plan->total_tiles;
    d.done_flag = done_flags ? done_flags[i] : nullptr;
    d.first_host = first_host ? first_host[i] : nullptr;
    d.done_value = done_value;
    plan->total_tiles += tiles;
    plan->total_elems += r.n;
    plan->reqs.push_back(d);
    plan->index.push_back(i);
  }
  for (auto &kv : last_of) plan->reqs[kv.second].last_of_handle = 1;
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

zg_status BatchSlot::ensure(zg_ctx *ctx, size_t nreq) {
  if (!done) {
    hipError_t e = hipEventCreateWithFlags(&done, hipEventDisableTiming);
    if (e != hipSuccess) return hip_fail(ctx, e, "slot event");
  }
  if (nreq <= cap) return ZG_OK;
  size_t want = std::max<size_t>(nreq, 256);
  want = std::min<size_t>(std::max(want, cap * 2), ZG_MAX_BATCH);
  if (want < nreq) return ZG_EINVAL;
  invalidate_graphs();
  if (h_buf) (void)hipHostFree(h_buf);
  if (d_buf) (void)hipFree(d_buf);
  h_buf = d_buf = nullptr;
  cap = 0;
  size_t bytes = sizeof(BatchHeader) + want * sizeof(DevRequest);
  hipError_t e = hipHostMalloc(&h_buf, bytes, hipHostMallocDefault);
  if (e != hipSuccess) return hip_fail(ctx, e, "slot staging");
  e = hipMalloc(&d_buf, bytes);
  if (e != hipSuccess) return hip_fail(ctx, e, "slot device buffer");
  cap = want;
  return ZG_OK;
}

zg_status BatchSlot::build_graphs(zg_ctx *ctx) {
  if (x_full) return ZG_OK;
  const zg_tune bt = ctx->tune[ZG_TUNE_BATCH];
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

  void *batch_args[] = {&dR, &dH, &T, &flags};
  hipKernelNodeParams kb{};
  kb.func = (void *)kernel_batch();
  kb.gridDim = dim3((uint32_t)(ctx->num_cus * bt.batch_blocks_per_cu));
  kb.blockDim = dim3(64 * bt.waves_per_block);
  kb.sharedMemBytes = (unsigned)batch_lds_bytes(bt.waves_per_block);
  kb.kernelParams = batch_args;
  kb.extra = nullptr;

  hipError_t e;
  hipGraphNode_t nr, nb;
  // full graph: copy -> reserve -> batch
  e = hipGraphCreate(&g_full, 0);
  if (e == hipSuccess)
    e = hipGraphAddMemcpyNode1D(&cpy_full, g_full, nullptr, 0, d_buf, h_buf, bytes,
                                hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipGraphAddKernelNode(&nr, g_full, &cpy_full, 1, &kr);
  if (e == hipSuccess) e = hipGraphAddKernelNode(&nb, g_full, &nr, 1, &kb);
  if (e == hipSuccess) e = hipGraphInstantiate(&x_full, g_full, nullptr, nullptr, 0);
  // split graphs for the serving loop: copy -> reserve, then batch
  if (e == hipSuccess) e = hipGraphCreate(&g_prep, 0);
  if (e == hipSuccess)
    e = hipGraphAddMemcpyNode1D(&cpy_prep, g_prep, nullptr, 0, d_buf, h_buf, bytes,
                                hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipGraphAddKernelNode(&nr, g_prep, &cpy_prep, 1, &kr);
  if (e == hipSuccess) e = hipGraphInstantiate(&x_prep, g_prep, nullptr, nullptr, 0);
  if (e == hipSuccess) e = hipGraphCreate(&g_run, 0);
  if (e == hipSuccess) e = hipGraphAddKernelNode(&nb, g_run, nullptr, 0, &kb);
  if (e == hipSuccess) e = hipGraphInstantiate(&x_run, g_run, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    invalidate_graphs();
    return hip_fail(ctx, e, "batch graph build");
  }
  return ZG_OK;
}

zg_status BatchSlot::launch(zg_ctx *ctx, const BatchPlan &plan, hipStream_t stream, bool full,
                            hipStream_t run_stream, hipEvent_t prep_done) {
  zg_status st = ensure(ctx, plan.reqs.size());
  if (st != ZG_OK) return st;
  st = build_graphs(ctx);
  if (st != ZG_OK) return st;
  BatchHeader *H = (BatchHeader *)h_buf;
  std::memset(H, 0, sizeof(*H));
  H->nreq = (uint32_t)plan.reqs.size();
  H->dmax = ctx->dmax;
  H->total_tiles = plan.total_tiles;
  std::memcpy((char *)h_buf + sizeof(BatchHeader), plan.reqs.data(),
              plan.reqs.size() * sizeof(DevRequest));
  size_t bytes = sizeof(BatchHeader) + plan.reqs.size() * sizeof(DevRequest);
  hipError_t e;
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
