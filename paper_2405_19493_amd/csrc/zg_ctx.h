// The context object behind the C ABI, and the batch machinery shared by
// zg_batch, zg_stream_fill and the serving loop.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "zg_internal.h"

namespace zg {

struct HandleInfo {
  uint64_t seed;
  uint32_t stream;
  uint32_t kind;
  uint32_t dtype;    // output mode the handle's counter serves
  uint32_t method;
  bool open;
};

// Whether a request in (dtype, method) may use a handle: the mode decides
// which uniform words a variate index reads, so a counter serves one mode.
inline bool handle_mode_ok(const HandleInfo &h, uint32_t dtype, uint32_t method) {
  return h.dtype == dtype && h.method == method;
}

// A validated batch ready for upload: only requests with n > 0, in order,
// and the workgroup tiles of each work class.
struct BatchPlan {
  std::vector<DevRequest> reqs;
  std::vector<uint32_t> index;   // position of each planned request in the caller's array
  std::vector<uint64_t> items;   // request << 32 | tile, grouped by class
  uint32_t cls_off[BATCH_CLASSES] = {};
  uint32_t cls_cnt[BATCH_CLASSES] = {};
  uint64_t total_elems = 0;
  zg_tune bt{};   // the batch launch shape the plan was made for
};

struct BatchSlot {
  void *h_buf = nullptr;   // pinned staging: BatchHeader, DevRequest[nreq], items[n_items]
  void *d_buf = nullptr;
  size_t cap = 0;
  size_t item_cap = 0;
  hipGraph_t g_full = nullptr, g_prep = nullptr, g_run = nullptr;
  hipGraphExec_t x_full = nullptr, x_prep = nullptr, x_run = nullptr;
  hipGraphNode_t cpy_full = nullptr, cpy_prep = nullptr;
  hipGraphNode_t cls_full[BATCH_CLASSES] = {}, cls_run[BATCH_CLASSES] = {};
  uint32_t mask_full = 0xFFu, mask_run = 0xFFu;   // class nodes currently enabled
  zg_tune graph_bt{};   // the launch shape the graphs were built for
  hipEvent_t done = nullptr;   // recorded after the last use of the staging buffer
  bool busy = false;
  bool recorded = false;

  DevRequest *d_reqs() const { return (DevRequest *)((char *)d_buf + sizeof(BatchHeader)); }
  zg_status ensure(struct ::zg_ctx *ctx, size_t nreq, size_t nitems);
  zg_status build_graphs(struct ::zg_ctx *ctx, const zg_tune &bt);
  void invalidate_graphs();
  void release();
  // Uploads the plan and launches.  full: one graph {copy, reserve, batch} on
  // `stream`.  Otherwise the graph {copy, reserve} goes on `stream`, an event
  // is recorded in *prep_done, and the batch kernel graph goes on run_stream
  // after waiting for that event.
  zg_status launch(struct ::zg_ctx *ctx, const BatchPlan &plan, hipStream_t stream, bool full,
                   hipStream_t run_stream, hipEvent_t prep_done = nullptr);
};

// Makes `dev` current for the scope and restores the previous device.
struct DeviceGuard {
  int prev = -1;
  explicit DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) (void)hipSetDevice(dev);
  }
  ~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
  }
};

zg_status hip_fail(const struct ::zg_ctx *ctx, hipError_t e, const char *what);
uint64_t window_of(uint32_t kind);
uint32_t max_streams_of(uint32_t kind);
zg_status check_gen(const void *out, uint64_t n_total, zg_dtype dtype, zg_method method,
                    zg_kind kind, uint32_t stream0, uint32_t n_streams, uint64_t first,
                    uint64_t n_per, uint32_t *op);
uint32_t head_of(const void *out, uint32_t op, uint64_t n);
zg_status launch_job(struct ::zg_ctx *ctx, const Job &J, hipStream_t stream);

// done_flags (host-visible, optional): completion word of request i is
// done_flags[i], written with done_value when its last tile finishes.
// first_host (host-visible, optional): receives request i's first index.
zg_status plan_batch(struct ::zg_ctx *ctx, const zg_request *reqs, uint32_t nreq,
                     uint32_t *const *done_flags, uint32_t done_value, BatchPlan *plan,
                     uint64_t *const *first_host = nullptr);
zg_status acquire_slot(struct ::zg_ctx *ctx, BatchSlot **out);
void release_slot(struct ::zg_ctx *ctx, BatchSlot *slot);

}  // namespace zg

struct zg_ctx {
  int device = 0;
  int num_cus = 256;
  std::string arch;
  zg_table_view table;
  zg::DevTables *d_tables = nullptr;
  uint32_t *d_flags = nullptr;
  uint64_t *d_counters = nullptr;
  void *d_seq_scratch = nullptr;      // the device's resident sequential workspace (not owned)
  uint32_t dmax = ZG_MAX_DRAWS;
  uint64_t seq_spans = 0;             // test knob: cap on the sequential scan (0 = automatic)
  zg_tune tune[ZG_TUNE_CLASSES];
  std::vector<zg::HandleInfo> handles;
  uint32_t next_handle = 0;
  std::vector<zg::BatchSlot> slots;   // reserved up front; never reallocated
  std::mutex mu;                      // handles, slots, tune
  mutable std::mutex err_mu;
  mutable std::string last_error;
};
