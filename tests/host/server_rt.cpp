// libzg's host code (context, batch planner, staging slots and graphs, the
// serving loop) built for the CPU against the runtime stand-in in
// tests/host/rt_shim, to run under ThreadSanitizer or AddressSanitizer.
//
// The kernels are host functions with the effects the serving loop relies
// on: the reservation kernel resolves first indices from the device counters
// in submission order; the class kernels write every element e of each of
// their tiles as first + e (so overlapping outputs would show); the
// completion kernel publishes the completion words with a release store.
//
//   server_rt STREAMS CLIENTS REQUESTS HANDLES MODE
// runs CLIENTS submitting threads (REQUESTS each, uneven sizes, handles of
// both dtypes), waiting and releasing from their own threads, then one
// zg_server_replay of the same size; checks every range against its handle's
// submission order and every output element; prints "server ok".
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <random>

#include "../../paper_2405_19493_amd/csrc/zg_ctx.h"

namespace zg {

// ---------------------------------------------------------- fake kernels
static void k_reserve_host(DevRequest *R, const BatchHeader *H, uint64_t *counters,
                           uint32_t *flags) {
  const uint32_t nreq = H->nreq;
  for (uint32_t i = 0; i < nreq; ++i) {
    DevRequest &r = R[i];
    if (r.handle >= 0) {
      const uint64_t first = counters[r.handle] + r.off;
      r.job.first = first;
      if (first + r.job.n_total > r.limit || first + r.job.n_total < first) {
        r.status = ZG_FLAG_RANGE;
        __atomic_fetch_or(flags, ZG_FLAG_RANGE, __ATOMIC_RELAXED);
      }
    }
  }
  for (uint32_t i = 0; i < nreq; ++i) {
    const DevRequest &r = R[i];
    if (r.handle >= 0 && r.last_of_handle) counters[r.handle] = r.job.first + r.job.n_total;
    if (r.first_host) __atomic_store_n(r.first_host, r.job.first, __ATOMIC_RELAXED);
  }
}

static void write_range(const DevRequest &rq, uint64_t b, uint64_t e) {
  const Job &J = rq.job;
  for (uint64_t k = b; k < e; ++k) {
    const double v = (double)(J.first + k);
    if (J.op == OP_ZIG32)
      ((float *)J.out)[k] = (float)v;
    else
      ((double *)J.out)[k] = v;
  }
}

static void k_class_host(int cls, const DevRequest *R, const BatchHeader *H, uint32_t waves) {
  const uint64_t *items = (const uint64_t *)((const char *)H + H->items_off);
  for (uint32_t k = 0; k < H->cls_cnt[cls]; ++k) {
    const uint64_t it = items[H->cls_off[cls] + k];
    const DevRequest &rq = R[(uint32_t)(it >> 32)];
    const uint32_t j = (uint32_t)it;
    if (rq.status) continue;
    const uint64_t bt = (uint64_t)rq.tile * waves;
    const uint64_t b0 = rq.head + j * bt;
    const uint64_t b1 = std::min<uint64_t>(b0 + bt, rq.job.n_total);
    if (b0 < b1) write_range(rq, b0, b1);
    if (j == 0 && rq.head) write_range(rq, 0, std::min<uint64_t>(rq.head, rq.job.n_total));
  }
}

static void k_complete_host(const DevRequest *R, const BatchHeader *H) {
  for (uint32_t i = 0; i < H->nreq; ++i) {
    const DevRequest &rq = R[i];
    if (!rq.done_flag) continue;
    const uint32_t val = rq.done_value | (rq.status ? 0x80000000u : 0u);
    __atomic_store_n(rq.done_flag, val, __ATOMIC_RELEASE);
  }
}

// distinct addresses standing for the kernels
static char tag_reserve, tag_complete, tag_class[BATCH_CLASSES];

const void *kernel_reserve() { return &tag_reserve; }
const void *kernel_complete() { return &tag_complete; }
const void *kernel_batch_class(int cls, bool) { return &tag_class[cls]; }
// a direct class launch: the same tagged launch on the stream, in its order
hipError_t launch_batch_class(int cls, bool, uint32_t grid, uint32_t waves, DevRequest *R,
                              const BatchHeader *H, const DevTables *T, uint32_t *flags,
                              hipStream_t stream) {
  void *args[] = {&R, &H, &T, &flags};
  return hipLaunchKernel(&tag_class[cls], dim3(grid), dim3(64 * waves), args, 0, stream);
}
size_t batch_class_lds_bytes(int, uint32_t) { return 0; }

// The plain paths are not part of this harness.
hipError_t launch_fill(const Job &, const DevTables *, uint32_t, uint32_t *, uint32_t, uint32_t,
                       uint32_t, uint32_t, uint32_t, uint32_t, uint32_t, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_ea(const EaJob &, const DevTables *, uint32_t, uint32_t *, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_words(uint64_t *, uint64_t, const DevTables *, uint32_t, uint64_t, uint32_t,
                        uint32_t, uint64_t, hipStream_t) {
  return hipErrorInvalidValue;
}
hipError_t launch_decide(const uint64_t *, uint64_t, const DevTables *, uint8_t *, double *,
                         hipStream_t) {
  return hipErrorInvalidValue;
}
SeqPlan seq_plan(uint64_t, uint64_t) { return SeqPlan{}; }
hipError_t launch_seq(const SeqJob &, const SeqPlan &, const DevTables *, void *, uint64_t,
                      uint32_t *, hipStream_t) {
  return hipErrorInvalidValue;
}
static unsigned char scratch_host[64];
hipError_t seq_scratch_ptr(int, void **out) {
  *out = scratch_host;
  return hipSuccess;
}

}  // namespace zg

using namespace zg;

std::vector<size_t> emu_kernel_arg_sizes(const void *func) {
  if (func == &tag_reserve) return {8, 8, 8, 8};
  if (func == &tag_complete) return {8, 8};
  return {8, 8, 8, 8};
}

void emu_run_kernel(const void *func, dim3, dim3 block, void **a) {
  if (func == &tag_reserve) {
    k_reserve_host(*(DevRequest **)a[0], *(const BatchHeader **)a[1], *(uint64_t **)a[2],
                   *(uint32_t **)a[3]);
  } else if (func == &tag_complete) {
    k_complete_host(*(const DevRequest **)a[0], *(const BatchHeader **)a[1]);
  } else {
    for (int c = 0; c < BATCH_CLASSES; ++c)
      if (func == &tag_class[c])
        k_class_host(c, *(const DevRequest **)a[0], *(const BatchHeader **)a[1], block.x / 64);
  }
}

// ------------------------------------------------------------- workload
namespace {

struct Rec {
  uint32_t handle;
  uint64_t n;
  uint8_t dtype;
  uint64_t first;
  bool ok;
};

int fail(const char *what) {
  std::fprintf(stderr, "FAIL: %s\n", what);
  return 1;
}

bool check_output(const void *p, uint64_t n, uint8_t dtype, uint64_t first) {
  for (uint64_t k = 0; k < n; ++k) {
    const double want = (double)(first + k);
    const double got = dtype == ZG_F32 ? (double)((const float *)p)[k] : ((const double *)p)[k];
    if (dtype == ZG_F32 ? (float)want != (float)got : want != got) return false;
  }
  return true;
}

}  // namespace

int main(int argc, char **argv) {
  if (argc < 6) return 2;
  const uint32_t n_streams = (uint32_t)atoi(argv[1]);
  const uint32_t clients = (uint32_t)atoi(argv[2]);
  const uint32_t per_client = (uint32_t)atoi(argv[3]);
  const uint32_t n_handles = (uint32_t)atoi(argv[4]);
  const uint32_t mode = (uint32_t)atoi(argv[5]);
  zg_ctx *ctx = nullptr;
  if (zg_create(0, &ctx) != ZG_OK) return fail("zg_create");
  std::vector<zg_handle> hs(n_handles);
  std::vector<uint8_t> hdt(n_handles);
  for (uint32_t h = 0; h < n_handles; ++h) {
    hdt[h] = (h % 3 == 2) ? ZG_F32 : ZG_F64;
    if (zg_stream_open(ctx, 100 + h, h, ZG_SPLITMIX64, (zg_dtype)hdt[h], ZG_ZIGGURAT, &hs[h]) !=
        ZG_OK)
      return fail("zg_stream_open");
  }
  zg_server_config cfg{};
  cfg.mem_cap_bytes = 8u << 20;   // small: admission waits for releases
  cfg.max_inflight = 64;
  cfg.max_batch = 32;
  cfg.batch_window_us = 0;
  cfg.n_streams = n_streams;
  cfg.mode = mode;
  zg_server *srv = nullptr;
  const zg_status cst = zg_server_create(ctx, &cfg, &srv);
  if (cst != ZG_OK) {
    std::printf("create status %d\n", cst);
    return 3;
  }
  // clients: submit, wait, check, release; a handle's submissions from one
  // client are in order, so each client owns a disjoint set of handles
  std::vector<std::vector<Rec>> recs(clients);
  std::vector<std::thread> th;
  std::atomic<int> bad{0};
  for (uint32_t c = 0; c < clients; ++c)
    th.emplace_back([&, c] {
      std::mt19937_64 rng(1234 + c);
      std::vector<uint64_t> tickets;
      for (uint32_t k = 0; k < per_client; ++k) {
        const uint32_t h = c + clients * (uint32_t)(rng() % (n_handles / clients));
        const uint64_t n = 1 + (uint64_t)std::exp(std::log(20000.0) * (double)(rng() % 1000) / 1000.0);
        zg_server_request r{};
        r.n = n;
        r.handle = hs[h];
        r.dtype = hdt[h];
        r.method = ZG_ZIGGURAT;
        uint64_t t = 0;
        if (zg_server_submit(srv, &r, &t) != ZG_OK) {
          ++bad;
          return;
        }
        tickets.push_back(t);
        recs[c].push_back(Rec{h, n, hdt[h], 0, false});
        // keep a few in flight, then collect the oldest
        while (tickets.size() > 4 || (k + 1 == per_client && !tickets.empty())) {
          zg_completion cpl{};
          if (zg_server_wait(srv, tickets.front(), 60.0, &cpl) != ZG_OK || cpl.status != ZG_OK) {
            ++bad;
            return;
          }
          Rec &rc = recs[c][recs[c].size() - tickets.size()];
          rc.first = cpl.first_index;
          rc.ok = check_output(cpl.d_out, rc.n, rc.dtype, rc.first);
          if (zg_server_release(srv, tickets.front()) != ZG_OK) ++bad;
          tickets.erase(tickets.begin());
        }
      }
    });
  for (auto &t : th) t.join();
  if (bad) return fail("a submission, wait or release failed");
  // every handle's ranges follow its submission order, back to back
  std::map<uint32_t, uint64_t> next;
  for (uint32_t c = 0; c < clients; ++c)
    for (const Rec &r : recs[c]) {
      if (!r.ok) return fail("output values");
      if (r.first != next[r.handle]) return fail("handle order");
      next[r.handle] += r.n;
    }
  // a replay (the C-driven open loop) of more requests, with a short deadline
  // for half of them so that late completions are released by the server
  const uint32_t m = clients * per_client;
  std::vector<zg_server_request> rr(m);
  for (uint32_t k = 0; k < m; ++k) {
    const uint32_t h = k % n_handles;
    rr[k].n = 1 + (k * 7919u) % 30000u;
    rr[k].handle = hs[h];
    rr[k].dtype = hdt[h];
    rr[k].arrival_s = 1e-6 * k;
  }
  std::vector<uint64_t> first(m);
  if (zg_server_replay(srv, rr.data(), m, first.data(), 600.0) != ZG_OK)
    return fail("replay");
  for (uint32_t k = 0; k < m; ++k) {
    const uint32_t h = k % n_handles;
    if (first[k] != next[h]) return fail("replay order");
    next[h] += rr[k].n;
  }
  (void)zg_server_replay(srv, rr.data(), m / 2, nullptr, 1e-4);   // may time out
  zg_server_drain(srv);
  zg_server_stats st{};
  zg_server_stats_get(srv, &st);
  if (st.inflight_bytes != 0) return fail("bytes left in flight after drain");
  zg_server_destroy(srv);
  for (uint32_t h = 0; h < n_handles; ++h) {
    uint64_t cnt = 0;
    if (zg_stream_get_counter(ctx, hs[h], &cnt) != ZG_OK) return fail("counter");
  }
  zg_destroy(ctx);
  std::printf("server ok streams=%u clients=%u requests=%u completed=%llu batches=%llu\n",
              n_streams, clients, m, (unsigned long long)st.completed,
              (unsigned long long)st.batches);
  return 0;
}
