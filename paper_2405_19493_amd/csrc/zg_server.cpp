// Continuous-batching serving loop over the batch path.
//
// Callers submit counter-keyed requests ("n variates from this stream
// handle").  A batcher thread admits them in arrival order while request
// slots and output memory (one device arena) are free, gathers what arrived
// within the batch window (or up to max_batch), and launches the batch as one
// graph {descriptor upload, counter reservation, persistent batch kernel} on
// one of n_streams HIP streams (the first idle one, else the next in turn),
// so several batches are in flight.
// Every request has a host-mapped completion record that the device writes
// (the resolved first index, then the completion word, with a system-scope
// release); a completion thread polls the records of the requests in flight
// and stamps their completion time.  In per-request mode every request is
// launched alone through the same path (what a caller of zg_stream_fill per
// request gets), which is the baseline the batched mode is measured against.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "zg_arena.h"
#include "zg_ctx.h"

using namespace zg;

namespace {

constexpr uint64_t ARENA_ALIGN = 256;
// Most HIP streams one server launches on (a build-time setting).
#ifndef ZG_SERVER_MAX_STREAMS
#define ZG_SERVER_MAX_STREAMS 2
#endif
// at most this many requests admitted together are launched one by one
constexpr size_t SOLO_MAX = 4;

// Completion record in host memory, written by the device.
struct HostRec {
  uint32_t done;    // 0 until complete; bit 31: the request was skipped (index window)
  uint32_t pad;
  uint64_t first;   // first index the request received
};

struct Ticket {
  zg_server_request req{};
  uint64_t bytes = 0;
  uint64_t off = 0;
  int32_t rec = -1;      // completion record while in flight
  bool has_mem = false;
  bool detached = false; // released by the library once complete (nobody waits for it)
  zg_completion c{};
};

uint64_t elem_bytes(uint8_t dtype) { return dtype == ZG_F32 ? 4 : 8; }

double percentile(std::vector<double> v, double q) {
  if (v.empty()) return 0.0;
  std::sort(v.begin(), v.end());
  const double pos = q * (double)(v.size() - 1);
  const size_t i = (size_t)pos;
  const double f = pos - (double)i;
  return i + 1 < v.size() ? v[i] * (1.0 - f) + v[i + 1] * f : v[i];
}

}  // namespace

struct zg_server {
  zg_ctx *ctx = nullptr;
  zg_server_config cfg{};
  char *arena_base = nullptr;
  Arena arena;
  HostRec *recs = nullptr;      // host pointer
  HostRec *d_recs = nullptr;    // the same records as the device sees them
  std::vector<int32_t> free_recs;
  std::vector<hipStream_t> streams;
  std::vector<hipEvent_t> stream_idle;   // recorded after each launch on the stream
  uint32_t next_stream = 0;
  // The stream for the next launch: the first idle one from the round-robin
  // position (a short request is not queued behind a long one while another
  // stream has nothing to do), else the round-robin one.
  uint32_t pick_stream() {
    const uint32_t n = (uint32_t)streams.size();
    uint32_t k = next_stream % n;
    for (uint32_t j = 0; j < n; ++j) {
      const uint32_t c = (next_stream + j) % n;
      if (hipEventQuery(stream_idle[c]) == hipSuccess) {
        k = c;
        break;
      }
    }
    next_stream = k + 1;
    return k;
  }
  // Per stream handle: the event after the last batch that reserved from it,
  // and that batch's stream.  A batch on another stream waits for it, so
  // that reservations of one handle happen in submission order.
  struct LastUse {
    hipEvent_t ev = nullptr;
    uint32_t si = 0;
  };
  std::vector<LastUse> last_use;
  std::chrono::steady_clock::time_point t0;

  std::mutex mu;
  std::condition_variable cv_work;   // batcher: new requests or freed capacity
  std::condition_variable cv_done;   // waiters: completions
  std::condition_variable cv_poll;   // completion thread: new requests in flight
  std::deque<uint64_t> pending;
  std::unordered_map<uint64_t, Ticket> tickets;
  // ticket that owns each completion record (0: free); read by the
  // completion thread without the lock
  std::unique_ptr<std::atomic<uint64_t>[]> owner;
  uint64_t n_inflight = 0;
  std::vector<uint32_t> active;       // records in use, in any order
  std::vector<uint32_t> active_pos;   // position of each record in `active`
  uint64_t next_ticket = 1;
  bool stop = false;

  uint64_t submitted = 0, completed = 0, rejected = 0, batches = 0, variates = 0;
  uint64_t inflight_bytes = 0, peak_inflight_bytes = 0;
  std::vector<double> latencies;
  double first_arrival = -1.0, last_complete = 0.0;

  std::thread batcher, completer;

  double now() const {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  }
  void batch_loop();
  void complete_loop();
  // Marks a request complete (lock held); a detached ticket is released and
  // erased, so `t` must not be used afterwards.
  void finish(uint64_t id, Ticket &t, int32_t status, uint64_t first);
  // Frees a complete ticket's output and forgets it (lock held).
  void drop(std::unordered_map<uint64_t, Ticket>::iterator it);
};

void zg_server::drop(std::unordered_map<uint64_t, Ticket>::iterator it) {
  if (it->second.has_mem) {
    arena.release(it->second.off, it->second.bytes);
    inflight_bytes -= it->second.bytes;
  }
  tickets.erase(it);
  cv_work.notify_one();
}

void zg_server::finish(uint64_t id, Ticket &t, int32_t status, uint64_t first) {
  t.c.status = status;
  t.c.first_index = first;
  t.c.complete_s = now();
  t.c.done = 1;
  if (t.rec >= 0) {
    owner[t.rec].store(0, std::memory_order_relaxed);
    const uint32_t pos = active_pos[t.rec];
    active[pos] = active.back();
    active_pos[active[pos]] = pos;
    active.pop_back();
    free_recs.push_back(t.rec);
    t.rec = -1;
    --n_inflight;
  }
  ++completed;
  if (status == ZG_OK) variates += t.req.n;
  latencies.push_back(t.c.complete_s - t.c.arrival_s);
  last_complete = std::max(last_complete, t.c.complete_s);
  cv_work.notify_one();
  cv_done.notify_all();
  if (t.detached) drop(tickets.find(id));
}

void zg_server::batch_loop() {
  DeviceGuard g(ctx->device);
  const uint32_t limit = cfg.mode == ZG_SERVE_PER_REQUEST ? 1u : cfg.max_batch;
  std::vector<uint64_t> batch;
  std::vector<zg_request> reqs;
  std::vector<uint32_t *> flags;
  std::vector<uint64_t *> firsts;
  std::unique_lock<std::mutex> lk(mu);
  for (;;) {
    cv_work.wait(lk, [&] { return stop || !pending.empty(); });
    if (pending.empty()) break;   // stopping
    if (cfg.mode == ZG_SERVE_BATCHED && cfg.batch_window_us && pending.size() < limit) {
      // gather what arrives within the window after the oldest pending request
      const double open = tickets[pending.front()].c.arrival_s;
      const double close = std::max(open, now()) + 1e-6 * cfg.batch_window_us;
      while (!stop && pending.size() < limit) {
        const double left = close - now();
        if (left <= 0) break;
        cv_work.wait_for(lk, std::chrono::duration<double>(left));
      }
    }
    // admit in arrival order while a record and arena space are free
    batch.clear();
    while (!pending.empty() && batch.size() < limit && !free_recs.empty()) {
      const uint64_t id = pending.front();
      Ticket &t = tickets[id];
      uint64_t off = 0;
      if (!arena.alloc(t.bytes, &off)) break;
      t.off = off;
      t.has_mem = true;
      t.rec = free_recs.back();
      free_recs.pop_back();
      recs[t.rec].done = 0;
      recs[t.rec].first = 0;
      owner[t.rec].store(id, std::memory_order_release);
      active_pos[t.rec] = (uint32_t)active.size();
      active.push_back((uint32_t)t.rec);
      ++n_inflight;
      t.c.d_out = arena_base + off;
      t.c.admit_s = now();
      inflight_bytes += t.bytes;
      peak_inflight_bytes = std::max(peak_inflight_bytes, inflight_bytes);
      pending.pop_front();
      batch.push_back(id);
    }
    if (batch.empty()) {
      // full: wait for a completion or a release
      cv_work.wait(lk);
      continue;
    }
    // A batch completes as a whole, so a short request batched with a long
    // one would wait for it: with no backlog (a few admitted at once) every
    // request is launched alone; batches form once requests queue up.
    const size_t groups = batch.size() <= SOLO_MAX ? batch.size() : 1;
    reqs.assign(batch.size(), zg_request{});
    flags.assign(batch.size(), nullptr);
    firsts.assign(batch.size(), nullptr);
    for (size_t k = 0; k < batch.size(); ++k) {
      const Ticket &t = tickets[batch[k]];
      zg_request &r = reqs[k];
      r.out = t.c.d_out;
      r.n = t.req.n;
      r.handle = (int32_t)t.req.handle;
      r.dtype = t.req.dtype;
      r.method = t.req.method;
      r.op = ZG_OP_FILL;
      flags[k] = &d_recs[t.rec].done;
      firsts[k] = &d_recs[t.rec].first;
    }
    const size_t per = batch.size() / groups;
    batches += groups;
    lk.unlock();
    std::vector<zg_status> sts(groups, ZG_OK);
    for (size_t g2 = 0; g2 < groups; ++g2) {
      const size_t k0 = g2 * per, k1 = g2 + 1 == groups ? batch.size() : k0 + per;
      const uint32_t si = pick_stream();
      hipStream_t stream = streams[si];
      BatchPlan plan;
      zg_status st = plan_batch(ctx, reqs.data() + k0, (uint32_t)(k1 - k0), flags.data() + k0, 1u,
                                &plan, firsts.data() + k0);
      BatchSlot *slot = nullptr;
      if (st == ZG_OK) st = acquire_slot(ctx, &slot);
      if (st == ZG_OK) {
        // earlier batches on other streams that reserve from the same handles
        for (size_t k = k0; k < k1 && st == ZG_OK; ++k) {
          const LastUse &u = last_use[reqs[k].handle];
          if (u.ev && u.si != si && hipStreamWaitEvent(stream, u.ev, 0) != hipSuccess)
            st = hip_fail(ctx, hipGetLastError(), "handle order");
        }
        if (st == ZG_OK) st = slot->launch(ctx, plan, stream, /*full=*/true, nullptr);
        if (st == ZG_OK)
          for (size_t k = k0; k < k1; ++k) last_use[reqs[k].handle] = LastUse{slot->done, si};
        release_slot(ctx, slot);
      }
      if (st == ZG_OK) (void)hipEventRecord(stream_idle[si], stream);
      sts[g2] = st;
    }
    lk.lock();
    for (size_t g2 = 0; g2 < groups; ++g2) {
      const size_t k0 = g2 * per, k1 = g2 + 1 == groups ? batch.size() : k0 + per;
      if (sts[g2] != ZG_OK)
        for (size_t k = k0; k < k1; ++k) finish(batch[k], tickets[batch[k]], sts[g2], 0);
    }
    cv_poll.notify_one();
  }
}

void zg_server::complete_loop() {
  std::vector<uint32_t> watch;
  std::vector<std::pair<uint64_t, uint32_t>> hits;   // (ticket, record)
  uint32_t idle = 0;
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(mu);
      if (n_inflight == 0) {
        if (stop && pending.empty()) break;
        cv_poll.wait_for(lk, std::chrono::microseconds(200));
        continue;
      }
      watch.assign(active.begin(), active.end());
    }
    // read the records without the lock; the device writes them
    hits.clear();
    for (uint32_t k : watch) {
      const uint64_t id = owner[k].load(std::memory_order_acquire);
      if (id && __atomic_load_n(&recs[k].done, __ATOMIC_ACQUIRE)) hits.emplace_back(id, k);
    }
    if (hits.empty()) {
      // yield for a while after the last completion, then back off to short sleeps
      if (++idle < 2000)
        std::this_thread::yield();
      else
        std::this_thread::sleep_for(std::chrono::microseconds(10));
      continue;
    }
    idle = 0;
    std::lock_guard<std::mutex> lk(mu);
    for (auto &h : hits) {
      if (owner[h.second].load(std::memory_order_relaxed) != h.first) continue;
      auto it = tickets.find(h.first);
      if (it == tickets.end() || it->second.c.done) continue;
      const uint32_t v = __atomic_load_n(&recs[h.second].done, __ATOMIC_ACQUIRE);
      const uint64_t first = __atomic_load_n(&recs[h.second].first, __ATOMIC_ACQUIRE);
      finish(h.first, it->second, (v & 0x80000000u) ? ZG_ERANGE : ZG_OK, first);
    }
  }
}

extern "C" {

zg_status zg_server_create(zg_ctx *ctx, const zg_server_config *cfg, zg_server **out) {
  if (!ctx || !cfg || !out) return ZG_EINVAL;
  if (cfg->mem_cap_bytes < ARENA_ALIGN || cfg->max_inflight == 0 || cfg->max_inflight > 1u << 20 ||
      cfg->max_batch == 0 || cfg->max_batch > ZG_MAX_BATCH || cfg->n_streams < 1 ||
      cfg->n_streams > ZG_SERVER_MAX_STREAMS || cfg->mode > ZG_SERVE_PER_REQUEST)
    return ZG_EINVAL;
  DeviceGuard g(ctx->device);
  zg_server *s = new zg_server();
  s->ctx = ctx;
  s->cfg = *cfg;
  s->cfg.mem_cap_bytes &= ~(ARENA_ALIGN - 1);
  s->t0 = std::chrono::steady_clock::now();
  hipError_t e = hipMalloc((void **)&s->arena_base, s->cfg.mem_cap_bytes);
  if (e == hipSuccess)
    e = hipHostMalloc((void **)&s->recs, sizeof(HostRec) * cfg->max_inflight,
                      hipHostMallocCoherent | hipHostMallocMapped);
  if (e == hipSuccess) e = hipHostGetDevicePointer((void **)&s->d_recs, s->recs, 0);
  for (uint32_t k = 0; k < cfg->n_streams && e == hipSuccess; ++k) {
    hipStream_t st = nullptr;
    e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) s->streams.push_back(st);
    hipEvent_t ev = nullptr;
    if (e == hipSuccess) e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
    if (e == hipSuccess) s->stream_idle.push_back(ev);
  }
  if (e != hipSuccess) {
    zg_status st = hip_fail(ctx, e, "server create");
    for (hipEvent_t ev : s->stream_idle) (void)hipEventDestroy(ev);
    for (hipStream_t st2 : s->streams) (void)hipStreamDestroy(st2);
    if (s->recs) (void)hipHostFree(s->recs);
    if (s->arena_base) (void)hipFree(s->arena_base);
    delete s;
    return st == ZG_OK ? ZG_EHIP : st;
  }
  std::memset(s->recs, 0, sizeof(HostRec) * cfg->max_inflight);
  s->owner.reset(new std::atomic<uint64_t>[cfg->max_inflight]);
  for (uint32_t k = 0; k < cfg->max_inflight; ++k) s->owner[k].store(0);
  s->active_pos.assign(cfg->max_inflight, 0);
  s->last_use.assign(ZG_MAX_HANDLES, zg_server::LastUse{});
  s->active.reserve(cfg->max_inflight);
  s->arena.init(s->cfg.mem_cap_bytes);
  for (int32_t k = (int32_t)cfg->max_inflight - 1; k >= 0; --k) s->free_recs.push_back(k);
  s->batcher = std::thread([s] { s->batch_loop(); });
  s->completer = std::thread([s] { s->complete_loop(); });
  *out = s;
  return ZG_OK;
}

zg_status zg_server_submit(zg_server *s, const zg_server_request *req, uint64_t *ticket) {
  if (!s || !req || !ticket) return ZG_EINVAL;
  if (req->dtype > ZG_F32 || req->method > ZG_POLAR) return ZG_EINVAL;
  if (req->method == ZG_POLAR && req->dtype == ZG_F32) return ZG_EINVAL;
  const uint64_t bytes =
      (req->n * elem_bytes(req->dtype) + ARENA_ALIGN - 1) & ~(ARENA_ALIGN - 1);
  if (req->n > (1ull << 40) || bytes > s->cfg.mem_cap_bytes) return ZG_EINVAL;
  {
    std::lock_guard<std::mutex> hl(s->ctx->mu);
    if (req->handle >= ZG_MAX_HANDLES || !s->ctx->handles[req->handle].open) return ZG_ENOENT;
    if (!handle_mode_ok(s->ctx->handles[req->handle], req->dtype, req->method)) return ZG_EINVAL;
  }
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) return ZG_ESTATE;
  const uint64_t id = s->next_ticket++;
  Ticket &t = s->tickets[id];
  t.req = *req;
  t.bytes = bytes;
  t.c.arrival_s = req->arrival_s > 0.0 ? req->arrival_s : s->now();
  if (s->first_arrival < 0.0 || t.c.arrival_s < s->first_arrival) s->first_arrival = t.c.arrival_s;
  ++s->submitted;
  *ticket = id;
  if (req->n == 0) {
    t.c.admit_s = s->now();
    s->finish(id, t, ZG_OK, 0);
    return ZG_OK;
  }
  s->pending.push_back(id);
  s->cv_work.notify_one();
  return ZG_OK;
}

zg_status zg_server_poll(zg_server *s, uint64_t ticket, zg_completion *out) {
  if (!s || !out) return ZG_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return ZG_ENOENT;
  *out = it->second.c;
  return ZG_OK;
}

zg_status zg_server_wait(zg_server *s, uint64_t ticket, double timeout_s, zg_completion *out) {
  if (!s) return ZG_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  auto done = [&] {
    auto it = s->tickets.find(ticket);
    return it == s->tickets.end() || it->second.c.done;
  };
  if (!s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), done)) return ZG_EBUSY;
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return ZG_ENOENT;
  if (out) *out = it->second.c;
  return ZG_OK;
}

zg_status zg_server_release(zg_server *s, uint64_t ticket) {
  if (!s) return ZG_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return ZG_ENOENT;
  if (!it->second.c.done) return ZG_EBUSY;
  s->drop(it);
  return ZG_OK;
}

namespace {
// Releases a ticket now if it is complete, else as soon as it completes.
void release_when_done(zg_server *s, uint64_t ticket) {
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->tickets.find(ticket);
  if (it == s->tickets.end()) return;
  if (it->second.c.done)
    s->drop(it);
  else
    it->second.detached = true;
}
}  // namespace

zg_status zg_server_drain(zg_server *s) {
  if (!s) return ZG_EINVAL;
  std::unique_lock<std::mutex> lk(s->mu);
  s->cv_done.wait(lk, [&] { return s->pending.empty() && s->n_inflight == 0; });
  return ZG_OK;
}

zg_status zg_server_stats_get(zg_server *s, zg_server_stats *out) {
  if (!s || !out) return ZG_EINVAL;
  std::lock_guard<std::mutex> lk(s->mu);
  std::memset(out, 0, sizeof(*out));
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->rejected = s->rejected;
  out->batches = s->batches;
  out->variates = s->variates;
  out->inflight_bytes = s->inflight_bytes;
  out->peak_inflight_bytes = s->peak_inflight_bytes;
  out->p50_latency_s = percentile(s->latencies, 0.50);
  out->p99_latency_s = percentile(s->latencies, 0.99);
  out->max_latency_s =
      s->latencies.empty() ? 0.0 : *std::max_element(s->latencies.begin(), s->latencies.end());
  out->first_arrival_s = s->first_arrival < 0.0 ? 0.0 : s->first_arrival;
  out->last_complete_s = s->last_complete;
  return ZG_OK;
}

double zg_server_now(const zg_server *s) { return s ? s->now() : 0.0; }

zg_status zg_server_replay(zg_server *s, const zg_server_request *reqs, uint32_t n,
                           uint64_t *first_out, double timeout_s) {
  if (!s || (n && !reqs)) return ZG_EINVAL;
  std::vector<uint64_t> tickets(n, 0);
  std::vector<char> ready(n, 0);
  std::mutex rmu;   // ready[], result
  std::condition_variable rcv;
  zg_status result = ZG_OK;
  auto note = [&](zg_status st) {   // keeps the first error
    std::lock_guard<std::mutex> lk(rmu);
    if (st != ZG_OK && result == ZG_OK) result = st;
  };
  const double base = s->now();
  const double deadline = base + timeout_s;
  // releases completed requests in submission order; a request still running
  // at the deadline is released by the server when it completes
  std::thread releaser([&] {
    for (uint32_t k = 0; k < n; ++k) {
      {
        std::unique_lock<std::mutex> lk(rmu);
        rcv.wait(lk, [&] { return ready[k] != 0; });
        if (ready[k] < 0) continue;
      }
      zg_completion c{};
      const double left = deadline - s->now();
      zg_status st = left > 0 ? zg_server_wait(s, tickets[k], left, &c) : ZG_EBUSY;
      if (st != ZG_OK) {
        note(st);
        release_when_done(s, tickets[k]);
        continue;
      }
      if (first_out) first_out[k] = c.first_index;
      note(c.status);
      zg_server_release(s, tickets[k]);
    }
  });
  for (uint32_t k = 0; k < n; ++k) {
    zg_server_request r = reqs[k];
    r.arrival_s = base + reqs[k].arrival_s;
    while (s->now() < r.arrival_s) {
    }
    zg_status st = zg_server_submit(s, &r, &tickets[k]);
    note(st);
    {
      std::lock_guard<std::mutex> lk(rmu);
      ready[k] = st == ZG_OK ? 1 : -1;
    }
    rcv.notify_one();
  }
  releaser.join();
  std::lock_guard<std::mutex> lk(rmu);
  return result;
}

zg_status zg_server_destroy(zg_server *s) {
  if (!s) return ZG_OK;
  zg_server_drain(s);
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  s->cv_poll.notify_all();
  if (s->batcher.joinable()) s->batcher.join();
  if (s->completer.joinable()) s->completer.join();
  DeviceGuard g(s->ctx->device);
  for (hipStream_t st : s->streams) {
    (void)hipStreamSynchronize(st);
    (void)hipStreamDestroy(st);
  }
  for (hipEvent_t ev : s->stream_idle) (void)hipEventDestroy(ev);
  if (s->recs) (void)hipHostFree(s->recs);
  if (s->arena_base) (void)hipFree(s->arena_base);
  delete s;
  return ZG_OK;
}

}  // extern "C"
