// CPU stand-in for the HIP runtime calls of libzg's host code (the batch
// planner, the staging slots and their graphs, the serving loop), so that
// this code can run under ThreadSanitizer and AddressSanitizer with no GPU.
//
// Device memory is host memory.  Each stream is a worker thread running its
// operations in order; an event records the position of its last record in
// its stream; a stream that waits on an event runs nothing until that
// position has run.  Graphs keep copies of their nodes and run them in order
// on the launching stream.  Kernels are host functions: tests/host/
// server_rt.cpp defines what each libzg kernel does here (emu_run_kernel).
#pragma once
#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <deque>
#include <functional>
#include <memory>
#include <mutex>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __align__(n) alignas(n)

struct dim3 {
  uint32_t x = 1, y = 1, z = 1;
  dim3(uint32_t a = 1, uint32_t b = 1, uint32_t c = 1) : x(a), y(b), z(c) {}
};

typedef int hipError_t;
enum : int {
  hipSuccess = 0,
  hipErrorInvalidValue = 1,
  hipErrorOutOfMemory = 2,
  hipErrorNotReady = 600,
  hipErrorInvalidDevice = 101,
};
enum hipMemcpyKind { hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2, hipMemcpyDeviceToDevice = 3 };
#define hipStreamNonBlocking 1
#define hipEventDisableTiming 2
#define hipHostMallocDefault 0
#define hipHostMallocMapped 2
#define hipHostMallocCoherent 0x40000000
#define hipDeviceAttributeMultiprocessorCount 1

struct hipDeviceProp_t {
  int multiProcessorCount = 256;
  char gcnArchName[256] = "gfx950-host-emulation";
};

// ------------------------------------------------------------ streams
struct EmuStream {
  std::mutex mu;
  std::condition_variable cv;
  std::deque<std::function<void()>> q;
  uint64_t pushed = 0, ran = 0;
  bool quit = false;
  std::thread th;
  EmuStream() {
    th = std::thread([this] {
      for (;;) {
        std::function<void()> f;
        {
          std::unique_lock<std::mutex> lk(mu);
          cv.wait(lk, [&] { return quit || !q.empty(); });
          if (q.empty()) return;
          f = std::move(q.front());
          q.pop_front();
        }
        f();
        {
          std::lock_guard<std::mutex> lk(mu);
          ++ran;
        }
        cv.notify_all();
      }
    });
  }
  ~EmuStream() {
    {
      std::lock_guard<std::mutex> lk(mu);
      quit = true;
    }
    cv.notify_all();
    th.join();
  }
  void push(std::function<void()> f) {
    {
      std::lock_guard<std::mutex> lk(mu);
      q.push_back(std::move(f));
      ++pushed;
    }
    cv.notify_all();
  }
  void sync() {
    std::unique_lock<std::mutex> lk(mu);
    const uint64_t want = pushed;
    cv.wait(lk, [&] { return ran >= want; });
  }
};
typedef EmuStream *hipStream_t;

// All streams (the null stream first); kept until the process ends.
inline std::mutex &emu_streams_mu() {
  static std::mutex m;
  return m;
}
inline std::vector<EmuStream *> &emu_streams() {
  static std::vector<EmuStream *> v;
  return v;
}
inline EmuStream *emu_null_stream() {
  static EmuStream *s = [] {
    EmuStream *x = new EmuStream();
    std::lock_guard<std::mutex> lk(emu_streams_mu());
    emu_streams().push_back(x);
    return x;
  }();
  return s;
}
inline EmuStream *emu_stream(hipStream_t s) { return s ? s : emu_null_stream(); }

inline hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
  emu_null_stream();
  *s = new EmuStream();
  std::lock_guard<std::mutex> lk(emu_streams_mu());
  emu_streams().push_back(*s);
  return hipSuccess;
}
inline hipError_t hipStreamSynchronize(hipStream_t s) {
  emu_stream(s)->sync();
  return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t s) {
  if (!s) return hipErrorInvalidValue;
  s->sync();
  std::lock_guard<std::mutex> lk(emu_streams_mu());
  auto &v = emu_streams();
  for (size_t i = 0; i < v.size(); ++i)
    if (v[i] == s) {
      v.erase(v.begin() + (long)i);
      break;
    }
  delete s;
  return hipSuccess;
}
inline hipError_t hipDeviceSynchronize() {
  std::vector<EmuStream *> all;
  {
    std::lock_guard<std::mutex> lk(emu_streams_mu());
    all = emu_streams();
  }
  for (EmuStream *s : all) s->sync();
  return hipSuccess;
}

// ------------------------------------------------------------- events
struct EmuEvent {
  std::mutex mu;
  std::condition_variable cv;
  uint64_t recorded = 0, reached = 0;
};
typedef EmuEvent *hipEvent_t;
inline hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) {
  *e = new EmuEvent();
  return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t e) {
  delete e;
  return hipSuccess;
}
inline hipError_t hipEventRecord(hipEvent_t e, hipStream_t s) {
  if (!e) return hipErrorInvalidValue;
  uint64_t gen;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    gen = ++e->recorded;
  }
  emu_stream(s)->push([e, gen] {
    {
      std::lock_guard<std::mutex> lk(e->mu);
      if (gen > e->reached) e->reached = gen;
    }
    e->cv.notify_all();
  });
  return hipSuccess;
}
inline hipError_t hipEventQuery(hipEvent_t e) {
  std::lock_guard<std::mutex> lk(e->mu);
  return e->reached >= e->recorded ? hipSuccess : hipErrorNotReady;
}
inline hipError_t hipEventSynchronize(hipEvent_t e) {
  std::unique_lock<std::mutex> lk(e->mu);
  const uint64_t want = e->recorded;
  e->cv.wait(lk, [&] { return e->reached >= want; });
  return hipSuccess;
}
inline hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned) {
  uint64_t want;
  {
    std::lock_guard<std::mutex> lk(e->mu);
    want = e->recorded;
  }
  emu_stream(s)->push([e, want] {
    std::unique_lock<std::mutex> lk(e->mu);
    e->cv.wait(lk, [&] { return e->reached >= want; });
  });
  return hipSuccess;
}

// ------------------------------------------------------------- memory
inline hipError_t hipMalloc(void **p, size_t n) {
  *p = std::aligned_alloc(256, (n + 255) / 256 * 256);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
template <typename T>
inline hipError_t hipMalloc(T **p, size_t n) {
  return hipMalloc((void **)p, n);
}
inline hipError_t hipFree(void *p) {
  hipDeviceSynchronize();
  std::free(p);
  return hipSuccess;
}
inline hipError_t hipHostMalloc(void **p, size_t n, unsigned) { return hipMalloc(p, n); }
template <typename T>
inline hipError_t hipHostMalloc(T **p, size_t n, unsigned f) {
  return hipHostMalloc((void **)p, n, f);
}
inline hipError_t hipHostFree(void *p) { return hipFree(p); }
inline hipError_t hipHostGetDevicePointer(void **d, void *h, unsigned) {
  *d = h;
  return hipSuccess;
}
inline hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind) {
  emu_null_stream()->sync();
  std::memcpy(d, s, n);
  return hipSuccess;
}
inline hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind,
                                 hipStream_t st) {
  emu_stream(st)->push([d, s, n] { std::memcpy(d, s, n); });
  return hipSuccess;
}
inline hipError_t hipMemset(void *p, int v, size_t n) {
  emu_null_stream()->sync();
  std::memset(p, v, n);
  return hipSuccess;
}

// ------------------------------------------------------------- device
inline hipError_t hipGetDeviceCount(int *n) {
  *n = 1;
  return hipSuccess;
}
inline hipError_t hipGetDevice(int *d) {
  *d = 0;
  return hipSuccess;
}
inline hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
inline hipError_t hipGetDeviceProperties(hipDeviceProp_t *p, int) {
  *p = hipDeviceProp_t{};
  return hipSuccess;
}
inline hipError_t hipDeviceGetAttribute(int *v, int, int) {
  *v = 256;
  return hipSuccess;
}
inline hipError_t hipGetLastError() { return hipSuccess; }
inline const char *hipGetErrorString(hipError_t) { return "host emulation error"; }

// ------------------------------------------------------------ kernels
// What a kernel does here: defined by the test program for every kernel
// function libzg launches (args as HIP passes them: pointers to each value).
void emu_run_kernel(const void *func, dim3 grid, dim3 block, void **args);
// Bytes of each argument of a kernel (so that launches copy them at once).
std::vector<size_t> emu_kernel_arg_sizes(const void *func);

struct EmuArgs {
  std::vector<std::vector<char>> vals;
  std::vector<void *> ptrs;
  EmuArgs() = default;
  EmuArgs(const void *func, void **args) {
    const std::vector<size_t> sz = emu_kernel_arg_sizes(func);
    vals.resize(sz.size());
    for (size_t i = 0; i < sz.size(); ++i) {
      vals[i].resize(sz[i]);
      std::memcpy(vals[i].data(), args[i], sz[i]);
    }
    relink();
  }
  EmuArgs(const EmuArgs &o) : vals(o.vals) { relink(); }
  EmuArgs &operator=(const EmuArgs &o) {
    vals = o.vals;
    relink();
    return *this;
  }
  void relink() {
    ptrs.resize(vals.size());
    for (size_t i = 0; i < vals.size(); ++i) ptrs[i] = vals[i].data();
  }
};

inline hipError_t hipLaunchKernel(const void *func, dim3 grid, dim3 block, void **args, size_t,
                                  hipStream_t st) {
  EmuArgs a(func, args);
  emu_stream(st)->push([func, grid, block, a]() mutable {
    emu_run_kernel(func, grid, block, a.ptrs.data());
  });
  return hipSuccess;
}

// ------------------------------------------------------------- graphs
struct hipKernelNodeParams {
  void *func = nullptr;
  dim3 gridDim, blockDim;
  unsigned sharedMemBytes = 0;
  void **kernelParams = nullptr;
  void **extra = nullptr;
};
struct EmuNode {
  bool is_copy = false;
  bool enabled = true;
  void *dst = nullptr;
  const void *src = nullptr;
  size_t bytes = 0;
  const void *func = nullptr;
  dim3 grid, block;
  EmuArgs args;
};
typedef EmuNode *hipGraphNode_t;
struct EmuGraph {
  std::vector<std::unique_ptr<EmuNode>> nodes;
};
typedef EmuGraph *hipGraph_t;
struct EmuGraphExec {
  std::vector<EmuNode> nodes;            // copies, in insertion (dependency) order
  std::vector<const EmuNode *> origin;   // the graph node each copy came from
  EmuNode *find(hipGraphNode_t n) {
    for (size_t i = 0; i < origin.size(); ++i)
      if (origin[i] == n) return &nodes[i];
    return nullptr;
  }
};
typedef EmuGraphExec *hipGraphExec_t;

inline hipError_t hipGraphCreate(hipGraph_t *g, unsigned) {
  *g = new EmuGraph();
  return hipSuccess;
}
inline hipError_t hipGraphDestroy(hipGraph_t g) {
  delete g;
  return hipSuccess;
}
inline hipError_t hipGraphAddMemcpyNode1D(hipGraphNode_t *n, hipGraph_t g, const hipGraphNode_t *,
                                          size_t, void *dst, const void *src, size_t bytes,
                                          hipMemcpyKind) {
  auto x = std::make_unique<EmuNode>();
  x->is_copy = true;
  x->dst = dst;
  x->src = src;
  x->bytes = bytes;
  *n = x.get();
  g->nodes.push_back(std::move(x));
  return hipSuccess;
}
inline hipError_t hipGraphAddKernelNode(hipGraphNode_t *n, hipGraph_t g, const hipGraphNode_t *,
                                        size_t, const hipKernelNodeParams *p) {
  auto x = std::make_unique<EmuNode>();
  x->func = p->func;
  x->grid = p->gridDim;
  x->block = p->blockDim;
  x->args = EmuArgs(p->func, p->kernelParams);
  *n = x.get();
  g->nodes.push_back(std::move(x));
  return hipSuccess;
}
inline hipError_t hipGraphInstantiate(hipGraphExec_t *x, hipGraph_t g, void *, void *, size_t) {
  auto *e = new EmuGraphExec();
  for (auto &n : g->nodes) {
    e->nodes.push_back(*n);
    e->origin.push_back(n.get());
  }
  *x = e;
  return hipSuccess;
}
inline hipError_t hipGraphExecDestroy(hipGraphExec_t x) {
  delete x;
  return hipSuccess;
}
inline hipError_t hipGraphExecMemcpyNodeSetParams1D(hipGraphExec_t x, hipGraphNode_t n, void *dst,
                                                    const void *src, size_t bytes,
                                                    hipMemcpyKind) {
  EmuNode *e = x->find(n);
  if (!e || !e->is_copy) return hipErrorInvalidValue;
  e->dst = dst;
  e->src = src;
  e->bytes = bytes;
  return hipSuccess;
}
inline hipError_t hipGraphNodeSetEnabled(hipGraphExec_t x, hipGraphNode_t n, unsigned on) {
  EmuNode *e = x->find(n);
  if (!e) return hipErrorInvalidValue;
  e->enabled = on != 0;
  return hipSuccess;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t x, hipStream_t st) {
  std::vector<EmuNode> nodes = x->nodes;   // the parameters as of this launch
  emu_stream(st)->push([nodes]() mutable {
    for (EmuNode &n : nodes) {
      if (!n.enabled) continue;
      if (n.is_copy)
        std::memcpy(n.dst, n.src, n.bytes);
      else
        emu_run_kernel(n.func, n.grid, n.block, n.args.ptrs.data());
    }
  });
  return hipSuccess;
}

// device-side atomics used by host code paths (none launch-side here)
#define __HIP_MEMORY_SCOPE_SYSTEM 0
