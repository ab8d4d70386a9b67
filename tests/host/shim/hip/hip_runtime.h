// CPU stand-in for the HIP names the kernel file uses, so that its device code
// can be built for the host and run under AddressSanitizer (tests/host/
// seq_emu.cpp): blocks run one at a time on a pool of blockDim.x threads,
// __shared__ data is block-static, and waves are groups of 64 whose ballot and
// readfirstlane are barrier-based collectives (valid where the kernel calls
// them with whole waves, as the sequential passes do).
#pragma once
#include <atomic>
#include <barrier>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <memory>
#include <thread>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __align__(n) alignas(n)
#define __restrict__

struct dim3 { uint32_t x = 1, y = 1, z = 1; dim3(uint32_t a = 1, uint32_t b = 1, uint32_t c = 1) : x(a), y(b), z(c) {} };
struct uint3_ { uint32_t x, y, z; };
extern thread_local uint3_ threadIdx;
extern uint3_ blockIdx, blockDim, gridDim;

struct double2 { double x, y; };
struct float4 { float x, y, z, w; };
inline double2 make_double2(double a, double b) { return {a, b}; }
inline float4 make_float4(float a, float b, float c, float d) { return {a, b, c, d}; }

typedef int hipError_t;
typedef void *hipStream_t;
#define hipSuccess 0
#define hipErrorInvalidValue 1
#define hipErrorInvalidDevice 101
#define HIP_SYMBOL(x) (&(x))
inline hipError_t hipGetSymbolAddress(void **p, const void *sym) { *p = const_cast<void *>(sym); return 0; }
#define hipDeviceAttributeMultiprocessorCount 1
inline hipError_t hipGetLastError() { return 0; }
inline hipError_t hipGetDevice(int *d) { *d = 0; return 0; }
// compute units: EMU_CUS from the environment (default 256), so that a test
// can make persistent grids of few, large workgroups
inline hipError_t hipDeviceGetAttribute(int *v, int, int) {
  const char *e = std::getenv("EMU_CUS");
  *v = e ? std::atoi(e) : 256;
  return 0;
}
// workgroups per compute unit that fit: EMU_OCC from the environment (default 1)
inline hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *o, const void *, int, size_t) {
  const char *e = std::getenv("EMU_OCC");
  *o = e ? std::atoi(e) : 1;
  return 0;
}

// ---- collectives
struct EmuWave {
  std::unique_ptr<std::barrier<>> bar;
  std::atomic<uint64_t> acc{0};
  uint64_t val = 0;
  uint32_t lanes[64] = {};
};
extern std::vector<std::unique_ptr<EmuWave>> emu_waves;
extern std::unique_ptr<std::barrier<>> emu_block_bar;

inline uint32_t __lane_id() { return threadIdx.x & 63u; }
inline void __syncthreads() { emu_block_bar->arrive_and_wait(); }
inline void __threadfence_block() { std::atomic_thread_fence(std::memory_order_seq_cst); }
inline void __threadfence_system() { std::atomic_thread_fence(std::memory_order_seq_cst); }
inline uint64_t emu_ballot(bool p) {
  EmuWave &w = *emu_waves[threadIdx.x >> 6];
  if (p) w.acc.fetch_or(1ull << (threadIdx.x & 63u));
  w.bar->arrive_and_wait();
  const uint64_t r = w.acc.load();
  w.bar->arrive_and_wait();
  if ((threadIdx.x & 63u) == 0) w.acc.store(0);
  w.bar->arrive_and_wait();
  return r;
}
inline uint32_t emu_rfl(uint32_t x) {
  EmuWave &w = *emu_waves[threadIdx.x >> 6];
  if ((threadIdx.x & 63u) == 0) w.val = x;
  w.bar->arrive_and_wait();
  const uint32_t r = (uint32_t)w.val;
  w.bar->arrive_and_wait();
  return r;
}
inline int emu_readlane(int x, int q) {
  EmuWave &w = *emu_waves[threadIdx.x >> 6];
  w.lanes[threadIdx.x & 63u] = (uint32_t)x;
  w.bar->arrive_and_wait();
  const int r = (int)w.lanes[q & 63];
  w.bar->arrive_and_wait();
  return r;
}
inline uint64_t __umul64hi(uint64_t a, uint64_t b) {
  return (uint64_t)(((unsigned __int128)a * b) >> 64);
}
#define __builtin_amdgcn_readlane(x, q) emu_readlane(x, q)
using std::isnan;
#define __builtin_amdgcn_ballot_w64(p) emu_ballot(p)
#define __builtin_amdgcn_readfirstlane(x) emu_rfl(x)
// a wave's lanes in step at this point: LDS writes made before it by any lane
// are seen after it by every lane, as they are in a wave on the GPU
inline void emu_wave_barrier() { emu_waves[threadIdx.x >> 6]->bar->arrive_and_wait(); }
#define __builtin_amdgcn_wave_barrier() emu_wave_barrier()
inline uint32_t emu_mbcnt_lo(uint32_t m, uint32_t a) { uint32_t l = threadIdx.x & 63u; return a + __builtin_popcount(l >= 32 ? m : (m & ((1u << l) - 1u))); }
inline uint32_t emu_mbcnt_hi(uint32_t m, uint32_t a) { uint32_t l = threadIdx.x & 63u; return a + (l < 32 ? 0 : __builtin_popcount(m & ((l == 32 ? 0u : (1u << (l - 32)) - 1u)))); }
#define __builtin_amdgcn_mbcnt_lo(m, a) emu_mbcnt_lo(m, a)
#define __builtin_amdgcn_mbcnt_hi(m, a) emu_mbcnt_hi(m, a)
#define __builtin_amdgcn_ubfe(x, o, w) ((uint32_t)(((uint32_t)(x) >> (o)) & ((1u << (w)) - 1u)))
#define __builtin_amdgcn_alignbit(h, l, s) ((uint32_t)(((((uint64_t)(uint32_t)(h)) << 32) | (uint32_t)(l)) >> (s)))

inline uint32_t atomicAdd(uint32_t *p, uint32_t v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline int32_t atomicAdd(int32_t *p, int32_t v) { return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST); }
inline uint32_t atomicOr(uint32_t *p, uint32_t v) { return __atomic_fetch_or(p, v, __ATOMIC_SEQ_CST); }
inline uint32_t atomicMax(uint32_t *p, uint32_t v) {
  uint32_t cur = __atomic_load_n(p, __ATOMIC_SEQ_CST);
  while (cur < v &&
         !__atomic_compare_exchange_n(p, &cur, v, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST)) {
  }
  return cur;
}
inline int32_t atomicSub(int32_t *p, int32_t v) { return __atomic_fetch_sub(p, v, __ATOMIC_SEQ_CST); }
inline uint32_t atomicCAS(uint32_t *p, uint32_t cmp, uint32_t val) {
  __atomic_compare_exchange_n(p, &cmp, val, false, __ATOMIC_SEQ_CST, __ATOMIC_SEQ_CST);
  return cmp;
}
#define __HIP_MEMORY_SCOPE_SYSTEM 0
#define __HIP_MEMORY_SCOPE_WORKGROUP 1
#define __hip_atomic_store(p, v, o, s) __atomic_store_n(p, v, __ATOMIC_SEQ_CST)
#define __hip_atomic_load(p, o, s) __atomic_load_n(p, __ATOMIC_SEQ_CST)
#define __builtin_amdgcn_fence(o, s) std::atomic_thread_fence(std::memory_order_seq_cst)
#define __builtin_amdgcn_s_sleep(n) std::this_thread::yield()
#define __builtin_amdgcn_s_setprio(n) ((void)0)

inline double __longlong_as_double(long long x) { double d; std::memcpy(&d, &x, 8); return d; }
inline long long __double_as_longlong(double x) { long long d; std::memcpy(&d, &x, 8); return d; }
inline float __int_as_float(int x) { float d; std::memcpy(&d, &x, 4); return d; }
inline int __float_as_int(float x) { int d; std::memcpy(&d, &x, 4); return d; }
inline int __double2hiint(double x) { return (int)(__double_as_longlong(x) >> 32); }
inline int __double2loint(double x) { return (int)(uint32_t)__double_as_longlong(x); }
using std::exp; using std::log; using std::fma; using std::sqrt; using std::frexp;

// ---- launches: every block of the grid in turn on blockDim.x threads
void emu_run_grid(dim3 grid, dim3 block, const std::function<void()> &body);
#define hipLaunchKernelGGL(k, g, b, shm, st, ...) emu_run_grid(dim3(g), dim3(b), [=]() { k(__VA_ARGS__); })
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline double __hiloint2double(int hi, int lo) { return __longlong_as_double(((long long)(uint32_t)hi << 32) | (uint32_t)lo); }
