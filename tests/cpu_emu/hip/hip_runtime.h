// A host-only stand-in for the HIP runtime and device intrinsics, for running
// the library's kernels on the CPU under AddressSanitizer (test
// infrastructure; the product never includes it).
//
// Every "device" buffer is host memory.  A kernel launch runs its blocks one
// after another; the threads of a block are fibers (ucontext) that switch
// only at __syncthreads and at the wavefront collectives (__shfl*, __ballot),
// which exchange values through a per-wavefront buffer.  Atomics are plain
// read-modify-writes (one OS thread).  Streams, events and graphs are no-ops
// or refused.
#pragma once
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>
#include <functional>
#include <limits>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __noinline__ __attribute__((noinline))
#define __shared__ static
#define __align__(n) __attribute__((aligned(n)))
#define __launch_bounds__(...)

struct dim3 {
  uint32_t x, y, z;
  constexpr dim3(uint32_t a = 1, uint32_t b = 1, uint32_t c = 1) : x(a), y(b), z(c) {}
};

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorInvalidValue = 1, hipErrorOutOfMemory = 2, hipErrorNotSupported = 801 };
typedef enum { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
               hipMemcpyDeviceToDevice = 3, hipMemcpyDefault = 4 } hipMemcpyKind;
typedef struct emu_stream_t *hipStream_t;
typedef struct emu_event_t *hipEvent_t;
typedef struct emu_graph_t *hipGraph_t;
typedef struct emu_graph_exec_t *hipGraphExec_t;
typedef struct emu_graph_node_t *hipGraphNode_t;
enum { hipStreamDefault = 0, hipStreamNonBlocking = 1 };
enum { hipEventDefault = 0, hipEventDisableTiming = 2 };
typedef enum { hipStreamCaptureModeGlobal = 0, hipStreamCaptureModeThreadLocal = 1,
               hipStreamCaptureModeRelaxed = 2 } hipStreamCaptureMode;

namespace emu {

struct Fiber;
extern Fiber *cur;            // the running thread of the block
extern dim3 block_idx, grid_dim, block_dim;
const dim3 &thread_idx();
void block_barrier();
// a sleeping thread parks its block (another block runs meanwhile)
void sleep_park();
// Exchanges 8 bytes per lane within the wavefront: every live lane of the
// wavefront stores its value, waits for the others, and gets the buffer.
const uint64_t *wave_exchange(uint64_t v);
int lane_id();
void launch(dim3 grid, dim3 block, const std::function<void()> &body);

template <class T> inline uint64_t to_bits(T v) {
  static_assert(sizeof(T) <= 8, "8 bytes at most");
  uint64_t b = 0;
  memcpy(&b, &v, sizeof v);
  return b;
}
template <class T> inline T from_bits(uint64_t b) {
  T v;
  memcpy(&v, &b, sizeof v);
  return v;
}

}  // namespace emu

#define threadIdx (emu::thread_idx())
#define blockIdx (emu::block_idx)
#define gridDim (emu::grid_dim)
#define blockDim (emu::block_dim)

inline void __syncthreads() { emu::block_barrier(); }

// HIP's integer min and max
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }
inline unsigned min(unsigned a, unsigned b) { return a < b ? a : b; }
inline unsigned max(unsigned a, unsigned b) { return a > b ? a : b; }
inline long long min(long long a, long long b) { return a < b ? a : b; }
inline long long max(long long a, long long b) { return a > b ? a : b; }
inline long min(long a, long b) { return a < b ? a : b; }
inline long max(long a, long b) { return a > b ? a : b; }

template <class T> inline T __shfl(T v, int src, int width = 64) {
  const uint64_t *b = emu::wave_exchange(emu::to_bits(v));
  const int l = emu::lane_id();
  return emu::from_bits<T>(b[(l & ~(width - 1)) + (src & (width - 1))]);
}
template <class T> inline T __shfl_down(T v, unsigned d, int width = 64) {
  const uint64_t *b = emu::wave_exchange(emu::to_bits(v));
  const int l = emu::lane_id();
  const int s = (l & (width - 1)) + (int)d < width ? l + (int)d : l;
  return emu::from_bits<T>(b[s]);
}
template <class T> inline T __shfl_up(T v, unsigned d, int width = 64) {
  const uint64_t *b = emu::wave_exchange(emu::to_bits(v));
  const int l = emu::lane_id();
  const int s = (l & (width - 1)) >= (int)d ? l - (int)d : l;
  return emu::from_bits<T>(b[s]);
}
template <class T> inline T __shfl_xor(T v, int mask, int width = 64) {
  const uint64_t *b = emu::wave_exchange(emu::to_bits(v));
  const int l = emu::lane_id();
  return emu::from_bits<T>(b[(l & ~(width - 1)) + ((l ^ mask) & (width - 1))]);
}
inline unsigned long long __ballot(int pred) {
  const uint64_t *b = emu::wave_exchange(pred ? 1u : 0u);
  unsigned long long m = 0;
  for (int k = 0; k < 64; k++)
    if (b[k] == 1u) m |= 1ull << k;
  return m;
}

inline int __ffs(unsigned x) { return __builtin_ffs((int)x); }
inline int __ffsll(unsigned long long x) { return __builtin_ffsll((long long)x); }
inline int __popc(unsigned x) { return __builtin_popcount(x); }
inline int __popcll(unsigned long long x) { return __builtin_popcountll(x); }
inline int __clzll(long long x) { return x == 0 ? 64 : __builtin_clzll((unsigned long long)x); }
inline long long __double_as_longlong(double x) { return emu::from_bits<long long>(emu::to_bits(x)); }
inline double __longlong_as_double(long long x) { return emu::from_bits<double>(emu::to_bits(x)); }
inline int __float_as_int(float x) { return emu::from_bits<int>(emu::to_bits(x)); }
inline float __int_as_float(int x) { return emu::from_bits<float>(emu::to_bits(x)); }
#define __builtin_amdgcn_rcpf(x) (1.0f / (x))

template <class T, class U> inline T atomicAdd(T *p, U v) {
  T o = *p;
  *p = (T)(o + (T)v);
  return o;
}
template <class T, class U> inline T atomicOr(T *p, U v) {
  T o = *p;
  *p = (T)(o | (T)v);
  return o;
}
template <class T, class U> inline T atomicMax(T *p, U v) {
  T o = *p;
  if ((T)v > o) *p = (T)v;
  return o;
}
template <class T, class U> inline T atomicMin(T *p, U v) {
  T o = *p;
  if ((T)v < o) *p = (T)v;
  return o;
}
template <class T, class U> inline T atomicExch(T *p, U v) {
  T o = *p;
  *p = (T)v;
  return o;
}

// the wavefront-wide intrinsics of the persistent kernel (its scoped atomics
// are clang builtins on the host too).  A sleep and a fence park the block:
// the persistent kernel sleeps while it waits and fences between work items,
// so blocks take turns there, as they would run side by side on the device
// (a fence has nothing to order on one OS thread).
#ifndef __HIP_MEMORY_SCOPE_AGENT
#define __HIP_MEMORY_SCOPE_AGENT 3
#endif
#define __builtin_amdgcn_fence(order, scope) emu::sleep_park()
#define __builtin_amdgcn_s_sleep(n) emu::sleep_park()
#define __builtin_amdgcn_wave_barrier() ((void)0)
// the first lane's value in every lane (lane 0 is always live where used)
#define __builtin_amdgcn_readfirstlane(x) __shfl((x), 0)
uint64_t wall_clock64();

// ---- host API ----------------------------------------------------------------
hipError_t hipMalloc(void **p, size_t bytes);
hipError_t hipFree(void *p);
hipError_t hipMallocAsync(void **p, size_t bytes, hipStream_t);
hipError_t hipFreeAsync(void *p, hipStream_t);
template <class T> inline hipError_t hipMalloc(T **p, size_t bytes) { return hipMalloc((void **)p, bytes); }
template <class T> inline hipError_t hipMallocAsync(T **p, size_t bytes, hipStream_t s) {
  return hipMallocAsync((void **)p, bytes, s);
}
hipError_t hipMemcpy(void *d, const void *s, size_t bytes, hipMemcpyKind);
hipError_t hipMemcpyAsync(void *d, const void *s, size_t bytes, hipMemcpyKind, hipStream_t);
hipError_t hipMemsetAsync(void *d, int v, size_t bytes, hipStream_t);
hipError_t hipStreamSynchronize(hipStream_t);
hipError_t hipDeviceSynchronize();
hipError_t hipGetLastError();
hipError_t hipPeekAtLastError();
const char *hipGetErrorString(hipError_t);
hipError_t hipEventCreate(hipEvent_t *);
hipError_t hipEventCreateWithFlags(hipEvent_t *, unsigned);
hipError_t hipEventDestroy(hipEvent_t);
hipError_t hipEventRecord(hipEvent_t, hipStream_t);
hipError_t hipEventSynchronize(hipEvent_t);
hipError_t hipEventElapsedTime(float *, hipEvent_t, hipEvent_t);
hipError_t hipStreamCreateWithFlags(hipStream_t *, unsigned);
hipError_t hipStreamDestroy(hipStream_t);
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned);
hipError_t hipStreamBeginCapture(hipStream_t, hipStreamCaptureMode);
hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t *);
hipError_t hipGraphInstantiate(hipGraphExec_t *, hipGraph_t, hipGraphNode_t *, char *, size_t);
hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t);
hipError_t hipGraphExecDestroy(hipGraphExec_t);
hipError_t hipGraphDestroy(hipGraph_t);
hipError_t hipLaunchKernel(const void *f, dim3 grid, dim3 block, void **args, size_t shmem, hipStream_t);
hipError_t hipGetSymbolAddress(void **p, const void *symbol);
hipError_t hipGetDevice(int *d);
enum { hipDeviceAttributeMultiprocessorCount = 63, hipDeviceAttributeWallClockRate = 88 };
hipError_t hipDeviceGetAttribute(int *v, int attr, int dev);
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int *nb, const void *f, int block, size_t shmem);
#define HIP_SYMBOL(x) (&(x))

#define hipLaunchKernelGGL(K, G, B, SH, ST, ...) \
  emu::launch(dim3(G), dim3(B), [=]() { K(__VA_ARGS__); })
