// The persistent batch kernel: one launch runs every iteration of every
// shape of a batch, with a work queue in place of the launches of the
// one-launch-per-kernel batch (the paper balances its points over CPU
// threads with a dynamic schedule, Sec. 5; here the items of many shapes of
// uneven size share the GPU the same way).
//
// Work items and their order are described with PersistArgs (launch.hpp).
// Each block is one wavefront and takes items until the queue is empty.  An
// item runs its kernel's block for each tile of its chunk through the
// kernel's one-wavefront form, whose results are those of the block (the
// same sums in the same order), so a persistent batch computes what the
// one-launch-per-kernel batch and the shapes run alone compute.
//
// Ordering: an item waits until its shape's count of finished items reaches
// the number of that shape's items before it in the queue; the items it
// waits for were handed out earlier, to blocks that are running, so every
// wait ends.  Finished work is published with an agent-scope release before
// the count is raised and read after an agent-scope acquire (the L2 caches
// of the XCDs are not coherent with each other).  The counts and the abort
// flag are read with atomic read-modify-writes (adding 0), which meet the
// increments at the one place where each counter's atomics are ordered,
// so an increment is seen as soon as it is made, whichever XCD made it;
// each counter has a 128-byte line of its own, and a waiting wavefront
// backs off between reads.  A wavefront still waiting past the launch's
// deadline (a fault of the schedule, never expected) raises the abort flag
// and ERR_SCHED in the shape's stats; from then on items are counted but not
// run and nothing waits, so the kernel ends soon after the deadline.
#include "bin_k.hpp"
#include "cells_k.hpp"
#include "dm_k.hpp"

namespace trime {

template <class T, class G, int MODE> struct PersistSet {
  using C = Cells<T, G, MODE, FAST_VMAX, fast_block<T, MODE>()>;
  using Post = CellsPost<G, MODE, WAVE_VMAX>;
  using X = CellsExact<G, MODE, REPLAY_VMAX, REPLAY_BLOCK>;
  // the LDS of the cell kernels' wavefront forms, one at a time
  union Shm {
    typename C::WaveShm c;
    typename Post::Shm p;
  };
  using XPoly = VRec<double>[REPLAY_VMAX][REPLAY_BLOCK];
};

template <class F> TRIME_D const typename F::Args &arg_of(const unsigned char *p) {
  return *(const typename F::Args *)p;
}

// One tile of each kernel kind, each a function of its own so that every
// kernel body gets its own register allocation (inlined into one function
// they would share the largest one's and spill).
template <class F> __device__ __noinline__ void tile_virt(const unsigned char *args, Blk blk) {
  wave_virt<F>(arg_of<F>(args), blk);
}
template <class F> __device__ __noinline__ void tile_wave(const unsigned char *args, Blk blk) {
  F::run_wave(arg_of<F>(args), blk);
}
template <class F> __device__ __noinline__ void tile_run(const unsigned char *args, Blk blk) {
  F::run(arg_of<F>(args), blk);
}
template <class C>
__device__ __noinline__ void tile_cells(const unsigned char *args, Blk blk, TRIME_LDS typename C::WaveShm *sh) {
  C::run_wave(arg_of<C>(args), blk, *(typename C::WaveShm *)sh);
}
template <class Post>
__device__ __noinline__ void tile_post(const unsigned char *args, Blk blk, TRIME_LDS typename Post::Shm *sh) {
  Post::body(arg_of<Post>(args), blk, *(typename Post::Shm *)sh);
}
template <class X, class XPoly>
__device__ __noinline__ void tile_exact(const unsigned char *args, Blk blk, XPoly *P, TRIME_LDS int *hist) {
  X::body(arg_of<X>(args), blk, *P, (int *)hist);
}

// Runs tile blk of kernel `code` on the arguments at `args`.  Returns false
// for a code this kernel does not run (refused on the host beforehand).
template <class T, class G, int MODE>
TRIME_D bool run_tile(uint32_t code, const unsigned char *args, Blk blk, typename PersistSet<T, G, MODE>::Shm &sh,
                      int *xhist, unsigned char *xws) {
  using S = PersistSet<T, G, MODE>;
  switch (code) {
    case KindOf<FillCond>::code: tile_virt<FillCond>(args, blk); return true;
    case KindOf<BinKeys>::code: tile_virt<BinKeys>(args, blk); return true;
    case KindOf<ScanTiles>::code: tile_wave<ScanTiles>(args, blk); return true;
    case KindOf<ScanSums>::code: tile_wave<ScanSums>(args, blk); return true;
    case KindOf<ScanAdd>::code: tile_virt<ScanAdd>(args, blk); return true;
    case KindOf<ScanAddFew>::code: tile_wave<ScanAddFew>(args, blk); return true;
    case KindOf<BinScatter>::code: tile_virt<BinScatter>(args, blk); return true;
    case KindOf<BinPlace>::code: tile_virt<BinPlace>(args, blk); return true;
    case KindOf<OrderScatter>::code: tile_virt<OrderScatter>(args, blk); return true;
    case KindOf<OrderAdd>::code: tile_wave<OrderAdd>(args, blk); return true;
    // kernels of one wavefront run as they are
    case KindOf<StatsReset>::code: tile_run<StatsReset>(args, blk); return true;
    case KindOf<FinishExtract>::code: tile_run<FinishExtract>(args, blk); return true;
    case KindOf<SetFlag>::code: tile_run<SetFlag>(args, blk); return true;
    case KindOf<typename S::C>::code:
      tile_cells<typename S::C>(args, blk, (TRIME_LDS typename S::C::WaveShm *)&sh.c);
      return true;
    case KindOf<typename S::Post>::code:
      tile_post<typename S::Post>(args, blk, (TRIME_LDS typename S::Post::Shm *)&sh.p);
      return true;
    case KindOf<typename S::X>::code:
      // the exact stage's polygons (48 KiB per wavefront) in this block's
      // slice of device memory instead of LDS
      tile_exact<typename S::X>(args, blk, (typename S::XPoly *)(xws + (size_t)blockIdx.x * sizeof(typename S::XPoly)),
                                (TRIME_LDS int *)xhist);
      return true;
    default: break;
  }
  if constexpr (MODE == MODE_EXTRACT) {
    switch (code) {
      case KindOf<DmBegin>::code: tile_run<DmBegin>(args, blk); return true;
      case KindOf<DmSums<G>>::code: tile_wave<DmSums<G>>(args, blk); return true;
      case KindOf<DmFinal>::code: tile_wave<DmFinal>(args, blk); return true;
      case KindOf<DmForce<T, G>>::code: tile_virt<DmForce<T, G>>(args, blk); return true;
      case KindOf<DmForceReplay<G>>::code: tile_virt<DmForceReplay<G>>(args, blk); return true;
      case KindOf<DmFlag>::code: tile_run<DmFlag>(args, blk); return true;
      default: break;
    }
  }
  return false;
}

template <class T, class G, int MODE> bool runs_code(uint32_t code) {
  using S = PersistSet<T, G, MODE>;
  const uint32_t common[] = {KindOf<FillCond>::code,   KindOf<BinKeys>::code,       KindOf<ScanTiles>::code,
                             KindOf<ScanSums>::code,   KindOf<ScanAdd>::code,       KindOf<ScanAddFew>::code,
                             KindOf<BinScatter>::code, KindOf<BinPlace>::code,      KindOf<OrderScatter>::code,
                             KindOf<OrderAdd>::code,   KindOf<StatsReset>::code,    KindOf<FinishExtract>::code,
                             KindOf<SetFlag>::code,    KindOf<typename S::C>::code, KindOf<typename S::Post>::code,
                             KindOf<typename S::X>::code};
  for (uint32_t c : common)
    if (c == code) return true;
  if (MODE == MODE_EXTRACT) {
    const uint32_t dm[] = {KindOf<DmBegin>::code,       KindOf<DmSums<G>>::code,         KindOf<DmFinal>::code,
                           KindOf<DmForce<T, G>>::code, KindOf<DmForceReplay<G>>::code, KindOf<DmFlag>::code};
    for (uint32_t c : dm)
      if (c == code) return true;
  }
  return false;
}

// The shape and chunk of item r of a period (phase p by binary search over
// ph_first, the shape's position by binary search over the phase's
// sh_first row).
struct ItemPos {
  uint32_t p, s, t0, t1, need;
};
TRIME_D ItemPos locate_item(const PersistArgs &P, uint32_t item) {
  ItemPos q;
  const uint32_t period = item / P.nper, r = item - period * P.nper;
  int lo = 0, hi = (int)P.nphase;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (gld(P.ph_first, mid) <= r)
      lo = mid;
    else
      hi = mid;
  }
  q.p = (uint32_t)lo;
  const uint32_t rr = r - gld(P.ph_first, lo);
  const uint32_t *sf = P.sh_first + (size_t)q.p * (P.ns + 1);
  lo = 0;
  hi = (int)P.ns;
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (gld(sf, mid) <= rr)
      lo = mid;
    else
      hi = mid;
  }
  q.s = (uint32_t)gld(P.order, lo);
  const uint32_t c = rr - gld(sf, lo);
  const uint32_t chunk = gld(P.ph_chunk, q.p);
  const uint32_t g = gld(P.grid, (int64_t)q.p * P.ns + q.s);
  q.t0 = c * chunk;
  q.t1 = q.t0 + chunk < g ? q.t0 + chunk : g;
  q.need = period * gld(P.per_shape, q.s) + gld(P.need, (int64_t)q.p * P.ns + q.s);
  return q;
}

// Waves per SIMD the kernel is built for: those of the fast cell kernel in
// its own launch (its register use sets the occupancy of the whole kernel).
template <class T> constexpr int persist_waves() { return sizeof(T) == 4 ? 3 : 2; }

// The current value of a counter, by an atomic that adds `zero` (a kernel
// argument, 0 at every launch: the compiler cannot see that the atomic
// changes nothing and turn it into a load).
TRIME_D uint32_t read_counter(uint32_t *p, uint32_t zero) {
  return __hip_atomic_fetch_add(p, zero, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <class T, class G, int MODE>
__global__ __launch_bounds__(64, persist_waves<T>()) void k_persist(PersistArgs P) {
  __shared__ typename PersistSet<T, G, MODE>::Shm sh;
  __shared__ int xhist[40];
  const int lane = threadIdx.x;
  const uint64_t total = (uint64_t)P.nper * P.nperiods;
  uint32_t *const head = P.ctl, *const abort_flag = P.ctl + PERSIST_LINE;
  const uint64_t deadline = (uint64_t)wall_clock64() + P.timeout;
  for (;;) {
    uint32_t item = 0;
    if (lane == 0) item = __hip_atomic_fetch_add(head, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    item = __builtin_amdgcn_readfirstlane(item);
    if (item >= total) break;
    const ItemPos q = locate_item(P, item);
    int ok = 1;
    if (lane == 0) {
      uint32_t *const cnt = P.done + (size_t)q.s * PERSIST_LINE;
      ok = read_counter(abort_flag, P.zero) == 0;
      int backoff = 1;
      while (ok && read_counter(cnt, P.zero) < q.need) {
        if ((uint64_t)wall_clock64() > deadline) {
          __hip_atomic_fetch_or(abort_flag, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          atomicOr(&gld(P.stats, q.s)->error, (int32_t)ERR_SCHED);
          ok = 0;
          break;
        }
        for (int k = 0; k < backoff; k++) __builtin_amdgcn_s_sleep(8);
        if (backoff < 32) {
          backoff *= 2;
        } else {
          ok = read_counter(abort_flag, P.zero) == 0;
        }
      }
    }
    ok = __builtin_amdgcn_readfirstlane(ok);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (ok) {
      const uint32_t code = gld(P.ph_code, q.p);
      const unsigned char *args = P.args + gld(P.ph_args, q.p) + (size_t)q.s * gld(P.ph_asz, q.p);
      const uint32_t g = gld(P.grid, (int64_t)q.p * P.ns + q.s);
      for (uint32_t t = q.t0; t < q.t1; t++) run_tile<T, G, MODE>(code, args, Blk{t, g}, sh, xhist, P.exact_ws);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __builtin_amdgcn_wave_barrier();
    if (lane == 0)
      __hip_atomic_fetch_add(P.done + (size_t)q.s * PERSIST_LINE, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// ------------------------------------------------------------ host side --
// cells_code bits: T double (1), G double (2), mode (<< 2)
#define TRIME_PERSIST_CASES(X)                     \
  X(float, float, MODE_EXTRACT)                    \
  X(double, float, MODE_EXTRACT)                   \
  X(float, double, MODE_EXTRACT)                   \
  X(double, double, MODE_EXTRACT)                  \
  X(float, float, MODE_CVD)                        \
  X(double, float, MODE_CVD)                       \
  X(float, double, MODE_CVD)                       \
  X(double, double, MODE_CVD)

bool persist_supported(uint32_t cells_code) {
#define X(T, G, M) \
  if (cells_code == KindOf<Cells<T, G, M, FAST_VMAX, fast_block<T, M>()>>::code) return true;
  TRIME_PERSIST_CASES(X)
#undef X
  return false;
}

bool persist_runs(uint32_t cells_code, uint32_t code) {
#define X(T, G, M) \
  if (cells_code == KindOf<Cells<T, G, M, FAST_VMAX, fast_block<T, M>()>>::code) return runs_code<T, G, M>(code);
  TRIME_PERSIST_CASES(X)
#undef X
  return false;
}

uint32_t persist_grid(uint32_t cells_code) {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return 0;
#define X(T, G, M)                                                                                     \
  if (cells_code == KindOf<Cells<T, G, M, FAST_VMAX, fast_block<T, M>()>>::code &&                           \
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void *)&k_persist<T, G, M>, 64, 0) != \
          hipSuccess)                                                                                  \
    return 0;
  TRIME_PERSIST_CASES(X)
#undef X
  return per > 0 && cus > 0 ? (uint32_t)per * (uint32_t)cus : 0;
}

size_t persist_exact_slice() { return sizeof(typename PersistSet<float, float, MODE_CVD>::XPoly); }

void launch_persist(uint32_t cells_code, const PersistArgs &p, uint32_t grid, hipStream_t s) {
#define X(T, G, M)                                                           \
  if (cells_code == KindOf<Cells<T, G, M, FAST_VMAX, fast_block<T, M>()>>::code) {   \
    hipLaunchKernelGGL((k_persist<T, G, M>), dim3(grid), dim3(64), 0, s, p); \
    return;                                                                  \
  }
  TRIME_PERSIST_CASES(X)
#undef X
}

}  // namespace trime
