// Binning of the points into Morton-ordered square bins (the role of the
// Voro++ container blocks, ~3.3 points per block as in the paper's example
// code unless tuned), by counting sort: keys + histogram, exclusive scan,
// scatter, then a per-bin sort by previous slot so the new slot order is the
// deterministic order (bin key, previous slot).  The gather then permutes every per-point array into the
// new slot order (coalesced: points move little between iterations).
#pragma once
#include "launch.hpp"

namespace trime {


constexpr int SCAN_BLOCK = 1024;
constexpr int SCAN_ITEMS = 4;  // elements per thread
constexpr int SCAN_TILE = SCAN_BLOCK * SCAN_ITEMS;

// Zeroes the bin fill counts (grid-stride).  With reset >= 0, block 0 also
// clears the stats and counters of the pass that follows the binning (the
// full flag of the stats reset), which spares that pass a launch of its own.
struct FillCond {
  struct Args {
    KArgs a;
    int32_t *p;
    int64_t n;
    int32_t reset;
  };
  static constexpr int BLOCK = 256;
  TRIME_D static void run(const Args &A, Blk b) { body(A, b, threadIdx.x); }
  TRIME_D static void body(const Args &A, Blk b, int t) {
    if (cond_off(A.a)) return;
    if (A.reset >= 0 && b.id == 0) stats_reset(A.a, A.reset, t);
    for (int64_t i = (int64_t)b.id * BLOCK + t; i < A.n; i += (int64_t)b.n * BLOCK) A.p[i] = 0;
  }
};

// Keys and ranks within the bins.  The points arrive in the previous slot
// order, so runs of equal keys fill a wavefront: the first lane of each run
// takes the run's ranks with one atomic and hands them out.
struct BinKeys {
  using Args = KArgs;
  static constexpr int BLOCK = 256;
  TRIME_D static void run(const KArgs &a, Blk blk) { body(a, blk, threadIdx.x); }
  TRIME_D static void body(const KArgs &a, Blk blk, int t);
};
TRIME_D void BinKeys::body(const KArgs &a, Blk blk, int t) {
  if (cond_off(a)) return;
  int64_t k = (int64_t)blk.id * BLOCK + t;
  const int lane = t & 63;
  const bool valid = k < a.n;
  int key = -1;
  if (valid) {
    int bx, by;
    bin_of(a, a.x[k], a.y[k], bx, by);
    key = (int)morton((uint32_t)bx, (uint32_t)by);
    a.key[k] = key;
  }
  const int prev = __shfl_up(key, 1);
  const bool head = valid && (lane == 0 || prev != key);
  const uint64_t H = __ballot(head), V = __ballot(valid);
  const uint64_t upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);  // lanes 0..lane
  int base = 0;
  if (head) {
    uint64_t above = (H | ~V) & ~upto;  // the next head or the first lane past the end
    int nxt = above ? __ffsll((unsigned long long)above) - 1 : 64;
    base = atomicAdd(&a.bin_fill[key], nxt - lane);
  }
  const int hl = 63 - __clzll((unsigned long long)(H & upto));
  const int b = __shfl(base, hl < 0 ? 0 : hl);
  if (valid) a.rank[k] = b + (lane - hl);
}

// Block-wide exclusive scan of 4096 ints per block; writes block totals.
__device__ __forceinline__ int block_excl_scan(int v, int *smem, int &total) {
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int x = v;
  for (int off = 1; off < 64; off <<= 1) {
    int y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  if (lane == 63) smem[w] = x;
  __syncthreads();
  if (threadIdx.x < 64) {
    int nw = blockDim.x >> 6;
    int s = threadIdx.x < nw ? smem[threadIdx.x] : 0;
    for (int off = 1; off < 64; off <<= 1) {
      int y = __shfl_up(s, off);
      if ((int)threadIdx.x >= off) s += y;
    }
    if (threadIdx.x < nw) smem[threadIdx.x] = s;
  }
  __syncthreads();
  int before = (w > 0 ? smem[w - 1] : 0) + x - v;
  total = smem[(blockDim.x >> 6) - 1];
  __syncthreads();
  return before;
}

// Inclusive prefix sum over the lanes of a wavefront.
TRIME_D int wave_incl_scan(int x) {
  const int lane = threadIdx.x & 63;
  for (int off = 1; off < 64; off <<= 1) {
    int y = __shfl_up(x, off);
    if (lane >= off) x += y;
  }
  return x;
}

// Sum over the lanes of a wavefront, in every lane.
TRIME_D int wave_sum_i(int x) {
  for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off);
  return x;
}

// The three passes of an exclusive scan share one argument set.
struct ScanArgs {
  const int32_t *in;
  int32_t *out;
  int64_t n, nt;
  int32_t *sums;  // nt + 1 tile sums
  const int32_t *cond;
};

struct ScanTiles {
  using Args = ScanArgs;
  static constexpr int BLOCK = SCAN_BLOCK;
  TRIME_D static void run(const ScanArgs &A, Blk blk);
  TRIME_D static void run_wave(const ScanArgs &A, Blk blk);
};
TRIME_D void ScanTiles::run(const ScanArgs &A, Blk blk) {
  __shared__ int smem[SCAN_BLOCK / 64];
  if (A.cond && gld(A.cond, 0) == 0) return;
  const int32_t *in = A.in;
  int32_t *out = A.out;
  const int64_t n = A.n;
  int64_t base = (int64_t)blk.id * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int v[SCAN_ITEMS];
  int s = 0;
#pragma unroll
  for (int q = 0; q < SCAN_ITEMS; q++) {
    v[q] = (base + q < n) ? in[base + q] : 0;
    s += v[q];
  }
  int total;
  int before = block_excl_scan(s, smem, total);
#pragma unroll
  for (int q = 0; q < SCAN_ITEMS; q++) {
    if (base + q < n) out[base + q] = before;
    before += v[q];
  }
  if (threadIdx.x == 0) A.sums[blk.id] = total;
}

// One wavefront does the block's tile: the 1024 threads' items 64 threads
// at a time, each group's scan offset by the sum of the groups before it.
TRIME_D void ScanTiles::run_wave(const ScanArgs &A, Blk blk) {
  if (A.cond && gld(A.cond, 0) == 0) return;
  const int lane = threadIdx.x & 63;
  int carry = 0;
  for (int sub = 0; sub < SCAN_BLOCK / 64; sub++) {
    const int64_t b0 = (int64_t)blk.id * SCAN_TILE + (int64_t)sub * 64 * SCAN_ITEMS;
    if (b0 >= A.n) break;  // the rest of the tile is past the end: it adds nothing
    const int64_t base = b0 + (int64_t)lane * SCAN_ITEMS;
    int v[SCAN_ITEMS];
    int s = 0;
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; q++) {
      v[q] = (base + q < A.n) ? A.in[base + q] : 0;
      s += v[q];
    }
    const int incl = wave_incl_scan(s);
    int before = carry + incl - s;
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; q++) {
      if (base + q < A.n) A.out[base + q] = before;
      before += v[q];
    }
    carry += __shfl(incl, 63);
  }
  if (lane == 0) A.sums[blk.id] = carry;
}

// Single block: exclusive scan of the tile sums (any count), total at [nt].
struct ScanSums {
  using Args = ScanArgs;
  static constexpr int BLOCK = SCAN_BLOCK;
  TRIME_D static void run(const ScanArgs &A, Blk blk);
  TRIME_D static void run_wave(const ScanArgs &A, Blk blk);
};
TRIME_D void ScanSums::run(const ScanArgs &A, Blk) {
  __shared__ int smem[SCAN_BLOCK / 64];
  if (A.cond && gld(A.cond, 0) == 0) return;
  int32_t *sums = A.sums;
  const int64_t nt = A.nt;
  int carry = 0;
  for (int64_t base = 0; base < nt; base += SCAN_BLOCK) {
    int64_t i = base + threadIdx.x;
    int v = i < nt ? sums[i] : 0;
    int total;
    int before = block_excl_scan(v, smem, total);
    if (i < nt) sums[i] = before + carry;
    carry += total;
  }
  if (threadIdx.x == 0) sums[nt] = carry;
}

TRIME_D void ScanSums::run_wave(const ScanArgs &A, Blk) {
  if (A.cond && gld(A.cond, 0) == 0) return;
  const int lane = threadIdx.x & 63;
  int carry = 0;
  for (int64_t base = 0; base < A.nt; base += 64) {
    const int64_t i = base + lane;
    const int v = i < A.nt ? A.sums[i] : 0;
    const int incl = wave_incl_scan(v);
    if (i < A.nt) A.sums[i] = carry + incl - v;
    carry += __shfl(incl, 63);
  }
  if (lane == 0) A.sums[A.nt] = carry;
}

struct ScanAdd {
  using Args = ScanArgs;
  static constexpr int BLOCK = SCAN_BLOCK;
  TRIME_D static void run(const ScanArgs &A, Blk blk) { body(A, blk, threadIdx.x); }
  TRIME_D static void body(const ScanArgs &A, Blk blk, int t) {
    if (A.cond && gld(A.cond, 0) == 0) return;
    int64_t base = (int64_t)blk.id * SCAN_TILE + (int64_t)t * SCAN_ITEMS;
    int add = A.sums[blk.id];
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; q++)
      if (base + q < A.n) A.out[base + q] += add;
    if (blk.id == 0 && t == 0) A.out[A.n] = A.sums[A.nt];
  }
};

// With few tiles, the second pass of its own: each block adds the tile sums
// before it (a block-wide sum of at most SCAN_FEW_TILES values) to its tile,
// and block 0 also writes the total, which spares the single-block pass.
constexpr int64_t SCAN_FEW_TILES = 2048;
struct ScanAddFew {
  using Args = ScanArgs;
  static constexpr int BLOCK = SCAN_BLOCK;
  TRIME_D static void run(const ScanArgs &A, Blk blk) {
    __shared__ int smem[SCAN_BLOCK / 64];
    if (A.cond && gld(A.cond, 0) == 0) return;
    const int64_t upto = blk.id == 0 ? A.nt : (int64_t)blk.id;  // block 0: every tile, for the total
    int v = 0;
    for (int64_t i = threadIdx.x; i < upto; i += SCAN_BLOCK) v += A.sums[i];
    int total;
    block_excl_scan(v, smem, total);
    const int add = blk.id == 0 ? 0 : total;
    int64_t base = (int64_t)blk.id * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; q++)
      if (base + q < A.n) A.out[base + q] += add;
    if (blk.id == 0 && threadIdx.x == 0) A.out[A.n] = total;
  }
  TRIME_D static void run_wave(const ScanArgs &A, Blk blk) {
    if (A.cond && gld(A.cond, 0) == 0) return;
    const int lane = threadIdx.x & 63;
    const int64_t upto = blk.id == 0 ? A.nt : (int64_t)blk.id;
    int v = 0;
    for (int64_t i = lane; i < upto; i += 64) v += A.sums[i];
    const int total = wave_sum_i(v);
    if (blk.id != 0) {
      for (int sub = 0; sub < SCAN_BLOCK / 64; sub++) {
        const int64_t base = (int64_t)blk.id * SCAN_TILE + (int64_t)(sub * 64 + lane) * SCAN_ITEMS;
#pragma unroll
        for (int q = 0; q < SCAN_ITEMS; q++)
          if (base + q < A.n) A.out[base + q] += total;
      }
    } else if (lane == 0) {
      A.out[A.n] = total;
    }
  }
};

struct BinScatter {
  using Args = KArgs;
  static constexpr int BLOCK = 256;
  TRIME_D static void run(const KArgs &a, Blk blk) { body(a, blk, threadIdx.x); }
  TRIME_D static void body(const KArgs &a, Blk blk, int t) {
    int64_t k = (int64_t)blk.id * BLOCK + t;
    if (k >= a.n || cond_off(a)) return;
    a.perm[a.bin_start[a.key[k]] + a.rank[k]] = (int)k;
  }
};

// The new slot of every point, and its arrays written there (the other
// buffer set).  Slots are ordered by (bin key, previous slot): a point's
// place in its bin is the number of the bin's points with a smaller
// previous slot, which is deterministic whatever order the atomics of the
// ranks took.  The positions of the last triangulation become the current
// ones, the octagon span S is recomputed from the point's cell, and the
// flag of the processing order (1 on the boundary) goes to rank[] at the
// new slot.  A conditional binning without work copies every array in
// place order instead (the buffer sets still swap), keeping the
// last-triangulation positions and spans, and leaves the processing order
// as it was.
struct BinPlace {
  struct Args {
    KArgs a;
    GatherArgs g;
  };
  static constexpr int BLOCK = 256;
  TRIME_D static void run(const Args &A, Blk blk) { body(A, blk, threadIdx.x); }
  TRIME_D static void body(const Args &A, Blk blk, int t);
};
TRIME_D void BinPlace::body(const Args &A, Blk blk, int t) {
  const KArgs &a = A.a;
  const GatherArgs &g = A.g;
  const int64_t k = (int64_t)blk.id * BLOCK + t;
  if (k >= a.n) return;
  if (cond_off(a)) {
    if (a.old_slot) {
      a.old_slot[k] = (int32_t)k;
      a.new_slot[k] = (int32_t)k;
    }
    g.xo[k] = g.x[k];
    g.yo[k] = g.y[k];
    g.dprevo[k] = g.dprev[k];
    g.cato[k] = g.cat[k];
    g.ido[k] = g.id[k];
    g.xlo[k] = g.xl[k];
    g.ylo[k] = g.yl[k];
    g.spano[k] = g.span[k];
    return;
  }
  const int key = a.key[k];
  const int s0 = a.bin_start[key], s1 = a.bin_start[key + 1];
  int s = s0;
  for (int t = s0; t < s1; t++) s += a.perm[t] < (int)k ? 1 : 0;
  const double x = g.x[k], y = g.y[k];
  g.xo[s] = x;
  g.yo[s] = y;
  g.xlo[s] = x;
  g.ylo[s] = y;
  g.dprevo[s] = g.dprev[k];
  const uint8_t c = g.cat[k];
  g.cato[s] = c;
  const int id = g.id[k];
  g.ido[s] = id;
  if (a.old_slot) {
    a.old_slot[s] = (int32_t)k;
    a.new_slot[k] = (int32_t)s;
  }
  g.spano[s] = span_at(a, x, y);
  a.rank[s] = c == TRIME_CAT_BOUNDARY ? 1 : 0;
}

// Processing order of the cell kernels: the slots of points on the boundary
// first (their cells reach the octagon walls outside the domain, so they scan
// the most bins), then all others, each group in slot order.  Heavy points
// then share wavefronts and start first instead of holding back 64-point
// wavefronts of light ones.  The flags (rank[], from BinPlace) are scanned
// into perm[]; the slot of the w-th point in processing order goes to
// order[w].
struct OrderScatter {
  using Args = KArgs;
  static constexpr int BLOCK = 256;
  TRIME_D static void run(const KArgs &a, Blk blk) { body(a, blk, threadIdx.x); }
  TRIME_D static void body(const KArgs &a, Blk blk, int t) {
    int64_t s = (int64_t)blk.id * BLOCK + t;
    if (s >= a.n || cond_off(a)) return;
    int before = a.perm[s];  // heavy slots before s
    int heavy = a.perm[a.n];
    if (s == 0) a.counters[CNT_HEAVY] = heavy;
    int64_t w = a.rank[s] ? before : heavy + (s - before);
    a.order[w] = (int)s;
  }
};

// With few scan tiles, the second scan pass and the order scatter in one:
// each block sums the tile totals before it and all of them (the number of
// heavy slots), adds the first to the tile's own exclusive scan and places
// its slots.
struct OrderAdd {
  struct Args {
    KArgs a;
    ScanArgs s;
  };
  static constexpr int BLOCK = SCAN_BLOCK;
  TRIME_D static void run(const Args &A, Blk blk) {
    __shared__ int smem[SCAN_BLOCK / 64];
    const KArgs &a = A.a;
    const ScanArgs &S = A.s;
    if (cond_off(a)) return;
    int vb = 0, va = 0;
    for (int64_t i = threadIdx.x; i < S.nt; i += SCAN_BLOCK) {
      const int t = S.sums[i];
      va += t;
      vb += i < (int64_t)blk.id ? t : 0;
    }
    int add, heavy;
    block_excl_scan(vb, smem, add);
    block_excl_scan(va, smem, heavy);
    if (blk.id == 0 && threadIdx.x == 0) a.counters[CNT_HEAVY] = heavy;
    const int64_t base = (int64_t)blk.id * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
#pragma unroll
    for (int q = 0; q < SCAN_ITEMS; q++) {
      const int64_t s = base + q;
      if (s < S.n) {
        const int before = S.out[s] + add;
        const int64_t w = S.in[s] ? before : heavy + (s - before);
        a.order[w] = (int)s;
      }
    }
  }
  TRIME_D static void run_wave(const Args &A, Blk blk) {
    const KArgs &a = A.a;
    const ScanArgs &S = A.s;
    if (cond_off(a)) return;
    const int lane = threadIdx.x & 63;
    int vb = 0, va = 0;
    for (int64_t i = lane; i < S.nt; i += 64) {
      const int t = S.sums[i];
      va += t;
      vb += i < (int64_t)blk.id ? t : 0;
    }
    const int add = wave_sum_i(vb), heavy = wave_sum_i(va);
    if (blk.id == 0 && lane == 0) a.counters[CNT_HEAVY] = heavy;
    for (int sub = 0; sub < SCAN_BLOCK / 64; sub++) {
      const int64_t base = (int64_t)blk.id * SCAN_TILE + (int64_t)(sub * 64 + lane) * SCAN_ITEMS;
#pragma unroll
      for (int q = 0; q < SCAN_ITEMS; q++) {
        const int64_t s = base + q;
        if (s < S.n) {
          const int before = S.out[s] + add;
          const int64_t w = S.in[s] ? before : heavy + (s - before);
          a.order[w] = (int)s;
        }
      }
    }
  }
};

// kinds (persistent batch kernel)
template <> struct KindOf<FillCond> { static constexpr uint32_t code = kcode(KF_FILL); };
template <> struct KindOf<BinKeys> { static constexpr uint32_t code = kcode(KF_BINKEYS); };
template <> struct KindOf<ScanTiles> { static constexpr uint32_t code = kcode(KF_SCANTILES); };
template <> struct KindOf<ScanSums> { static constexpr uint32_t code = kcode(KF_SCANSUMS); };
template <> struct KindOf<ScanAdd> { static constexpr uint32_t code = kcode(KF_SCANADD); };
template <> struct KindOf<ScanAddFew> { static constexpr uint32_t code = kcode(KF_SCANADDFEW); };
template <> struct KindOf<BinScatter> { static constexpr uint32_t code = kcode(KF_BINSCATTER); };
template <> struct KindOf<BinPlace> { static constexpr uint32_t code = kcode(KF_BINPLACE); };
template <> struct KindOf<OrderScatter> { static constexpr uint32_t code = kcode(KF_ORDERSCATTER); };
template <> struct KindOf<OrderAdd> { static constexpr uint32_t code = kcode(KF_ORDERADD); };

}  // namespace trime
