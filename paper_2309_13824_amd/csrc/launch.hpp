// Launch-side declarations shared by the kernel files and the ABI.
#pragma once
#include <vector>

#include "trime_dev.hpp"

namespace trime {

// ---- one kernel for one shape, or for a whole batch of shapes --------------
// A kernel of the iteration loop is a functor F: F::Args its arguments,
// F::BLOCK its block size, F::run(args, blk) its body, written against the
// block coordinates blk instead of blockIdx / gridDim.  k_one runs it for one
// shape; k_many runs it for every shape of a batch in one launch: first[s] is
// the first block of shape s (first[ns] the grid size) and tab[s] its
// arguments, so each block finds its shape and runs the same body on that
// shape's buffers as if it were launched alone.
struct Blk {
  uint32_t id, n;  // block index and block count within the shape's grid
};

// The shape of block blk: the s with first[s] <= blk < first[s + 1] (shapes
// with no blocks are never returned).
TRIME_D int shape_of(const uint32_t *first, int ns, uint32_t blk) {
  int lo = 0, hi = ns;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (gld(first, mid) <= blk)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

template <class F> __global__ __launch_bounds__(F::BLOCK) void k_one(typename F::Args a) {
  F::run(a, Blk{blockIdx.x, gridDim.x});
}

template <class F>
__global__ __launch_bounds__(F::BLOCK) void k_many(const typename F::Args *__restrict__ tab,
                                                   const uint32_t *__restrict__ first, int ns) {
  const int s = shape_of(first, ns, blockIdx.x);
  const uint32_t f0 = gld(first, s), f1 = gld(first, s + 1);
  F::run(tab[s], Blk{blockIdx.x - f0, f1 - f0});
}

// ---- kernel kinds, for the persistent batch kernel --------------------------
// Every kernel of an iteration has a code naming its functor and template
// arguments: family << 8 | (T is double) | (G is double) << 1 | mode << 2.
// KindOf<F>::code is 0 for a kernel the persistent kernel cannot run.
enum KFam : uint32_t {
  KF_NONE = 0, KF_FILL, KF_BINKEYS, KF_SCANTILES, KF_SCANSUMS, KF_SCANADD, KF_SCANADDFEW, KF_BINSCATTER,
  KF_BINPLACE, KF_ORDERSCATTER, KF_ORDERADD, KF_CELLS, KF_POST, KF_EXACT, KF_DMSUMS, KF_DMFINAL, KF_DMFORCE,
  KF_DMREPLAY, KF_DMFLAG, KF_SETFLAG, KF_DMBEGIN, KF_STATSRESET, KF_FINISH
};
constexpr uint32_t kcode(uint32_t fam, bool tdbl = false, bool gdbl = false, uint32_t mode = 0) {
  return fam << 8 | (tdbl ? 1u : 0u) | (gdbl ? 2u : 0u) | mode << 2;
}
template <class T> constexpr bool is_dbl() { return sizeof(T) == 8; }
template <class F> struct KindOf {
  static constexpr uint32_t code = 0;
};

// The work of block blk of F by one wavefront (a block of 64 threads): F's
// BLOCK threads 64 at a time, for kernels whose threads never meet at a
// barrier (F::body(args, blk, t) is thread t of the block).
template <class F> TRIME_D void wave_virt(const typename F::Args &A, Blk blk) {
  const int lane = threadIdx.x & 63;
  for (int sub = 0; sub < F::BLOCK / 64; sub++) F::body(A, blk, sub * 64 + lane);
}

// A launch as recorded for a batch: the batched kernel, its kind, the grid
// of one shape, and that shape's argument bytes.
struct LaunchRec {
  const void *many;
  uint32_t code;
  uint32_t grid, block;
  std::vector<unsigned char> args;
};
// When set (on the calling host thread), launches are recorded, not issued.
extern thread_local std::vector<LaunchRec> *g_launch_log;

template <class F> void launch(const typename F::Args &a, uint32_t grid, hipStream_t s) {
  if (g_launch_log) {
    LaunchRec r;
    r.many = (const void *)&k_many<F>;
    r.code = KindOf<F>::code;
    r.grid = grid;
    r.block = F::BLOCK;
    r.args.assign((const unsigned char *)&a, (const unsigned char *)&a + sizeof a);
    g_launch_log->push_back(std::move(r));
    return;
  }
  if (grid) hipLaunchKernelGGL((k_one<F>), dim3(grid), dim3(F::BLOCK), 0, s, a);
}

enum { MODE_CELLS = 0, MODE_EXTRACT = 1, MODE_CVD = 2 };

// ---- the persistent batch kernel (persist.hip) -------------------------------
// One launch runs n_iter iterations of every shape of a batch.  Its work
// items are (period, phase, shape, chunk of tiles): a phase is one kernel of
// the recorded period (two iterations), a tile one block of that kernel for
// that shape, run by one wavefront.  Items are handed out in the order
// period, phase, shape (larger shapes first), chunk; an item waits until
// every item of its shape before it in that order is done (a per-shape
// count), so a shape's phases follow each other while other shapes are in
// other phases, and no wait is on an item handed out later.
struct PersistArgs {
  const unsigned char *args;   // per (phase, shape) kernel arguments: args + ph_args[p] + s * ph_asz[p]
  const uint64_t *ph_args;     // [P]
  const uint32_t *ph_asz;      // [P]
  const uint32_t *ph_code;     // [P] kernel kind (KindOf)
  const uint32_t *ph_chunk;    // [P] tiles per item
  const uint32_t *ph_first;    // [P + 1] first item of each phase within a period
  const uint32_t *sh_first;    // [P][ns + 1] first item of the i-th shape (in order) within the phase
  const uint32_t *grid;        // [P][ns] tiles of shape s in phase p
  const uint32_t *need;        // [P][ns] items of shape s in the phases before p
  const uint32_t *per_shape;   // [ns] items of shape s in one period
  const int32_t *order;        // [ns] the shape at position i
  trime_stats *const *stats;   // [ns] where a wait past the deadline is reported
  uint32_t *done;              // items done by shape s at done[s * PERSIST_LINE] (zero at launch)
  uint32_t *ctl;               // next item at ctl[0], abort flag at ctl[PERSIST_LINE] (zero at launch)
  unsigned char *exact_ws;     // the exact stage's polygons: one slice per block
  uint32_t nphase, ns, nper, nperiods;
  uint32_t zero;               // 0: the addend of the counters' reads
  uint64_t timeout;            // wall-clock ticks from a block's start to the launch's deadline
};
// counters of the persistent kernel one 128-byte line apart (in uint32_t)
constexpr int PERSIST_LINE = 32;
// cells_code: the code of the batch's fast cell kernel (its precision, grid
// type and mode).  persist_supported: false if no persistent kernel exists
// for it; persist_runs: whether that kernel runs the kernel kind `code`;
// persist_grid: its grid (resident blocks on the device); launch_persist
// enqueues it.
bool persist_supported(uint32_t cells_code);
bool persist_runs(uint32_t cells_code, uint32_t code);
uint32_t persist_grid(uint32_t cells_code);
size_t persist_exact_slice();
void launch_persist(uint32_t cells_code, const PersistArgs &p, uint32_t grid, hipStream_t s);

// Binning gather: current buffers in, the other buffer set out.
struct GatherArgs {
  const double *x, *y, *dprev;
  const uint8_t *cat;
  const int32_t *id;
  const double *xl, *yl;  // current last-triangulation positions and spans
  const float *span;
  double *xo, *yo, *dprevo, *xlo, *ylo;
  uint8_t *cato;
  int32_t *ido;
  float *spano;
};

struct LoadArgs {
  const double *xin, *yin;
  double *x, *y, *dprev, *xl, *yl;
  uint8_t *cat;
  int32_t *id;
  float *span;
};

void launch_cells(const KArgs &a, int mode, int grid_bytes, hipStream_t s);
// reset >= 0: the first binning kernel also clears the stats and counters
// (the full flag of launch_stats_reset) for the pass that follows
void launch_bin(const KArgs &a, const GatherArgs &g, int64_t nkeys, int32_t *scan_tmp, hipStream_t s,
                int32_t reset = -1);
void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
void launch_iota_i32(int32_t *p, int64_t n, hipStream_t s);
void scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *tmp, hipStream_t s,
              const int32_t *cond = nullptr);
size_t scan_tmp_ints(int64_t n);
void launch_dm(const KArgs &a, int grid_bytes, hipStream_t s);
int dm_partials(int64_t n);
void launch_load(const KArgs &a, const LoadArgs &l, int grid_bytes, hipStream_t s);
void launch_export_points(const KArgs &a, double *xo, double *yo, uint8_t *co, hipStream_t s);
void launch_export_tri(const KArgs &a, int32_t *off, int32_t *scan_tmp, int32_t *out, uint8_t *valid,
                       int64_t cap, int64_t *count, hipStream_t s);
void launch_export_adj(const KArgs &a, int32_t *deg_o, int32_t *col_o, hipStream_t s);
void launch_quality(const KArgs &a, hipStream_t s);
void launch_stats_reset(const KArgs &a, int full, hipStream_t s);
void launch_finish_extract(const KArgs &a, hipStream_t s);
void launch_set_flag(const KArgs &a, hipStream_t s);

// adaptive runs (adapt.hip): the gates of the control block, one per group
// of kernels of an iteration
enum { G_BIN = 0, G_DMTRI = 1, G_DMQ = 2, G_CVD = 3, G_DM = 4, G_COPY = 5, G_RUN = 6 };
void launch_adapt_init(const KArgs &a, int method, hipStream_t s);
void launch_adapt_pre(const KArgs &a, hipStream_t s);
// t_add < 0: no point addition (the request is never raised)
void launch_adapt_end(const KArgs &a, int hybrid, double t_quality, double t_amax, double t_switch,
                      double t_add, hipStream_t s);
const int32_t *adapt_gate(const trime_state *st, int g);

// point addition (grow.hip); the selection keys and state live in the
// caller's scratch (grow_key_bytes / grow_sel_bytes each)
void launch_grow_count(const KArgs &a, int32_t *cnt, hipStream_t s);
void launch_grow_select(const KArgs &a, const int32_t *off, void *keys, int64_t nk, void *sel, int64_t n_add,
                        hipStream_t s);
void launch_grow_mark(const KArgs &a, const void *sel, int32_t *cnt_id, hipStream_t s);
// a: the state after the addition's h scale; h_sel: the selection's
void launch_grow_write(const KArgs &a, double h_sel, int grid_bytes, const void *sel, const int32_t *base, double *x,
                       double *y, double *dprev, uint8_t *cat, int32_t *id, float *span, double *xl, double *yl,
                       hipStream_t s);
void launch_grow_state(const KArgs &a, int growing, int added, hipStream_t s);
size_t grow_key_bytes();
size_t grow_sel_bytes();
}  // namespace trime
