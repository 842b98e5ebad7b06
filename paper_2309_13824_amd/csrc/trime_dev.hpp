// Internal device-side definitions of the trime library (gfx950).
//
// Everything here follows the definitions stated in include/trime.h; the
// comments cite the paper (TriMe++, arXiv 2309.13824) by section/equation.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/trime.h"

#define TRIME_HD __host__ __device__ __forceinline__
#define TRIME_D __device__ __forceinline__

namespace trime {

// Unit roundoff of the two working precisions.
template <class T> struct U;
template <> struct U<float> { static constexpr float v = 5.9604645e-8f; };          // 2^-24
template <> struct U<double> { static constexpr double v = 1.1102230246251565e-16; }; // 2^-53

// Loads and stores through the global address space (plain pointers would
// compile to flat memory operations).
#define TRIME_GLOBAL __attribute__((address_space(1)))
// a pointer to LDS handed to a function that is not inlined (the callee then
// still addresses it as LDS)
#define TRIME_LDS __attribute__((address_space(3)))
template <class T> TRIME_D T gld(const T *p, int64_t i) { return ((const TRIME_GLOBAL T *)p)[i]; }
template <class T> TRIME_D void gst(T *p, int64_t i, T v) { ((TRIME_GLOBAL T *)p)[i] = v; }

// Everything a kernel needs, passed by value (well under the 4 KiB limit).
struct KArgs {
  int64_t n;
  // per-point arrays in slot order: current positions, next positions
  const double *x, *y;
  double *xn, *yn;
  const double *xl, *yl;  // positions at the last triangulation
  const double *dprev;
  double *dprevn;
  const uint8_t *cat;
  uint8_t *catn;
  const float *span;
  const int32_t *id;
  // binning
  int32_t *perm;
  int32_t *bin_start, *bin_fill, *key, *rank;
  int32_t *order;  // processing order of the slots in the cell kernels
  int32_t nbx, nby, lbits;
  double bx0, by0, bw, inv_bw;
  // grid
  int32_t nx, ny;
  double gx0, gy0, gdx, gdy, inv_dx, inv_dy;
  double box_x0, box_y0, box_x1, box_y1;
  const void *sdf, *mu;
  const uint8_t *cgrid;
  const float *hcell;
  const trime_grid_scalars *scal;
  // connectivity
  int32_t max_deg;
  int32_t *adj, *deg;
  int32_t *tri;  // TRIME_TRI_PER_POINT triangles per owner slot
  uint8_t *tri_valid;
  int32_t *tri_n;
  // work queues / counters / stats
  int32_t *queue;   // points for the FP64 replay
  int32_t *queue2;  // points for the exact replay
  int32_t *queue3;  // points whose centroid and treatment are redone in FP64
  int32_t *cq_cons; // per queue3 entry: n, then the n constraints of the cell
  int32_t *counters;
  double *partials;
  trime_stats *stats;
  // cell output (trime_voronoi_cells)
  int32_t *cell_cons, *cell_n;
  int32_t cell_cap;
  trime_params prm;
  int32_t precision;
  void *ev0, *ev1;  // optional timing events around the fused cell kernel
  // When set, the binning and extraction kernels work only if *cond != 0
  // (the re-triangulation flag of a DistMesh step, read on the device).
  const int32_t *cond;
  // every h of the grid times this (the grid built for more points than are
  // in the mesh, Sec. 3.7)
  double h_scale;
  // neighbours of each point's last cell by id (clipped first), and the slot
  // of each id in the current binning
  // warm start: the lists of the previous slot order (read), of this one
  // (written), and the slot maps of the last binning
  const int32_t *warm_n_prev, *warm_nb_prev;
  int32_t *warm_n, *warm_nb;
  int32_t *old_slot, *new_slot;
  int32_t xcd_run;  // blocks per XCD run of the fused cell kernel (>= 1)
};

// Whether a conditional launch has work (uniform over the grid).
TRIME_D bool cond_off(const KArgs &a) { return a.cond && gld(a.cond, 0) == 0; }

// counters[]: queue lengths, error bits, and the reasons of FP64 replays
enum { CNT_QUEUE = 0, CNT_TRI = 1, CNT_ERR = 2, CNT_MOVED = 3, CNT_QUEUE2 = 4, CNT_QUEUE3 = 5,
       CNT_REASON = 8, CNT_HEAVY = 24, CNT_NCOUNTERS = 32 };
// ints per entry of the deferred-centroid queue (count + constraints)
constexpr int CQ_STRIDE = 16;
// ERR_SCHED: a wait of the persistent batch kernel ran past its time limit
// (the batch's results are then incomplete)
enum { ERR_TRI_CAP = 1, ERR_DEG_CAP = 2, ERR_POLY_CAP = 4, ERR_EXACT_CAP = 8, ERR_QUEUE = 16, ERR_SCHED = 32 };
// why a point left the fast path
enum { WHY_PRED = 1, WHY_VERTEX = 2, WHY_POLY = 3, WHY_AND = 4, WHY_LEVEL = 5, WHY_TREAT = 6,
       WHY_BOX = 7, WHY_HEAVY = 8, WHY_PREC = 9 };

// ------------------------------------------------ exact quality sums ----
// The quality sums (Eq. 10-11) are kept as 128-bit fixed-point integers in
// units of 2^-52 (trime_stats.quality_acc, low word first).  A contribution
// v >= 0 is truncated to the unit; the sum of truncated values is exact, so
// it does not depend on the order in which blocks add them.  v = m 2^(e-1075)
// with the 53-bit significand m, so v 2^52 = m 2^(e-1023).  Values of 2^60 and
// more (or not finite) saturate at 2^60.
TRIME_D void fx_add(uint64_t *acc, double v) {
  if (!(v > 0.0)) return;
  if (!(v < 0x1p60)) v = 0x1p60;
  const uint64_t bits = (uint64_t)__double_as_longlong(v);
  const int e = (int)((bits >> 52) & 0x7ff);
  if (e == 0) return;  // subnormal: below the unit
  const uint64_t m = (bits & 0xfffffffffffffull) | 0x10000000000000ull;
  const int sh = e - 1023;  // <= 59
  uint64_t lo, hi;
  if (sh >= 0) {
    lo = m << sh;
    hi = sh == 0 ? 0 : m >> (64 - sh);
  } else if (sh > -64) {
    lo = m >> (-sh);
    hi = 0;
  } else {
    return;
  }
  typedef unsigned long long ull;
  const uint64_t old = (uint64_t)atomicAdd((ull *)&acc[0], (ull)lo);
  const uint64_t c = (old + lo < old) ? 1u : 0u;
  if (hi + c) atomicAdd((ull *)&acc[1], (ull)(hi + c));
}

TRIME_HD double fx_value(const uint64_t *acc) {
  return ((double)acc[1] * 0x1p64 + (double)acc[0]) * 0x1p-52;
}

// The finished quality fields of the stats (Eq. 11 with p = 1/2, mean and
// min q), from the exact sums; the host (trime_stats_read) and the adaptive
// control kernel evaluate the same expressions.
TRIME_HD void quality_finish(trime_stats *S) {
  S->sum_sqrt_alpha = fx_value(S->quality_acc + 0);
  S->sum_sqrt_beta = fx_value(S->quality_acc + 2);
  S->sum_q = fx_value(S->quality_acc + 4);
  if (S->nq > 0) {
    const double n = (double)S->nq;
    const double ma = S->sum_sqrt_alpha / n, mb = S->sum_sqrt_beta / n;
    S->half_mean_alpha = ma * ma;
    S->half_mean_beta = mb * mb;
    S->mean_q = S->sum_q / n;
    S->min_q = S->max_alpha > 0.0 ? 1.0 / S->max_alpha : 0.0;
  } else {
    S->half_mean_alpha = S->half_mean_beta = S->mean_q = S->min_q = 0.0;
  }
}

// Adds one partial of the quality sums (a block's or one point's, summed in a
// fixed order) and its max alpha (ordered as integers: alpha >= 0).
TRIME_D void quality_add(trime_stats *S, double sa, double sb, double sq, double amax) {
  fx_add(S->quality_acc + 0, sa);
  fx_add(S->quality_acc + 2, sb);
  fx_add(S->quality_acc + 4, sq);
  if (amax > 0.0) atomicMax((unsigned long long *)&S->max_alpha, (unsigned long long)__double_as_longlong(amax));
}

// Clears the quality part of the stats and the per-pass counters, and with
// full set every run statistic and counter; thread t of one block (at least
// 64 threads) takes its share.
TRIME_D void stats_reset(const KArgs &a, int full, int t) {
  trime_stats *S = a.stats;
  if (t < 40) S->hist_beta[t] = 0;
  if (t == 0) {
    S->sum_sqrt_alpha = 0;
    S->sum_sqrt_beta = 0;
    S->sum_q = 0;
    S->max_alpha = 0;
    for (int q = 0; q < 6; q++) S->quality_acc[q] = 0;
    S->half_mean_alpha = S->half_mean_beta = S->mean_q = S->min_q = 0;
    S->nq = 0;
    S->ntri = 0;
    S->nvalid = 0;
    S->moved = 0;
    if (full) {
      S->fp64_replays = 0;
      S->exact_points = 0;
      S->exact_calls = 0;
      S->sos_calls = 0;
      S->overflow_points = 0;
      S->newton_fail = 0;
      S->trace_fail = 0;
      S->level_cap_hits = 0;
      S->empty_cells = 0;
      S->triangulations = 0;
      S->iterations = 0;
      S->retri_flag = 1;
      S->error = 0;
      S->sum_l2 = 0;
      S->sum_mu2 = 0;
      S->fac_mu = 0;
      S->work_candidates = 0;
      S->work_margins = 0;
      S->work_cuts = 0;
      S->work_leaves = 0;
    }
  }
  if (t < (full ? CNT_NCOUNTERS : CNT_REASON)) a.counters[t] = 0;
}

// ---------------------------------------------------------------- grid ----

template <class G> TRIME_D double gval(const void *p, int64_t k) {
  return (double)gld((const G *)p, k);
}

// An integral float or double v as an int, saturated at +-2^24: the grid
// indices and offsets this converts are far smaller, and every caller clamps
// its result to the grid (one conversion instead of the 64-bit sequence).
template <class V> TRIME_D int sat_int(V v) { return (int)fmin(fmax(v, (V)-16777216.0), (V)16777216.0); }

// Bin of beta in the quality histogram (Eq. 11): 40 bins of width 0.05 from
// beta = 1, the last one open (beta >= 2.95, and the infinite or undefined
// beta of a triangle with a zero edge).  The bin is picked in floating point
// before the conversion, so a beta of any size converts in range.
TRIME_D int beta_bin(double be) {
  const double f = floor((be - 1.0) / 2.0 * 40.0);
  return f < 39.0 ? (f > 0.0 ? (int)f : 0) : 39;
}

// A grid cell by column i and row j; the cell arrays hold cell (i, j) at
// j (nx - 1) + i, the node arrays its lower-left node at j nx + i.
struct GCell {
  int i, j;
};
TRIME_D int64_t cell_index(const KArgs &a, const GCell &c) { return (int64_t)c.j * (a.nx - 1) + c.i; }
TRIME_D int64_t node_index(const KArgs &a, const GCell &c) { return (int64_t)c.j * a.nx + c.i; }

// Cell of (x, y): f = (x - x0) * (1/dx), cell = floor(f), t = f - cell.
// Returns false off the grid.
TRIME_D bool locate(const KArgs &a, double x, double y, GCell &cell, double &tx, double &ty) {
  double fx = (x - a.gx0) * a.inv_dx;
  double fy = (y - a.gy0) * a.inv_dy;
  if (!(fx >= 0.0) || !(fy >= 0.0)) return false;
  double ix = floor(fx), iy = floor(fy);
  if (ix >= (double)(a.nx - 1) || iy >= (double)(a.ny - 1)) return false;
  cell.i = (int)ix;  // 0 <= ix < nx - 1 (checked above)
  cell.j = (int)iy;
  tx = fx - ix;
  ty = fy - iy;
  return true;
}

// Bilinear value inside a cell: (f00 (1-tx) + f10 tx)(1-ty) + (f01 (1-tx) + f11 tx) ty.
template <class G>
TRIME_D double bilinear(const KArgs &a, const void *f, const GCell &cell, double tx, double ty) {
  const int64_t n0 = node_index(a, cell);
  double f00 = gval<G>(f, n0), f10 = gval<G>(f, n0 + 1);
  double f01 = gval<G>(f, n0 + a.nx), f11 = gval<G>(f, n0 + a.nx + 1);
  return (f00 * (1.0 - tx) + f10 * tx) * (1.0 - ty) + (f01 * (1.0 - tx) + f11 * tx) * ty;
}

TRIME_D uint8_t cell_cat(const KArgs &a, const GCell &cell) { return gld(a.cgrid, cell_index(a, cell)); }
// h of a cell, scaled for the current point count (fl32(h * h_scale))
TRIME_D float cell_h(const KArgs &a, const GCell &cell) {
  const float h = gld(a.hcell, cell_index(a, cell));
  return a.h_scale == 1.0 ? h : (float)((double)h * a.h_scale);
}
TRIME_D double h_avg(const KArgs &a) {
  return gld((const double *)a.scal, 1) * a.h_scale;  // trime_grid_scalars.h_avg
}

// geps of a cell (Sec. 3.7): fac_geps * min(h_cell, h_avg).
TRIME_D double geps_of(const KArgs &a, const GCell &cell) {
  return a.prm.fac_geps * fmin((double)cell_h(a, cell), h_avg(a));
}

// mu anywhere (cells clamped to the grid), used by the quadrature and forces.
template <class G> TRIME_D double mu_clamped(const KArgs &a, double x, double y) {
  double fx = (x - a.gx0) * a.inv_dx, fy = (y - a.gy0) * a.inv_dy;
  double ix = floor(fx), iy = floor(fy);
  ix = fmin(fmax(ix, 0.0), (double)(a.nx - 2));
  iy = fmin(fmax(iy, 0.0), (double)(a.ny - 2));
  double tx = fmin(fmax(fx - ix, 0.0), 1.0), ty = fmin(fmax(fy - iy, 0.0), 1.0);
  GCell cell;
  cell.i = (int)ix;  // clamped to [0, nx - 2]
  cell.j = (int)iy;
  return bilinear<G>(a, a.mu, cell, tx, ty);
}

// ------------------------------------------------------------- morton ----
TRIME_HD uint32_t spread2(uint32_t v) {
  v &= 0xffff;
  v = (v | (v << 8)) & 0x00ff00ff;
  v = (v | (v << 4)) & 0x0f0f0f0f;
  v = (v | (v << 2)) & 0x33333333;
  v = (v | (v << 1)) & 0x55555555;
  return v;
}
TRIME_HD uint32_t morton(uint32_t bx, uint32_t by) { return spread2(bx) | (spread2(by) << 1); }

TRIME_D void bin_of(const KArgs &a, double x, double y, int &bx, int &by) {
  bx = (int)floor((x - a.bx0) * a.inv_bw);
  by = (int)floor((y - a.by0) * a.inv_bw);
  bx = bx < 0 ? 0 : (bx >= a.nbx ? a.nbx - 1 : bx);
  by = by < 0 ? 0 : (by >= a.nby ? a.nby - 1 : by);
}

// Span S of the octagon of a point (Sec. 4.1): fac_voro * h of its cell, in
// float; D = fl32(fl32(sqrt 2) * S).
TRIME_D float span_at(const KArgs &a, double x, double y) {
  GCell cell;
  double tx, ty;
  if (!locate(a, x, y, cell, tx, ty)) return -1.0f;
  return (float)a.prm.fac_voro * cell_h(a, cell);
}

}  // namespace trime
