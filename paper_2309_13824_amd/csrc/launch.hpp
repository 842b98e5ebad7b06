// Launch-side declarations shared by the kernel files and the ABI.
#pragma once
#include "trime_dev.hpp"

namespace trime {

enum { MODE_CELLS = 0, MODE_EXTRACT = 1, MODE_CVD = 2 };

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

// Geometry for the grid build (device copies of the primitive lists).
struct GridPrims {
  int nprims;
  const trime_prim *prims;
  const double *poly;
  trime_sizing sz;  // cent / holes point into device memory
  const double *cent;
  const int32_t *holes;
  int nx, ny;
  double x0, y0, dx, dy;
  int64_t n_total;
};

void launch_cells(const KArgs &a, int mode, int grid_bytes, hipStream_t s);
void launch_bin(const KArgs &a, const GatherArgs &g, int64_t nkeys, int32_t *scan_tmp, hipStream_t s);
void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s);
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
void launch_adapt_end(const KArgs &a, int hybrid, double t_quality, double t_amax, double t_switch,
                      hipStream_t s);
const int32_t *adapt_gate(const trime_state *st, int g);
int64_t grid_partials(int nx, int ny);
void launch_grid_build(const GridPrims &g, int dtype_bytes, void *sdf, void *mu, uint8_t *cat,
                       float *hcell, trime_grid_scalars *scal, double *part, hipStream_t s);

}  // namespace trime
