// Host side of the C ABI declared in include/trime.h: argument checks,
// workspace layout and the launch sequence of each entry point.
#include <math.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <stdio.h>
#include <string.h>

#include "trime_dev.hpp"

#include "launch.hpp"
#include "setup.hpp"

using namespace trime;

namespace trime {
thread_local std::vector<LaunchRec> *g_launch_log = nullptr;
}

static thread_local char g_err[512] = "";

static trime_status fail(trime_status st, const char *msg) {
  snprintf(g_err, sizeof g_err, "%s", msg);
  return st;
}

static trime_status check_hip(const char *where) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    snprintf(g_err, sizeof g_err, "%s: %s", where, hipGetErrorString(e));
    return TRIME_EHIP;
  }
  return TRIME_OK;
}

#define TRY_HIP(call, where)                                                   \
  do {                                                                         \
    hipError_t e_ = (call);                                                    \
    if (e_ != hipSuccess) {                                                    \
      snprintf(g_err, sizeof g_err, "%s: %s", where, hipGetErrorString(e_));   \
      return TRIME_EHIP;                                                       \
    }                                                                          \
  } while (0)

// entry points: C linkage from the declarations in trime.h

const char *trime_last_error(void) { return g_err; }
const char *trime_version(void) { return "trime-gfx950 0.1"; }

void trime_default_params(trime_params *p) {
  if (!p) return;
  p->fac_F = 1.2;
  p->fac_voro = 5.0;
  p->fac_pt = 0.4;
  p->fac_retria = 0.1;
  p->fac_end = 0.001;
  p->fac_geps = 0.01;
  p->T_tria = 0.4;
  p->alpha_hat = 1.0;
  p->T_newton = 10;
  p->k_spring = 1.0;
  p->dt = 0.2;
  p->cvd_max_level = 12;
  p->trace_max_steps = 64;
  p->trace_bisect = 8;
  p->test2_mode = 0;
}

static bool grid_ok(const trime_grid *g) {
  return g && g->nx >= 2 && g->ny >= 2 && g->dx > 0 && g->dy > 0 &&
         (g->dtype_bytes == 4 || g->dtype_bytes == 8) && isfinite(g->x0) && isfinite(g->y0);
}

// ------------------------------------------------------ automatic sizing --

static trime_status auto_ok(const trime_geometry *geo, const trime_sizing *sz, const char *who) {
  static thread_local char msg[160];
  const char *why = nullptr;
  if (!sz || sz->kind != TRIME_SZ_AUTO)
    why = "the sizing kind is not AUTO";
  else if (!(sz->a1 > 0) || !(sz->a0 >= 0) || !isfinite(sz->a0) || !isfinite(sz->a1))
    why = "automatic sizing needs a0 = K >= 0 and a1 = fac_s > 0";
  else if (sz->n_thres < 0 || !(sz->fac_nei >= 0) || !(sz->fac_geps >= 0))
    why = "automatic sizing: negative n_thres or fac_nei";
  if (!why) return TRIME_OK;
  snprintf(msg, sizeof msg, "%s: %s", who, why);
  return fail(TRIME_EINVAL, msg);
}

struct AutoSetup {
  double d_s, geps, r_nei, box[4], gbox[4];
  int n_thres;
};

static AutoSetup auto_setup(const trime_sizing *sz, const trime_grid *grid) {
  AutoSetup a;
  a.d_s = sz->a1 * fmin(grid->dx, grid->dy);
  a.geps = (sz->fac_geps > 0 ? sz->fac_geps : 0.01) * fmin(grid->dx, grid->dy);
  a.n_thres = sz->n_thres > 0 ? sz->n_thres : 3;
  const double fac_nei = sz->fac_nei > 0 ? sz->fac_nei : 2.0;
  a.r_nei = fac_nei * a.n_thres * a.d_s;
  const double W = (grid->nx - 1) * grid->dx, H = (grid->ny - 1) * grid->dy;
  a.gbox[0] = grid->x0;
  a.gbox[1] = grid->y0;
  a.gbox[2] = grid->x0 + W;
  a.gbox[3] = grid->y0 + H;
  a.box[0] = grid->x0 - W;
  a.box[1] = grid->y0 - H;
  a.box[2] = grid->x0 + 2 * W;
  a.box[3] = grid->y0 + 2 * H;
  return a;
}

trime_status trime_auto_sizing(const trime_geometry *geo, const trime_sizing *sz, const trime_grid *grid,
                               double *d_pts, int64_t s_cap, int64_t *ns_out, double *d_medial, uint8_t *d_keep,
                               int64_t m_cap, int64_t *nm_out, double *d_lfs, void *stream) {
  if (!geo || !grid_ok(grid) || !ns_out || !nm_out || !d_pts || !d_medial || !d_keep || !d_lfs ||
      geo->nprims <= 0 || !geo->prims)
    return fail(TRIME_EINVAL, "trime_auto_sizing: null or invalid argument");
  for (int k = 0; k < geo->nprims; k++) {
    const trime_prim &p = geo->prims[k];
    if ((p.kind == TRIME_PRIM_SEGMENTS || p.kind == TRIME_PRIM_POLYGON) &&
        (p.nv < 3 || p.voff < 0 || p.voff + p.nv > geo->npoly || !geo->poly))
      return fail(TRIME_EINVAL, "trime_auto_sizing: bad polygon range");
    if (p.kind < 0 || p.kind > TRIME_PRIM_SEGMENTS || p.op < 0 || p.op > 3)
      return fail(TRIME_EINVAL, "trime_auto_sizing: bad primitive op/kind");
  }
  trime_status e = auto_ok(geo, sz, "trime_auto_sizing");
  if (e) return e;
  const AutoSetup A = auto_setup(sz, grid);
  std::vector<double> S = trim_boundary(geo, A.d_s, A.geps, boundary_points(geo, A.d_s, A.geps));
  const int64_t ns = (int64_t)S.size() / 2;
  *ns_out = ns;
  *nm_out = -1;
  if (s_cap < ns || m_cap < 2 * ns) return fail(TRIME_ECAPACITY, "trime_auto_sizing: output buffers too small");
  if (ns >= ((int64_t)1 << 30)) return fail(TRIME_EUNSUPPORTED, "trime_auto_sizing: too many boundary points");
  hipStream_t s = (hipStream_t)stream;
  TRY_HIP(hipMemcpyAsync(d_pts, S.data(), sizeof(double) * S.size(), hipMemcpyHostToDevice, s), "copy points");
  std::vector<void *> allocs;
  int64_t nm = 0;
  const char *err = auto_sizing_build(d_pts, ns, A.box, A.gbox, A.r_nei, A.n_thres, sz->a0, 0.0, d_medial, d_keep,
                                      d_lfs, &nm, nullptr, allocs, s);
  for (void *a : allocs) (void)hipFreeAsync(a, s);
  TRY_HIP(hipStreamSynchronize(s), "trime_auto_sizing (sync)");
  if (err) return fail(TRIME_EINVAL, err);
  *nm_out = nm;
  return check_hip("trime_auto_sizing");
}

// The argument checks of both grid builds.
static trime_status grid_build_ok(const trime_geometry *geo, const trime_sizing *sz, const trime_grid *grid,
                                  int64_t n_total, void *d_sdf, void *d_mu, uint8_t *d_cat, float *d_hcell,
                                  trime_grid_scalars *d_scal) {
  if (!geo || !sz || !grid_ok(grid) || n_total <= 0 || !d_sdf || !d_mu || !d_cat || !d_hcell || !d_scal)
    return fail(TRIME_EINVAL, "trime_sdf_grid_build: null or invalid argument");
  if (geo->nprims <= 0 || !geo->prims || geo->prims[0].op != TRIME_OP_INIT)
    return fail(TRIME_EINVAL, "trime_sdf_grid_build: the first primitive must be INIT");
  for (int k = 0; k < geo->nprims; k++) {
    const trime_prim &p = geo->prims[k];
    if (p.op < 0 || p.op > 3 || p.kind < 0 || p.kind > TRIME_PRIM_SEGMENTS)
      return fail(TRIME_EINVAL, "trime_sdf_grid_build: bad primitive op/kind");
    if ((p.kind == TRIME_PRIM_POLYGON || p.kind == TRIME_PRIM_SEGMENTS) &&
        (p.nv < 3 || p.voff < 0 || p.voff + p.nv > geo->npoly || !geo->poly))
      return fail(TRIME_EINVAL, "trime_sdf_grid_build: bad polygon range");
    if ((p.kind == TRIME_PRIM_DISK && !(p.p[2] > 0)) ||
        (p.kind == TRIME_PRIM_ELLIPSE && !(p.p[2] > 0 && p.p[3] > 0)))
      return fail(TRIME_EINVAL, "trime_sdf_grid_build: nonpositive radius");
  }
  if (sz->kind < 0 || sz->kind > TRIME_SZ_AUTO) return fail(TRIME_EINVAL, "trime_sdf_grid_build: bad sizing kind");
  if (sz->kind == TRIME_SZ_AUTO) {
    trime_status e = auto_ok(geo, sz, "trime_sdf_grid_build");
    if (e) return e;
  }
  if (sz->kind == TRIME_SZ_GAUSS_RHO && (sz->ncent < 0 || (sz->ncent > 0 && !sz->cent) || !(sz->s2 > 0)))
    return fail(TRIME_EINVAL, "trime_sdf_grid_build: bad density centres");
  if (sz->kind == TRIME_SZ_HOLE_RAMP) {
    if (sz->nholes <= 0 || !sz->holes || !(sz->a1 > 0))
      return fail(TRIME_EINVAL, "trime_sdf_grid_build: bad hole list");
    for (int k = 0; k < sz->nholes; k++)
      if (sz->holes[k] < 0 || sz->holes[k] >= geo->nprims)
        return fail(TRIME_EINVAL, "trime_sdf_grid_build: hole index out of range");
  }
  return TRIME_OK;
}

trime_status trime_sdf_grid_build(const trime_geometry *geo, const trime_sizing *sz,
                                  const trime_grid *grid, int64_t n_total, void *d_sdf, void *d_mu,
                                  uint8_t *d_cat, float *d_hcell, trime_grid_scalars *d_scal,
                                  void *stream) {
  trime_status e0 = grid_build_ok(geo, sz, grid, n_total, d_sdf, d_mu, d_cat, d_hcell, d_scal);
  if (e0) return e0;
  hipStream_t s = (hipStream_t)stream;
  // one temporary device buffer: prims | poly | cent | holes | partials |
  // segment candidate trees (their lists are allocated while they are built)
  size_t b_prims = sizeof(trime_prim) * (size_t)geo->nprims;
  size_t b_segs = sizeof(SegTree) * (size_t)geo->nprims;
  size_t b_poly = sizeof(double) * 2 * (size_t)(geo->npoly > 0 ? geo->npoly : 0);
  size_t b_cent = sizeof(double) * 2 * (size_t)(sz->kind == TRIME_SZ_GAUSS_RHO ? sz->ncent : 0);
  size_t b_holes = sizeof(int32_t) * (size_t)(sz->kind == TRIME_SZ_HOLE_RAMP ? sz->nholes : 0);
  size_t b_part = sizeof(double) * 2 * (size_t)grid_partials(grid->nx, grid->ny);
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  size_t total = al(b_prims) + al(b_poly) + al(b_cent) + al(b_holes) + al(b_part) + al(b_segs);
  char *buf = nullptr;
  TRY_HIP(hipMallocAsync((void **)&buf, total, s), "trime_sdf_grid_build: hipMallocAsync");
  char *q = buf;
  trime_prim *d_prims = (trime_prim *)q; q += al(b_prims);
  double *d_poly = (double *)q; q += al(b_poly);
  double *d_cent = (double *)q; q += al(b_cent);
  int32_t *d_holes = (int32_t *)q; q += al(b_holes);
  double *d_part = (double *)q; q += al(b_part);
  SegTree *d_segs = (SegTree *)q;
  TRY_HIP(hipMemcpyAsync(d_prims, geo->prims, b_prims, hipMemcpyHostToDevice, s), "copy prims");
  if (b_poly) TRY_HIP(hipMemcpyAsync(d_poly, geo->poly, b_poly, hipMemcpyHostToDevice, s), "copy poly");
  if (b_cent) TRY_HIP(hipMemcpyAsync(d_cent, sz->cent, b_cent, hipMemcpyHostToDevice, s), "copy cent");
  if (b_holes) TRY_HIP(hipMemcpyAsync(d_holes, sz->holes, b_holes, hipMemcpyHostToDevice, s), "copy holes");
  // segment loops: the candidate hierarchy over the grid's box and the loop's
  std::vector<SegTree> trees((size_t)geo->nprims);
  memset(trees.data(), 0, sizeof(SegTree) * trees.size());
  std::vector<void *> allocs;
  bool any_seg = false;
  const char *seg_err = nullptr;
  for (int k = 0; k < geo->nprims && !seg_err; k++) {
    const trime_prim &p = geo->prims[k];
    if (p.kind != TRIME_PRIM_SEGMENTS) continue;
    any_seg = true;
    double bx0 = grid->x0, by0 = grid->y0;
    double bx1 = grid->x0 + (grid->nx - 1) * grid->dx, by1 = grid->y0 + (grid->ny - 1) * grid->dy;
    for (int i = 0; i < p.nv; i++) {
      const double *v = geo->poly + 2 * (size_t)(p.voff + i);
      bx0 = fmin(bx0, v[0]);
      by0 = fmin(by0, v[1]);
      bx1 = fmax(bx1, v[0]);
      by1 = fmax(by1, v[1]);
    }
    seg_err = seg_tree_build(d_poly + 2 * (size_t)p.voff, p.nv, bx0, by0, bx1, by1,
                             8.0 * fmax(grid->dx, grid->dy), &trees[k], allocs, s);
  }
  if (!seg_err && any_seg &&
      (hipMemcpyAsync(d_segs, trees.data(), b_segs, hipMemcpyHostToDevice, s) != hipSuccess ||
       hipStreamSynchronize(s) != hipSuccess))
    seg_err = "copy segment trees";
  LfsField auto_field;
  memset(&auto_field, 0, sizeof auto_field);
  std::vector<double> S;
  if (!seg_err && sz->kind == TRIME_SZ_AUTO) {
    const AutoSetup A = auto_setup(sz, grid);
    S = trim_boundary(geo, A.d_s, A.geps, boundary_points(geo, A.d_s, A.geps));
    const int64_t ns = (int64_t)S.size() / 2;
    double *d_S = nullptr, *d_med = nullptr, *d_lfs = nullptr;
    uint8_t *d_keep = nullptr;
    if (ns >= ((int64_t)1 << 30) ||
        hipMallocAsync((void **)&d_S, sizeof(double) * S.size(), s) != hipSuccess ||
        hipMallocAsync((void **)&d_med, sizeof(double) * 4 * (size_t)ns, s) != hipSuccess ||
        hipMallocAsync((void **)&d_keep, 2 * (size_t)ns, s) != hipSuccess ||
        hipMallocAsync((void **)&d_lfs, sizeof(double) * (size_t)ns, s) != hipSuccess) {
      seg_err = "automatic sizing: allocation";
    } else {
      for (void *a : {(void *)d_S, (void *)d_med, (void *)d_keep, (void *)d_lfs}) allocs.push_back(a);
      int64_t nm = 0;
      if (hipMemcpyAsync(d_S, S.data(), sizeof(double) * S.size(), hipMemcpyHostToDevice, s) != hipSuccess)
        seg_err = "automatic sizing: copy the boundary points";
      else
        seg_err = auto_sizing_build(d_S, ns, A.box, A.gbox, A.r_nei, A.n_thres, sz->a0,
                                    8.0 * fmax(grid->dx, grid->dy), d_med, d_keep, d_lfs, &nm, &auto_field, allocs,
                                    s);
    }
  }
  if (seg_err) {
    for (void *a : allocs) (void)hipFreeAsync(a, s);
    (void)hipFreeAsync(buf, s);
    (void)hipGetLastError();
    return fail(TRIME_EINVAL, seg_err);
  }
  GridPrims g;
  g.nprims = geo->nprims;
  g.prims = d_prims;
  g.poly = d_poly;
  g.segs = d_segs;
  g.auto_mu = auto_field;
  g.sz = *sz;
  g.cent = d_cent;
  g.holes = d_holes;
  g.nx = grid->nx;
  g.ny = grid->ny;
  g.x0 = grid->x0;
  g.y0 = grid->y0;
  g.dx = grid->dx;
  g.dy = grid->dy;
  g.n_total = n_total;
  launch_grid_build(g, grid->dtype_bytes, d_sdf, d_mu, d_cat, d_hcell, d_scal, d_part, s);
  trime_status st = check_hip("trime_sdf_grid_build: launch");
  for (void *a : allocs) (void)hipFreeAsync(a, s);
  (void)hipFreeAsync(buf, s);
  return st;
}

// ------------------------------------------- grid build without allocation --
//
// The scratch of trime_sdf_grid_build_noalloc: the primitive list, polygon
// vertices, density centres and hole indices copied from the host, and the
// per-block partial sums of H (written before they are read), in one device
// array of fixed size.  Each GPU the library runs on holds its own copy until
// the process ends; every call on a GPU shares it, so calls that overlap on
// one GPU race.  Host code uses the address hipGetSymbolAddress gives on
// each device, never the array's name (a host-side stand-in).
constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)6 << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];
constexpr int NOALLOC_MAX_DEVICES = 64;
static void *g_scratch_ptr[NOALLOC_MAX_DEVICES];
static std::mutex g_scratch_mu;

// The scratch's device address on the current device, looked up once per
// device, with that device current.
static trime_status noalloc_scratch(void **out) {
  int dev = -1;
  TRY_HIP(hipGetDevice(&dev), "trime_sdf_grid_build_noalloc: hipGetDevice");
  if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
    return fail(TRIME_EUNSUPPORTED, "trime_sdf_grid_build_noalloc: device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *p = nullptr;
    TRY_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)), "trime_sdf_grid_build_noalloc: hipGetSymbolAddress");
    if (!p) return fail(TRIME_EHIP, "trime_sdf_grid_build_noalloc: no scratch address");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TRIME_OK;
}

trime_status trime_sdf_grid_build_noalloc(const trime_geometry *geo, const trime_sizing *sz,
                                          const trime_grid *grid, int64_t n_total, void *d_sdf, void *d_mu,
                                          uint8_t *d_cat, float *d_hcell, trime_grid_scalars *d_scal,
                                          void *stream) {
  trime_status e = grid_build_ok(geo, sz, grid, n_total, d_sdf, d_mu, d_cat, d_hcell, d_scal);
  if (e) return e;
  for (int k = 0; k < geo->nprims; k++)
    if (geo->prims[k].kind == TRIME_PRIM_SEGMENTS)
      return fail(TRIME_EUNSUPPORTED,
                  "trime_sdf_grid_build_noalloc: segment loops need candidate lists (trime_sdf_grid_build)");
  if (sz->kind == TRIME_SZ_AUTO)
    return fail(TRIME_EUNSUPPORTED,
                "trime_sdf_grid_build_noalloc: automatic sizing needs scratch of its own (trime_sdf_grid_build)");
  auto al = [](size_t v) { return (v + 255) & ~(size_t)255; };
  const size_t b_prims = sizeof(trime_prim) * (size_t)geo->nprims;
  const size_t b_poly = sizeof(double) * 2 * (size_t)(geo->npoly > 0 ? geo->npoly : 0);
  const size_t b_cent = sizeof(double) * 2 * (size_t)(sz->kind == TRIME_SZ_GAUSS_RHO ? sz->ncent : 0);
  const size_t b_holes = sizeof(int32_t) * (size_t)(sz->kind == TRIME_SZ_HOLE_RAMP ? sz->nholes : 0);
  const size_t b_part = sizeof(double) * 2 * (size_t)grid_partials(grid->nx, grid->ny);
  const size_t total = al(b_prims) + al(b_poly) + al(b_cent) + al(b_holes) + al(b_part);
  if (total > NOALLOC_SCRATCH_BYTES) {
    snprintf(g_err, sizeof g_err,
             "trime_sdf_grid_build_noalloc: needs %zu bytes of scratch, %zu available (fewer primitives or "
             "vertices, or a grid of fewer cells)",
             total, NOALLOC_SCRATCH_BYTES);
    return TRIME_ECAPACITY;
  }
  void *base = nullptr;
  e = noalloc_scratch(&base);
  if (e) return e;
  hipStream_t s = (hipStream_t)stream;
  char *q = (char *)base;
  trime_prim *d_prims = (trime_prim *)q; q += al(b_prims);
  double *d_poly = (double *)q; q += al(b_poly);
  double *d_cent = (double *)q; q += al(b_cent);
  int32_t *d_holes = (int32_t *)q; q += al(b_holes);
  double *d_part = (double *)q;
  TRY_HIP(hipMemcpyAsync(d_prims, geo->prims, b_prims, hipMemcpyHostToDevice, s), "copy prims");
  if (b_poly) TRY_HIP(hipMemcpyAsync(d_poly, geo->poly, b_poly, hipMemcpyHostToDevice, s), "copy poly");
  if (b_cent) TRY_HIP(hipMemcpyAsync(d_cent, sz->cent, b_cent, hipMemcpyHostToDevice, s), "copy cent");
  if (b_holes) TRY_HIP(hipMemcpyAsync(d_holes, sz->holes, b_holes, hipMemcpyHostToDevice, s), "copy holes");
  GridPrims g;
  memset(&g, 0, sizeof g);
  g.nprims = geo->nprims;
  g.prims = d_prims;
  g.poly = d_poly;
  g.segs = nullptr;
  g.sz = *sz;
  g.cent = d_cent;
  g.holes = d_holes;
  g.nx = grid->nx;
  g.ny = grid->ny;
  g.x0 = grid->x0;
  g.y0 = grid->y0;
  g.dx = grid->dx;
  g.dy = grid->dy;
  g.n_total = n_total;
  launch_grid_build(g, grid->dtype_bytes, d_sdf, d_mu, d_cat, d_hcell, d_scal, d_part, s);
  return check_hip("trime_sdf_grid_build_noalloc: launch");
}

// ------------------------------------------------------------ workspace --

static int64_t defaults_deg(const trime_state *st) { return st->max_deg > 0 ? st->max_deg : 16; }

static trime_status bin_geometry(trime_state *st, void *stream) {
  if (st->area_sel <= 0) {
    trime_grid_scalars h;
    TRY_HIP(hipMemcpyAsync(&h, st->scal, sizeof h, hipMemcpyDeviceToHost, (hipStream_t)stream),
            "read grid scalars");
    TRY_HIP(hipStreamSynchronize((hipStream_t)stream), "read grid scalars (sync)");
    st->area_sel = h.area_sel;
  }
  const trime_grid &g = st->grid;
  double W = (g.nx - 1) * g.dx, H = (g.ny - 1) * g.dy;
  double dens = st->bin_density > 0 ? st->bin_density : 3.3;
  double area = st->area_sel > 0 ? st->area_sel : W * H;
  double bw = sqrt(dens * area / (double)st->n);
  if (!(bw > 0)) bw = fmax(W, H);
  int nbx = (int)ceil(W / bw), nby = (int)ceil(H / bw);
  nbx = nbx < 1 ? 1 : nbx;
  nby = nby < 1 ? 1 : nby;
  int lb = 0;
  while ((1 << lb) < nbx || (1 << lb) < nby) lb++;
  if (lb > 15) return fail(TRIME_EUNSUPPORTED, "bin grid wider than 32768 bins");
  st->bw = bw;
  st->nbx = nbx;
  st->nby = nby;
  st->lbits = lb;
  st->nkeys = (int64_t)1 << (2 * lb);
  st->bx0 = g.x0;
  st->by0 = g.y0;
  return TRIME_OK;
}

// The bin keys of the capacity n_cap (more points, smaller bins, more keys).
static trime_status cap_geometry(trime_state *st) {
  st->nkeys_cap = st->nkeys;
  if (st->n_cap > st->n) {
    trime_state t = *st;
    t.n = st->n_cap;
    trime_status e = bin_geometry(&t, nullptr);  // area_sel is known by now
    if (e) return e;
    st->nkeys_cap = t.nkeys > st->nkeys ? t.nkeys : st->nkeys;
  }
  return TRIME_OK;
}

// The int32 queue: the FP64 replay, exact and deferred-centroid queues
// (3 (n + 1) + CQ_STRIDE n), and room for the point-addition selection.
static int64_t queue_ints(int64_t n) { return 3 * (n + 1) + (int64_t)CQ_STRIDE * n + 512; }

struct Layout {
  size_t off = 0;
  char *base;
  template <class T> T *take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T *p = base ? (T *)(base + off) : nullptr;
    off += sizeof(T) * count;
    return p;
  }
};

// Sizes follow the capacity n_cap (points that trime_add_points may add)
// and the bin keys of that many points.
static void layout(trime_state *st, Layout &L) {
  const int64_t n = st->n_cap > st->n ? st->n_cap : st->n;
  const int64_t nkeys = st->nkeys_cap > st->nkeys ? st->nkeys_cap : st->nkeys;
  int64_t md = defaults_deg(st);
  for (int b = 0; b < 2; b++) {
    st->pos[b].x = L.take<double>(n);
    st->pos[b].y = L.take<double>(n);
    st->pos[b].dprev = L.take<double>(n);
    st->pos[b].cat = L.take<uint8_t>(n);
    st->ord[b].id = L.take<int32_t>(n);
    st->ord[b].span = L.take<float>(n);
    st->ord[b].xl = L.take<double>(n);
    st->ord[b].yl = L.take<double>(n);
  }
  st->adj = L.take<int32_t>(md * n);
  st->deg = L.take<int32_t>(n);
  st->tri = L.take<int32_t>(3 * TRIME_TRI_PER_POINT * n);
  st->tri_valid = L.take<uint8_t>(TRIME_TRI_PER_POINT * n);
  st->tri_n = L.take<int32_t>(n + 1);
  st->perm = L.take<int32_t>(n + 1);
  st->key = L.take<int32_t>(n);
  st->rank = L.take<int32_t>(n);
  st->order = L.take<int32_t>(n);
  st->bin_start = L.take<int32_t>(nkeys + 1);
  st->bin_fill = L.take<int32_t>(nkeys);
  int64_t scan_n = nkeys > n ? nkeys : n;
  st->scan_tmp = L.take<int32_t>(scan_tmp_ints(scan_n) + 1);
  // FP64 replay queue, exact queue, deferred-centroid queue and its cells
  st->queue = L.take<int32_t>(queue_ints(n));
  st->counters = L.take<int32_t>(CNT_NCOUNTERS);
  for (int b = 0; b < 2; b++) {
    st->warm_n[b] = L.take<int32_t>(n);
    st->warm_nb[b] = L.take<int32_t>((size_t)TRIME_WARM * n);
  }
  st->old_slot = L.take<int32_t>(n);
  st->new_slot = L.take<int32_t>(n);
  int64_t np = dm_partials(n);
  st->partials = L.take<double>(2 * (np > 1 ? np : 1));
  st->stats = L.take<trime_stats>(1);
}

// h of the grid is read times sqrt(n_grid / n) with n points in the mesh
// (Sec. 3.7: the desired edge length of N points goes as 1/sqrt(N)).
static double h_scale_of(const trime_state *st, int64_t n) {
  const int64_t ng = st->n_grid > 0 ? st->n_grid : n;
  return ng == n ? 1.0 : sqrt((double)ng / (double)n);
}

static trime_status state_ok(const trime_state *st) {
  if (!st || st->n <= 0 || st->n > (int64_t)1 << 30) return fail(TRIME_EINVAL, "state: bad n");
  if (st->n_cap != 0 && (st->n_cap < st->n || st->n_cap > (int64_t)1 << 30))
    return fail(TRIME_EINVAL, "state: n_cap must be 0 or in [n, 2^30]");
  if (st->n_grid < 0 || st->n_grid > (int64_t)1 << 40) return fail(TRIME_EINVAL, "state: bad n_grid");
  if (st->precision != TRIME_FP64 && st->precision != TRIME_FP32)
    return fail(TRIME_EINVAL, "state: bad precision");
  if (!grid_ok(&st->grid)) return fail(TRIME_EINVAL, "state: bad grid");
  if (!st->sdf || !st->mu || !st->cat_grid || !st->hcell || !st->scal)
    return fail(TRIME_EINVAL, "state: grid arrays missing");
  if (st->max_deg < 0 || st->max_deg > 64) return fail(TRIME_EINVAL, "state: max_deg out of range");
  if (st->xcd_run < 0 || st->xcd_run > 256) return fail(TRIME_EINVAL, "state: xcd_run outside [0, 256]");
  return TRIME_OK;
}

trime_status trime_state_workspace_bytes(const trime_state *st_in, size_t *bytes) {
  trime_status e = state_ok(st_in);
  if (e) return e;
  if (!bytes) return fail(TRIME_EINVAL, "trime_state_workspace_bytes: null bytes");
  trime_state st = *st_in;
  e = bin_geometry(&st, 0);
  if (e) return e;
  e = cap_geometry(&st);
  if (e) return e;
  Layout L;
  L.base = nullptr;
  layout(&st, L);
  *bytes = (L.off + 255) & ~(size_t)255;
  return TRIME_OK;
}

trime_status trime_state_bind(trime_state *st, void *d_ws, size_t bytes, void *stream) {
  trime_status e = state_ok(st);
  if (e) return e;
  if (!d_ws) return fail(TRIME_EINVAL, "trime_state_bind: null workspace");
  if (((uintptr_t)d_ws) & 255) return fail(TRIME_EINVAL, "trime_state_bind: workspace not 256-aligned");
  e = bin_geometry(st, stream);
  if (e) return e;
  e = cap_geometry(st);
  if (e) return e;
  Layout probe;
  probe.base = nullptr;
  trime_state tmp = *st;
  layout(&tmp, probe);
  if (probe.off > bytes) return fail(TRIME_ECAPACITY, "trime_state_bind: workspace too small");
  Layout L;
  L.base = (char *)d_ws;
  layout(st, L);
  if (st->max_deg <= 0) st->max_deg = 16;
  st->cur_pos = 0;
  st->cur_ord = 0;
  if (st->n_grid == 0) st->n_grid = st->n;
  st->h_scale = h_scale_of(st, st->n);
  return TRIME_OK;
}

// Kernel arguments with the current buffers (cur) and the next position
// buffers (the other set).
static KArgs make_args(const trime_state *st) {
  KArgs a;
  memset(&a, 0, sizeof a);
  const trime_posbuf &P = st->pos[st->cur_pos], &Q = st->pos[st->cur_pos ^ 1];
  const trime_ordbuf &O = st->ord[st->cur_ord];
  a.n = st->n;
  a.x = P.x;
  a.y = P.y;
  a.dprev = P.dprev;
  a.cat = P.cat;
  a.xn = Q.x;
  a.yn = Q.y;
  a.dprevn = Q.dprev;
  a.catn = Q.cat;
  a.xl = O.xl;
  a.yl = O.yl;
  a.span = O.span;
  a.id = O.id;
  a.perm = st->perm;
  a.key = st->key;
  a.rank = st->rank;
  a.order = st->order;
  a.bin_start = st->bin_start;
  a.bin_fill = st->bin_fill;
  a.nbx = st->nbx;
  a.nby = st->nby;
  a.lbits = st->lbits;
  a.bx0 = st->bx0;
  a.by0 = st->by0;
  a.bw = st->bw;
  a.inv_bw = 1.0 / st->bw;
  const trime_grid &g = st->grid;
  a.nx = g.nx;
  a.ny = g.ny;
  a.gx0 = g.x0;
  a.gy0 = g.y0;
  a.gdx = g.dx;
  a.gdy = g.dy;
  a.inv_dx = 1.0 / g.dx;
  a.inv_dy = 1.0 / g.dy;
  a.box_x0 = g.x0;
  a.box_y0 = g.y0;
  a.box_x1 = g.x0 + (g.nx - 1) * g.dx;
  a.box_y1 = g.y0 + (g.ny - 1) * g.dy;
  a.sdf = st->sdf;
  a.mu = st->mu;
  a.cgrid = st->cat_grid;
  a.hcell = st->hcell;
  a.scal = st->scal;
  a.max_deg = st->max_deg > 0 ? st->max_deg : 16;
  a.adj = st->adj;
  a.deg = st->deg;
  a.tri = st->tri;
  a.tri_valid = st->tri_valid;
  a.tri_n = st->tri_n;
  a.queue = st->queue;
  a.queue2 = st->queue + st->n + 1;
  a.queue3 = st->queue + 2 * (st->n + 1);
  a.cq_cons = st->queue + 3 * (st->n + 1);
  a.counters = st->counters;
  a.partials = st->partials;
  a.stats = st->stats;
  a.prm = st->params;
  a.h_scale = st->h_scale > 0 ? st->h_scale : 1.0;
  a.warm_n = st->warm_n[st->cur_ord];
  a.warm_nb = st->warm_nb[st->cur_ord];
  a.warm_n_prev = st->warm_n[st->cur_ord ^ 1];
  a.warm_nb_prev = st->warm_nb[st->cur_ord ^ 1];
  a.old_slot = st->old_slot;
  a.new_slot = st->new_slot;
  a.xcd_run = st->xcd_run > 0 ? st->xcd_run : 8;
  a.precision = st->precision;
  a.ev0 = st->ev_cells[0];
  a.ev1 = st->ev_cells[1];
  return a;
}

static trime_status bound_ok(const trime_state *st) {
  if (!st || !st->stats || !st->pos[0].x) return fail(TRIME_EINVAL, "state not bound");
  return state_ok(st);
}

trime_status trime_state_load(trime_state *st, const double *d_x, const double *d_y, void *stream) {
  trime_status e = bound_ok(st);
  if (e) return e;
  if (!d_x || !d_y) return fail(TRIME_EINVAL, "trime_state_load: null positions");
  hipStream_t s = (hipStream_t)stream;
  st->cur_pos = 0;
  st->cur_ord = 0;
  KArgs a = make_args(st);
  LoadArgs l;
  l.xin = d_x;
  l.yin = d_y;
  l.x = st->pos[0].x;
  l.y = st->pos[0].y;
  l.dprev = st->pos[0].dprev;
  l.cat = st->pos[0].cat;
  l.id = st->ord[0].id;
  l.span = st->ord[0].span;
  l.xl = st->ord[0].xl;
  l.yl = st->ord[0].yl;
  launch_stats_reset(a, 1, s);
  launch_load(a, l, st->grid.dtype_bytes, s);
  launch_fill_i32(st->deg, st->n, 0, s);
  launch_fill_i32(st->tri_n, st->n, 0, s);
  const int64_t ncap = st->n_cap > st->n ? st->n_cap : st->n;
  launch_fill_i32(st->warm_n[0], ncap, 0, s);
  launch_fill_i32(st->warm_n[1], ncap, 0, s);
  launch_iota_i32(st->old_slot, ncap, s);
  launch_iota_i32(st->new_slot, ncap, s);
  return check_hip("trime_state_load");
}

// Binning; with cond set it runs only if *cond != 0 on the device (else the
// buffer sets are copied in place order), and the host-side swap of the
// buffer sets is the same either way.  reset >= 0 also clears the stats for
// the pass that follows (launch_stats_reset's full flag).
static void bin_points(trime_state *st, hipStream_t s, const int32_t *cond, int32_t reset = -1) {
  KArgs a = make_args(st);
  a.cond = cond;
  GatherArgs g;
  const trime_posbuf &P = st->pos[st->cur_pos], &Q = st->pos[st->cur_pos ^ 1];
  const trime_ordbuf &O = st->ord[st->cur_ord], &R = st->ord[st->cur_ord ^ 1];
  g.x = P.x;
  g.y = P.y;
  g.dprev = P.dprev;
  g.cat = P.cat;
  g.id = O.id;
  g.xo = Q.x;
  g.yo = Q.y;
  g.dprevo = Q.dprev;
  g.cato = Q.cat;
  g.ido = R.id;
  g.spano = R.span;
  g.xlo = R.xl;
  g.ylo = R.yl;
  g.xl = O.xl;
  g.yl = O.yl;
  g.span = O.span;
  launch_bin(a, g, st->nkeys, st->scan_tmp, s, reset);
  st->cur_pos ^= 1;
  st->cur_ord ^= 1;
}

trime_status trime_bin_points(trime_state *st, void *stream) {
  trime_status e = bound_ok(st);
  if (e) return e;
  bin_points(st, (hipStream_t)stream, nullptr);
  return check_hip("trime_bin_points");
}

trime_status trime_voronoi_cells(trime_state *st, const trime_cells *out, void *stream) {
  trime_status e = bound_ok(st);
  if (e) return e;
  if (!out || !out->cons || !out->ncons || out->cap <= 0)
    return fail(TRIME_EINVAL, "trime_voronoi_cells: bad output");
  hipStream_t s = (hipStream_t)stream;
  KArgs a = make_args(st);
  a.cell_cons = out->cons;
  a.cell_n = out->ncons;
  a.cell_cap = out->cap;
  launch_fill_i32(st->counters, CNT_NCOUNTERS, 0, s);
  launch_cells(a, MODE_CELLS, st->grid.dtype_bytes, s);
  return check_hip("trime_voronoi_cells");
}

static void extract(trime_state *st, hipStream_t s, const int32_t *cond = nullptr) {
  KArgs a = make_args(st);
  a.cond = cond;
  launch_stats_reset(a, 0, s);
  launch_cells(a, MODE_EXTRACT, st->grid.dtype_bytes, s);
  launch_finish_extract(a, s);
}

trime_status trime_delaunay_extract(trime_state *st, void *stream) {
  trime_status e = bound_ok(st);
  if (e) return e;
  extract(st, (hipStream_t)stream);
  return check_hip("trime_delaunay_extract");
}

trime_status trime_step_dm(trime_state *st, int32_t n_iter, int32_t fresh, int32_t always,
                           void *stream) {
  trime_status e = bound_ok(st);
  if (e) return e;
  if (n_iter < 0) return fail(TRIME_EINVAL, "trime_step_dm: negative iteration count");
  hipStream_t s = (hipStream_t)stream;
  // the re-triangulation decision stays on the device: binning and
  // extraction run every iteration and do their work only when the flag
  // (set by the previous iteration's large-movement test) is raised
  const int32_t *flag = &st->stats->retri_flag;
  for (int it = 0; it < n_iter; it++) {
    if (always || (it == 0 && fresh)) launch_set_flag(make_args(st), s);
    bin_points(st, s, flag);
    extract(st, s, flag);
    KArgs a = make_args(st);
    launch_dm(a, st->grid.dtype_bytes, s);
    st->cur_pos ^= 1;
    e = check_hip("trime_step_dm");
    if (e) return e;
  }
  return TRIME_OK;
}

trime_status trime_step_cvd(trime_state *st, int32_t n_iter, void *stream) {
  trime_status e = bound_ok(st);
  if (e) return e;
  if (n_iter < 0) return fail(TRIME_EINVAL, "trime_step_cvd: negative iteration count");
  hipStream_t s = (hipStream_t)stream;
  for (int it = 0; it < n_iter; it++) {
    bin_points(st, s, nullptr, 0);  // with the stats reset of the CVD pass
    KArgs a = make_args(st);
    launch_cells(a, MODE_CVD, st->grid.dtype_bytes, s);
    launch_finish_extract(a, s);
    st->cur_pos ^= 1;
    e = check_hip("trime_step_cvd");
    if (e) return e;
  }
  return TRIME_OK;
}

trime_status trime_step_hybrid(trime_state *st, const trime_schedule *sch, void *stream) {
  trime_status e = bound_ok(st);
  if (e) return e;
  if (!sch || sch->nseg < 0 || (sch->nseg > 0 && (!sch->method || !sch->iters)))
    return fail(TRIME_EINVAL, "trime_step_hybrid: bad schedule");
  for (int k = 0; k < sch->nseg; k++) {
    if (sch->iters[k] < 0) return fail(TRIME_EINVAL, "trime_step_hybrid: negative count");
    if (sch->method[k] == TRIME_METHOD_DM)
      e = trime_step_dm(st, sch->iters[k], 1, 0, stream);
    else if (sch->method[k] == TRIME_METHOD_CVD)
      e = trime_step_cvd(st, sch->iters[k], stream);
    else
      return fail(TRIME_EUNSUPPORTED, "trime_step_hybrid: unknown method");
    if (e) return e;
  }
  return TRIME_OK;
}

static trime_status adapt_cfg_ok(const trime_adaptive *cfg, const char *who) {
  static thread_local char msg[128];
  const char *why = nullptr;
  if (!cfg)
    why = "null configuration";
  else if (cfg->mode != TRIME_ADAPT_DM && cfg->mode != TRIME_ADAPT_CVD && cfg->mode != TRIME_ADAPT_HYBRID)
    why = "unknown mode";
  else if (cfg->max_iter < 0)
    why = "negative iteration count";
  else if (!(cfg->t_quality >= 0.0) || !(cfg->t_amax >= 0.0) || !(cfg->t_switch >= 0.0))
    why = "thresholds must be >= 0";
  if (!why) return TRIME_OK;
  snprintf(msg, sizeof msg, "%s: %s", who, why);
  return fail(TRIME_EINVAL, msg);
}

// One iteration of an adaptive run: every group of kernels runs only when
// its gate is raised; the buffer swaps are the same whatever the gates say.
static void adapt_iteration(trime_state *st, const trime_adaptive *cfg, double t_add, hipStream_t s) {
  launch_adapt_pre(make_args(st), s);
  bin_points(st, s, adapt_gate(st, G_BIN));
  extract(st, s, adapt_gate(st, G_DMTRI));  // DistMesh, re-triangulating
  KArgs a = make_args(st);
  a.cond = adapt_gate(st, G_DMQ);  // DistMesh on the last triangulation: its quality now
  launch_quality(a, s);
  a.cond = adapt_gate(st, G_CVD);
  launch_stats_reset(a, 0, s);
  launch_cells(a, MODE_CVD, st->grid.dtype_bytes, s);
  launch_finish_extract(a, s);
  a.cond = adapt_gate(st, G_DM);
  launch_dm(a, st->grid.dtype_bytes, s);
  a.cond = nullptr;
  launch_adapt_end(a, cfg->mode == TRIME_ADAPT_HYBRID, cfg->t_quality, cfg->t_amax, cfg->t_switch, t_add, s);
  st->cur_pos ^= 1;
}

trime_status trime_step_adaptive(trime_state *st, const trime_adaptive *cfg, void *stream) {
  trime_status e = bound_ok(st);
  if (e) return e;
  e = adapt_cfg_ok(cfg, "trime_step_adaptive");
  if (e) return e;
  hipStream_t s = (hipStream_t)stream;
  launch_adapt_init(make_args(st), cfg->mode == TRIME_ADAPT_CVD ? TRIME_METHOD_CVD : TRIME_METHOD_DM, s);
  for (int it = 0; it < cfg->max_iter; it++) {
    adapt_iteration(st, cfg, -1.0, s);
    e = check_hip("trime_step_adaptive");
    if (e) return e;
  }
  return TRIME_OK;
}

// ------------------------------------------------------ point addition --
//
// Scratch: the int32 queue holds the valid-triangle count per slot and its
// scan, the selected count per owner id and its scan, then the selection
// state; the selection keys overwrite the adjacency (rebuilt by the next
// triangulation, which an addition always forces).

static trime_status add_points(trime_state *st, int64_t n_add, int growing, hipStream_t s) {
  const int64_t n = st->n;
  const int64_t cap = st->n_cap > n ? st->n_cap : n;
  if (n_add < 0 || n + n_add > cap) return fail(TRIME_EINVAL, "trime_add_points: n + n_add exceeds n_cap");
  KArgs a = make_args(st);
  int32_t *cnt = st->queue, *off = cnt + (n + 1), *cnt_id = off + (n + 1), *base = cnt_id + (n + 1);
  void *sel = (void *)(st->queue + ((4 * (n + 1) + 63) & ~(int64_t)63));
  const int64_t sel_end = ((4 * (n + 1) + 63) & ~(int64_t)63) + (int64_t)((grow_sel_bytes() + 3) / 4);
  if (sel_end > queue_ints(cap)) return fail(TRIME_ECAPACITY, "trime_add_points: selection scratch too small");
  if (n_add > 0) {
    launch_grow_count(a, cnt, s);
    scan_i32(cnt, off, n, st->scan_tmp, s);
    int32_t nk = 0;
    TRY_HIP(hipMemcpyAsync(&nk, off + n, sizeof nk, hipMemcpyDeviceToHost, s), "read triangle count");
    TRY_HIP(hipStreamSynchronize(s), "read triangle count (sync)");
    if (n_add > nk) return fail(TRIME_EINVAL, "trime_add_points: more points than valid triangles");
    const int64_t key_cap = (int64_t)defaults_deg(st) * cap * 4 / (int64_t)grow_key_bytes();
    if (nk > key_cap) return fail(TRIME_ECAPACITY, "trime_add_points: too many triangles for the key buffer");
    launch_grow_select(a, off, st->adj, nk, sel, n_add, s);
    launch_grow_mark(a, sel, cnt_id, s);
    scan_i32(cnt_id, base, n, st->scan_tmp, s);
    st->h_scale = h_scale_of(st, n + n_add);
    KArgs b = make_args(st);  // new points: categories and spans at the new h
    const trime_posbuf &P = st->pos[st->cur_pos];
    const trime_ordbuf &O = st->ord[st->cur_ord];
    launch_grow_write(b, a.h_scale, st->grid.dtype_bytes, sel, base, P.x, P.y, P.dprev, P.cat, O.id, O.span, O.xl,
                      O.yl, s);
    st->n = n + n_add;
    trime_status e = bin_geometry(st, s);
    if (e) return e;
    if (st->nkeys > (st->nkeys_cap > 0 ? st->nkeys_cap : st->nkeys))
      return fail(TRIME_ECAPACITY, "trime_add_points: bin keys beyond the workspace");
  }
  launch_grow_state(make_args(st), growing, n_add > 0, s);
  TRY_HIP(hipStreamSynchronize(s), "trime_add_points (sync)");
  return check_hip("trime_add_points");
}

trime_status trime_add_points(trime_state *st, int64_t n_add, void *stream) {
  trime_status e = bound_ok(st);
  if (e) return e;
  if (n_add < 0 || n_add > (st->n_cap > st->n ? st->n_cap : st->n) - st->n)
    return fail(TRIME_EINVAL, "trime_add_points: n_add must be in [0, n_cap - n]");
  hipStream_t s = (hipStream_t)stream;
  trime_adapt_ctl c;
  TRY_HIP(hipMemcpyAsync(&c, &st->stats->adapt, sizeof c, hipMemcpyDeviceToHost, s), "read control block");
  TRY_HIP(hipStreamSynchronize(s), "read control block (sync)");
  return add_points(st, n_add, c.growing, s);
}

trime_status trime_run_growing(trime_state *st, const trime_growing *cfg, void *stream) {
  trime_status e = bound_ok(st);
  if (e) return e;
  if (!cfg) return fail(TRIME_EINVAL, "trime_run_growing: null configuration");
  e = adapt_cfg_ok(&cfg->base, "trime_run_growing");
  if (e) return e;
  const int64_t cap = st->n_cap > st->n ? st->n_cap : st->n;
  if (cfg->n_total < st->n || cfg->n_total > cap)
    return fail(TRIME_EINVAL, "trime_run_growing: n_total must be in [n, n_cap]");
  if (!(cfg->t_add >= 0.0) || !(cfg->fac_add > 0.0) || !isfinite(cfg->fac_add))
    return fail(TRIME_EINVAL, "trime_run_growing: t_add must be >= 0 and fac_add > 0");
  hipStream_t s = (hipStream_t)stream;
  const trime_adaptive *base = &cfg->base;
  launch_adapt_init(make_args(st), base->mode == TRIME_ADAPT_CVD ? TRIME_METHOD_CVD : TRIME_METHOD_DM, s);
  launch_grow_state(make_args(st), st->n < cfg->n_total, 0, s);
  for (int it = 0; it < base->max_iter; it++) {
    adapt_iteration(st, base, cfg->t_add, s);
    trime_adapt_ctl c;
    TRY_HIP(hipMemcpyAsync(&c, &st->stats->adapt, sizeof c, hipMemcpyDeviceToHost, s), "read control block");
    TRY_HIP(hipStreamSynchronize(s), "read control block (sync)");
    e = check_hip("trime_run_growing");
    if (e) return e;
    if (c.stopped) break;
    if (c.add_request) {
      int64_t n_add = (int64_t)floor(cfg->fac_add * (double)st->n);
      if (n_add > cfg->n_total - st->n) n_add = cfg->n_total - st->n;
      if (n_add <= 0) continue;
      const int64_t n_new = st->n + n_add;
      e = add_points(st, n_add, n_new < cfg->n_total, s);
      if (e) return e;
    }
  }
  return TRIME_OK;
}

trime_status trime_quality(trime_state *st, void *stream) {
  trime_status e = bound_ok(st);
  if (e) return e;
  launch_quality(make_args(st), (hipStream_t)stream);
  return check_hip("trime_quality");
}

trime_status trime_export_points(const trime_state *st, double *d_x, double *d_y, uint8_t *d_cat,
                                 void *stream) {
  trime_status e = bound_ok(st);
  if (e) return e;
  launch_export_points(make_args(st), d_x, d_y, d_cat, (hipStream_t)stream);
  return check_hip("trime_export_points");
}

trime_status trime_export_triangles(const trime_state *st, int32_t *d_tri, uint8_t *d_valid, int64_t cap,
                                    int64_t *d_count, void *stream) {
  trime_status e = bound_ok(st);
  if (e) return e;
  if (!d_tri || !d_valid || cap < 0) return fail(TRIME_EINVAL, "trime_export_triangles: bad output");
  // offsets go to the perm buffer (n + 1 ints), free outside a binning
  launch_export_tri(make_args(st), st->perm, st->scan_tmp, d_tri, d_valid, cap, d_count,
                    (hipStream_t)stream);
  return check_hip("trime_export_triangles");
}

trime_status trime_export_adjacency(const trime_state *st, int32_t *d_deg, int32_t *d_col, void *stream) {
  trime_status e = bound_ok(st);
  if (e) return e;
  if (!d_deg || !d_col) return fail(TRIME_EINVAL, "trime_export_adjacency: bad output");
  launch_export_adj(make_args(st), d_deg, d_col, (hipStream_t)stream);
  return check_hip("trime_export_adjacency");
}

trime_status trime_stats_read(const trime_state *st, trime_stats *host, void *stream) {
  if (!st || !st->stats || !host) return fail(TRIME_EINVAL, "trime_stats_read: null argument");
  TRY_HIP(hipMemcpyAsync(host, st->stats, sizeof *host, hipMemcpyDeviceToHost, (hipStream_t)stream),
          "trime_stats_read");
  TRY_HIP(hipStreamSynchronize((hipStream_t)stream), "trime_stats_read (sync)");
  quality_finish(host);
  return TRIME_OK;
}

struct trime_graph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int nside = 0;
  hipStream_t side[64] = {};
  hipEvent_t ev[65] = {};
};

trime_status trime_graph_destroy(trime_graph *g) {
  if (!g) return fail(TRIME_EINVAL, "trime_graph_destroy: null graph");
  if (g->exec) (void)hipGraphExecDestroy(g->exec);
  if (g->graph) (void)hipGraphDestroy(g->graph);
  for (int i = 0; i < g->nside; i++)
    if (g->side[i]) (void)hipStreamDestroy(g->side[i]);
  for (int i = 0; i < 65; i++)
    if (g->ev[i]) (void)hipEventDestroy(g->ev[i]);
  delete g;
  return TRIME_OK;
}

trime_status trime_batch_graph_create(trime_state *const *states, int32_t nstates, int32_t method,
                                      int32_t n_iter, int32_t nstreams, trime_graph **out, void *stream) {
  if (!states || nstates <= 0 || !out || !stream)
    return fail(TRIME_EINVAL, "trime_batch_graph_create: bad argument (the stream must not be null)");
  if (method != TRIME_METHOD_DM && method != TRIME_METHOD_CVD)
    return fail(TRIME_EINVAL, "trime_batch_graph_create: bad method");
  if (n_iter <= 0 || (n_iter & 1)) return fail(TRIME_EINVAL, "trime_batch_graph_create: n_iter must be even");
  if (nstreams < 1 || nstreams > 64) return fail(TRIME_EINVAL, "trime_batch_graph_create: 1 <= nstreams <= 64");
  for (int k = 0; k < nstates; k++) {
    trime_status e = bound_ok(states[k]);
    if (e) return e;
    if (states[k]->ev_cells[0] || states[k]->ev_cells[1])
      return fail(TRIME_EINVAL, "trime_batch_graph_create: a state requests timing events");
  }
  *out = nullptr;
  trime_graph *g = new (std::nothrow) trime_graph;
  if (!g) return fail(TRIME_EINVAL, "trime_batch_graph_create: out of host memory");
  hipStream_t cap = (hipStream_t)stream;
  trime_status e = TRIME_OK;
  g->nside = nstreams - 1;
  for (int i = 0; i < g->nside && !e; i++)
    if (hipStreamCreateWithFlags(&g->side[i], hipStreamNonBlocking) != hipSuccess)
      e = fail(TRIME_EHIP, "trime_batch_graph_create: stream");
  for (int i = 0; i < nstreams && !e; i++)
    if (hipEventCreateWithFlags(&g->ev[i], hipEventDisableTiming) != hipSuccess)
      e = fail(TRIME_EHIP, "trime_batch_graph_create: event");
  if (e) {
    trime_graph_destroy(g);
    return e;
  }
  if (hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal) != hipSuccess) {
    trime_graph_destroy(g);
    return fail(TRIME_EHIP, "trime_batch_graph_create: begin capture");
  }
  // fork: every side stream joins the capture after the first event
  if (hipEventRecord(g->ev[0], cap) != hipSuccess) e = fail(TRIME_EHIP, "trime_batch_graph_create: fork");
  for (int i = 0; i < g->nside && !e; i++)
    if (hipStreamWaitEvent(g->side[i], g->ev[0], 0) != hipSuccess) e = fail(TRIME_EHIP, "trime_batch_graph_create: fork");
  for (int k = 0; k < nstates && !e; k++) {
    int b = k % nstreams;
    void *s = b == 0 ? (void *)cap : (void *)g->side[b - 1];
    e = method == TRIME_METHOD_DM ? trime_step_dm(states[k], n_iter, 0, 0, s)
                                       : trime_step_cvd(states[k], n_iter, s);
  }
  // join: the capture stream waits for every side stream
  for (int i = 0; i < g->nside && !e; i++) {
    if (hipEventRecord(g->ev[i + 1], g->side[i]) != hipSuccess ||
        hipStreamWaitEvent(cap, g->ev[i + 1], 0) != hipSuccess)
      e = fail(TRIME_EHIP, "trime_batch_graph_create: join");
  }
  hipGraph_t graph = nullptr;
  hipError_t ec = hipStreamEndCapture(cap, &graph);
  g->graph = graph;
  if (!e && ec != hipSuccess) e = fail(TRIME_EHIP, "trime_batch_graph_create: end capture");
  if (!e && hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0) != hipSuccess)
    e = fail(TRIME_EHIP, "trime_batch_graph_create: instantiate");
  if (e) {
    trime_graph_destroy(g);
    return e;
  }
  *out = g;
  return TRIME_OK;
}

trime_status trime_graph_launch(trime_graph *g, void *stream) {
  if (!g || !g->exec) return fail(TRIME_EINVAL, "trime_graph_launch: null graph");
  TRY_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream), "trime_graph_launch");
  return TRIME_OK;
}

// ---- one launch per kernel for a batch of shapes ----
struct BatchLaunch {
  const void *fn;       // k_many<F>
  uint32_t total, block;
  const void *tab;      // per-shape arguments (device)
  const uint32_t *first;  // per-shape first block, ns + 1 (device)
};

struct trime_batch {
  int32_t ns = 0;
  std::vector<BatchLaunch> launches;
  void *mem = nullptr;  // one device allocation for every table
  // as recorded, per launch: kind, argument table offset and size, and the
  // grid of every shape ([launch][shape])
  std::vector<uint32_t> code, asz, grids;
  std::vector<size_t> off_tab;
  std::vector<trime_stats *> stats;  // per shape
  // persistent execution (trime_batch_make_persistent)
  bool persistent = false;
  uint32_t cells_code = 0, pgrid = 0;
  void *pmem = nullptr;
  PersistArgs pa = {};
  int32_t *pclear = nullptr;  // done[] and ctl[], cleared before each launch
  int64_t pclear_n = 0;
};

trime_status trime_batch_destroy(trime_batch *b) {
  if (!b) return TRIME_OK;
  if (b->mem) (void)hipFree(b->mem);
  if (b->pmem) (void)hipFree(b->pmem);
  delete b;
  return TRIME_OK;
}

trime_status trime_batch_create(trime_state *const *states, int32_t nstates, int32_t method, trime_batch **out) {
  if (!states || nstates <= 0 || !out) return fail(TRIME_EINVAL, "trime_batch_create: bad argument");
  if (method != TRIME_METHOD_DM && method != TRIME_METHOD_CVD && method != TRIME_METHOD_DM_ALWAYS)
    return fail(TRIME_EINVAL, "trime_batch_create: bad method");
  *out = nullptr;
  for (int k = 0; k < nstates; k++) {
    trime_status e = bound_ok(states[k]);
    if (e) return e;
    if (states[k]->ev_cells[0] || states[k]->ev_cells[1])
      return fail(TRIME_EINVAL, "trime_batch_create: a state requests timing events");
  }
  // record one period (two iterations) of every state; nothing is launched
  std::vector<std::vector<LaunchRec>> logs(nstates);
  for (int k = 0; k < nstates; k++) {
    g_launch_log = &logs[k];
    trime_status e = method == TRIME_METHOD_CVD ? trime_step_cvd(states[k], 2, nullptr)
                                                : trime_step_dm(states[k], 2, 0, method == TRIME_METHOD_DM_ALWAYS,
                                                                nullptr);
    g_launch_log = nullptr;
    if (e) return e;
  }
  const size_t m = logs[0].size();
  for (int k = 1; k < nstates; k++) {
    if (logs[k].size() != m) return fail(TRIME_EINVAL, "trime_batch_create: the states' kernel sequences differ");
    for (size_t i = 0; i < m; i++)
      if (logs[k][i].many != logs[0][i].many || logs[k][i].block != logs[0][i].block ||
          logs[k][i].args.size() != logs[0][i].args.size())
        return fail(TRIME_EINVAL, "trime_batch_create: the states' kernel sequences differ");
  }
  // layout: per launch, the argument table then the block offsets, each
  // 256-byte aligned, in one device allocation
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  std::vector<size_t> off_tab(m), off_first(m);
  size_t bytes = 0;
  for (size_t i = 0; i < m; i++) {
    off_tab[i] = bytes;
    bytes += up(logs[0][i].args.size() * (size_t)nstates);
    off_first[i] = bytes;
    bytes += up(sizeof(uint32_t) * ((size_t)nstates + 1));
  }
  std::vector<unsigned char> host(bytes, 0);
  trime_batch *b = new (std::nothrow) trime_batch;
  if (!b) return fail(TRIME_EINVAL, "trime_batch_create: out of host memory");
  b->ns = nstates;
  b->grids.resize(m * (size_t)nstates);
  for (int k = 0; k < nstates; k++) b->stats.push_back(states[k]->stats);
  for (size_t i = 0; i < m; i++) {
    const size_t asz = logs[0][i].args.size();
    uint32_t *first = (uint32_t *)&host[off_first[i]];
    uint64_t tot = 0;
    b->code.push_back(logs[0][i].code);
    b->asz.push_back((uint32_t)asz);
    b->off_tab.push_back(off_tab[i]);
    for (int k = 0; k < nstates; k++) {
      memcpy(&host[off_tab[i] + asz * (size_t)k], logs[k][i].args.data(), asz);
      first[k] = (uint32_t)tot;
      tot += logs[k][i].grid;
      b->grids[i * (size_t)nstates + k] = logs[k][i].grid;
    }
    if (tot > 0x7fffffffull) {
      trime_batch_destroy(b);
      return fail(TRIME_EINVAL, "trime_batch_create: batched grid too large");
    }
    first[nstates] = (uint32_t)tot;
    BatchLaunch L;
    L.fn = logs[0][i].many;
    L.total = (uint32_t)tot;
    L.block = logs[0][i].block;
    L.tab = nullptr;
    L.first = nullptr;
    b->launches.push_back(L);
  }
  if (hipMalloc(&b->mem, bytes ? bytes : 256) != hipSuccess) {
    b->mem = nullptr;
    trime_batch_destroy(b);
    return fail(TRIME_EHIP, "trime_batch_create: device allocation");
  }
  if (bytes && hipMemcpy(b->mem, host.data(), bytes, hipMemcpyHostToDevice) != hipSuccess) {
    trime_batch_destroy(b);
    return fail(TRIME_EHIP, "trime_batch_create: copy of the argument tables");
  }
  for (size_t i = 0; i < m; i++) {
    b->launches[i].tab = (const unsigned char *)b->mem + off_tab[i];
    b->launches[i].first = (const uint32_t *)((const unsigned char *)b->mem + off_first[i]);
  }
  *out = b;
  return TRIME_OK;
}

trime_status trime_batch_make_persistent(trime_batch *b, int32_t tiles_cells, int32_t tiles_other) {
#ifndef TRIME_PERSIST_ENABLE
  // switched off: on MI355X a launch of the persistent kernel has not
  // completed, its cause not yet found; the schedule and the kernels'
  // one-wavefront forms are checked by the CPU emulation of the library,
  // which builds with TRIME_PERSIST_ENABLE
  (void)b;
  (void)tiles_cells;
  (void)tiles_other;
  return fail(TRIME_EINVAL,
              "trime_batch_make_persistent: switched off (the persistent kernel has not completed on MI355X; "
              "build with TRIME_PERSIST_ENABLE to enable it)");
#endif
  if (!b) return fail(TRIME_EINVAL, "trime_batch_make_persistent: null batch");
  if (b->persistent) return fail(TRIME_EINVAL, "trime_batch_make_persistent: the batch is persistent already");
  if (tiles_cells < 1 || tiles_cells > 4096 || tiles_other < 1 || tiles_other > 4096)
    return fail(TRIME_EINVAL, "trime_batch_make_persistent: tiles per item must be in [1, 4096]");
  const size_t P = b->code.size(), ns = (size_t)b->ns;
  uint32_t cells = 0;
  for (uint32_t c : b->code)
    if ((c >> 8) == KF_CELLS) cells = c;
  if (!cells || !persist_supported(cells))
    return fail(TRIME_EINVAL, "trime_batch_make_persistent: no persistent kernel for this batch's cell kernel");
  for (uint32_t c : b->code)
    if (!c || !persist_runs(cells, c))
      return fail(TRIME_EINVAL, "trime_batch_make_persistent: a kernel of the batch has no wavefront form");
  // items: ceil(grid / chunk) per (phase, shape); shapes with more work first
  std::vector<uint32_t> chunk(P), items(P * ns);
  for (size_t p = 0; p < P; p++) {
    const uint32_t fam = b->code[p] >> 8;
    chunk[p] = fam == KF_CELLS ? (uint32_t)tiles_cells
                               : (fam == KF_POST || fam == KF_EXACT || fam == KF_DMREPLAY) ? 1u : (uint32_t)tiles_other;
    for (size_t s = 0; s < ns; s++) items[p * ns + s] = (b->grids[p * ns + s] + chunk[p] - 1) / chunk[p];
  }
  std::vector<uint64_t> work(ns, 0);
  for (size_t p = 0; p < P; p++)
    for (size_t s = 0; s < ns; s++) work[s] += b->grids[p * ns + s];
  std::vector<int32_t> order(ns);
  for (size_t s = 0; s < ns; s++) order[s] = (int32_t)s;
  std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return work[x] > work[y]; });
  std::vector<uint32_t> ph_first(P + 1), sh_first(P * (ns + 1)), need(P * ns), per_shape(ns, 0);
  uint64_t tot = 0;
  for (size_t p = 0; p < P; p++) {
    ph_first[p] = (uint32_t)tot;
    uint64_t in_phase = 0;
    for (size_t i = 0; i < ns; i++) {
      sh_first[p * (ns + 1) + i] = (uint32_t)in_phase;
      in_phase += items[p * ns + order[i]];
    }
    sh_first[p * (ns + 1) + ns] = (uint32_t)in_phase;
    for (size_t s = 0; s < ns; s++) {
      need[p * ns + s] = per_shape[s];
      per_shape[s] += items[p * ns + s];
    }
    tot += in_phase;
    if (tot > 0x7fffffffull) return fail(TRIME_EINVAL, "trime_batch_make_persistent: too many work items");
  }
  ph_first[P] = (uint32_t)tot;
  const uint32_t grid = persist_grid(cells);
  if (!grid) return fail(TRIME_EHIP, "trime_batch_make_persistent: occupancy query");
  int dev = 0, khz = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess ||
      khz <= 0)
    return fail(TRIME_EHIP, "trime_batch_make_persistent: wall clock rate");
  // one device allocation: tables, counters, the exact stage's polygons
  auto up = [](size_t v) { return (v + 255) & ~(size_t)255; };
  std::vector<uint64_t> ph_args(P);
  for (size_t p = 0; p < P; p++) ph_args[p] = b->off_tab[p];
  size_t off = 0;
  auto place = [&](size_t bytes) {
    size_t o = off;
    off += up(bytes);
    return o;
  };
  const size_t o_args = place(P * 8), o_asz = place(P * 4), o_code = place(P * 4), o_chunk = place(P * 4),
               o_phf = place((P + 1) * 4), o_shf = place(P * (ns + 1) * 4), o_grid = place(P * ns * 4),
               o_need = place(P * ns * 4), o_per = place(ns * 4), o_order = place(ns * 4),
               o_stats = place(ns * sizeof(trime_stats *)), o_clear = place((ns + 2) * PERSIST_LINE * 4);
  const size_t table_bytes = off;
  const size_t o_ws = place(persist_exact_slice() * (size_t)grid);
  std::vector<unsigned char> host(table_bytes, 0);
  memcpy(&host[o_args], ph_args.data(), P * 8);
  memcpy(&host[o_asz], b->asz.data(), P * 4);
  memcpy(&host[o_code], b->code.data(), P * 4);
  memcpy(&host[o_chunk], chunk.data(), P * 4);
  memcpy(&host[o_phf], ph_first.data(), (P + 1) * 4);
  memcpy(&host[o_shf], sh_first.data(), P * (ns + 1) * 4);
  memcpy(&host[o_grid], b->grids.data(), P * ns * 4);
  memcpy(&host[o_need], need.data(), P * ns * 4);
  memcpy(&host[o_per], per_shape.data(), ns * 4);
  memcpy(&host[o_order], order.data(), ns * 4);
  memcpy(&host[o_stats], b->stats.data(), ns * sizeof(trime_stats *));
  void *mem = nullptr;
  if (hipMalloc(&mem, off) != hipSuccess) return fail(TRIME_EHIP, "trime_batch_make_persistent: device allocation");
  if (hipMemcpy(mem, host.data(), table_bytes, hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(mem);
    return fail(TRIME_EHIP, "trime_batch_make_persistent: copy of the tables");
  }
  unsigned char *d = (unsigned char *)mem;
  PersistArgs &pa = b->pa;
  pa.args = (const unsigned char *)b->mem;
  pa.ph_args = (const uint64_t *)(d + o_args);
  pa.ph_asz = (const uint32_t *)(d + o_asz);
  pa.ph_code = (const uint32_t *)(d + o_code);
  pa.ph_chunk = (const uint32_t *)(d + o_chunk);
  pa.ph_first = (const uint32_t *)(d + o_phf);
  pa.sh_first = (const uint32_t *)(d + o_shf);
  pa.grid = (const uint32_t *)(d + o_grid);
  pa.need = (const uint32_t *)(d + o_need);
  pa.per_shape = (const uint32_t *)(d + o_per);
  pa.order = (const int32_t *)(d + o_order);
  pa.stats = (trime_stats *const *)(d + o_stats);
  pa.done = (uint32_t *)(d + o_clear);
  pa.ctl = pa.done + ns * PERSIST_LINE;
  pa.exact_ws = d + o_ws;
  pa.nphase = (uint32_t)P;
  pa.ns = (uint32_t)ns;
  pa.nper = (uint32_t)tot;
  pa.nperiods = 0;
  pa.zero = 0;
  pa.timeout = (uint64_t)khz * 1000ull * 20ull;  // 20 s
  b->pclear = (int32_t *)(d + o_clear);
  b->pclear_n = (int64_t)(ns + 2) * PERSIST_LINE;
  b->pmem = mem;
  b->cells_code = cells;
  b->pgrid = grid;
  b->persistent = true;
  return TRIME_OK;
}

trime_status trime_batch_run(trime_batch *b, int32_t n_iter, void *stream) {
  if (!b) return fail(TRIME_EINVAL, "trime_batch_run: null batch");
  if (n_iter < 0 || (n_iter & 1)) return fail(TRIME_EINVAL, "trime_batch_run: n_iter must be even and >= 0");
  hipStream_t s = (hipStream_t)stream;
  if (b->persistent) {
    if (n_iter == 0 || b->pa.nper == 0) return TRIME_OK;
    if ((uint64_t)b->pa.nper * (uint64_t)(n_iter / 2) > 0xffffffffull)
      return fail(TRIME_EINVAL, "trime_batch_run: too many work items for one launch (run fewer iterations)");
    PersistArgs pa = b->pa;
    pa.nperiods = (uint32_t)(n_iter / 2);
    launch_fill_i32(b->pclear, b->pclear_n, 0, s);
    launch_persist(b->cells_code, pa, b->pgrid, s);
    return check_hip("trime_batch_run");
  }
  for (int it = 0; it < n_iter; it += 2) {
    for (const BatchLaunch &L : b->launches) {
      if (!L.total) continue;
      const void *tab = L.tab;
      const uint32_t *first = L.first;
      int ns = b->ns;
      void *args[3] = {(void *)&tab, (void *)&first, (void *)&ns};
      if (hipLaunchKernel(L.fn, dim3(L.total), dim3(L.block), args, 0, s) != hipSuccess)
        return fail(TRIME_EHIP, "trime_batch_run: launch");
    }
  }
  return check_hip("trime_batch_run");
}

trime_status trime_autotune_workspace_bytes(const trime_state *st_in, const double *dens, int32_t nd,
                                            size_t *bytes) {
  if (!st_in || !dens || nd <= 0 || !bytes) return fail(TRIME_EINVAL, "trime_autotune_workspace_bytes: bad argument");
  size_t most = 0;
  for (int i = 0; i < nd; i++) {
    if (!(dens[i] > 0)) return fail(TRIME_EINVAL, "trime_autotune_workspace_bytes: density must be positive");
    trime_state st = *st_in;
    st.bin_density = dens[i];
    size_t b = 0;
    trime_status e = trime_state_workspace_bytes(&st, &b);
    if (e) return e;
    most = b > most ? b : most;
  }
  *bytes = most;
  return TRIME_OK;
}

trime_status trime_autotune(trime_state *st, void *d_ws, size_t bytes, const double *d_x, const double *d_y,
                            const double *dens, int32_t nd, const int32_t *runs, int32_t nr, int32_t n_iter,
                            double *best_density, int32_t *best_run, float *ms_out, void *stream) {
  if (!st || !d_ws || !d_x || !d_y || !dens || nd <= 0 || n_iter <= 0 || !best_density || nr < 0)
    return fail(TRIME_EINVAL, "trime_autotune: bad argument");
  const int32_t own = st->xcd_run;
  if (!runs || nr == 0) {
    runs = &own;
    nr = 1;
  }
  for (int j = 0; j < nr; j++)
    if (runs[j] < 0 || runs[j] > 256) return fail(TRIME_EINVAL, "trime_autotune: XCD run outside [0, 256]");
  size_t need = 0;
  trime_status e = trime_autotune_workspace_bytes(st, dens, nd, &need);
  if (e) return e;
  if (bytes < need) return fail(TRIME_ECAPACITY, "trime_autotune: workspace too small");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  TRY_HIP(hipEventCreate(&t0), "trime_autotune: event");
  if (hipEventCreate(&t1) != hipSuccess) {
    (void)hipEventDestroy(t0);
    return fail(TRIME_EHIP, "trime_autotune: event");
  }
  double best = dens[0];
  int32_t best_r = runs[0];
  float best_ms = INFINITY;
  for (int i = 0; i < nd && !e; i++) {
    st->bin_density = dens[i];
    e = trime_state_bind(st, d_ws, bytes, stream);
    for (int j = 0; j < nr && !e; j++) {
      st->xcd_run = runs[j];
      e = trime_state_load(st, d_x, d_y, stream);
      if (!e) e = trime_step_cvd(st, 1, stream);  // warm-up
      if (!e && hipEventRecord(t0, s) != hipSuccess) e = fail(TRIME_EHIP, "trime_autotune: record");
      if (!e) e = trime_step_cvd(st, n_iter, stream);
      if (!e && hipEventRecord(t1, s) != hipSuccess) e = fail(TRIME_EHIP, "trime_autotune: record");
      if (!e && hipEventSynchronize(t1) != hipSuccess) e = fail(TRIME_EHIP, "trime_autotune: sync");
      float ms = 0;
      if (!e && hipEventElapsedTime(&ms, t0, t1) != hipSuccess) e = fail(TRIME_EHIP, "trime_autotune: time");
      if (e) break;
      ms /= (float)n_iter;
      if (ms_out) ms_out[(size_t)i * nr + j] = ms;
      if (ms < best_ms) {
        best_ms = ms;
        best = dens[i];
        best_r = runs[j];
      }
    }
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (e) return e;
  st->bin_density = best;
  st->xcd_run = best_r;
  e = trime_state_bind(st, d_ws, bytes, stream);
  if (!e) e = trime_state_load(st, d_x, d_y, stream);
  if (e) return e;
  *best_density = best;
  if (best_run) *best_run = best_r;
  return TRIME_OK;
}

trime_status trime_stats_check(const trime_stats *h) {
  if (!h) return fail(TRIME_EINVAL, "trime_stats_check: null");
  if (h->error & (ERR_TRI_CAP | ERR_DEG_CAP | ERR_POLY_CAP | ERR_EXACT_CAP))
    return fail(TRIME_ECAPACITY, "a device capacity was exceeded (see stats.error)");
  if (h->empty_cells > 0) return fail(TRIME_EDEGENERATE, "coincident points (empty cells)");
  return TRIME_OK;
}


