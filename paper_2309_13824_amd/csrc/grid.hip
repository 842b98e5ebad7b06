// Geometry grid (Sec. 3.1-3.3, Sec. 3.7): the signed distance of a
// constructive geometry at the nodes (union = min, difference = max(a, -b),
// intersection = max), the sizing field mu (rho = mu^-2, Eq. 9), the cell
// categories (boundary iff |sdf(mid)| <= cell diagonal, else inner iff
// sdf(mid) < 0, else outer) and h_cell = mu_cell * H with
// H = sqrt(dx dy sum_sel mu_cell^-2 / N) over the selected cells (inner, and
// boundary cells with sdf(mid) <= 0.5 min(dx, dy)); h_avg is the mean h of
// the selected cells.  Midpoint values are the means of the 4 corner nodes.
//
// One thread per node.  A primitive whose distance bound cannot change the
// running value (a hole far from the node) is skipped, so hundreds of holes
// cost a few flops each.
#include "prim_sdf.hpp"
#include "segsdf_dev.hpp"

namespace trime {


// Signed distance of primitive k of the geometry.
TRIME_D double prim_sdf(const GridPrims &g, int k, double x, double y) {
  const trime_prim &pr = g.prims[k];
  if (pr.kind == TRIME_PRIM_SEGMENTS) return segments_sdf(g.segs[k], x, y);
  return analytic_sdf(pr, g.poly, x, y);
}

// A radius R and centre with |sdf| >= dist(x, c) - R outside the circle, for
// disks and ellipses; other primitives have no cheap bound (R < 0).
TRIME_D double prim_bound(const trime_prim &pr, double &cx, double &cy) {
  if (pr.kind == TRIME_PRIM_DISK) {
    cx = pr.p[0];
    cy = pr.p[1];
    return pr.p[2];
  }
  if (pr.kind == TRIME_PRIM_ELLIPSE) {
    cx = pr.p[0];
    cy = pr.p[1];
    return fmax(pr.p[2], pr.p[3]);
  }
  return -1.0;
}

TRIME_D double csg_sdf(const GridPrims &g, double x, double y) {
  double s = INFINITY;
  for (int k = 0; k < g.nprims; k++) {
    const trime_prim &pr = g.prims[k];
    double cx, cy, R = prim_bound(pr, cx, cy);
    if (R >= 0 && k > 0) {
      double dist = sqrt((x - cx) * (x - cx) + (y - cy) * (y - cy)) - R;
      // t >= dist (outside the bound circle)
      if (dist > 0) {
        if (pr.op == TRIME_OP_DIFF && -dist <= s) continue;
        if (pr.op == TRIME_OP_UNION && dist >= s) continue;
      }
    }
    double t = prim_sdf(g, k, x, y);
    switch (pr.op) {
      case TRIME_OP_INIT: s = t; break;
      case TRIME_OP_UNION: s = fmin(s, t); break;
      case TRIME_OP_DIFF: s = fmax(s, -t); break;
      default: s = fmax(s, t); break;
    }
  }
  return s;
}

TRIME_D double sizing_mu(const GridPrims &g, double x, double y, double sdf) {
  switch (g.sz.kind) {
    case TRIME_SZ_AUTO: return auto_mu(g.auto_mu, x, y);
    case TRIME_SZ_UNIFORM: return 1.0;
    case TRIME_SZ_ABS_SDF: return g.sz.a0 + g.sz.a1 * fabs(sdf);
    case TRIME_SZ_GAUSS_RHO: {
      double acc = 0.0;
      for (int k = 0; k < g.sz.ncent; k++) {
        double dx = x - g.cent[2 * k], dy = y - g.cent[2 * k + 1];
        acc += exp(-(dx * dx + dy * dy) / g.sz.s2);
      }
      return 1.0 / sqrt(g.sz.a0 + g.sz.a1 * acc);
    }
    default: {
      double dh = INFINITY;
      for (int k = 0; k < g.sz.nholes; k++) {
        const trime_prim &pr = g.prims[g.holes[k]];
        double cx, cy, R = prim_bound(pr, cx, cy);
        if (R >= 0) {
          double lb = sqrt((x - cx) * (x - cx) + (y - cy) * (y - cy)) - R;
          if (lb > dh) continue;
        }
        dh = fmin(dh, fabs(prim_sdf(g, g.holes[k], x, y)));
      }
      double r = fmin(dh / g.sz.a1, 1.0);
      return 1.0 + (g.sz.a0 - 1.0) * r;
    }
  }
}

template <class G> __global__ void k_grid_nodes(GridPrims g, G *sdf, G *mu) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t nn = (int64_t)g.nx * g.ny;
  if (k >= nn) return;
  int i = (int)(k % g.nx), j = (int)(k / g.nx);
  double x = g.x0 + i * g.dx, y = g.y0 + j * g.dy;
  double s = csg_sdf(g, x, y);
  sdf[k] = (G)s;
  mu[k] = (G)sizing_mu(g, x, y, s);
}

constexpr int GB = 256;

template <class G>
__global__ __launch_bounds__(GB) void k_grid_cells(GridPrims g, const G *sdf, const G *mu,
                                                   uint8_t *cat, double *part) {
  __shared__ double s1[GB], s2[GB];
  int64_t c = (int64_t)blockIdx.x * GB + threadIdx.x;
  int cxn = g.nx - 1;
  int64_t nc = (int64_t)cxn * (g.ny - 1);
  double rho = 0.0, cnt = 0.0;
  if (c < nc) {
    int i = (int)(c % cxn), j = (int)(c / cxn);
    int64_t n0 = (int64_t)j * g.nx + i;
    double sm = (((double)sdf[n0] + (double)sdf[n0 + 1]) + ((double)sdf[n0 + g.nx] + (double)sdf[n0 + g.nx + 1])) * 0.25;
    double ld = sqrt(g.dx * g.dx + g.dy * g.dy);
    uint8_t ct = fabs(sm) <= ld ? TRIME_CAT_BOUNDARY : (sm < 0 ? TRIME_CAT_INNER : TRIME_CAT_OUTER);
    cat[c] = ct;
    bool sel = ct == TRIME_CAT_INNER || (ct == TRIME_CAT_BOUNDARY && sm <= 0.5 * fmin(g.dx, g.dy));
    if (sel) {
      double mm = (((double)mu[n0] + (double)mu[n0 + 1]) + ((double)mu[n0 + g.nx] + (double)mu[n0 + g.nx + 1])) * 0.25;
      rho = 1.0 / (mm * mm);
      cnt = 1.0;
    }
  }
  s1[threadIdx.x] = rho;
  s2[threadIdx.x] = cnt;
  __syncthreads();
  for (int w = GB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1[0];
    part[2 * blockIdx.x + 1] = s2[0];
  }
}

__global__ __launch_bounds__(GB) void k_grid_reduce(GridPrims g, const double *part, int np,
                                                    trime_grid_scalars *scal, int stage) {
  __shared__ double s1[GB], s2[GB];
  double A = 0, B = 0;
  for (int q = threadIdx.x; q < np; q += GB) {
    A += part[2 * q];
    B += part[2 * q + 1];
  }
  s1[threadIdx.x] = A;
  s2[threadIdx.x] = B;
  __syncthreads();
  for (int w = GB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (stage == 0) {
      scal->H = sqrt(g.dx * g.dy * s1[0] / (double)g.n_total);
      scal->n_sel = (int64_t)s2[0];
      scal->area_sel = s2[0] * g.dx * g.dy;
    } else {
      scal->h_avg = s2[0] > 0 ? s1[0] / s2[0] : 0.0;
    }
  }
}

template <class G>
__global__ __launch_bounds__(GB) void k_grid_h(GridPrims g, const G *sdf, const G *mu,
                                               const uint8_t *cat, const trime_grid_scalars *scal,
                                               float *hcell, double *part) {
  __shared__ double s1[GB], s2[GB];
  int64_t c = (int64_t)blockIdx.x * GB + threadIdx.x;
  int cxn = g.nx - 1;
  int64_t nc = (int64_t)cxn * (g.ny - 1);
  double hs = 0.0, cnt = 0.0;
  if (c < nc) {
    int i = (int)(c % cxn), j = (int)(c / cxn);
    int64_t n0 = (int64_t)j * g.nx + i;
    double mm = (((double)mu[n0] + (double)mu[n0 + 1]) + ((double)mu[n0 + g.nx] + (double)mu[n0 + g.nx + 1])) * 0.25;
    float h = (float)(mm * scal->H);
    hcell[c] = h;
    uint8_t ct = cat[c];
    double sm = (((double)sdf[n0] + (double)sdf[n0 + 1]) + ((double)sdf[n0 + g.nx] + (double)sdf[n0 + g.nx + 1])) * 0.25;
    if (ct == TRIME_CAT_INNER || (ct == TRIME_CAT_BOUNDARY && sm <= 0.5 * fmin(g.dx, g.dy))) {
      hs = (double)h;
      cnt = 1.0;
    }
  }
  s1[threadIdx.x] = hs;
  s2[threadIdx.x] = cnt;
  __syncthreads();
  for (int w = GB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s1[0];
    part[2 * blockIdx.x + 1] = s2[0];
  }
}

template <class G>
static void grid_build_g(const GridPrims &g, void *sdf, void *mu, uint8_t *cat, float *hcell,
                         trime_grid_scalars *scal, double *part, hipStream_t s) {
  int64_t nn = (int64_t)g.nx * g.ny;
  int64_t nc = (int64_t)(g.nx - 1) * (g.ny - 1);
  int nbn = (int)((nn + 255) / 256);
  int nbc = (int)((nc + GB - 1) / GB);
  hipLaunchKernelGGL(k_grid_nodes<G>, dim3(nbn), dim3(256), 0, s, g, (G *)sdf, (G *)mu);
  hipLaunchKernelGGL(k_grid_cells<G>, dim3(nbc), dim3(GB), 0, s, g, (const G *)sdf, (const G *)mu, cat, part);
  hipLaunchKernelGGL(k_grid_reduce, dim3(1), dim3(GB), 0, s, g, part, nbc, scal, 0);
  hipLaunchKernelGGL(k_grid_h<G>, dim3(nbc), dim3(GB), 0, s, g, (const G *)sdf, (const G *)mu, cat, scal, hcell, part);
  hipLaunchKernelGGL(k_grid_reduce, dim3(1), dim3(GB), 0, s, g, part, nbc, scal, 1);
}

int64_t grid_partials(int nx, int ny) { return ((int64_t)(nx - 1) * (ny - 1) + GB - 1) / GB; }

void launch_grid_build(const GridPrims &g, int dtype_bytes, void *sdf, void *mu, uint8_t *cat,
                       float *hcell, trime_grid_scalars *scal, double *part, hipStream_t s) {
  if (dtype_bytes == 4)
    grid_build_g<float>(g, sdf, mu, cat, hcell, scal, part, s);
  else
    grid_build_g<double>(g, sdf, mu, cat, hcell, scal, part, s);
}

}  // namespace trime
