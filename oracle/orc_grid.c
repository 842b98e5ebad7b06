/*
 * Oracle: geometry, sizing field and the geometry grid (test infrastructure
 * only).
 *
 * Sec. 3.1: the shape is a signed distance field (negative inside), built
 * from analytic primitives combined by union = min, difference =
 * max(a, -b), intersection = max.
 * Sec. 3.2: every grid cell is boundary if |sdf(midpoint)| <= l_diag (the
 * cell diagonal), otherwise inner if sdf(midpoint) < 0, else outer.
 * Sec. 3.3-3.5, 3.7: the sizing field mu gives relative edge lengths,
 * rho = mu^-2 (Eq. 9); the local desired edge length of a cell is
 * h_i = sqrt(dx*dy / n_i^E) with n_i^E = rho_i^norm * N, rho normalised over
 * the inner cells and the boundary cells whose midpoint sdf is at most
 * eta*min(dx, dy) ("selected" cells, eta = 0.5); h_avg is the mean h over
 * the selected cells.
 *
 * Readings (where the paper leaves the grid unspecified): the geometry grid
 * is a vertex-centred node grid with bilinear interpolation inside each cell;
 * the midpoint value of a cell is the mean of its four corner nodes (the
 * bilinear value there); mu_i of a cell is likewise the mean of its corner
 * mu nodes, so h_i = mu_i * H with H = sqrt(dx*dy*sum_sel mu_i^-2 / N).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "orc.h"

void orc_default_params(orc_params *p) {
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

/* distance from (x, y) to segment (ax, ay)-(bx, by) */
static double seg_dist(double x, double y, double ax, double ay, double bx, double by) {
  double ex = bx - ax, ey = by - ay;
  double wx = x - ax, wy = y - ay;
  double L2 = ex * ex + ey * ey;
  double t = L2 > 0 ? (wx * ex + wy * ey) / L2 : 0.0;
  if (t < 0) t = 0;
  if (t > 1) t = 1;
  double dx = wx - t * ex, dy = wy - t * ey;
  return sqrt(dx * dx + dy * dy);
}

/* Signed distance to an ellipse (centre c, semi-axes a, b, rotation phi).
   Closest point by the published method of D. Eberly ("Distance from a point
   to an ellipse"): in the first quadrant with e0 >= e1 the Lagrange
   parameter solves a strictly monotone scalar equation, found by bisection. */
static double ellipse_dist_q1(double e0, double e1, double y0, double y1) {
  if (y1 > 0) {
    if (y0 > 0) {
      double z0 = y0 / e0, z1 = y1 / e1, g = z0 * z0 + z1 * z1 - 1.0;
      if (g == 0.0) return 0.0;
      double r0 = (e0 / e1) * (e0 / e1);
      double n0 = r0 * z0, s0 = z1 - 1.0, s1 = g < 0 ? 0.0 : sqrt(n0 * n0 + z1 * z1) - 1.0;
      double s = 0.0;
      for (int it = 0; it < 2000; it++) {
        s = 0.5 * (s0 + s1);
        if (s == s0 || s == s1) break;
        double q0 = n0 / (s + r0), q1 = z1 / (s + 1.0);
        double gg = q0 * q0 + q1 * q1 - 1.0;
        if (gg > 0)
          s0 = s;
        else if (gg < 0)
          s1 = s;
        else
          break;
      }
      double x0 = r0 * y0 / (s + r0), x1 = y1 / (s + 1.0);
      return sqrt((x0 - y0) * (x0 - y0) + (x1 - y1) * (x1 - y1));
    }
    return fabs(y1 - e1);
  }
  double numer0 = e0 * y0, denom0 = e0 * e0 - e1 * e1;
  if (numer0 < denom0) {
    double xd = numer0 / denom0;
    double x0 = e0 * xd, x1 = e1 * sqrt(1.0 - xd * xd);
    return sqrt((x0 - y0) * (x0 - y0) + x1 * x1);
  }
  return fabs(y0 - e0);
}

static double ellipse_sdf(const double *p, double x, double y) {
  double cx = p[0], cy = p[1], a = p[2], b = p[3], phi = p[4];
  double c = cos(phi), s = sin(phi);
  double u = fabs(c * (x - cx) + s * (y - cy));
  double v = fabs(-s * (x - cx) + c * (y - cy));
  double inside = (u / a) * (u / a) + (v / b) * (v / b) - 1.0;
  double d = a >= b ? ellipse_dist_q1(a, b, u, v) : ellipse_dist_q1(b, a, v, u);
  return inside < 0 ? -d : d;
}

/* Unit inward normal of the segment a -> b of a clockwise loop: the
   direction (ex, ey) turned clockwise, (ey, -ex) / |e|. */
static void seg_normal(double ax, double ay, double bx, double by, double *nx, double *ny) {
  double ex = bx - ax, ey = by - ay;
  double L = sqrt(ex * ex + ey * ey);
  *nx = L > 0 ? ey / L : 0.0;
  *ny = L > 0 ? -ex / L : 0.0;
}

double orc_segments_sdf(const double *v, int32_t nv, double x, double y, int32_t *seg_out) {
  double best = INFINITY, bt = 0.0;
  int32_t kb = -1;
  for (int32_t k = 0; k < nv; k++) {
    int32_t k1 = k + 1 == nv ? 0 : k + 1;
    double ax = v[2 * k], ay = v[2 * k + 1], bx = v[2 * k1], by = v[2 * k1 + 1];
    double ex = bx - ax, ey = by - ay, wx = x - ax, wy = y - ay;
    double L2 = ex * ex + ey * ey;
    double t = L2 > 0 ? (wx * ex + wy * ey) / L2 : 0.0;
    if (t < 0) t = 0;
    if (t > 1) t = 1;
    double qx = wx - t * ex, qy = wy - t * ey;
    double d = sqrt(qx * qx + qy * qy);
    if (d < best) { /* strict: equal distances keep the lower index */
      best = d;
      bt = t;
      kb = k;
    }
  }
  if (seg_out) *seg_out = kb;
  int32_t k1 = kb + 1 == nv ? 0 : kb + 1;
  double ax = v[2 * kb], ay = v[2 * kb + 1], bx = v[2 * k1], by = v[2 * k1 + 1];
  double nx, ny;
  seg_normal(ax, ay, bx, by, &nx, &ny);
  double px = ax + bt * (bx - ax), py = ay + bt * (by - ay);
  if (bt == 0.0 || bt == 1.0) {
    /* an end point: the mean of the normals of the two segments there */
    int32_t ko = bt == 0.0 ? (kb == 0 ? nv - 1 : kb - 1) : k1;
    int32_t ko1 = ko + 1 == nv ? 0 : ko + 1;
    double mx, my;
    seg_normal(v[2 * ko], v[2 * ko + 1], v[2 * ko1], v[2 * ko1 + 1], &mx, &my);
    nx = 0.5 * (nx + mx);
    ny = 0.5 * (ny + my);
    px = bt == 0.0 ? ax : bx;
    py = bt == 0.0 ? ay : by;
  }
  double dot = (x - px) * nx + (y - py) * ny;
  return dot > 0 ? -best : best;
}

static double prim_sdf(const orc_prim *pr, const double *poly, double x, double y) {
  switch (pr->kind) {
    case ORC_PRIM_DISK: {
      double dx = x - pr->p[0], dy = y - pr->p[1];
      return sqrt(dx * dx + dy * dy) - pr->p[2];
    }
    case ORC_PRIM_BOX: {
      double ex = fmax(pr->p[0] - x, x - pr->p[2]);
      double ey = fmax(pr->p[1] - y, y - pr->p[3]);
      if (ex <= 0 && ey <= 0) return fmax(ex, ey);
      double qx = fmax(ex, 0.0), qy = fmax(ey, 0.0);
      return sqrt(qx * qx + qy * qy);
    }
    case ORC_PRIM_ELLIPSE:
      return ellipse_sdf(pr->p, x, y);
    case ORC_PRIM_POLYGON: {
      const double *v = poly + 2 * (size_t)pr->voff;
      int nv = pr->nv;
      double d = INFINITY;
      int inside = 0;
      for (int k = 0; k < nv; k++) {
        int k1 = (k + 1) % nv;
        double ax = v[2 * k], ay = v[2 * k + 1], bx = v[2 * k1], by = v[2 * k1 + 1];
        double dk = seg_dist(x, y, ax, ay, bx, by);
        if (dk < d) d = dk;
        /* crossing number along +x */
        if ((ay > y) != (by > y)) {
          double xc = ax + (y - ay) * (bx - ax) / (by - ay);
          if (x < xc) inside = !inside;
        }
      }
      return inside ? -d : d;
    }
    case ORC_PRIM_SEGMENTS:
      return orc_segments_sdf(poly + 2 * (size_t)pr->voff, pr->nv, x, y, NULL);
  }
  return INFINITY;
}

double orc_sdf_eval(const orc_prim *prims, int32_t nprims, const double *poly, double x,
                    double y) {
  double s = INFINITY;
  for (int k = 0; k < nprims; k++) {
    double t = prim_sdf(&prims[k], poly, x, y);
    switch (prims[k].op) {
      case ORC_OP_INIT: s = t; break;
      case ORC_OP_UNION: s = fmin(s, t); break;
      case ORC_OP_DIFF: s = fmax(s, -t); break;
      case ORC_OP_INTERSECT: s = fmax(s, t); break;
    }
  }
  return s;
}

static double sizing_mu(const orc_sizing *sz, const orc_prim *prims, const double *poly,
                        double x, double y, double sdf) {
  switch (sz->kind) {
    case ORC_SZ_AUTO:
      return orc_auto_mu(sz->cent, sz->lfs, sz->ncent, sz->a0, x, y);
    case ORC_SZ_UNIFORM: return 1.0;
    case ORC_SZ_ABS_SDF: return sz->a0 + sz->a1 * fabs(sdf);
    case ORC_SZ_GAUSS_RHO: {
      double acc = 0.0;
      for (int k = 0; k < sz->ncent; k++) {
        double dx = x - sz->cent[2 * k], dy = y - sz->cent[2 * k + 1];
        acc += exp(-(dx * dx + dy * dy) / sz->s2);
      }
      double rho = sz->a0 + sz->a1 * acc;
      return 1.0 / sqrt(rho);
    }
    case ORC_SZ_HOLE_RAMP: {
      double dh = INFINITY;
      for (int k = 0; k < sz->nholes; k++) {
        double t = fabs(prim_sdf(&prims[sz->holes[k]], poly, x, y));
        if (t < dh) dh = t;
      }
      double r = dh / sz->a1;
      if (r > 1.0) r = 1.0;
      return 1.0 + (sz->a0 - 1.0) * r;
    }
  }
  return 1.0;
}

int orc_grid_build(const orc_prim *prims, int32_t nprims, const double *poly,
                   const orc_sizing *sz, int32_t nx, int32_t ny, double x0, double y0,
                   double dx, double dy, int32_t dtype_bytes, int64_t n_total, double *sdf,
                   double *mu, uint8_t *cat, float *hcell, double *h_avg, double *H_out) {
  if (nx < 2 || ny < 2 || n_total <= 0 || !(dx > 0) || !(dy > 0)) return -1;
#pragma omp parallel for schedule(dynamic, 4)
  for (int j = 0; j < ny; j++)
    for (int i = 0; i < nx; i++) {
      double x = x0 + i * dx, y = y0 + j * dy;
      double s = orc_sdf_eval(prims, nprims, poly, x, y);
      double m = sizing_mu(sz, prims, poly, x, y, s);
      size_t k = (size_t)j * nx + i;
      sdf[k] = dtype_bytes == 4 ? (double)(float)s : s;
      mu[k] = dtype_bytes == 4 ? (double)(float)m : m;
    }
  int cx = nx - 1, cy = ny - 1;
  double ldiag = sqrt(dx * dx + dy * dy);
  double band = 0.5 * fmin(dx, dy);
  double sum_rho = 0.0;
  for (int j = 0; j < cy; j++)
    for (int i = 0; i < cx; i++) {
      size_t n0 = (size_t)j * nx + i;
      double sm = ((sdf[n0] + sdf[n0 + 1]) + (sdf[n0 + nx] + sdf[n0 + nx + 1])) * 0.25;
      uint8_t c;
      if (fabs(sm) <= ldiag)
        c = ORC_CAT_BOUNDARY;
      else if (sm < 0)
        c = ORC_CAT_INNER;
      else
        c = ORC_CAT_OUTER;
      cat[(size_t)j * cx + i] = c;
      int sel = c == ORC_CAT_INNER || (c == ORC_CAT_BOUNDARY && sm <= band);
      if (sel) {
        double mm = ((mu[n0] + mu[n0 + 1]) + (mu[n0 + nx] + mu[n0 + nx + 1])) * 0.25;
        sum_rho += 1.0 / (mm * mm);
      }
    }
  double H = sqrt(dx * dy * sum_rho / (double)n_total);
  double hsum = 0.0;
  int64_t nsel = 0;
  for (int j = 0; j < cy; j++)
    for (int i = 0; i < cx; i++) {
      size_t n0 = (size_t)j * nx + i;
      double mm = ((mu[n0] + mu[n0 + 1]) + (mu[n0 + nx] + mu[n0 + nx + 1])) * 0.25;
      float h = (float)(mm * H);
      hcell[(size_t)j * cx + i] = h;
      uint8_t c = cat[(size_t)j * cx + i];
      double sm = ((sdf[n0] + sdf[n0 + 1]) + (sdf[n0 + nx] + sdf[n0 + nx + 1])) * 0.25;
      if (c == ORC_CAT_INNER || (c == ORC_CAT_BOUNDARY && sm <= band)) {
        hsum += (double)h;
        nsel++;
      }
    }
  *h_avg = nsel ? hsum / (double)nsel : 0.0;
  if (H_out) *H_out = H;
  return 0;
}

void orc_grid_init(orc_grid *g, int32_t nx, int32_t ny, double x0, double y0, double dx,
                   double dy, const double *sdf, const double *mu, const uint8_t *cat,
                   const float *hcell, double h_avg) {
  g->nx = nx;
  g->ny = ny;
  g->x0 = x0;
  g->y0 = y0;
  g->dx = dx;
  g->dy = dy;
  g->inv_dx = 1.0 / dx;
  g->inv_dy = 1.0 / dy;
  g->sdf = sdf;
  g->mu = mu;
  g->cat = cat;
  g->hcell = hcell;
  g->h_avg = h_avg;
}

/* Cell of (x, y): fx = (x - x0) * (1/dx), cell = floor(fx), t = fx - cell. */
int orc_locate(const orc_grid *g, double x, double y, int64_t *cell, double *tx, double *ty) {
  double fx = (x - g->x0) * g->inv_dx;
  double fy = (y - g->y0) * g->inv_dy;
  if (!(fx >= 0.0) || !(fy >= 0.0)) return 0;
  double ix = floor(fx), iy = floor(fy);
  if (ix >= (double)(g->nx - 1) || iy >= (double)(g->ny - 1)) return 0;
  *cell = (int64_t)iy * (g->nx - 1) + (int64_t)ix;
  *tx = fx - ix;
  *ty = fy - iy;
  return 1;
}
