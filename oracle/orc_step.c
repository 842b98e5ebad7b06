/*
 * Oracle: the position updates (test infrastructure only).
 *
 * DistMesh (Sec. 2.2, Alg. 1, Eq. 2-5): every edge of the valid triangles is
 * a repulsive spring, f = k*(l0 - l) if l < l0 else 0, with
 * l0 = mu(m)*fac_F*fac_mu, m the edge midpoint and
 * fac_mu = (sum l^2 / sum mu(m)^2)^(1/2) over all edges; forward Euler
 * p <- p + dt*F.  k = 1 and dt = 0.2 are the DistMesh defaults (the paper's
 * table leaves them open).
 *
 * CVD (Sec. 2.3, Eq. 6, Alg. 2, Sec. 4.2 II): the new position is the
 * rho-weighted centroid of the bounded cell, rho = mu^-2 (Eq. 9), by the
 * adaptive quadrature of Sec. 4.2: level 0 uses the generator itself, level 1
 * the fan of triangles (p, v_k, v_k+1) with one point at each centroid, each
 * further level halves every triangle through the midpoint of its longest
 * edge; stop at the first k with |c_k - c_k+1| < sqrt(A_V)*max(d_prev/h,
 * fac_end) and use c_k+1.  Readings: "longest" compares squared lengths and
 * ties go to the first of (v0v1, v1v2, v2v0); the level is capped at
 * cvd_max_level; d_prev < 0 marks the first iteration and means d_prev = h.
 *
 * Treatment (Sec. 4.3, Eq. 12-14): cap the movement at fac_pt*h of the old
 * cell; a new point in an inner cell is kept; in a boundary cell it is kept
 * when sdf <= geps; otherwise (outside, an outer cell or off the grid) it is
 * brought to the boundary by sphere tracing from p_old (p_old inner) or by
 * damped Newton projection from p_new (p_old on the boundary), which falls
 * back to p_old when it does not reach a boundary point within T_newton
 * steps.  Readings: Eq. 13 is followed (gradient at the iterate), with the
 * derivatives of the bilinear sdf patch of the iterate's cell (f_xx = f_yy =
 * 0); sphere tracing stops at |sdf| <= geps, bisects back on an overshoot
 * and keeps the last inside point on failure; the category of the final
 * point follows Sec. 3.5.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "orc_internal.h"

static double bilin_f(const orc_grid *g, const double *f, int64_t cell, double tx, double ty) {
  int64_t ci = cell % (g->nx - 1), cj = cell / (g->nx - 1);
  size_t n0 = (size_t)cj * g->nx + (size_t)ci;
  double f00 = f[n0], f10 = f[n0 + 1], f01 = f[n0 + g->nx], f11 = f[n0 + g->nx + 1];
  return (f00 * (1.0 - tx) + f10 * tx) * (1.0 - ty) + (f01 * (1.0 - tx) + f11 * tx) * ty;
}

/* mu anywhere: bilinear in the cell, cells clamped to the grid outside it */
static double mu_at(const orc_grid *g, double x, double y) {
  double fx = (x - g->x0) * g->inv_dx, fy = (y - g->y0) * g->inv_dy;
  double ix = floor(fx), iy = floor(fy);
  if (ix < 0) ix = 0;
  if (iy < 0) iy = 0;
  if (ix > g->nx - 2) ix = g->nx - 2;
  if (iy > g->ny - 2) iy = g->ny - 2;
  double tx = fx - ix, ty = fy - iy;
  if (tx < 0) tx = 0;
  if (tx > 1) tx = 1;
  if (ty < 0) ty = 0;
  if (ty > 1) ty = 1;
  int64_t cell = (int64_t)iy * (g->nx - 1) + (int64_t)ix;
  return bilin_f(g, g->mu, cell, tx, ty);
}

static double geps_cell(const orc_grid *g, const orc_params *prm, int64_t cell) {
  return prm->fac_geps * fmin((double)g->hcell[cell], g->h_avg);
}

uint8_t orc_point_category(const orc_grid *g, const orc_params *prm, double x, double y) {
  int64_t cell;
  double tx, ty;
  if (!orc_locate(g, x, y, &cell, &tx, &ty)) return ORC_CAT_OUTER;
  uint8_t c = g->cat[cell];
  if (c != ORC_CAT_BOUNDARY) return c;
  double s = bilin_f(g, g->sdf, cell, tx, ty), ge = geps_cell(g, prm, cell);
  if (s > ge) return ORC_CAT_OUTER;
  return fabs(s) <= ge ? ORC_CAT_BOUNDARY : ORC_CAT_INNER;
}

/* ---------------- treatment ---------------- */

static int sdf_probe(const orc_grid *g, const orc_params *prm, double x, double y, double *s,
                     double *ge) {
  int64_t cell;
  double tx, ty;
  if (!orc_locate(g, x, y, &cell, &tx, &ty)) return 0;
  *s = bilin_f(g, g->sdf, cell, tx, ty);
  *ge = geps_cell(g, prm, cell);
  return 1;
}

static void sphere_trace(const orc_grid *g, const orc_params *prm, double xo, double yo,
                         double xn, double yn, double *xf, double *yf, orc_counters *cnt) {
  double dx = xn - xo, dy = yn - yo;
  double L = sqrt(dx * dx + dy * dy);
  double ux = dx / L, uy = dy / L;
  double t_in = 0.0, t = 0.0, t_out = -1.0;
  for (int it = 0; it < prm->trace_max_steps; it++) {
    double x = xo + t * ux, y = yo + t * uy, s, ge;
    int on = sdf_probe(g, prm, x, y, &s, &ge);
    if (on && fabs(s) <= ge) {
      *xf = x;
      *yf = y;
      return;
    }
    if (!on || s > 0) {
      t_out = t;
      break;
    }
    t_in = t;
    t = t + fabs(s);
    if (t > L) t = L;
  }
  if (t_out >= 0) {
    double lo = t_in, hi = t_out;
    for (int b = 0; b < prm->trace_bisect; b++) {
      double mid = 0.5 * (lo + hi);
      double x = xo + mid * ux, y = yo + mid * uy, s, ge;
      int on = sdf_probe(g, prm, x, y, &s, &ge);
      if (on && fabs(s) <= ge) {
        *xf = x;
        *yf = y;
        return;
      }
      if (!on || s > 0)
        hi = mid;
      else
        lo = mid;
    }
    t_in = lo;
  }
  if (cnt) cnt->trace_fail++;
  *xf = xo + t_in * ux;
  *yf = yo + t_in * uy;
}

static int newton_project(const orc_grid *g, const orc_params *prm, double xn, double yn,
                          double *xf, double *yf) {
  double xk = xn, yk = yn;
  for (int it = 0; it < prm->T_newton; it++) {
    int64_t cell;
    double tx, ty;
    if (!orc_locate(g, xk, yk, &cell, &tx, &ty)) return 0;
    int64_t ci = cell % (g->nx - 1), cj = cell / (g->nx - 1);
    size_t n0 = (size_t)cj * g->nx + (size_t)ci;
    double s00 = g->sdf[n0], s10 = g->sdf[n0 + 1], s01 = g->sdf[n0 + g->nx],
           s11 = g->sdf[n0 + g->nx + 1];
    double f = (s00 * (1.0 - tx) + s10 * tx) * (1.0 - ty) + (s01 * (1.0 - tx) + s11 * tx) * ty;
    double fx = ((s10 - s00) * (1.0 - ty) + (s11 - s01) * ty) * g->inv_dx;
    double fy = ((s01 - s00) * (1.0 - tx) + (s11 - s10) * tx) * g->inv_dy;
    double fxy = (((s11 - s10) - (s01 - s00)) * g->inv_dx) * g->inv_dy;
    double ex = xk - xn, ey = yk - yn;
    double L1 = f, L2 = ex * fy - ey * fx;
    double J00 = fx, J01 = fy;
    double J10 = fy + ex * fxy, J11 = -fx - ey * fxy;
    double det = J00 * J11 - J01 * J10;
    if (det == 0.0 || !isfinite(det)) return 0;
    double sx = (J11 * L1 - J01 * L2) / det;
    double sy = (J00 * L2 - J10 * L1) / det;
    xk = xk - prm->alpha_hat * sx;
    yk = yk - prm->alpha_hat * sy;
    double tx2, ty2;
    if (orc_locate(g, xk, yk, &cell, &tx2, &ty2) && g->cat[cell] == ORC_CAT_BOUNDARY) {
      double s = bilin_f(g, g->sdf, cell, tx2, ty2);
      if (fabs(s) <= geps_cell(g, prm, cell)) {
        *xf = xk;
        *yf = yk;
        return 1;
      }
    }
  }
  return 0;
}

void orc_treat(const orc_grid *g, const orc_params *prm, double xo, double yo, uint8_t cat_old,
               double xnew, double ynew, double *xf, double *yf, uint8_t *catf,
               orc_counters *cnt) {
  int64_t cell;
  double tx, ty;
  /* 1. movement cap T_pt = fac_pt * h of the old cell */
  if (orc_locate(g, xo, yo, &cell, &tx, &ty)) {
    double T = prm->fac_pt * (double)g->hcell[cell];
    double dx = xnew - xo, dy = ynew - yo, d2 = dx * dx + dy * dy;
    if (d2 > T * T) {
      double sc = T / sqrt(d2);
      xnew = xo + dx * sc;
      ynew = yo + dy * sc;
    }
  }
  /* 2. inner / boundary-inside points are kept */
  if (orc_locate(g, xnew, ynew, &cell, &tx, &ty)) {
    uint8_t c = g->cat[cell];
    if (c == ORC_CAT_INNER) {
      *xf = xnew;
      *yf = ynew;
      *catf = ORC_CAT_INNER;
      return;
    }
    if (c == ORC_CAT_BOUNDARY) {
      double s = bilin_f(g, g->sdf, cell, tx, ty), ge = geps_cell(g, prm, cell);
      if (s <= ge) {
        *xf = xnew;
        *yf = ynew;
        *catf = fabs(s) <= ge ? ORC_CAT_BOUNDARY : ORC_CAT_INNER;
        return;
      }
    }
  }
  /* 3. outside: bring it back to the boundary */
  if (cat_old == ORC_CAT_INNER) {
    sphere_trace(g, prm, xo, yo, xnew, ynew, xf, yf, cnt);
    *catf = orc_point_category(g, prm, *xf, *yf);
  } else {
    if (newton_project(g, prm, xnew, ynew, xf, yf)) {
      *catf = ORC_CAT_BOUNDARY;
    } else {
      if (cnt) cnt->newton_fail++;
      *xf = xo;
      *yf = yo;
      *catf = cat_old;
    }
  }
}

/* ---------------- DistMesh ---------------- */

double orc_fac_mu(const orc_grid *g, int64_t n, const double *x, const double *y,
                  const int64_t *rowptr, const int32_t *col, double *sum_l2, double *sum_mu2) {
  double sl = 0.0, sm = 0.0;
  for (int64_t i = 0; i < n; i++)
    for (int64_t t = rowptr[i]; t < rowptr[i + 1]; t++) {
      int32_t j = col[t];
      if (j <= i) continue;
      double dx = x[i] - x[j], dy = y[i] - y[j];
      double m = mu_at(g, (x[i] + x[j]) * 0.5, (y[i] + y[j]) * 0.5);
      sl += dx * dx + dy * dy;
      sm += m * m;
    }
  if (sum_l2) *sum_l2 = sl;
  if (sum_mu2) *sum_mu2 = sm;
  return sm > 0 ? sqrt(sl / sm) : 0.0;
}

int64_t orc_dm_step(const orc_grid *g, const orc_params *prm, int64_t n, const double *x,
                    const double *y, const uint8_t *cat, const int64_t *rowptr,
                    const int32_t *col, const double *xl, const double *yl, double *xn,
                    double *yn, uint8_t *catn, double *fac_mu_out, orc_counters *cnt) {
  double fac_mu = orc_fac_mu(g, n, x, y, rowptr, col, NULL, NULL);
  if (fac_mu_out) *fac_mu_out = fac_mu;
  int64_t moved = 0;
  for (int64_t i = 0; i < n; i++) {
    double Fx = 0.0, Fy = 0.0;
    for (int64_t t = rowptr[i]; t < rowptr[i + 1]; t++) {
      int32_t j = col[t];
      double dx = x[i] - x[j], dy = y[i] - y[j];
      double l = sqrt(dx * dx + dy * dy);
      if (l == 0.0) continue;
      double m = mu_at(g, (x[i] + x[j]) * 0.5, (y[i] + y[j]) * 0.5);
      double l0 = m * prm->fac_F * fac_mu;
      double f = l < l0 ? prm->k_spring * (l0 - l) : 0.0;
      double w = f / l;
      Fx += w * dx;
      Fy += w * dy;
    }
    double px = x[i] + prm->dt * Fx, py = y[i] + prm->dt * Fy;
    orc_treat(g, prm, x[i], y[i], cat[i], px, py, &xn[i], &yn[i], &catn[i], cnt);
    int64_t cell;
    double tx, ty;
    if (xl && orc_locate(g, xn[i], yn[i], &cell, &tx, &ty)) {
      double h = prm->fac_retria * (double)g->hcell[cell];
      double ex = xn[i] - xl[i], ey = yn[i] - yl[i];
      if (ex * ex + ey * ey > h * h) moved++;
    }
  }
  return moved;
}

/* ---------------- CVD ---------------- */

typedef struct {
  double w, wx, wy;
} acc3;

static void quad_tri(const orc_grid *g, double px, double py, double ax, double ay, double bx,
                     double by, double cx, double cy, int depth, acc3 *acc, int64_t *nq) {
  if (depth == 0) {
    double A = 0.5 * ((bx - ax) * (cy - ay) - (by - ay) * (cx - ax));
    double gx = (ax + bx + cx) / 3.0, gy = (ay + by + cy) / 3.0;
    double m = mu_at(g, px + gx, py + gy);
    double w = A / (m * m);
    acc->w += w;
    acc->wx += w * gx;
    acc->wy += w * gy;
    (*nq)++;
    return;
  }
  double l0 = (bx - ax) * (bx - ax) + (by - ay) * (by - ay);
  double l1 = (cx - bx) * (cx - bx) + (cy - by) * (cy - by);
  double l2 = (ax - cx) * (ax - cx) + (ay - cy) * (ay - cy);
  if (l0 >= l1 && l0 >= l2) {
    double mx = (ax + bx) * 0.5, my = (ay + by) * 0.5;
    quad_tri(g, px, py, ax, ay, mx, my, cx, cy, depth - 1, acc, nq);
    quad_tri(g, px, py, mx, my, bx, by, cx, cy, depth - 1, acc, nq);
  } else if (l1 >= l2) {
    double mx = (bx + cx) * 0.5, my = (by + cy) * 0.5;
    quad_tri(g, px, py, ax, ay, bx, by, mx, my, depth - 1, acc, nq);
    quad_tri(g, px, py, ax, ay, mx, my, cx, cy, depth - 1, acc, nq);
  } else {
    double mx = (cx + ax) * 0.5, my = (cy + ay) * 0.5;
    quad_tri(g, px, py, ax, ay, bx, by, mx, my, depth - 1, acc, nq);
    quad_tri(g, px, py, mx, my, bx, by, cx, cy, depth - 1, acc, nq);
  }
}

/* centroid at quadrature level L >= 1 (relative to p) */
static void level_centroid(const orc_grid *g, double px, double py, const double *vx,
                           const double *vy, int m, int L, double *cx, double *cy,
                           int64_t *nq) {
  acc3 acc = {0, 0, 0};
  for (int k = 0; k < m; k++) {
    int k1 = (k + 1) % m;
    quad_tri(g, px, py, 0.0, 0.0, vx[k], vy[k], vx[k1], vy[k1], L - 1, &acc, nq);
  }
  *cx = acc.wx / acc.w;
  *cy = acc.wy / acc.w;
}

int orc_cvd_centroid(const orc_grid *g, const orc_params *prm, int64_t n, const double *x,
                     const double *y, int64_t i, double dprev, double *cx, double *cy,
                     double *area, orc_counters *cnt) {
  orc_cellctx *cc = orc_cellctx_new(g, prm, n, x, y);
  int L = orc_cvd_centroid_ctx(cc, g, prm, x, y, i, dprev, cx, cy, area, cnt);
  orc_cellctx_free(cc);
  return L;
}

int orc_cvd_centroid_ctx(const orc_cellctx *cc, const orc_grid *g, const orc_params *prm,
                         const double *x, const double *y, int64_t i, double dprev, double *cx,
                         double *cy, double *area, orc_counters *cnt) {
  int32_t cons[256];
  double vx[256], vy[256];
  int m = orc_cellctx_cell(cc, i, cons, vx, vy, 256, cnt);
  if (m <= 0) {
    *cx = 0;
    *cy = 0;
    if (area) *area = 0;
    return 0;
  }
  double A = 0.0;
  for (int k = 0; k < m; k++) {
    int k1 = (k + 1) % m;
    A += 0.5 * (vx[k] * vy[k1] - vy[k] * vx[k1]);
  }
  if (area) *area = A;
  int64_t cell;
  double tx, ty;
  orc_locate(g, x[i], y[i], &cell, &tx, &ty);
  double h = (double)g->hcell[cell];
  double dp = dprev < 0 ? h : dprev;
  double eps = fmax(dp / h, prm->fac_end);
  double E = sqrt(A) * eps;
  double c0x = 0.0, c0y = 0.0, c1x, c1y;
  int64_t nq = 0;
  int L;
  for (L = 1;; L++) {
    level_centroid(g, x[i], y[i], vx, vy, m, L, &c1x, &c1y, &nq);
    double ex = c0x - c1x, ey = c0y - c1y;
    if (ex * ex + ey * ey < E * E) break;
    if (L == prm->cvd_max_level) {
      if (cnt) cnt->level_cap_hits++;
      break;
    }
    c0x = c1x;
    c0y = c1y;
  }
  if (cnt) cnt->quad_points += nq;
  *cx = c1x;
  *cy = c1y;
  return L;
}

int orc_cvd_step(const orc_grid *g, const orc_params *prm, int64_t n, const double *x,
                 const double *y, const uint8_t *cat, const double *dprev, double *xn,
                 double *yn, uint8_t *catn, double *dprevn, int32_t *levels, int nthreads,
                 orc_counters *cnt) {
  orc_counters tot;
  memset(&tot, 0, sizeof tot);
  orc_cellctx *cc = orc_cellctx_new(g, prm, n, x, y);
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
  {
    orc_counters loc;
    memset(&loc, 0, sizeof loc);
#pragma omp for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; i++) {
      double cx, cy;
      int L = orc_cvd_centroid_ctx(cc, g, prm, x, y, i, dprev[i], &cx, &cy, NULL, &loc);
      if (levels) levels[i] = L;
      orc_treat(g, prm, x[i], y[i], cat[i], x[i] + cx, y[i] + cy, &xn[i], &yn[i], &catn[i], &loc);
      double ex = xn[i] - x[i], ey = yn[i] - y[i];
      dprevn[i] = sqrt(ex * ex + ey * ey);
    }
#pragma omp critical
    {
      int64_t *a = (int64_t *)&tot, *b = (int64_t *)&loc;
      for (size_t k = 0; k < sizeof(orc_counters) / sizeof(int64_t); k++) a[k] += b[k];
    }
  }
  orc_cellctx_free(cc);
  if (cnt) {
    int64_t *a = (int64_t *)cnt, *b = (int64_t *)&tot;
    for (size_t k = 0; k < sizeof(orc_counters) / sizeof(int64_t); k++) a[k] += b[k];
  }
  return 0;
}

void orc_point_categories(const orc_grid *g, const orc_params *prm, int64_t n, const double *x,
                          const double *y, uint8_t *out) {
  for (int64_t i = 0; i < n; i++) out[i] = orc_point_category(g, prm, x[i], y[i]);
}
