// Device geometry on the geometry grid, in FP64: validity of a triangle
// (Sec. 4.1 Tests 1-3, the check of Procedure I), point categories (Sec. 3.5) and the
// treatment of an updated point (Sec. 4.3: movement cap, restriction to
// inner/boundary cells, sphere tracing, damped Newton projection Eq. 12-14).
#pragma once
#include "trime_dev.hpp"

namespace trime {

// Triangle validity on the id-sorted triple (a < b < c by id).
// Test 1: centroid in an inner cell -> valid; outer/off-grid -> invalid;
//         boundary cell with sdf > geps -> invalid.
// Test 2: count edge midpoints in inner cells or with sdf <= geps in boundary
//         cells; >= 2 -> valid, 0 -> invalid, 1 -> Test 3 (test2_mode 0) or
//         invalid (test2_mode 1).
// Test 3: |sdf(circumcentre)| / R <= T_tria -> valid.
template <class G>
TRIME_D bool tri_valid(const KArgs &a, double ax, double ay, double bx, double by, double cx,
                       double cy) {
  GCell cell;
  double tx, ty;
  double gx = ((ax + bx) + cx) / 3.0, gy = ((ay + by) + cy) / 3.0;
  if (!locate(a, gx, gy, cell, tx, ty)) return false;
  uint8_t ct = cell_cat(a, cell);
  if (ct == TRIME_CAT_INNER) return true;
  if (ct == TRIME_CAT_OUTER) return false;
  if (bilinear<G>(a, a.sdf, cell, tx, ty) > geps_of(a, cell)) return false;
  int count = 0;
  {
    double mx[3] = {(ax + bx) * 0.5, (bx + cx) * 0.5, (ax + cx) * 0.5};
    double my[3] = {(ay + by) * 0.5, (by + cy) * 0.5, (ay + cy) * 0.5};
#pragma unroll
    for (int e = 0; e < 3; e++) {
      if (!locate(a, mx[e], my[e], cell, tx, ty)) continue;
      uint8_t cm = cell_cat(a, cell);
      if (cm == TRIME_CAT_INNER)
        count++;
      else if (cm == TRIME_CAT_BOUNDARY && bilinear<G>(a, a.sdf, cell, tx, ty) <= geps_of(a, cell))
        count++;
    }
  }
  if (count >= 2) return true;
  if (count == 0 || a.prm.test2_mode == 1) return false;
  double ux_ = bx - ax, uy_ = by - ay, qx = cx - ax, qy = cy - ay;
  double d = 2.0 * (ux_ * qy - uy_ * qx);
  if (d == 0.0) return false;
  double b2 = ux_ * ux_ + uy_ * uy_, q2 = qx * qx + qy * qy;
  double ccx = (qy * b2 - uy_ * q2) / d, ccy = (ux_ * q2 - qx * b2) / d;
  double R = sqrt(ccx * ccx + ccy * ccy);
  if (!locate(a, ax + ccx, ay + ccy, cell, tx, ty)) return false;
  double s = bilinear<G>(a, a.sdf, cell, tx, ty);
  return fabs(s) / R <= a.prm.T_tria;
}

// Category of a point (Sec. 3.5): inner cell -> inner; boundary cell ->
// boundary when |sdf| <= geps, inner when sdf < -geps, outer when outside.
// `unsure` is raised when a comparison falls within `band`.
template <class G>
TRIME_D uint8_t point_category(const KArgs &a, double x, double y, double band, bool &unsure) {
  GCell cell;
  double tx, ty;
  if (!locate(a, x, y, cell, tx, ty)) return TRIME_CAT_OUTER;
  uint8_t c = cell_cat(a, cell);
  if (c != TRIME_CAT_BOUNDARY) return c;
  double s = bilinear<G>(a, a.sdf, cell, tx, ty), ge = geps_of(a, cell);
  if (fabs(s - ge) <= band || fabs(fabs(s) - ge) <= band) unsure = true;
  if (s > ge) return TRIME_CAT_OUTER;
  return fabs(s) <= ge ? TRIME_CAT_BOUNDARY : TRIME_CAT_INNER;
}

// Failures of one treatment as bits of one word (bit 0 sphere tracing, bit 1
// Newton), so the two paths update one register rather than two fields.
struct TreatCount {
  int fail = 0;
  TRIME_D int trace_fail() const { return fail & 1; }
  TRIME_D int newton_fail() const { return (fail >> 1) & 1; }
};

template <class G>
TRIME_D bool sdf_probe(const KArgs &a, double x, double y, double &s, double &ge) {
  GCell cell;
  double tx, ty;
  if (!locate(a, x, y, cell, tx, ty)) return false;
  s = bilinear<G>(a, a.sdf, cell, tx, ty);
  ge = geps_of(a, cell);
  return true;
}

// Sphere tracing from p_old (inside) towards p_new (outside): step by |sdf|
// until |sdf| <= geps; on an overshoot bisect back; on failure keep the last
// inside point.
template <class G>
TRIME_D void sphere_trace(const KArgs &a, double xo, double yo, double xn, double yn, double band,
                          double &xf, double &yf, bool &unsure, TreatCount &tc) {
  double dx = xn - xo, dy = yn - yo;
  double L = sqrt(dx * dx + dy * dy);
  double ux = dx / L, uy = dy / L;
  double t_in = 0.0, t = 0.0, t_out = -1.0;
  for (int it = 0; it < a.prm.trace_max_steps; it++) {
    double x = xo + t * ux, y = yo + t * uy, s, ge;
    bool on = sdf_probe<G>(a, x, y, s, ge);
    if (on && (fabs(fabs(s) - ge) <= band || fabs(s) <= band)) unsure = true;
    if (on && fabs(s) <= ge) {
      xf = x;
      yf = y;
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
    for (int b = 0; b < a.prm.trace_bisect; b++) {
      double mid = 0.5 * (lo + hi);
      double x = xo + mid * ux, y = yo + mid * uy, s, ge;
      bool on = sdf_probe<G>(a, x, y, s, ge);
      if (on && (fabs(fabs(s) - ge) <= band || fabs(s) <= band)) unsure = true;
      if (on && fabs(s) <= ge) {
        xf = x;
        yf = y;
        return;
      }
      if (!on || s > 0)
        hi = mid;
      else
        lo = mid;
    }
    t_in = lo;
  }
  tc.fail |= 1;
  xf = xo + t_in * ux;
  yf = yo + t_in * uy;
}

// Damped Newton projection of p_new onto the boundary (Eq. 12-14) with the
// derivatives of the bilinear patch of the iterate's cell (f_xx = f_yy = 0).
template <class G>
TRIME_D bool newton_project(const KArgs &a, double xn, double yn, double band, double &xf,
                            double &yf, bool &unsure) {
  double xk = xn, yk = yn;
  for (int it = 0; it < a.prm.T_newton; it++) {
    GCell cell;
    double tx, ty;
    if (!locate(a, xk, yk, cell, tx, ty)) return false;
    const int64_t n0 = node_index(a, cell);
    double s00 = gval<G>(a.sdf, n0), s10 = gval<G>(a.sdf, n0 + 1);
    double s01 = gval<G>(a.sdf, n0 + a.nx), s11 = gval<G>(a.sdf, n0 + a.nx + 1);
    double f = (s00 * (1.0 - tx) + s10 * tx) * (1.0 - ty) + (s01 * (1.0 - tx) + s11 * tx) * ty;
    double fx = ((s10 - s00) * (1.0 - ty) + (s11 - s01) * ty) * a.inv_dx;
    double fy = ((s01 - s00) * (1.0 - tx) + (s11 - s10) * tx) * a.inv_dy;
    double fxy = (((s11 - s10) - (s01 - s00)) * a.inv_dx) * a.inv_dy;
    double ex = xk - xn, ey = yk - yn;
    double L1 = f, L2 = ex * fy - ey * fx;
    double J00 = fx, J01 = fy, J10 = fy + ex * fxy, J11 = -fx - ey * fxy;
    double det = J00 * J11 - J01 * J10;
    if (det == 0.0 || !isfinite(det)) return false;
    double sx = (J11 * L1 - J01 * L2) / det;
    double sy = (J00 * L2 - J10 * L1) / det;
    xk = xk - a.prm.alpha_hat * sx;
    yk = yk - a.prm.alpha_hat * sy;
    double tx2, ty2;
    if (locate(a, xk, yk, cell, tx2, ty2) && cell_cat(a, cell) == TRIME_CAT_BOUNDARY) {
      double s = bilinear<G>(a, a.sdf, cell, tx2, ty2), ge = geps_of(a, cell);
      if (fabs(fabs(s) - ge) <= band) unsure = true;
      if (fabs(s) <= ge) {
        xf = xk;
        yf = yk;
        return true;
      }
    }
  }
  return false;
}

// Treatment of an updated point (Sec. 4.3).  band > 0 marks comparisons
// whose inputs carry FP32 error; then `unsure` asks for an FP64 replay.
template <class G>
TRIME_D void treat(const KArgs &a, double xo, double yo, uint8_t cat_old, double xnew, double ynew,
                   double band, double &xf, double &yf, uint8_t &catf, bool &unsure,
                   TreatCount &tc) {
  GCell cell;
  double tx, ty;
  if (locate(a, xo, yo, cell, tx, ty)) {
    double T = a.prm.fac_pt * (double)cell_h(a, cell);
    double dx = xnew - xo, dy = ynew - yo, d2 = dx * dx + dy * dy;
    if (d2 > T * T) {
      double sc = T / sqrt(d2);
      xnew = xo + dx * sc;
      ynew = yo + dy * sc;
    }
  }
  if (locate(a, xnew, ynew, cell, tx, ty)) {
    uint8_t c = cell_cat(a, cell);
    if (c == TRIME_CAT_INNER) {
      xf = xnew;
      yf = ynew;
      catf = TRIME_CAT_INNER;
      return;
    }
    if (c == TRIME_CAT_BOUNDARY) {
      double s = bilinear<G>(a, a.sdf, cell, tx, ty), ge = geps_of(a, cell);
      if (fabs(s - ge) <= band) unsure = true;
      if (s <= ge) {
        if (fabs(fabs(s) - ge) <= band) unsure = true;
        xf = xnew;
        yf = ynew;
        catf = fabs(s) <= ge ? TRIME_CAT_BOUNDARY : TRIME_CAT_INNER;
        return;
      }
    }
  }
  if (cat_old == TRIME_CAT_INNER) {
    sphere_trace<G>(a, xo, yo, xnew, ynew, band, xf, yf, unsure, tc);
    catf = point_category<G>(a, xf, yf, band, unsure);
  } else {
    if (newton_project<G>(a, xnew, ynew, band, xf, yf, unsure)) {
      catf = TRIME_CAT_BOUNDARY;
    } else {
      tc.fail |= 2;
      xf = xo;
      yf = yo;
      catf = cat_old;
    }
  }
}

}  // namespace trime
