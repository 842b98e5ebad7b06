// Device side of the segment-loop distance (Sec. 3.2), shared by the
// candidate build and the grid's node kernel.
#pragma once
#include "setup.hpp"

namespace trime {

// Distance from (x, y) to segment k of the loop; t: the clamped parameter of
// the closest point.  The same operations as the reference definition.
TRIME_HD double seg_dist_t(const double *v, int nv, int k, double x, double y, double &t) {
  const int k1 = k + 1 == nv ? 0 : k + 1;
  const double ax = v[2 * k], ay = v[2 * k + 1], bx = v[2 * k1], by = v[2 * k1 + 1];
  const double ex = bx - ax, ey = by - ay, wx = x - ax, wy = y - ay;
  const double L2 = ex * ex + ey * ey;
  t = L2 > 0 ? (wx * ex + wy * ey) / L2 : 0.0;
  t = t < 0 ? 0.0 : (t > 1 ? 1.0 : t);
  const double qx = wx - t * ex, qy = wy - t * ey;
  return sqrt(qx * qx + qy * qy);
}

TRIME_HD void seg_normal_unit(const double *v, int nv, int k, double &nx, double &ny) {
  const int k1 = k + 1 == nv ? 0 : k + 1;
  const double ex = v[2 * k1] - v[2 * k], ey = v[2 * k1 + 1] - v[2 * k + 1];
  const double L = sqrt(ex * ex + ey * ey);
  nx = L > 0 ? ey / L : 0.0;
  ny = L > 0 ? -ex / L : 0.0;
}

// The signed distance at (x, y) from the nearest segment kb, its clamped
// parameter bt and its distance best.
TRIME_HD double seg_signed(const double *v, int nv, int kb, double bt, double best, double x, double y) {
  const int k1 = kb + 1 == nv ? 0 : kb + 1;
  const double ax = v[2 * kb], ay = v[2 * kb + 1], bx = v[2 * k1], by = v[2 * k1 + 1];
  double nx, ny;
  seg_normal_unit(v, nv, kb, nx, ny);
  double px = ax + bt * (bx - ax), py = ay + bt * (by - ay);
  if (bt == 0.0 || bt == 1.0) {
    const int ko = bt == 0.0 ? (kb == 0 ? nv - 1 : kb - 1) : k1;
    double mx, my;
    seg_normal_unit(v, nv, ko, mx, my);
    nx = 0.5 * (nx + mx);
    ny = 0.5 * (ny + my);
    px = bt == 0.0 ? ax : bx;
    py = bt == 0.0 ? ay : by;
  }
  const double dot = (x - px) * nx + (y - py) * ny;
  return dot > 0 ? -best : best;
}

// The loop's signed distance by brute force over its segments (host use).
TRIME_HD double segments_sdf_brute(const double *v, int nv, double x, double y) {
  double best = INFINITY, bt = 0.0;
  int kb = -1;
  for (int k = 0; k < nv; k++) {
    double t;
    const double d = seg_dist_t(v, nv, k, x, y, t);
    if (d < best) {
      best = d;
      bt = t;
      kb = k;
    }
  }
  return kb < 0 ? INFINITY : seg_signed(v, nv, kb, bt, best, x, y);
}

TRIME_D int64_t cand_cell(const CandGrid &G, double x, double y) {
  double fx = floor((x - G.x0) / G.cw), fy = floor((y - G.y0) / G.ch);
  fx = fmin(fmax(fx, 0.0), (double)(G.nx - 1));
  fy = fmin(fmax(fy, 0.0), (double)(G.ny - 1));
  return (int64_t)fy * G.nx + (int64_t)fx;
}

// The function families the candidate lists are built for: value(k, x, y)
// is L-Lipschitz in (x, y) for every item k, slack(r) = 2 L r.
struct SegMetric {
  const double *v;
  int nv;
  TRIME_D double value(int k, double x, double y) const {
    double t;
    return seg_dist_t(v, nv, k, x, y, t);
  }
  TRIME_D double slack(double r) const { return 2.0 * r; }
};

// K |x - s_k| + lfs(s_k), in the operation order of Eq. 8's reference.
struct LfsMetric {
  const double *s, *lfs;
  double K;
  TRIME_D double value(int k, double x, double y) const {
    const double dx = x - s[2 * k], dy = y - s[2 * k + 1];
    return K * sqrt(dx * dx + dy * dy) + lfs[k];
  }
  TRIME_D double slack(double r) const { return 2.0 * K * r; }
};

// mu at (x, y): the minimum over the cell's candidates (order-free).
TRIME_D double auto_mu(const LfsField &F, double x, double y) {
  const int64_t c = cand_cell(F.g, x, y);
  const LfsMetric M{F.s, F.lfs, F.K};
  double best = INFINITY;
  const int32_t e = F.g.start[c + 1];
  for (int32_t i = F.g.start[c]; i < e; i++) best = fmin(best, M.value(F.g.cand[i], x, y));
  return best;
}

TRIME_D double segments_sdf(const SegTree &T, double x, double y) {
  const int64_t c = cand_cell(T.g, x, y);
  const int32_t e = T.g.start[c + 1];
  double best = INFINITY, bt = 0.0;
  int kb = -1;
  for (int32_t i = T.g.start[c]; i < e; i++) {
    const int k = T.g.cand[i];  // ascending: strict < keeps the lowest index
    double t;
    const double d = seg_dist_t(T.v, T.nv, k, x, y, t);
    if (d < best) {
      best = d;
      bt = t;
      kb = k;
    }
  }
  return kb < 0 ? INFINITY : seg_signed(T.v, T.nv, kb, bt, best, x, y);
}

}  // namespace trime
