// Signed distances of the analytic primitives (Sec. 3.1), for the grid's
// node pass on the device and for the boundary points of automatic sizing
// on the host (the same operations on both).
#pragma once
#include <math.h>

#include "trime_dev.hpp"

namespace trime {

// D. Eberly's point-ellipse distance, first quadrant, e0 >= e1.
TRIME_HD double ellipse_q1(double e0, double e1, double y0, double y1) {
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

// Disk, box, ellipse and polygon (segment loops have their own search).
TRIME_HD double analytic_sdf(const trime_prim &pr, const double *poly, double x, double y) {
  switch (pr.kind) {
    case TRIME_PRIM_DISK: {
      double dx = x - pr.p[0], dy = y - pr.p[1];
      return sqrt(dx * dx + dy * dy) - pr.p[2];
    }
    case TRIME_PRIM_BOX: {
      double ex = fmax(pr.p[0] - x, x - pr.p[2]);
      double ey = fmax(pr.p[1] - y, y - pr.p[3]);
      if (ex <= 0 && ey <= 0) return fmax(ex, ey);
      double qx = fmax(ex, 0.0), qy = fmax(ey, 0.0);
      return sqrt(qx * qx + qy * qy);
    }
    case TRIME_PRIM_ELLIPSE: {
      double c = cos(pr.p[4]), s = sin(pr.p[4]);
      double u = fabs(c * (x - pr.p[0]) + s * (y - pr.p[1]));
      double v = fabs(-s * (x - pr.p[0]) + c * (y - pr.p[1]));
      double a = pr.p[2], b = pr.p[3];
      double in = (u / a) * (u / a) + (v / b) * (v / b) - 1.0;
      double d = a >= b ? ellipse_q1(a, b, u, v) : ellipse_q1(b, a, v, u);
      return in < 0 ? -d : d;
    }
    default: {  // polygon: segment distance, crossing-number sign
      const double *v = poly + 2 * (int64_t)pr.voff;
      int nv = pr.nv;
      double d = INFINITY;
      bool inside = false;
      for (int k = 0; k < nv; k++) {
        int k1 = (k + 1 == nv) ? 0 : k + 1;
        double ax = v[2 * k], ay = v[2 * k + 1], bx = v[2 * k1], by = v[2 * k1 + 1];
        double ex = bx - ax, ey = by - ay, wx = x - ax, wy = y - ay;
        double L2 = ex * ex + ey * ey;
        double t = L2 > 0 ? (wx * ex + wy * ey) / L2 : 0.0;
        t = fmin(fmax(t, 0.0), 1.0);
        double qx = wx - t * ex, qy = wy - t * ey;
        d = fmin(d, sqrt(qx * qx + qy * qy));
        if ((ay > y) != (by > y)) {
          double xc = ax + (y - ay) * (bx - ax) / (by - ay);
          if (x < xc) inside = !inside;
        }
      }
      return inside ? -d : d;
    }
  }
}


}  // namespace trime
