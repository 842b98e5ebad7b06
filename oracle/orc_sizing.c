/* Automatic sizing field (Sec. 3.3, Eq. 8), oracle side: boundary points
   of segment loops (App. A), medial-axis approximating points from the
   Voronoi cells of the boundary points, their trimming, the local feature
   size lfs(s) and mu(x) = min over s of K |s - x| + lfs(s).  Brute force
   throughout: every Voronoi cell is clipped by every other point's
   bisector, every count and minimum runs over all points.  Test
   infrastructure only. */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "orc.h"

/* The vertices of a closed loop, then floor(L / d_s) points splitting each
   segment of length L > d_s evenly (spacing below d_s); returns the new
   count (writes below cap only). */
static int64_t loop_points(const double *v, int32_t nv, double d_s, double *out, int64_t n, int64_t cap) {
  for (int32_t k = 0; k < nv; k++) {
    int32_t k1 = k + 1 == nv ? 0 : k + 1;
    double ax = v[2 * k], ay = v[2 * k + 1], bx = v[2 * k1], by = v[2 * k1 + 1];
    double L = sqrt((bx - ax) * (bx - ax) + (by - ay) * (by - ay));
    int64_t pieces = L > d_s ? (int64_t)floor(L / d_s) + 1 : 1;
    for (int64_t i = 0; i < pieces; i++) {
      if (n < cap) {
        double t = (double)i / (double)pieces;
        out[2 * n] = ax + t * (bx - ax);
        out[2 * n + 1] = ay + t * (by - ay);
      }
      n++;
    }
  }
  return n;
}

#define ORC_TWO_PI 6.283185307179586

int64_t orc_boundary_points(const orc_prim *prims, int32_t nprims, const double *poly, double d_s, double geps,
                            double *out, int64_t cap) {
  int64_t n = 0;
  for (int32_t q = 0; q < nprims; q++) {
    const orc_prim *p = &prims[q];
    /* sample this primitive's boundary into a scratch list */
    int64_t m = 0;
    double *raw = NULL;
    if (p->kind == ORC_PRIM_DISK || p->kind == ORC_PRIM_ELLIPSE) {
      double rmax = p->kind == ORC_PRIM_DISK ? p->p[2] : fmax(p->p[2], p->p[3]);
      m = (int64_t)floor(ORC_TWO_PI * rmax / d_s) + 1;
      if (m < 3) m = 3;
      raw = (double *)malloc(sizeof(double) * 2 * (size_t)m);
      double c = p->kind == ORC_PRIM_ELLIPSE ? cos(p->p[4]) : 1.0, sn = p->kind == ORC_PRIM_ELLIPSE ? sin(p->p[4]) : 0.0;
      for (int64_t k = 0; k < m; k++) {
        double th = ORC_TWO_PI * (double)k / (double)m;
        if (p->kind == ORC_PRIM_DISK) {
          raw[2 * k] = p->p[0] + p->p[2] * cos(th);
          raw[2 * k + 1] = p->p[1] + p->p[2] * sin(th);
        } else {
          double u = p->p[2] * cos(th), w = p->p[3] * sin(th);
          raw[2 * k] = p->p[0] + (c * u - sn * w);
          raw[2 * k + 1] = p->p[1] + (sn * u + c * w);
        }
      }
    } else {
      double box[8];
      const double *v;
      int32_t nv;
      if (p->kind == ORC_PRIM_BOX) {
        /* the clockwise loop (x0,y0) (x0,y1) (x1,y1) (x1,y0) */
        box[0] = p->p[0]; box[1] = p->p[1]; box[2] = p->p[0]; box[3] = p->p[3];
        box[4] = p->p[2]; box[5] = p->p[3]; box[6] = p->p[2]; box[7] = p->p[1];
        v = box;
        nv = 4;
      } else {
        v = poly + 2 * (size_t)p->voff;
        nv = p->nv;
      }
      m = loop_points(v, nv, d_s, NULL, 0, 0);
      raw = (double *)malloc(sizeof(double) * 2 * (size_t)(m > 0 ? m : 1));
      loop_points(v, nv, d_s, raw, 0, m);
    }
    /* keep the points on the boundary of the whole geometry */
    for (int64_t k = 0; k < m; k++) {
      if (fabs(orc_sdf_eval(prims, nprims, poly, raw[2 * k], raw[2 * k + 1])) > geps) continue;
      if (n < cap) {
        out[2 * n] = raw[2 * k];
        out[2 * n + 1] = raw[2 * k + 1];
      }
      n++;
    }
    free(raw);
  }
  return n;
}

/* Voronoi cell of point i among s[0..ns), clipped to the box: a convex
   polygon (x, y) with, per edge k (from vertex k to k+1), the index of the
   point whose bisector carries it, or -1 for a box edge.  Points equal to
   s_i are skipped.  Returns the vertex count. */
#define ORC_VMAX 256
static int voronoi_cell(const double *s, int64_t ns, int64_t i, const double box[4], double *px, double *py,
                        int64_t *pe) {
  int n = 4;
  px[0] = box[0]; py[0] = box[1]; pe[0] = -1;
  px[1] = box[2]; py[1] = box[1]; pe[1] = -1;
  px[2] = box[2]; py[2] = box[3]; pe[2] = -1;
  px[3] = box[0]; py[3] = box[3]; pe[3] = -1;
  double qx[ORC_VMAX], qy[ORC_VMAX], val[ORC_VMAX];
  int64_t qe[ORC_VMAX];
  const double sx = s[2 * i], sy = s[2 * i + 1];
  for (int64_t j = 0; j < ns; j++) {
    if (j == i) continue;
    const double tx = s[2 * j], ty = s[2 * j + 1];
    if (tx == sx && ty == sy) continue;
    /* inside the cell: (x - m) . (t - s) <= 0, m the midpoint */
    const double nx = tx - sx, ny = ty - sy, mx = 0.5 * (sx + tx), my = 0.5 * (sy + ty);
    int out = 0;
    for (int k = 0; k < n; k++) {
      val[k] = (px[k] - mx) * nx + (py[k] - my) * ny;
      out |= val[k] > 0;
    }
    if (!out) continue;
    int m = 0;
    for (int k = 0; k < n; k++) {
      int k1 = k + 1 == n ? 0 : k + 1;
      if (val[k] <= 0) {
        qx[m] = px[k]; qy[m] = py[k]; qe[m] = pe[k]; m++;
      }
      if ((val[k] <= 0) != (val[k1] <= 0)) {
        /* the edge k crosses the bisector: the crossing starts the next
           piece of edge k (entering) or the bisector edge (leaving) */
        double t = val[k] / (val[k] - val[k1]);
        qx[m] = px[k] + t * (px[k1] - px[k]);
        qy[m] = py[k] + t * (py[k1] - py[k]);
        qe[m] = val[k] <= 0 ? j : pe[k];
        m++;
      }
      if (m >= ORC_VMAX - 2) return -1;
    }
    n = m;
    memcpy(px, qx, sizeof(double) * n);
    memcpy(py, qy, sizeof(double) * n);
    memcpy(pe, qe, sizeof(int64_t) * n);
  }
  return n;
}

/* The poles of point i (v1 then v2) into out[0..4), returns a 2-bit mask
   of the poles found. */
static int poles(const double *s, int64_t ns, int64_t i, const double box[4], double *out) {
  double px[ORC_VMAX], py[ORC_VMAX];
  int64_t pe[ORC_VMAX];
  int n = voronoi_cell(s, ns, i, box, px, py, pe);
  if (n < 3) return 0;
  const double sx = s[2 * i], sy = s[2 * i + 1];
  int found = 0;
  /* v1: the farthest vertex; a vertex with a box edge on either side
     stands for infinity and is never a medial point */
  int b1 = -1;
  double d1 = -1.0;
  for (int k = 0; k < n; k++) {
    double d = (px[k] - sx) * (px[k] - sx) + (py[k] - sy) * (py[k] - sy);
    if (d > d1) { d1 = d; b1 = k; }
  }
  const double ux = px[b1] - sx, uy = py[b1] - sy;
  if (pe[b1] >= 0 && pe[b1 == 0 ? n - 1 : b1 - 1] >= 0) {
    out[0] = px[b1];
    out[1] = py[b1];
    found |= 1;
  }
  /* v2: the farthest real vertex in the open half plane (v - s) . u < 0 */
  int b2 = -1;
  double d2 = -1.0;
  for (int k = 0; k < n; k++) {
    int real = pe[k] >= 0 && pe[k == 0 ? n - 1 : k - 1] >= 0;
    if (!real || (px[k] - sx) * ux + (py[k] - sy) * uy >= 0) continue;
    double d = (px[k] - sx) * (px[k] - sx) + (py[k] - sy) * (py[k] - sy);
    if (d > d2) { d2 = d; b2 = k; }
  }
  if (b2 >= 0) {
    out[2] = px[b2];
    out[3] = py[b2];
    found |= 2;
  }
  return found;
}

int64_t orc_medial_points(const double *s, int64_t ns, const double box[4], double *out, int64_t cap) {
  double *tmp = (double *)malloc(sizeof(double) * 4 * (size_t)(ns > 0 ? ns : 1));
  unsigned char *mask = (unsigned char *)malloc((size_t)(ns > 0 ? ns : 1));
  if (!tmp || !mask) {
    free(tmp);
    free(mask);
    return -1;
  }
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t i = 0; i < ns; i++) mask[i] = (unsigned char)poles(s, ns, i, box, tmp + 4 * i);
  int64_t nm = 0;
  for (int64_t i = 0; i < ns; i++)
    for (int q = 0; q < 2; q++) {
      if (!(mask[i] >> q & 1)) continue;
      if (nm < cap) {
        out[2 * nm] = tmp[4 * i + 2 * q];
        out[2 * nm + 1] = tmp[4 * i + 2 * q + 1];
      }
      nm++;
    }
  free(tmp);
  free(mask);
  return nm;
}

int64_t orc_trim_medial(const double *m, int64_t nm, double r_nei, int32_t n_thres, uint8_t *keep) {
  int64_t kept = 0;
  const double r2 = r_nei * r_nei;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : kept)
  for (int64_t i = 0; i < nm; i++) {
    int64_t c = 0;
    for (int64_t j = 0; j < nm; j++) {
      if (j == i) continue;
      double dx = m[2 * j] - m[2 * i], dy = m[2 * j + 1] - m[2 * i + 1];
      c += dx * dx + dy * dy <= r2;
    }
    keep[i] = c >= n_thres;
    kept += keep[i];
  }
  return kept;
}

void orc_lfs(const double *s, int64_t ns, const double *m, int64_t nm, const uint8_t *keep, double *lfs) {
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t i = 0; i < ns; i++) {
    double best = INFINITY;
    for (int64_t j = 0; j < nm; j++) {
      if (!keep[j]) continue;
      double dx = m[2 * j] - s[2 * i], dy = m[2 * j + 1] - s[2 * i + 1];
      double d = sqrt(dx * dx + dy * dy);
      if (d < best) best = d;
    }
    lfs[i] = best;
  }
}

double orc_auto_mu(const double *s, const double *lfs, int64_t ns, double K, double x, double y) {
  double best = INFINITY;
  for (int64_t i = 0; i < ns; i++) {
    double dx = x - s[2 * i], dy = y - s[2 * i + 1];
    double f = K * sqrt(dx * dx + dy * dy) + lfs[i];
    if (f < best) best = f;
  }
  return best;
}

int64_t orc_trim_boundary(const orc_prim *prims, int32_t nprims, const double *poly, double d_s, double geps,
                          double *pts, int64_t n) {
  unsigned char *gone = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
  unsigned char *done = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
  unsigned char *bad = (unsigned char *)calloc((size_t)(n > 0 ? n : 1), 1);
  double *d = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  if (!gone || !done || !bad || !d) {
    free(gone); free(done); free(bad); free(d);
    return -1;
  }
  int changed = 1;
  while (changed) {
    changed = 0;
    for (int64_t i = 0; i < n; i++) {
      if (gone[i] || done[i]) continue;
      const double xi = pts[2 * i], yi = pts[2 * i + 1];
#pragma omp parallel for schedule(static)
      for (int64_t j = 0; j < n; j++) {
        double dx = pts[2 * j] - xi, dy = pts[2 * j + 1] - yi;
        d[j] = sqrt(dx * dx + dy * dy);
        bad[j] = (unsigned char)(gone[j] || j == i);
      }
      /* the closest point whose midpoint with p_i is on the boundary: the
         nearest (ties: lower index), then the next nearest, ... */
      int64_t bj = -1;
      double mx = 0, my = 0;
      for (;;) {
        int64_t c = -1;
        for (int64_t j = 0; j < n; j++)
          if (!bad[j] && (c < 0 || d[j] < d[c])) c = j;
        if (c < 0) break;
        mx = 0.5 * (xi + pts[2 * c]);
        my = 0.5 * (yi + pts[2 * c + 1]);
        if (fabs(orc_sdf_eval(prims, nprims, poly, mx, my)) <= geps) {
          bj = c;
          break;
        }
        bad[c] = 1;
      }
      if (bj < 0 || d[bj] >= d_s) {
        done[i] = 1;
        continue;
      }
      gone[bj] = 1;
      pts[2 * i] = mx;
      pts[2 * i + 1] = my;
      changed = 1;
    }
  }
  int64_t m = 0;
  for (int64_t i = 0; i < n; i++)
    if (!gone[i]) {
      pts[2 * m] = pts[2 * i];
      pts[2 * m + 1] = pts[2 * i + 1];
      m++;
    }
  free(gone); free(done); free(bad); free(d);
  return m;
}
