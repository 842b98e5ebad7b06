// Boundary points of segment loops for the automatic sizing field (App. A):
// the dense initial set and its trimming.  Host code: the trimming is a
// serial pass whose result depends on its order (points move and disappear
// one after another), so it runs on the CPU, with a uniform grid for the
// nearest-point searches and a bucket grid of segments for the on-boundary
// test of midpoints.
#include <math.h>

#include <algorithm>
#include <vector>

#include "launch.hpp"

namespace trime {

std::vector<double> boundary_points(const trime_geometry *geo, double d_s) {
  std::vector<double> out;
  for (int q = 0; q < geo->nprims; q++) {
    const trime_prim &p = geo->prims[q];
    if (p.kind != TRIME_PRIM_SEGMENTS) continue;
    const double *v = geo->poly + 2 * (size_t)p.voff;
    for (int k = 0; k < p.nv; k++) {
      const int k1 = k + 1 == p.nv ? 0 : k + 1;
      const double ax = v[2 * k], ay = v[2 * k + 1], bx = v[2 * k1], by = v[2 * k1 + 1];
      const double L = sqrt((bx - ax) * (bx - ax) + (by - ay) * (by - ay));
      // the vertex, then floor(L / d_s) points splitting a longer segment
      const int64_t pieces = L > d_s ? (int64_t)floor(L / d_s) + 1 : 1;
      for (int64_t i = 0; i < pieces; i++) {
        const double t = (double)i / (double)pieces;
        out.push_back(ax + t * (bx - ax));
        out.push_back(ay + t * (by - ay));
      }
    }
  }
  return out;
}

namespace {

struct Buckets {
  double x0 = 0, y0 = 0, cs = 1;
  int nx = 1, ny = 1;
  std::vector<std::vector<int32_t>> cell;
  void init(double bx0, double by0, double bx1, double by1, double size) {
    const double W = fmax(bx1 - bx0, 1e-300), H = fmax(by1 - by0, 1e-300);
    cs = fmax(size, fmax(W, H) / 1024.0);
    nx = (int)fmin(ceil(W / cs) + 1, 1025.0);
    ny = (int)fmin(ceil(H / cs) + 1, 1025.0);
    x0 = bx0;
    y0 = by0;
    cell.assign((size_t)nx * ny, {});
  }
  int cx(double x) const { return std::min(std::max((int)floor((x - x0) / cs), 0), nx - 1); }
  int cy(double y) const { return std::min(std::max((int)floor((y - y0) / cs), 0), ny - 1); }
};

struct Seg {
  double ax, ay, bx, by;
};

// Distance from (x, y) to the segment, by the operations of the segment
// distance everywhere else in the library.
double seg_dist(const Seg &g, double x, double y) {
  const double ex = g.bx - g.ax, ey = g.by - g.ay, wx = x - g.ax, wy = y - g.ay;
  const double L2 = ex * ex + ey * ey;
  double t = L2 > 0 ? (wx * ex + wy * ey) / L2 : 0.0;
  t = t < 0 ? 0.0 : (t > 1 ? 1.0 : t);
  const double qx = wx - t * ex, qy = wy - t * ey;
  return sqrt(qx * qx + qy * qy);
}

}  // namespace

// App. A trimming, in place; returns the remaining points in order.
std::vector<double> trim_boundary(const trime_geometry *geo, double d_s, double geps, const std::vector<double> &in) {
  // segments of the loops, bucketed by the cells their boxes overlap (cells
  // of at least geps: a segment within geps of a point meets the 3 x 3
  // cells around it)
  std::vector<Seg> segs;
  double sx0 = INFINITY, sy0 = INFINITY, sx1 = -INFINITY, sy1 = -INFINITY, len = 0;
  for (int q = 0; q < geo->nprims; q++) {
    const trime_prim &p = geo->prims[q];
    if (p.kind != TRIME_PRIM_SEGMENTS) continue;
    const double *v = geo->poly + 2 * (size_t)p.voff;
    for (int k = 0; k < p.nv; k++) {
      const int k1 = k + 1 == p.nv ? 0 : k + 1;
      Seg g{v[2 * k], v[2 * k + 1], v[2 * k1], v[2 * k1 + 1]};
      segs.push_back(g);
      sx0 = fmin(sx0, fmin(g.ax, g.bx));
      sy0 = fmin(sy0, fmin(g.ay, g.by));
      sx1 = fmax(sx1, fmax(g.ax, g.bx));
      sy1 = fmax(sy1, fmax(g.ay, g.by));
      len += hypot(g.bx - g.ax, g.by - g.ay);
    }
  }
  std::vector<double> pts = in;
  const int64_t n = (int64_t)pts.size() / 2;
  if (segs.empty() || n == 0) return pts;
  Buckets SB;
  SB.init(sx0, sy0, sx1, sy1, fmax(len / segs.size(), 2.0 * geps));
  for (size_t k = 0; k < segs.size(); k++) {
    const Seg &g = segs[k];
    for (int j = SB.cy(fmin(g.ay, g.by)); j <= SB.cy(fmax(g.ay, g.by)); j++)
      for (int i = SB.cx(fmin(g.ax, g.bx)); i <= SB.cx(fmax(g.ax, g.bx)); i++)
        SB.cell[(size_t)j * SB.nx + i].push_back((int32_t)k);
  }
  auto on_boundary = [&](double x, double y) {
    const int ci = SB.cx(x), cj = SB.cy(y);
    double d = INFINITY;
    for (int j = std::max(cj - 1, 0); j <= std::min(cj + 1, SB.ny - 1); j++)
      for (int i = std::max(ci - 1, 0); i <= std::min(ci + 1, SB.nx - 1); i++)
        for (int32_t k : SB.cell[(size_t)j * SB.nx + i]) d = fmin(d, seg_dist(segs[k], x, y));
    return d <= geps;
  };
  // points, bucketed by cells of about d_s (they only ever move to midpoints
  // of two of them, so they stay in the box of the initial set)
  double px0 = INFINITY, py0 = INFINITY, px1 = -INFINITY, py1 = -INFINITY;
  for (int64_t i = 0; i < n; i++) {
    px0 = fmin(px0, pts[2 * i]);
    py0 = fmin(py0, pts[2 * i + 1]);
    px1 = fmax(px1, pts[2 * i]);
    py1 = fmax(py1, pts[2 * i + 1]);
  }
  Buckets PB;
  PB.init(px0, py0, px1, py1, d_s);
  std::vector<int> where((size_t)n);
  for (int64_t i = 0; i < n; i++) {
    const int c = PB.cy(pts[2 * i + 1]) * PB.nx + PB.cx(pts[2 * i]);
    where[i] = c;
    PB.cell[c].push_back((int32_t)i);
  }
  std::vector<unsigned char> gone((size_t)n, 0), done((size_t)n, 0);
  std::vector<std::pair<double, int64_t>> pend;
  bool changed = true;
  while (changed) {
    changed = false;
    for (int64_t i = 0; i < n; i++) {
      if (gone[i] || done[i]) continue;
      const double xi = pts[2 * i], yi = pts[2 * i + 1];
      const int ci = PB.cx(xi), cj = PB.cy(yi);
      const int rmax = std::max(std::max(ci, PB.nx - 1 - ci), std::max(cj, PB.ny - 1 - cj));
      // rings outward; a candidate is settled once it is nearer than every
      // cell not yet visited (ring r + 1 lies at least r cells away)
      pend.clear();
      int64_t bj = -1;
      double mx = 0, my = 0, bd = 0;
      size_t head = 0;
      for (int r = 0; r <= rmax && bj < 0; r++) {
        for (int j = cj - r; j <= cj + r; j++) {
          if (j < 0 || j >= PB.ny) continue;
          const bool edge_row = j == cj - r || j == cj + r;
          for (int ii = ci - r; ii <= ci + r; ii += (edge_row || r == 0) ? 1 : 2 * r) {
            if (ii < 0 || ii >= PB.nx) continue;
            for (int32_t k : PB.cell[(size_t)j * PB.nx + ii]) {
              if (k == i || gone[k]) continue;
              const double dx = pts[2 * k] - xi, dy = pts[2 * k + 1] - yi;
              pend.emplace_back(sqrt(dx * dx + dy * dy), (int64_t)k);
            }
          }
        }
        std::sort(pend.begin() + head, pend.end());
        const double lb = r < rmax ? (double)r * PB.cs : INFINITY;
        while (head < pend.size() && pend[head].first < lb) {
          const int64_t c = pend[head].second;
          const double cxm = 0.5 * (xi + pts[2 * c]), cym = 0.5 * (yi + pts[2 * c + 1]);
          if (on_boundary(cxm, cym)) {
            bj = c;
            bd = pend[head].first;
            mx = cxm;
            my = cym;
            break;
          }
          head++;
        }
      }
      if (bj < 0 || bd >= d_s) {
        done[i] = 1;
        continue;
      }
      gone[bj] = 1;
      auto &vb = PB.cell[where[bj]];
      vb.erase(std::find(vb.begin(), vb.end(), (int32_t)bj));
      pts[2 * i] = mx;
      pts[2 * i + 1] = my;
      const int c = PB.cy(my) * PB.nx + PB.cx(mx);
      if (c != where[i]) {
        auto &vi = PB.cell[where[i]];
        vi.erase(std::find(vi.begin(), vi.end(), (int32_t)i));
        PB.cell[c].push_back((int32_t)i);
        where[i] = c;
      }
      changed = true;
    }
  }
  std::vector<double> out;
  for (int64_t i = 0; i < n; i++)
    if (!gone[i]) {
      out.push_back(pts[2 * i]);
      out.push_back(pts[2 * i + 1]);
    }
  return out;
}

}  // namespace trime
