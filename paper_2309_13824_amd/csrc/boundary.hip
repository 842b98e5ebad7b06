// Boundary points for the automatic sizing field (App. A): the dense initial
// set and its trimming.  Host code: the trimming is a serial pass whose
// result depends on its order (points move and disappear one after
// another), so it runs on the CPU, with a uniform grid for the nearest-point
// searches.  The on-boundary tests evaluate the geometry's signed distance
// exactly (every primitive, the set operations of Sec. 3.1).
#include <math.h>

#include <algorithm>
#include <vector>

#include "prim_sdf.hpp"
#include "segsdf_dev.hpp"

namespace trime {

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
  bool inside(double x, double y) const { return x >= x0 && y >= y0 && x < x0 + nx * cs && y < y0 + ny * cs; }
};

// A segment loop with its segments bucketed by the cells their boxes meet:
// the nearest segment (ties to the lower index) by rings of cells outward,
// settled once nearer than every cell not yet visited.  Points off the grid,
// and points so far from the loop that the rings would hold many more cells
// than the loop has segments, search every segment instead.  Either way the
// same segment as a brute-force scan.
struct LoopIndex {
  const double *v = nullptr;
  int nv = 0;
  Buckets B;
  void build(const double *verts, int n) {
    v = verts;
    nv = n;
    double x0 = INFINITY, y0 = INFINITY, x1 = -INFINITY, y1 = -INFINITY, len = 0;
    for (int k = 0; k < nv; k++) {
      const int k1 = k + 1 == nv ? 0 : k + 1;
      x0 = fmin(x0, v[2 * k]);
      y0 = fmin(y0, v[2 * k + 1]);
      x1 = fmax(x1, v[2 * k]);
      y1 = fmax(y1, v[2 * k + 1]);
      len += hypot(v[2 * k1] - v[2 * k], v[2 * k1 + 1] - v[2 * k + 1]);
    }
    B.init(x0, y0, x1, y1, len / nv);
    for (int k = 0; k < nv; k++) {
      const int k1 = k + 1 == nv ? 0 : k + 1;
      for (int j = B.cy(fmin(v[2 * k + 1], v[2 * k1 + 1])); j <= B.cy(fmax(v[2 * k + 1], v[2 * k1 + 1])); j++)
        for (int i = B.cx(fmin(v[2 * k], v[2 * k1])); i <= B.cx(fmax(v[2 * k], v[2 * k1])); i++)
          B.cell[(size_t)j * B.nx + i].push_back(k);
    }
  }
  double sdf(double x, double y) const {
    if (!B.inside(x, y)) return segments_sdf_brute(v, nv, x, y);
    double best = INFINITY, bt = 0.0;
    int kb = -1;
    const int ci = B.cx(x), cj = B.cy(y);
    const int rmax = std::max(std::max(ci, B.nx - 1 - ci), std::max(cj, B.ny - 1 - cj));
    for (int r = 0; r <= rmax; r++) {
      if ((int64_t)(2 * r + 1) * (2 * r + 1) > 2 * (int64_t)nv) return segments_sdf_brute(v, nv, x, y);
      for (int j = cj - r; j <= cj + r; j++) {
        if (j < 0 || j >= B.ny) continue;
        const bool edge_row = j == cj - r || j == cj + r;
        for (int i = ci - r; i <= ci + r; i += (edge_row || r == 0) ? 1 : 2 * r) {
          if (i < 0 || i >= B.nx) continue;
          for (int32_t k : B.cell[(size_t)j * B.nx + i]) {
            double t;
            const double d = seg_dist_t(v, nv, k, x, y, t);
            if (d < best || (d == best && k < kb)) {
              best = d;
              bt = t;
              kb = k;
            }
          }
        }
      }
      if (kb >= 0 && best < (double)r * B.cs) break;  // ring r + 1 lies at least r cells away
    }
    return kb < 0 ? INFINITY : seg_signed(v, nv, kb, bt, best, x, y);
  }
};

}  // namespace

// The geometry's signed distance at (x, y): every primitive, combined by
// its set operation; segment loops through their indexes.
struct GeometryEval {
  const trime_geometry *geo;
  std::vector<LoopIndex> loops;
  explicit GeometryEval(const trime_geometry *g) : geo(g), loops((size_t)g->nprims) {
    for (int k = 0; k < g->nprims; k++)
      if (g->prims[k].kind == TRIME_PRIM_SEGMENTS) loops[k].build(g->poly + 2 * (size_t)g->prims[k].voff, g->prims[k].nv);
  }
  double operator()(double x, double y) const {
    double sd = INFINITY;
    for (int k = 0; k < geo->nprims; k++) {
      const trime_prim &pr = geo->prims[k];
      const double t = pr.kind == TRIME_PRIM_SEGMENTS ? loops[k].sdf(x, y) : analytic_sdf(pr, geo->poly, x, y);
      switch (pr.op) {
        case TRIME_OP_INIT: sd = t; break;
        case TRIME_OP_UNION: sd = fmin(sd, t); break;
        case TRIME_OP_DIFF: sd = fmax(sd, -t); break;
        default: sd = fmax(sd, t); break;
      }
    }
    return sd;
  }
};

double geometry_sdf(const trime_geometry *geo, double x, double y) { return GeometryEval(geo)(x, y); }

namespace {

constexpr double TWO_PI = 6.283185307179586;

// The vertices of a closed loop and floor(L / d_s) points splitting each of
// its segments longer than d_s.
void loop_points(const double *v, int nv, double d_s, std::vector<double> &out) {
  for (int k = 0; k < nv; k++) {
    const int k1 = k + 1 == nv ? 0 : k + 1;
    const double ax = v[2 * k], ay = v[2 * k + 1], bx = v[2 * k1], by = v[2 * k1 + 1];
    const double L = sqrt((bx - ax) * (bx - ax) + (by - ay) * (by - ay));
    const int64_t pieces = L > d_s ? (int64_t)floor(L / d_s) + 1 : 1;
    for (int64_t i = 0; i < pieces; i++) {
      const double t = (double)i / (double)pieces;
      out.push_back(ax + t * (bx - ax));
      out.push_back(ay + t * (by - ay));
    }
  }
}

}  // namespace

std::vector<double> boundary_points(const trime_geometry *geo, double d_s, double geps) {
  const GeometryEval sdf(geo);
  std::vector<double> raw, out;
  for (int q = 0; q < geo->nprims; q++) {
    const trime_prim &p = geo->prims[q];
    raw.clear();
    switch (p.kind) {
      case TRIME_PRIM_DISK: {
        const int64_t m = std::max<int64_t>(3, (int64_t)floor(TWO_PI * p.p[2] / d_s) + 1);
        for (int64_t k = 0; k < m; k++) {
          const double th = TWO_PI * (double)k / (double)m;
          raw.push_back(p.p[0] + p.p[2] * cos(th));
          raw.push_back(p.p[1] + p.p[2] * sin(th));
        }
        break;
      }
      case TRIME_PRIM_ELLIPSE: {
        const double c = cos(p.p[4]), sn = sin(p.p[4]);
        const int64_t m = std::max<int64_t>(3, (int64_t)floor(TWO_PI * fmax(p.p[2], p.p[3]) / d_s) + 1);
        for (int64_t k = 0; k < m; k++) {
          const double th = TWO_PI * (double)k / (double)m;
          const double u = p.p[2] * cos(th), w = p.p[3] * sin(th);
          raw.push_back(p.p[0] + (c * u - sn * w));
          raw.push_back(p.p[1] + (sn * u + c * w));
        }
        break;
      }
      case TRIME_PRIM_BOX: {
        const double v[8] = {p.p[0], p.p[1], p.p[0], p.p[3], p.p[2], p.p[3], p.p[2], p.p[1]};
        loop_points(v, 4, d_s, raw);
        break;
      }
      default:  // polygon or segment loop
        loop_points(geo->poly + 2 * (size_t)p.voff, p.nv, d_s, raw);
        break;
    }
    // the parts of this primitive's boundary that bound the whole geometry
    for (size_t i = 0; i < raw.size(); i += 2)
      if (fabs(sdf(raw[i], raw[i + 1])) <= geps) {
        out.push_back(raw[i]);
        out.push_back(raw[i + 1]);
      }
  }
  return out;
}


// App. A trimming, in place; returns the remaining points in order.
std::vector<double> trim_boundary(const trime_geometry *geo, double d_s, double geps, const std::vector<double> &in) {
  std::vector<double> pts = in;
  const int64_t n = (int64_t)pts.size() / 2;
  if (n == 0) return pts;
  const GeometryEval sdf(geo);
  auto on_boundary = [&](double x, double y) { return fabs(sdf(x, y)) <= geps; };
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
