// Bounded Voronoi cells, Delaunay extraction and the CVD centroid step.
//
// One lane per point (slot order = Morton bins), 64 consecutive points per
// wavefront.  A lane builds its cell (Sec. 2.1, Sec. 4.1): the octagon of
// span S around p, cut by the bisector of every neighbour found in the rings
// of bins around p, stopping once the nearest unvisited ring is farther than
// twice the largest vertex distance.  The polygon lives in LDS, one column
// per lane ([vertex][lane], conflict-free).
//
// Every cut decision is a margin with a forward error bound: FP32 (or FP64)
// vertex coordinates carry an error bound E; a decision whose |margin| is
// within the bound is "unsure".  The fast kernels push such points to a
// queue; the replay kernel recomputes them in FP64 and settles what FP64
// cannot with the exact expansion predicate (exact_dev.hpp) and symbolic
// perturbation.  The cells are therefore the exact cells of one perturbed
// configuration, whatever the precision, order, bin size or batching.
//
// After the cell: triangles at the cell vertices between two bisectors
// (Proc. I line 2) that are vertices of all three cells, validity Tests 1-3
// (line 3), adjacency of valid triangles, quality statistics (Eq. 10-11),
// and in CVD mode the adaptive-quadrature centroid (Sec. 4.2 II) and the
// treatment of the new point (Sec. 4.3).
#include "exact_dev.hpp"
#include "geom_dev.hpp"
#include "launch.hpp"

namespace trime {

template <class T> struct Row {
  T nx, ny, s;
};

TRIME_D void oct_normal(int w, int &nx, int &ny) {
  // outward normals of the octagon walls, counter-clockwise from +x
  nx = (w == 0 || w == 1 || w == 7) ? 1 : ((w == 3 || w == 4 || w == 5) ? -1 : 0);
  ny = (w == 1 || w == 2 || w == 3) ? 1 : ((w == 5 || w == 6 || w == 7) ? -1 : 0);
}

// Constraint row in the frame of p: >= 0 a slot (bisector), -1-w a wall.
template <class T>
TRIME_D Row<T> row_of(const KArgs &a, int con, double px, double py, float S, float D) {
  Row<T> r;
  if (con >= 0) {
    r.nx = (T)(a.x[con] - px);
    r.ny = (T)(a.y[con] - py);
    r.s = (r.nx * r.nx + r.ny * r.ny) * (T)0.5;
  } else {
    int w = -1 - con;
    if (w < 8) {
      int nx, ny;
      oct_normal(w, nx, ny);
      r.nx = (T)nx;
      r.ny = (T)ny;
      r.s = (w & 1) ? (T)D : (T)S;
    } else if (w == 8) {
      r.nx = 1; r.ny = 0; r.s = (T)(a.box_x1 - px);
    } else if (w == 9) {
      r.nx = 0; r.ny = 1; r.s = (T)(a.box_y1 - py);
    } else if (w == 10) {
      r.nx = -1; r.ny = 0; r.s = (T)(px - a.box_x0);
    } else {
      r.nx = 0; r.ny = -1; r.s = (T)(py - a.box_y0);
    }
  }
  return r;
}

TRIME_D void xrow_of(const KArgs &a, ex::XRow &r, int con, double px, double py, float S, float D,
                     int *err) {
  if (con >= 0) {
    ex::bisector(r, a.id[con], a.x[con], a.y[con], px, py, err);
  } else {
    int w = -1 - con;
    if (w < 8) {
      int nx, ny;
      oct_normal(w, nx, ny);
      ex::wall(r, nx, ny, false, (w & 1) ? (double)D : (double)S, 0.0, px, py);
    } else if (w == 8) {
      ex::wall(r, 1, 0, true, 0.0, a.box_x1, px, py);
    } else if (w == 9) {
      ex::wall(r, 0, 1, true, 0.0, a.box_y1, px, py);
    } else if (w == 10) {
      ex::wall(r, -1, 0, true, 0.0, a.box_x0, px, py);
    } else {
      ex::wall(r, 0, -1, true, 0.0, a.box_y0, px, py);
    }
  }
}

struct ExactCount {
  int calls = 0, sos = 0, err = 0;
};

// Exact sign of the margin of c3 at the vertex (c1, c2) in the frame of the
// point at (px, py) with id pid.
TRIME_D int exact_cut(const KArgs &a, int c1, int c2, int c3, int pid, double px, double py,
                      float S, float D, ExactCount &ec) {
  ex::XRow r1, r2, r3;
  int err = 0, sos = 0;
  xrow_of(a, r1, c1, px, py, S, D, &err);
  xrow_of(a, r2, c2, px, py, S, D, &err);
  xrow_of(a, r3, c3, px, py, S, D, &err);
  int s = ex::margin_sign(&r1, &r2, &r3, pid, &err, &sos);
  ec.calls++;
  ec.sos += sos;
  ec.err |= err;
  return s;
}

// Vertex of two constraint rows by Cramer's rule with a forward error bound
// E on each coordinate (inputs: n with relative error u, s with 4u):
//   |dv| <= (7u max|num| + 4u |v| detabs) / |det| + 2u |v|,
// doubled, plus the 6u|v| term of the cut test's own rounding.  Returns false
// (E = inf) for an ill-conditioned pair (|det| <= 64u detabs).
template <class T>
TRIME_D bool make_vertex(const Row<T> &r1, const Row<T> &r2, T &vx, T &vy, float &E) {
  const T u = U<T>::v;
  T det = r1.nx * r2.ny - r1.ny * r2.nx;
  T detabs = fabs(r1.nx * r2.ny) + fabs(r1.ny * r2.nx);
  T numx = r1.s * r2.ny - r2.s * r1.ny;
  T numy = r1.nx * r2.s - r2.nx * r1.s;
  vx = numx / det;
  vy = numy / det;
  T vmax = fmax(fabs(vx), fabs(vy));
  if (!(fabs(det) > (T)64 * u * detabs) || !isfinite(vmax)) {
    E = INFINITY;
    if (!isfinite(vx) || !isfinite(vy)) {
      vx = 0;
      vy = 0;
    }
    return false;
  }
  T ax = fabs(r1.s * r2.ny) + fabs(r2.s * r1.ny);
  T ay = fabs(r1.nx * r2.s) + fabs(r2.nx * r1.s);
  T e = ((T)7 * u * fmax(ax, ay) + (T)4 * u * vmax * detabs) / fabs(det) + (T)2 * u * vmax;
  E = (float)((T)2 * e + (T)6 * u * vmax) * 1.00001f;
  return true;
}

template <class T, int VMAX, int BLOCK> struct Poly {
  T vx[VMAX][BLOCK];
  T vy[VMAX][BLOCK];
  float ev[VMAX][BLOCK];
  int con[VMAX][BLOCK];
};

struct LaneStats {
  double sa = 0, sb = 0, sq = 0, amax = 0;
  int nq = 0, ntri = 0, nvalid = 0;
  int replays = 0, exact_pts = 0, exact_calls = 0, sos = 0, overflow = 0, empty = 0;
  int newton_fail = 0, trace_fail = 0, cap_hits = 0;
};

template <class T, class G, int MODE, bool EXACT, int VMAX, int BLOCK> struct CellLane {
  const KArgs &a;
  Poly<T, VMAX, BLOCK> &P;
  int tid;
  int64_t k;
  int pid;
  double px, py;
  float S, D;
  int n = 0;
  bool bad = false;
  bool overflow = false;
  T R2 = 0;
  ExactCount ec;
  int hb[TRIME_TRI_PER_POINT];  // beta-histogram bins of the owned valid triangles
  int nhb = 0;

  TRIME_D CellLane(const KArgs &a_, Poly<T, VMAX, BLOCK> &P_, int tid_, int64_t k_)
      : a(a_), P(P_), tid(tid_), k(k_) {}

  TRIME_D void set_vertex(int j, T vx, T vy, float e, int con) {
    P.vx[j][tid] = vx;
    P.vy[j][tid] = vy;
    P.ev[j][tid] = e;
    P.con[j][tid] = con;
  }

  TRIME_D void copy_vertex(int dst, int src) {
    P.vx[dst][tid] = P.vx[src][tid];
    P.vy[dst][tid] = P.vy[src][tid];
    P.ev[dst][tid] = P.ev[src][tid];
    P.con[dst][tid] = P.con[src][tid];
  }

  // |v_true|^2 bound over all vertices, capped by the octagon's circumradius
  TRIME_D void update_R2() {
    const T u = U<T>::v;
    T r2 = 0;
    for (int j = 0; j < n; j++) {
      T vx = P.vx[j][tid], vy = P.vy[j][tid];
      T E = (T)P.ev[j][tid];
      T l1 = fabs(vx) + fabs(vy);
      T t = (vx * vx + vy * vy) * ((T)1 + (T)8 * u) + (T)4 * l1 * E + (T)4 * E * E;
      r2 = fmax(r2, t);
    }
    T cap = (T)((double)S * (double)S * 1.1717 * 1.00001);
    R2 = isfinite(r2) ? fmin(r2, cap) : cap;
  }

  // Initial polygon: the octagon, or (replay kernel) the octagon clipped by
  // the box when the box is within reach.
  TRIME_D void init_polygon() {
    for (int w = 0; w < 8; w++) {
      Row<T> r1 = row_of<T>(a, -1 - ((w + 7) & 7), px, py, S, D);
      Row<T> r2 = row_of<T>(a, -1 - w, px, py, S, D);
      T vx, vy;
      float e;
      make_vertex<T>(r1, r2, vx, vy, e);
      set_vertex(w, vx, vy, e, -1 - w);
    }
    n = 8;
    double reach = (double)S * 1.0001 + 1e-300;
    bool clear = (a.box_x1 - px) > reach && (px - a.box_x0) > reach && (a.box_y1 - py) > reach &&
                 (py - a.box_y0) > reach;
    if (!clear) {
      if constexpr (!EXACT) {
        bad = true;
        return;
      } else {
        for (int w = 8; w < 12 && n > 0; w++) {
          Row<T> r3 = row_of<T>(a, -1 - w, px, py, S, D);
          clip(r3, -1 - w);
          if (bad) return;
        }
      }
    }
    update_R2();
  }

  // Cut the polygon by constraint c3 (row r3).
  TRIME_D void clip(const Row<T> &r3, int c3) {
    const T u = U<T>::v;
    uint32_t M = 0;
    T n1 = fabs(r3.nx) + fabs(r3.ny);
    T b0 = (T)12 * u * fabs(r3.s);
    for (int j = 0; j < n; j++) {
      T vx = P.vx[j][tid], vy = P.vy[j][tid];
      T E = (T)P.ev[j][tid];
      T m = fma(r3.nx, vx, fma(r3.ny, vy, -r3.s));
      T b = fma(n1, E, b0);
      if (m > b) {
        M |= 1u << j;
      } else if (m >= -b) {
        if constexpr (EXACT) {
          int c1 = P.con[j == 0 ? n - 1 : j - 1][tid], c2 = P.con[j][tid];
          if (exact_cut(a, c1, c2, c3, pid, px, py, S, D, ec) > 0) M |= 1u << j;
        } else {
          bad = true;
          return;
        }
      }
    }
    if (M == 0) return;
    uint32_t full = (n == 32) ? 0xffffffffu : ((1u << n) - 1u);
    if (M == full) {
      n = 0;
      return;
    }
    uint32_t Pm = ((M << 1) | (M >> (n - 1))) & full;
    uint32_t Nm = ((M >> 1) | (M << (n - 1))) & full;
    uint32_t starts = M & ~Pm, ends = M & ~Nm;
    if (__popc(starts) != 1) {  // impossible with exact decisions
      bad = true;
      return;
    }
    int k0 = __ffs(starts) - 1, k1 = __ffs(ends) - 1;
    int r = __popc(M);
    int nn = n - r + 2;
    if (nn > VMAX) {
      bad = true;
      overflow = true;
      return;
    }
    int cin = P.con[k0 == 0 ? n - 1 : k0 - 1][tid];
    int cout = P.con[k1][tid];
    Row<T> ri = row_of<T>(a, cin, px, py, S, D);
    Row<T> ro = row_of<T>(a, cout, px, py, S, D);
    T x1, y1, x2, y2;
    float e1, e2;
    bool ok1 = make_vertex<T>(ri, r3, x1, y1, e1);
    bool ok2 = make_vertex<T>(r3, ro, x2, y2, e2);
    if constexpr (!EXACT) {
      if (!ok1 || !ok2) {
        bad = true;
        return;
      }
    }
    if (k0 <= k1) {
      if (r >= 2) {
        int sh = r - 2;
        if (sh > 0)
          for (int j = k1 + 1; j < n; j++) copy_vertex(j - sh, j);
      } else {
        for (int j = n - 1; j > k1; j--) copy_vertex(j + 1, j);
      }
      set_vertex(k0, x1, y1, e1, c3);
      set_vertex(k0 + 1, x2, y2, e2, cout);
    } else {
      int m = 0;
      for (int j = k1 + 1; j < k0; j++, m++) copy_vertex(m, j);
      set_vertex(m, x1, y1, e1, c3);
      set_vertex(m + 1, x2, y2, e2, cout);
    }
    n = nn;
    update_R2();
  }

  // Scan the rings of bins around p.
  TRIME_D void scan() {
    const T u = U<T>::v;
    int bx, by;
    bin_of(a, px, py, bx, by);
    double ox = px - (a.bx0 + bx * a.bw), oy = py - (a.by0 + by * a.bw);
    double edge = fmax(0.0, fmin(fmin(ox, a.bw - ox), fmin(oy, a.bw - oy)));
    int rmax = max(a.nbx, a.nby);
    for (int r = 0; r <= rmax; r++) {
      if (r > 0) {
        double dmin = (r - 1) * a.bw + edge;
        if (dmin * dmin > 4.0 * (double)R2 * 1.00001) break;
      }
      for (int dy = -r; dy <= r; dy++) {
        int yy = by + dy;
        if (yy < 0 || yy >= a.nby) continue;
        int step = (r == 0 || dy == -r || dy == r) ? 1 : 2 * r;
        for (int dx = -r; dx <= r; dx += step) {
          int xx = bx + dx;
          if (xx < 0 || xx >= a.nbx) continue;
          uint32_t key = morton((uint32_t)xx, (uint32_t)yy);
          int s0 = a.bin_start[key], s1 = a.bin_start[key + 1];
          for (int s = s0; s < s1; s++) {
            if (s == (int)k) continue;
            Row<T> r3;
            r3.nx = (T)(a.x[s] - px);
            r3.ny = (T)(a.y[s] - py);
            T sq = r3.nx * r3.nx + r3.ny * r3.ny;
            r3.s = sq * (T)0.5;
            if (sq * ((T)1 - (T)8 * u) > (T)4 * R2) continue;
            clip(r3, s);
            if (bad || n == 0) return;
          }
        }
      }
    }
  }

  // Is the cell vertex j (circumcentre of p, q and `other`) inside the
  // octagon of the point in slot q?  1 inside, 0 outside; may set bad.
  TRIME_D int inside_octagon(int j, int q, int other) {
    const T u = U<T>::v;
    T vx = P.vx[j][tid], vy = P.vy[j][tid];
    T E = (T)P.ev[j][tid];
    T qx = (T)(a.x[q] - px), qy = (T)(a.y[q] - py);
    T cx = vx - qx, cy = vy - qy;
    float Sq = a.span[q], Dq = 1.41421356f * Sq;
    T base = E + (T)2 * u * (fabs(qx) + fabs(qy)) + (T)2 * u * (fabs(cx) + fabs(cy));
    for (int w = 0; w < 8; w++) {
      int nx, ny;
      oct_normal(w, nx, ny);
      T s = (w & 1) ? (T)Dq : (T)Sq;
      T m = (T)nx * cx + (T)ny * cy - s;
      T b = (T)2 * ((T)(abs(nx) + abs(ny)) * base + (T)2 * u * s);
      if (m > b) return 0;
      if (m >= -b) {
        if constexpr (EXACT) {
          // in the frame of q: rows bisector(q, p), bisector(q, other), wall w of q
          if (exact_cut(a, (int)k, other, -1 - w, a.id[q], a.x[q], a.y[q], Sq, Dq, ec) > 0)
            return 0;
        } else {
          bad = true;
          return 0;
        }
      }
    }
    return 1;
  }

  TRIME_D bool valid_triangle(int s1, int s2) {
    int i0 = pid, i1 = a.id[s1], i2 = a.id[s2];
    double x0 = px, y0 = py, x1 = a.x[s1], y1 = a.y[s1], x2 = a.x[s2], y2 = a.y[s2];
    // sort by id
    if (i0 > i1) { int t = i0; i0 = i1; i1 = t; double u = x0; x0 = x1; x1 = u; u = y0; y0 = y1; y1 = u; }
    if (i1 > i2) { int t = i1; i1 = i2; i2 = t; double u = x1; x1 = x2; x2 = u; u = y1; y1 = y2; y2 = u; }
    if (i0 > i1) { int t = i0; i0 = i1; i1 = t; double u = x0; x0 = x1; x1 = u; u = y0; y0 = y1; y1 = u; }
    return tri_valid<G>(a, x0, y0, x1, y1, x2, y2);
  }

  TRIME_D void write_cell() {
    int cap = a.cell_cap;
    if (n > cap) {
      a.cell_n[pid] = -1;
      return;
    }
    int s = 0, best = 0x7fffffff;
    for (int j = 0; j < n; j++) {
      int c = P.con[j][tid];
      int v = c >= 0 ? a.id[c] : c;
      if (v < best) {
        best = v;
        s = j;
      }
    }
    for (int t = 0; t < n; t++) {
      int c = P.con[(s + t) % n][tid];
      a.cell_cons[(int64_t)pid * cap + t] = c >= 0 ? a.id[c] : c;
    }
    a.cell_n[pid] = n;
  }

  // Adaptive-quadrature weighted centroid (relative to p) at level L >= 1.
  TRIME_D void level_centroid(int L, double fx0, double fy0, int64_t cx0, int64_t cy0, T &cx,
                              T &cy) {
    T sw = 0, swx = 0, swy = 0;
    const T idx = (T)a.inv_dx, idy = (T)a.inv_dy;
    const T fxf = (T)(fx0 - (double)cx0), fyf = (T)(fy0 - (double)cy0);
    int nleaf = 1 << (L - 1);
    for (int t = 0; t < n; t++) {
      int t1 = (t + 1 == n) ? 0 : t + 1;
      T bx = P.vx[t][tid], by = P.vy[t][tid], ccx = P.vx[t1][tid], ccy = P.vy[t1][tid];
      for (int b = 0; b < nleaf; b++) {
        T x0 = 0, y0 = 0, x1 = bx, y1 = by, x2 = ccx, y2 = ccy;
        for (int d = L - 2; d >= 0; d--) {
          int bit = (b >> d) & 1;
          T l0 = (x1 - x0) * (x1 - x0) + (y1 - y0) * (y1 - y0);
          T l1 = (x2 - x1) * (x2 - x1) + (y2 - y1) * (y2 - y1);
          T l2 = (x0 - x2) * (x0 - x2) + (y0 - y2) * (y0 - y2);
          if (l0 >= l1 && l0 >= l2) {
            T mx = (x0 + x1) * (T)0.5, my = (y0 + y1) * (T)0.5;
            if (!bit) { x1 = mx; y1 = my; } else { x0 = mx; y0 = my; }
          } else if (l1 >= l2) {
            T mx = (x1 + x2) * (T)0.5, my = (y1 + y2) * (T)0.5;
            if (!bit) { x2 = mx; y2 = my; } else { x1 = mx; y1 = my; }
          } else {
            T mx = (x2 + x0) * (T)0.5, my = (y2 + y0) * (T)0.5;
            if (!bit) { x2 = mx; y2 = my; } else { x0 = mx; y0 = my; }
          }
        }
        T A = (T)0.5 * ((x1 - x0) * (y2 - y0) - (y1 - y0) * (x2 - x0));
        T gx = (x0 + x1 + x2) / (T)3, gy = (y0 + y1 + y2) / (T)3;
        // mu at p + g, bilinear in the cell (cells clamped to the grid)
        T fx = fxf + gx * idx, fy = fyf + gy * idy;
        T flx = floor(fx), fly = floor(fy);
        int64_t ci = cx0 + (int64_t)flx, cj = cy0 + (int64_t)fly;
        T tx = fx - flx, ty = fy - fly;
        if (ci < 0) { ci = 0; tx = 0; }
        if (ci > a.nx - 2) { ci = a.nx - 2; tx = 1; }
        if (cj < 0) { cj = 0; ty = 0; }
        if (cj > a.ny - 2) { cj = a.ny - 2; ty = 1; }
        int64_t n0 = cj * a.nx + ci;
        const G *mu = (const G *)a.mu;
        T m = ((T)mu[n0] * ((T)1 - tx) + (T)mu[n0 + 1] * tx) * ((T)1 - ty) +
              ((T)mu[n0 + a.nx] * ((T)1 - tx) + (T)mu[n0 + a.nx + 1] * tx) * ty;
        T w = A / (m * m);
        sw += w;
        swx += w * gx;
        swy += w * gy;
      }
    }
    cx = swx / sw;
    cy = swy / sw;
  }

  TRIME_D void run(LaneStats &st) {
    pid = a.id[k];
    px = a.x[k];
    py = a.y[k];
    S = a.span[k];
    D = 1.41421356f * S;
    if (!(S > 0.0f)) {  // off the grid: the replay kernel keeps the point as is
      bad = true;
      return;
    }
    init_polygon();
    if (!bad) scan();
    if (bad) return;
    if (ec.calls) {
      st.exact_pts++;
      st.exact_calls += ec.calls;
      st.sos += ec.sos;
      if (ec.err) atomicOr(&a.counters[CNT_ERR], ERR_EXACT_CAP);
    }
    if (n == 0) st.empty++;
    if constexpr (MODE == MODE_CELLS) {
      write_cell();
      return;
    } else {
      // ---- triangles, validity, adjacency
      uint32_t exists = 0, valid = 0;
      for (int j = 0; j < n; j++) {
        int jin = P.con[j == 0 ? n - 1 : j - 1][tid], jout = P.con[j][tid];
        if (jin < 0 || jout < 0) continue;
        int e = inside_octagon(j, jin, jout);
        if (bad) return;
        if (e) e = inside_octagon(j, jout, jin);
        if (bad) return;
        if (!e) continue;
        exists |= 1u << j;
        if (valid_triangle(jin, jout)) valid |= 1u << j;
      }
      // owned triangles and their quality
      int nt = 0;
      int64_t tbase = k * TRIME_TRI_PER_POINT;
      for (int j = 0; j < n; j++) {
        if (!((exists >> j) & 1)) continue;
        int jin = P.con[j == 0 ? n - 1 : j - 1][tid], jout = P.con[j][tid];
        if (!(pid < a.id[jin] && pid < a.id[jout])) continue;
        bool v = (valid >> j) & 1;
        if (nt < TRIME_TRI_PER_POINT) {
          a.tri[(tbase + nt) * 3 + 0] = (int)k;
          a.tri[(tbase + nt) * 3 + 1] = jin;
          a.tri[(tbase + nt) * 3 + 2] = jout;
          a.tri_valid[tbase + nt] = v;
        } else {
          atomicOr(&a.counters[CNT_ERR], ERR_TRI_CAP);
        }
        nt++;
        st.ntri++;
        if (v) {
          st.nvalid++;
          double x1 = a.x[jin], y1 = a.y[jin], x2 = a.x[jout], y2 = a.y[jout];
          double l0 = sqrt((x1 - px) * (x1 - px) + (y1 - py) * (y1 - py));
          double l1 = sqrt((x2 - x1) * (x2 - x1) + (y2 - y1) * (y2 - y1));
          double l2 = sqrt((px - x2) * (px - x2) + (py - y2) * (py - y2));
          double A2 = fabs((x1 - px) * (y2 - py) - (y1 - py) * (x2 - px));
          double al = (l0 * l1 * l2) * (l0 + l1 + l2) / (4.0 * A2 * A2);
          double be = fmax(l0, fmax(l1, l2)) / fmin(l0, fmin(l1, l2));
          st.sa += sqrt(al);
          st.sb += sqrt(be);
          st.sq += 1.0 / al;
          st.amax = fmax(st.amax, al);
          st.nq++;
          int bin = (int)floor((be - 1.0) / 2.0 * 40.0);
          bin = bin < 0 ? 0 : (bin > 39 ? 39 : bin);
          if (nhb < TRIME_TRI_PER_POINT) hb[nhb++] = bin;
        }
      }
      a.tri_n[k] = nt < TRIME_TRI_PER_POINT ? nt : TRIME_TRI_PER_POINT;
      if constexpr (MODE == MODE_EXTRACT) {
        // adjacency row: edge j is kept when a valid triangle sits at one of
        // its two ends (vertices j and j + 1); sorted by slot
        int cnt = 0;
        int *row = (int *)&P.ev[0][0];  // reuse the error-bound column
        for (int j = 0; j < n; j++) {
          int c = P.con[j][tid];
          int jn = (j + 1 == n) ? 0 : j + 1;
          if (c < 0 || !(((valid >> j) & 1) || ((valid >> jn) & 1))) continue;
          int t = cnt++;
          while (t > 0 && row[(t - 1) * BLOCK + tid] > c) {
            row[t * BLOCK + tid] = row[(t - 1) * BLOCK + tid];
            t--;
          }
          row[t * BLOCK + tid] = c;
        }
        int md = a.max_deg;
        if (cnt > md) atomicOr(&a.counters[CNT_ERR], ERR_DEG_CAP);
        int w = cnt < md ? cnt : md;
        for (int t = 0; t < w; t++) a.adj[(int64_t)t * a.n + k] = row[t * BLOCK + tid];
        a.deg[k] = w;
      }
      if constexpr (MODE == MODE_CVD) {
        // ---- CVD centroid (Sec. 4.2 II) and treatment (Sec. 4.3)
        double xo = px, yo = py;
        uint8_t cat_old = a.cat[k];
        double dp = a.dprev[k];
        double xnew = px, ynew = py;
        int64_t cell;
        double tx, ty;
        locate(a, px, py, cell, tx, ty);
        double h = (double)a.hcell[cell];
        if (n > 0) {
          T A = 0;
          for (int j = 0; j < n; j++) {
            int j1 = (j + 1 == n) ? 0 : j + 1;
            A += (T)0.5 * (P.vx[j][tid] * P.vy[j1][tid] - P.vy[j][tid] * P.vx[j1][tid]);
          }
          double eps = fmax((dp < 0 ? h : dp) / h, a.prm.fac_end);
          T E = (T)(sqrt((double)A) * eps);
          T E2 = E * E;
          double fx0 = (px - a.gx0) * a.inv_dx, fy0 = (py - a.gy0) * a.inv_dy;
          int64_t cx0 = (int64_t)floor(fx0), cy0 = (int64_t)floor(fy0);
          T c0x = 0, c0y = 0, c1x = 0, c1y = 0;
          int L;
          for (L = 1;; L++) {
            level_centroid(L, fx0, fy0, cx0, cy0, c1x, c1y);
            T ex_ = c0x - c1x, ey_ = c0y - c1y;
            T d2 = ex_ * ex_ + ey_ * ey_;
            if constexpr (!EXACT && sizeof(T) == 4) {
              if (fabs(d2 - E2) <= (T)1e-2 * E2) {
                bad = true;
                return;
              }
            }
            if (d2 < E2) break;
            if (L >= a.prm.cvd_max_level) {
              st.cap_hits++;
              break;
            }
            c0x = c1x;
            c0y = c1y;
          }
          xnew = px + (double)c1x;
          ynew = py + (double)c1y;
        }
        double band = (!EXACT && sizeof(T) == 4) ? 1e-6 * h : 0.0;
        double xf, yf;
        uint8_t cf;
        bool unsure = false;
        TreatCount tc;
        treat<G>(a, xo, yo, cat_old, xnew, ynew, band, xf, yf, cf, unsure, tc);
        if (unsure) {
          bad = true;
          return;
        }
        st.newton_fail += tc.newton_fail;
        st.trace_fail += tc.trace_fail;
        a.xn[k] = xf;
        a.yn[k] = yf;
        a.catn[k] = cf;
        a.dprevn[k] = sqrt((xf - xo) * (xf - xo) + (yf - yo) * (yf - yo));
      }
    }
  }
};

TRIME_D void merge(LaneStats &d, const LaneStats &s) {
  d.sa += s.sa; d.sb += s.sb; d.sq += s.sq; d.amax = fmax(d.amax, s.amax);
  d.nq += s.nq; d.ntri += s.ntri; d.nvalid += s.nvalid; d.replays += s.replays;
  d.exact_pts += s.exact_pts; d.exact_calls += s.exact_calls; d.sos += s.sos;
  d.overflow += s.overflow; d.empty += s.empty; d.newton_fail += s.newton_fail;
  d.trace_fail += s.trace_fail; d.cap_hits += s.cap_hits;
}

// Block reduction of the lane statistics into the device stats.
template <int BLOCK> TRIME_D void flush_stats(const KArgs &a, LaneStats &st, int *hist) {
  __shared__ double rs[4][BLOCK / 64];
  __shared__ int ri[12][BLOCK / 64];
  double v[4] = {st.sa, st.sb, st.sq, st.amax};
  int iv[12] = {st.nq, st.ntri, st.nvalid, st.replays, st.exact_pts, st.exact_calls,
                st.sos, st.overflow, st.empty, st.newton_fail, st.trace_fail, st.cap_hits};
  int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int off = 32; off > 0; off >>= 1) {
    v[0] += __shfl_down(v[0], off);
    v[1] += __shfl_down(v[1], off);
    v[2] += __shfl_down(v[2], off);
    v[3] = fmax(v[3], __shfl_down(v[3], off));
#pragma unroll
    for (int q = 0; q < 12; q++) iv[q] += __shfl_down(iv[q], off);
  }
  if (lane == 0) {
    for (int q = 0; q < 4; q++) rs[q][wv] = v[q];
    for (int q = 0; q < 12; q++) ri[q][wv] = iv[q];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < BLOCK / 64; w++) {
      rs[0][0] += rs[0][w];
      rs[1][0] += rs[1][w];
      rs[2][0] += rs[2][w];
      rs[3][0] = fmax(rs[3][0], rs[3][w]);
      for (int q = 0; q < 12; q++) ri[q][0] += ri[q][w];
    }
    trime_stats *S = a.stats;
    if (ri[0][0]) {
      atomicAdd(&S->sum_sqrt_alpha, rs[0][0]);
      atomicAdd(&S->sum_sqrt_beta, rs[1][0]);
      atomicAdd(&S->sum_q, rs[2][0]);
      atomicMax((unsigned long long *)&S->max_alpha, (unsigned long long)__double_as_longlong(rs[3][0]));
      atomicAdd((unsigned long long *)&S->nq, (unsigned long long)ri[0][0]);
    }
    unsigned long long *c = (unsigned long long *)S;
    if (ri[1][0]) atomicAdd((unsigned long long *)&S->ntri, (unsigned long long)ri[1][0]);
    if (ri[2][0]) atomicAdd((unsigned long long *)&S->nvalid, (unsigned long long)ri[2][0]);
    if (ri[3][0]) atomicAdd((unsigned long long *)&S->fp64_replays, (unsigned long long)ri[3][0]);
    if (ri[4][0]) atomicAdd((unsigned long long *)&S->exact_points, (unsigned long long)ri[4][0]);
    if (ri[5][0]) atomicAdd((unsigned long long *)&S->exact_calls, (unsigned long long)ri[5][0]);
    if (ri[6][0]) atomicAdd((unsigned long long *)&S->sos_calls, (unsigned long long)ri[6][0]);
    if (ri[7][0]) atomicAdd((unsigned long long *)&S->overflow_points, (unsigned long long)ri[7][0]);
    if (ri[8][0]) atomicAdd((unsigned long long *)&S->empty_cells, (unsigned long long)ri[8][0]);
    if (ri[9][0]) atomicAdd((unsigned long long *)&S->newton_fail, (unsigned long long)ri[9][0]);
    if (ri[10][0]) atomicAdd((unsigned long long *)&S->trace_fail, (unsigned long long)ri[10][0]);
    if (ri[11][0]) atomicAdd((unsigned long long *)&S->level_cap_hits, (unsigned long long)ri[11][0]);
    (void)c;
  }
  for (int b = threadIdx.x; b < 40; b += BLOCK)
    if (hist[b]) atomicAdd((unsigned long long *)&a.stats->hist_beta[b], (unsigned long long)hist[b]);
}

template <int BLOCK> TRIME_D void zero_hist(int *hist) {
  for (int b = threadIdx.x; b < 40; b += BLOCK) hist[b] = 0;
  __syncthreads();
}

// Fast kernel: one point per lane; unsure points are queued for replay.
template <class T, class G, int MODE, int VMAX, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_cells(KArgs a) {
  __shared__ Poly<T, VMAX, BLOCK> P;
  __shared__ int hist[40];
  zero_hist<BLOCK>(hist);
  LaneStats st;
  int64_t k = (int64_t)blockIdx.x * BLOCK + threadIdx.x;
  if (k < a.n) {
    CellLane<T, G, MODE, false, VMAX, BLOCK> L(a, P, threadIdx.x, k);
    LaneStats loc;
    L.run(loc);
    if (L.bad) {
      int q = atomicAdd(&a.counters[CNT_QUEUE], 1);
      a.queue[q] = (int)k;
      if (L.overflow) st.overflow++;
      st.replays++;
    } else {
      merge(st, loc);
      for (int b = 0; b < L.nhb; b++) atomicAdd(&hist[L.hb[b]], 1);
    }
  }
  flush_stats<BLOCK>(a, st, hist);
}

// Replay kernel: FP64 with the exact stage, over the queue (grid-stride).
template <class G, int MODE, int VMAX, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_cells_replay(KArgs a) {
  __shared__ Poly<double, VMAX, BLOCK> P;
  __shared__ int hist[40];
  zero_hist<BLOCK>(hist);
  LaneStats st;
  int64_t nq = a.counters[CNT_QUEUE];
  for (int64_t w = (int64_t)blockIdx.x * BLOCK + threadIdx.x; w < nq;
       w += (int64_t)gridDim.x * BLOCK) {
    int64_t k = a.queue[w];
    CellLane<double, G, MODE, true, VMAX, BLOCK> L(a, P, threadIdx.x, k);
    LaneStats loc;
    L.run(loc);
    if (!L.bad) {
      merge(st, loc);
      for (int b = 0; b < L.nhb; b++) atomicAdd(&hist[L.hb[b]], 1);
    } else {  // capacity beyond the replay polygon: leave the point as is
      st.overflow++;
      atomicOr(&a.counters[CNT_ERR], ERR_POLY_CAP);
      if constexpr (MODE == MODE_CVD) {
        a.xn[k] = a.x[k];
        a.yn[k] = a.y[k];
        a.catn[k] = a.cat[k];
        a.dprevn[k] = 0.0;
      }
      if constexpr (MODE == MODE_EXTRACT) a.deg[k] = 0;
      if constexpr (MODE != MODE_CELLS) a.tri_n[k] = 0;
      if constexpr (MODE == MODE_CELLS) a.cell_n[a.id[k]] = -1;
    }
  }
  flush_stats<BLOCK>(a, st, hist);
}

// ------------------------------------------------------------ launchers --
constexpr int FAST_BLOCK = 128;
constexpr int FAST_VMAX = 16;
constexpr int REPLAY_BLOCK = 64;
constexpr int REPLAY_VMAX = 32;

template <class T, class G, int MODE> static void launch_mode(const KArgs &a, hipStream_t s) {
  int nb = (int)((a.n + FAST_BLOCK - 1) / FAST_BLOCK);
  if (a.ev0) (void)hipEventRecord((hipEvent_t)a.ev0, s);
  if (nb > 0) hipLaunchKernelGGL((k_cells<T, G, MODE, FAST_VMAX, FAST_BLOCK>), dim3(nb), dim3(FAST_BLOCK), 0, s, a);
  if (a.ev1) (void)hipEventRecord((hipEvent_t)a.ev1, s);
  hipLaunchKernelGGL((k_cells_replay<G, MODE, REPLAY_VMAX, REPLAY_BLOCK>), dim3(256), dim3(REPLAY_BLOCK), 0, s, a);
}

template <class G> static void launch_g(const KArgs &a, int mode, hipStream_t s) {
  if (a.precision == TRIME_FP32) {
    if (mode == MODE_CELLS) launch_mode<float, G, MODE_CELLS>(a, s);
    else if (mode == MODE_EXTRACT) launch_mode<float, G, MODE_EXTRACT>(a, s);
    else launch_mode<float, G, MODE_CVD>(a, s);
  } else {
    if (mode == MODE_CELLS) launch_mode<double, G, MODE_CELLS>(a, s);
    else if (mode == MODE_EXTRACT) launch_mode<double, G, MODE_EXTRACT>(a, s);
    else launch_mode<double, G, MODE_CVD>(a, s);
  }
}

void launch_cells(const KArgs &a, int mode, int grid_bytes, hipStream_t s) {
  if (grid_bytes == 4)
    launch_g<float>(a, mode, s);
  else
    launch_g<double>(a, mode, s);
}

}  // namespace trime
