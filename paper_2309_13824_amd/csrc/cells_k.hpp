// Bounded Voronoi cells, Delaunay extraction and the CVD centroid step.
//
// One lane per point (slot order = Morton bins), 64 consecutive points per
// wavefront.  A lane builds its cell (Sec. 2.1, Sec. 4.1): the octagon of
// span S around p, cut by the bisector of every neighbour found in the rings
// of bins around p, stopping once the nearest unvisited ring is farther than
// twice the largest vertex distance.  The polygon lives in LDS as one
// 16-byte record (x, y, error bound, constraint) per vertex and lane,
// [vertex][lane] so that a wavefront reads 64 consecutive records.  The
// bin/candidate scan is one flat loop (each iteration either opens the next
// bin or tests one candidate), which keeps the lanes of a wavefront in step.
//
// Every cut decision is a margin with a forward error bound: vertex
// coordinates carry an error bound E; a decision whose |margin| is within
// its bound is undecided.  The fast kernel (FP32 or FP64) re-evaluates an
// undecided FP32 cut or octagon test in FP64 on the spot and sends what is
// left to a queue; the FP64 replay kernel (one wavefront per point)
// recomputes those points and passes what FP64 cannot decide to the exact
// kernel, which settles it with expansion arithmetic (exact_dev.hpp) and
// symbolic perturbation.  The cells are
// therefore the exact cells of one perturbed configuration, whatever the
// precision, order, bin size or batching.
//
// After the cell: triangles at the cell vertices between two bisectors
// (Procedure I, Sec. 4.1) that are vertices of all three cells, validity
// Tests 1-3 (Sec. 4.1), adjacency of valid triangles, quality statistics (Eq. 10-11),
// and in CVD mode the adaptive-quadrature centroid (Sec. 4.2 II) and the
// treatment of the new point (Sec. 4.3).  All decisions are taken before
// anything is written, so a point sent to a replay leaves no partial output.
#pragma once
#include "exact_dev.hpp"
#include "geom_dev.hpp"
#include "launch.hpp"

#ifndef TRIME_HEAVY_WAVE
#define TRIME_HEAVY_WAVE 0  // 1: boundary points go to the wavefront-per-point kernel
#endif

namespace trime {

// bins per group of the lane scan (a divisor of 8)
#ifndef TRIME_SCAN_GROUP
#define TRIME_SCAN_GROUP 4
#endif
constexpr int SCAN_GROUP = TRIME_SCAN_GROUP;
static_assert(8 % SCAN_GROUP == 0, "a ring's bins must split into whole groups");

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
    r.nx = (T)(gld(a.x, con) - px);
    r.ny = (T)(gld(a.y, con) - py);
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
    ex::bisector(r, gld(a.id, con), gld(a.x, con), gld(a.y, con), px, py, err);
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
static __device__ __noinline__ int exact_cut(const KArgs &a, int c1, int c2, int c3, int pid, double px,
                                      double py, float S, float D, ExactCount &ec) {
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

template <class T> TRIME_D T recip(T x);
template <> TRIME_D float recip<float>(float x) { return __builtin_amdgcn_rcpf(x); }  // <= 1 ulp
template <> TRIME_D double recip<double>(double x) { return 1.0 / x; }

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
  T inv = recip<T>(det);
  vx = numx * inv;
  vy = numy * inv;
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
  T e = ((T)7 * u * fmax(ax, ay) + (T)4 * u * vmax * detabs) * fabs(inv) + (T)2 * u * vmax;
  E = (float)((T)2 * e + (T)6 * u * vmax) * 1.00001f;
  return true;
}

// One polygon vertex of one lane in LDS.
template <class T> struct VRec;
template <> struct alignas(16) VRec<float> {
  float x, y, e;
  int c;  // constraint of the edge leaving this vertex
};
template <> struct alignas(8) VRec<double> {
  double x, y;
  float e;
  int c;
};

struct LaneStats {
  double sa = 0, sb = 0, sq = 0, amax = 0;
  int nq = 0, ntri = 0, nvalid = 0;
  int replays = 0, exact_pts = 0, exact_calls = 0, sos = 0, overflow = 0, empty = 0;
  int newton_fail = 0, trace_fail = 0, cap_hits = 0;
  int candidates = 0, margins = 0, cuts = 0, leaves = 0;
};

// Algorithmic work of one point: neighbours tested against the range,
// vertex margins evaluated, cuts, quadrature leaf triangles.
struct Work {
  int candidates = 0, margins = 0, cuts = 0, leaves = 0;
};

// Longest-edge bisection of the triangle (x0, y0), (x1, y1), (x2, y2)
// (Sec. 4.2 II): the longest edge (ties to the first of l01, l12, l20) is
// split at its midpoint m; child 0 keeps the endpoint of lower vertex index
// and child 1 the other.
template <class V>
TRIME_D void longest_edge(V x0, V y0, V x1, V y1, V x2, V y2, int &e, V &mx, V &my) {
  V l0 = (x1 - x0) * (x1 - x0) + (y1 - y0) * (y1 - y0);
  V l1 = (x2 - x1) * (x2 - x1) + (y2 - y1) * (y2 - y1);
  V l2 = (x0 - x2) * (x0 - x2) + (y0 - y2) * (y0 - y2);
  if (l0 >= l1 && l0 >= l2) {
    e = 0;
    mx = (x0 + x1) * (V)0.5;
    my = (y0 + y1) * (V)0.5;
  } else if (l1 >= l2) {
    e = 1;
    mx = (x1 + x2) * (V)0.5;
    my = (y1 + y2) * (V)0.5;
  } else {
    e = 2;
    mx = (x2 + x0) * (V)0.5;
    my = (y2 + y0) * (V)0.5;
  }
}

template <class V>
TRIME_D void take_child(int e, int bit, V mx, V my, V &x0, V &y0, V &x1, V &y1, V &x2, V &y2) {
  // the vertex replaced by the midpoint, as selects (no indexed temporaries)
  int r = e == 0 ? (bit ? 0 : 1) : (e == 1 ? (bit ? 1 : 2) : (bit ? 0 : 2));
  x0 = r == 0 ? mx : x0;
  y0 = r == 0 ? my : y0;
  x1 = r == 1 ? mx : x1;
  y1 = r == 1 ? my : y1;
  x2 = r == 2 ? mx : x2;
  y2 = r == 2 ? my : y2;
}

// All leaves K bisections below a triangle, child 0 first (the order of the
// leaf sums is the depth-first order of the bisection tree at every level).
template <int K, class V, class Leaf>
TRIME_D void subtree(V x0, V y0, V x1, V y1, V x2, V y2, Leaf &leaf) {
  if constexpr (K == 0) {
    leaf(x0, y0, x1, y1, x2, y2);
  } else {
    int e;
    V mx, my;
    longest_edge(x0, y0, x1, y1, x2, y2, e, mx, my);
#pragma unroll 1
    for (int bit = 0; bit < 2; bit++) {
      V a0 = x0, b0 = y0, a1 = x1, b1 = y1, a2 = x2, b2 = y2;
      take_child(e, bit, mx, my, a0, b0, a1, b1, a2, b2);
      subtree<K - 1>(a0, b0, a1, b1, a2, b2, leaf);
    }
  }
}

template <class T, class G, int MODE, bool EXACT, int VMAX, int BLOCK> struct Lane {
  const KArgs &a;
  VRec<T> (&P)[VMAX][BLOCK];
  int tid;
  int64_t k;
  int pid;
  double px, py;
  float S, D;
  int n;
  int why;  // nonzero: the point leaves this kernel (WHY_*)
  T R2;
  float Emax = 0.0f;  // >= the error bound of every vertex of the polygon (clip_reg)
  ExactCount ec;
  Work wk;
  double cqx = 0, cqy = 0;  // FP64 offset of the candidate being clipped

  TRIME_D Lane(const KArgs &a_, VRec<T> (&P_)[VMAX][BLOCK], int tid_, int64_t k_)
      : a(a_), P(P_), tid(tid_), k(k_), n(0), why(0), R2(0) {}

  TRIME_D void set_v(int j, T x, T y, float e, int c) {
    VRec<T> r;
    r.x = x;
    r.y = y;
    r.e = e;
    r.c = c;
    P[j][tid] = r;
  }
  TRIME_D int con(int j) const { return P[j][tid].c; }

  // FP64 re-evaluation of one undecided FP32 cut decision: the vertex of
  // constraints (c1, c2) rebuilt in FP64 against constraint c3.  +1 cut,
  // -1 kept, 0 still undecided (then only the exact stage can decide).
  TRIME_D int margin64(int c1, int c2, int c3) const {
    const double u = U<double>::v;
    Row<double> r1 = row_of<double>(a, c1, px, py, S, D), r2 = row_of<double>(a, c2, px, py, S, D);
    Row<double> r3 = row_of<double>(a, c3, px, py, S, D);
    double vx, vy;
    float E;
    if (!make_vertex<double>(r1, r2, vx, vy, E)) return 0;
    double m = fma(r3.nx, vx, fma(r3.ny, vy, -r3.s));
    double b = fma(fabs(r3.nx) + fabs(r3.ny), (double)E, 12.0 * u * fabs(r3.s));
    return m > b ? 1 : (m < -b ? -1 : 0);
  }

  // FP64 vertex j (between the edges j-1 and j), rebuilt from its constraints.
  TRIME_D bool vertex64(int j, double &vx, double &vy, float &E) const {
    int c1 = con(j == 0 ? n - 1 : j - 1), c2 = con(j);
    return make_vertex<double>(row_of<double>(a, c1, px, py, S, D), row_of<double>(a, c2, px, py, S, D),
                               vx, vy, E);
  }

  // A new polygon vertex, between the edges of constraints c1 and c2 (r the
  // row of c3 == c2 or c1, already at hand).  The FP32 mode builds it in
  // FP64 from the FP64 rows and rounds it: an FP32 intersection of two
  // bisectors at angle t carries an error of ~20u h / sin t, which the cells
  // would pass on to their centroids; the rounded FP64 vertex is within
  // u|v| of the true one.  The bound E then covers that rounding plus the
  // FP32 cut test's own (6u|v|).  MI355X issues FP64 FMA at the FP32 rate.
  TRIME_D Row<double> row64(int c, int c3) const {
    if (c == c3 && c3 >= 0) {  // the candidate: its FP64 offset is at hand
      Row<double> r;
      r.nx = cqx;
      r.ny = cqy;
      r.s = (cqx * cqx + cqy * cqy) * 0.5;
      return r;
    }
    return row_of<double>(a, c, px, py, S, D);
  }
  TRIME_D bool new_vertex(int c1, int c2, const Row<T> &r1, const Row<T> &r2, T &vx, T &vy, float &E,
                          int c3) const {
    if constexpr (sizeof(T) == 4) {
      double dx, dy;
      float E64;
      if (!make_vertex<double>(row64(c1, c3), row64(c2, c3), dx, dy, E64)) {
        vx = 0;
        vy = 0;
        E = INFINITY;
        return false;
      }
      vx = (T)dx;
      vy = (T)dy;
      const double vmax = fmax(fabs(dx), fabs(dy));
      E = (float)(((double)E64 + 7.0 * (double)U<float>::v * vmax) * 1.00001);
      return true;
    } else {
      return make_vertex<T>(r1, r2, vx, vy, E);
    }
  }

  // The octagon test of vertex j against wall w of the point q at (qxd, qyd)
  // in FP64, from the FP64 vertex: +1 outside, -1 inside, 0 undecided.
  TRIME_D int oct_margin64(int j, double qxd, double qyd, float Sq, float Dq, int w) const {
    const double u = U<double>::v;
    double vx, vy;
    float E;
    if (!vertex64(j, vx, vy, E)) return 0;
    double qx = qxd - px, qy = qyd - py;
    double cx = vx - qx, cy = vy - qy;
    int nx, ny;
    oct_normal(w, nx, ny);
    double s = (w & 1) ? (double)Dq : (double)Sq;
    double base = (double)E + 2 * u * (fabs(qx) + fabs(qy)) + 2 * u * (fabs(cx) + fabs(cy));
    double m = (double)nx * cx + (double)ny * cy - s;
    double b = 2 * ((double)(abs(nx) + abs(ny)) * base + 2 * u * s);
    return m > b ? 1 : (m < -b ? -1 : 0);
  }

  // bound on |v_true|^2 of one vertex with error bound e
  TRIME_D static T vert_r2(T x, T y, float e) {
    const T u = U<T>::v;
    T E = (T)e;
    T l1 = fabs(x) + fabs(y);
    return (x * x + y * y) * ((T)1 + (T)8 * u) + (T)4 * l1 * E + (T)4 * E * E;
  }
  // R2 from the largest vertex bound, capped by the octagon's circumradius
  TRIME_D void set_R2(T r2) {
    T cap = (T)((double)S * (double)S * 1.1717 * 1.00001);
    R2 = isfinite(r2) ? fmin(r2, cap) : cap;
  }
  TRIME_D void update_R2() {
    T r2 = 0;
    for (int j = 0; j < n; j++) {
      VRec<T> v = P[j][tid];
      r2 = fmax(r2, vert_r2(v.x, v.y, v.e));
    }
    set_R2(r2);
  }

  // The octagon: vertex w between walls w-1 and w, exact in float and double
  // (S - D is exact by Sterbenz).  When the grid box is within reach the
  // replay kernels clip it by the box walls; the fast kernel defers.
  TRIME_D void init_polygon() {
    T s = (T)S, dmS = (T)D - (T)S;
    set_v(0, s, -dmS, 0.0f, -1);
    set_v(1, s, dmS, 0.0f, -2);
    set_v(2, dmS, s, 0.0f, -3);
    set_v(3, -dmS, s, 0.0f, -4);
    set_v(4, -s, dmS, 0.0f, -5);
    set_v(5, -s, -dmS, 0.0f, -6);
    set_v(6, -dmS, -s, 0.0f, -7);
    set_v(7, dmS, -s, 0.0f, -8);
    n = 8;
    double reach = (double)S * 1.0001 + 1e-300;
    bool clear = (a.box_x1 - px) > reach && (px - a.box_x0) > reach && (a.box_y1 - py) > reach &&
                 (py - a.box_y0) > reach;
    if (!clear) {
      if constexpr (!EXACT) {
        why = WHY_BOX;
        return;
      } else {
        for (int w = 8; w < 12 && n > 0; w++) {
          clip(row_of<T>(a, -1 - w, px, py, S, D), -1 - w);
          if (why) return;
        }
      }
    }
    update_R2();
  }

  // Cut the polygon by constraint c3 (row r3).  Small polygons go through
  // registers: all records are read at once, the margins are taken with
  // every load in flight, and the kept records are written back to their new
  // places (no dependent LDS round trips per vertex).  DUP false: c3 is
  // known not to bound the polygon yet (the previous cell's distinct
  // neighbours; one that did would leave its margins undecided and send the
  // point to the FP64 replay).
  template <bool DUP = true> TRIME_D void clip(const Row<T> &r3, int c3) {
    if constexpr (VMAX <= 16 && !EXACT)
      clip_reg<DUP>(r3, c3);
    else
      clip_lds(r3, c3);
  }

  template <bool DUP> TRIME_D void clip_reg(const Row<T> &r3, int c3) {
    const T u = U<T>::v;
    VRec<T> v[VMAX];
#pragma unroll
    for (int j = 0; j < VMAX; j++) v[j] = P[j][tid];
    // a neighbour whose bisector already bounds the cell (clipped first, from
    // the point's previous cell) is not clipped again: two vertices lie on
    // its bisector, where the margins vanish
    if constexpr (DUP) {
      uint32_t dup = 0;
#pragma unroll
      for (int j = 0; j < VMAX; j++) dup |= (uint32_t)(j < n && v[j].c == c3);
      if (dup) return;
    }
    const T n1 = fabs(r3.nx) + fabs(r3.ny);
    // one bound for every vertex: the largest vertex error bound of the
    // polygon stands for each vertex's own (a larger bound only leaves more
    // margins to the FP64 re-evaluation)
    const T b = fma(n1, (T)Emax, (T)12 * u * fabs(r3.s));
    uint32_t M = 0, Un = 0;
#pragma unroll
    for (int j = 0; j < VMAX; j++) {
      T m = fma(r3.nx, v[j].x, fma(r3.ny, v[j].y, -r3.s));
      // as bits, not branches: one exec-mask branch per vertex would cost
      // more than the comparisons
      uint32_t in = j < n, gt = m > b, ge = m >= -b;
      M |= (in & gt) << j;
      Un |= (in & ge & (gt ^ 1u)) << j;
    }
    wk.margins += n;
    while (Un) {  // undecided in the kernel's precision: FP64 in place
      int j = __ffs(Un) - 1;
      Un &= Un - 1;
      int s64 = sizeof(T) == 4 ? margin64(con(j == 0 ? n - 1 : j - 1), con(j), c3) : 0;
      if (s64 > 0) {
        M |= 1u << j;
      } else if (s64 == 0) {
        why = WHY_PRED;
        return;
      }
    }
    if (M == 0) return;
    wk.cuts++;
    uint32_t full = (1u << n) - 1u;
    if (M == full) {
      n = 0;
      return;
    }
    uint32_t Pm = ((M << 1) | (M >> (n - 1))) & full;
    uint32_t Nm = ((M >> 1) | (M << (n - 1))) & full;
    uint32_t starts = M & ~Pm, ends = M & ~Nm;
    if (__popc(starts) != 1) {  // impossible with exact decisions
      why = WHY_PRED;
      return;
    }
    int k0 = __ffs(starts) - 1, k1 = __ffs(ends) - 1;
    int r = __popc(M);
    int nn = n - r + 2;
    if (nn > VMAX) {
      why = WHY_POLY;
      return;
    }
    int cin = con(k0 == 0 ? n - 1 : k0 - 1);
    int cout = con(k1);
    T x1, y1, x2, y2;
    float e1, e2;
    bool ok1 = new_vertex(cin, c3, row_of<T>(a, cin, px, py, S, D), r3, x1, y1, e1, c3);
    bool ok2 = new_vertex(c3, cout, r3, row_of<T>(a, cout, px, py, S, D), x2, y2, e2, c3);
    if (!ok1 || !ok2) {
      why = WHY_VERTEX;
      return;
    }
    // kept vertex j moves to d(j); the two new vertices go to dn, dn + 1.
    // R2 bounds |v|^2 of every vertex with the polygon's largest error bound
    // (vert_r2 grows with the bound): the largest x^2 + y^2 and |x| + |y|
    // over the vertices, then one bound.
    const bool plain = k0 <= k1;
    const int dn = plain ? k0 : k0 - k1 - 1;
    Emax = fmax(Emax, fmax(e1, e2));
    T q2 = fmax(x1 * x1 + y1 * y1, x2 * x2 + y2 * y2);
    T l1 = fmax(fabs(x1) + fabs(y1), fabs(x2) + fabs(y2));
#pragma unroll
    for (int j = 0; j < VMAX; j++) {
      if (j < n && !((M >> j) & 1)) {
        int d = plain ? (j < k0 ? j : j - r + 2) : j - (k1 + 1);
        P[d][tid] = v[j];
        q2 = fmax(q2, v[j].x * v[j].x + v[j].y * v[j].y);
        l1 = fmax(l1, fabs(v[j].x) + fabs(v[j].y));
      }
    }
    set_v(dn, x1, y1, e1, c3);
    set_v(dn + 1, x2, y2, e2, cout);
    n = nn;
    const T E = (T)Emax;
    set_R2(q2 * ((T)1 + (T)8 * u) + (T)4 * l1 * E + (T)4 * E * E);
  }

  TRIME_D void clip_lds(const Row<T> &r3, int c3) {
    const T u = U<T>::v;
    uint32_t M = 0;
    T n1 = fabs(r3.nx) + fabs(r3.ny);
    T b0 = (T)12 * u * fabs(r3.s);
    for (int j = 0; j < n; j++) {
      VRec<T> v = P[j][tid];
      T m = fma(r3.nx, v.x, fma(r3.ny, v.y, -r3.s));
      T b = fma(n1, (T)v.e, b0);
      if (m > b) {
        M |= 1u << j;
      } else if (m >= -b) {
        if constexpr (EXACT) {
          if (exact_cut(a, con(j == 0 ? n - 1 : j - 1), v.c, c3, pid, px, py, S, D, ec) > 0)
            M |= 1u << j;
        } else {
          int s64 = sizeof(T) == 4 ? margin64(con(j == 0 ? n - 1 : j - 1), v.c, c3) : 0;
          if (s64 > 0) {
            M |= 1u << j;
          } else if (s64 == 0) {
            why = WHY_PRED;
            return;
          }
        }
      }
    }
    wk.margins += n;
    if (M == 0) return;
    wk.cuts++;
    uint32_t full = (n == 32) ? 0xffffffffu : ((1u << n) - 1u);
    if (M == full) {
      n = 0;
      return;
    }
    uint32_t Pm = ((M << 1) | (M >> (n - 1))) & full;
    uint32_t Nm = ((M >> 1) | (M << (n - 1))) & full;
    uint32_t starts = M & ~Pm, ends = M & ~Nm;
    if (__popc(starts) != 1) {  // impossible with exact decisions
      why = WHY_PRED;
      return;
    }
    int k0 = __ffs(starts) - 1, k1 = __ffs(ends) - 1;
    int r = __popc(M);
    int nn = n - r + 2;
    if (nn > VMAX) {
      why = WHY_POLY;
      return;
    }
    int cin = con(k0 == 0 ? n - 1 : k0 - 1);
    int cout = con(k1);
    T x1, y1, x2, y2;
    float e1, e2;
    bool ok1 = new_vertex(cin, c3, row_of<T>(a, cin, px, py, S, D), r3, x1, y1, e1, c3);
    bool ok2 = new_vertex(c3, cout, r3, row_of<T>(a, cout, px, py, S, D), x2, y2, e2, c3);
    if constexpr (!EXACT) {
      if (!ok1 || !ok2) {
        why = WHY_VERTEX;
        return;
      }
    }
    if (k0 <= k1) {
      if (r >= 2) {
        int sh = r - 2;
        if (sh > 0)
          for (int j = k1 + 1; j < n; j++) P[j - sh][tid] = P[j][tid];
      } else {
        for (int j = n - 1; j > k1; j--) P[j + 1][tid] = P[j][tid];
      }
      set_v(k0, x1, y1, e1, c3);
      set_v(k0 + 1, x2, y2, e2, cout);
    } else {
      int m = 0;
      for (int j = k1 + 1; j < k0; j++, m++) P[m][tid] = P[j][tid];
      set_v(m, x1, y1, e1, c3);
      set_v(m + 1, x2, y2, e2, cout);
    }
    n = nn;
    update_R2();
  }

  // bin (dx, dy) number bi of ring r: top row, bottom row, then the sides
  TRIME_D static void ring_bin(int r, int bi, int &dx, int &dy) {
    if (r == 0) {
      dx = 0;
      dy = 0;
    } else if (bi <= 2 * r) {
      dy = -r;
      dx = bi - r;
    } else if (bi <= 4 * r + 1) {
      dy = r;
      dx = bi - (3 * r + 1);
    } else {
      int q = bi - (4 * r + 2);
      dy = -r + 1 + (q >> 1);
      dx = (q & 1) ? r : -r;
    }
  }

  // bin (dx, dy) number bi of ring r, nearest first: rings 1 and 2 take the
  // bins that share a side with the inner rings before the corners (packed
  // tables: 2 bits per coordinate in ring 1, 3 bits in ring 2); rings from 3
  // on use the plain order
  TRIME_D static void ring_bin_near(int r, int bi, int &dx, int &dy) {
    if (r == 1) {
      uint32_t e = (0xa8206491u >> (4 * bi)) & 15u;
      dx = (int)(e & 3u) - 1;
      dy = (int)(e >> 2) - 1;
    } else if (r == 2) {
      uint64_t w = bi < 8 ? 0x8e10c1510882ull : 0x92010070c608ull;
      uint32_t e = (uint32_t)(w >> (6 * (bi & 7))) & 63u;
      dx = (int)(e & 7u) - 2;
      dy = (int)(e >> 3) - 2;
    } else {
      ring_bin(r, bi, dx, dy);
    }
  }

  // Scan the rings of bins around p, nearest bins first.  The scan is bound
  // by the latency of dependent loads and by the lanes of a wavefront
  // waiting on the lane with the most candidates, so:
  //  - the bins go in groups, ring 0 alone, then SCAN_GROUP bins of a ring
  //    at a time (rings have 8 r bins), and one loop takes the candidates of
  //    every bin of a group: the wavefront makes as many trips as its lane
  //    with the most candidates in the whole group, instead of, bin by bin,
  //    as many as the lane with the most in that bin;
  //  - the ranges of the next group's bins are loaded while the current
  //    group's candidates are clipped, and the candidates are loaded two at a
  //    time (four would take the FP32 kernel past the registers of three
  //    wavefronts per SIMD);
  //  - a bin whose distance from p exceeds the reach 2 R (R of the cell when
  //    the bin is fetched, never smaller than later) is not loaded.
  // Every candidate is still tested against the current R, in the same order
  // as one bin at a time, so the clips are the same.  The loop is one group
  // per trip with a single back edge: branches that skip a bin inside the
  // loop let the compiler split it into nested loops in which the lanes wait
  // on each other's loads.
  TRIME_D void fetch_bin(int r, int bi, int bx, int by, double ox, double oy, int &s, int &se) const {
    int dx, dy;
    ring_bin_near(r, bi, dx, dy);
    int xx = bx + dx, yy = by + dy;
    double gx = dx > 0 ? (dx - 1) * a.bw + (a.bw - ox) : (dx < 0 ? (-dx - 1) * a.bw + ox : 0.0);
    double gy = dy > 0 ? (dy - 1) * a.bw + (a.bw - oy) : (dy < 0 ? (-dy - 1) * a.bw + oy : 0.0);
    gx = fmax(gx, 0.0);
    gy = fmax(gy, 0.0);
    s = 0;
    se = 0;
    if (xx >= 0 && yy >= 0 && xx < a.nbx && yy < a.nby && !(gx * gx + gy * gy > 4.0 * (double)R2 * 1.00001)) {
      uint32_t key = morton((uint32_t)xx, (uint32_t)yy);
      s = gld(a.bin_start, (int64_t)key);
      se = gld(a.bin_start, (int64_t)key + 1);
    }
  }

  TRIME_D void scan() {
    const T u = U<T>::v;
    constexpr int NG = SCAN_GROUP;
    int bx, by;
    bin_of(a, px, py, bx, by);
    double ox = px - (a.bx0 + bx * a.bw), oy = py - (a.by0 + by * a.bw);
    double edge = fmax(0.0, fmin(fmin(ox, a.bw - ox), fmin(oy, a.bw - oy)));
    const int rmax = max(a.nbx, a.nby);
    // the current group: ring r from bin bi, bin g's candidates in [gs[g], ge[g])
    int r = 0, bi = 0;
    int gs[NG], ge[NG];
    fetch_bin(0, 0, bx, by, ox, oy, gs[0], ge[0]);
#pragma unroll
    for (int g = 1; g < NG; g++) gs[g] = ge[g] = 0;
    for (;;) {
      int r1 = r, bi1 = bi + NG;
      if (r == 0 || bi1 == 8 * r) {
        r1 = r + 1;
        bi1 = 0;
      }
      int ns[NG], ne[NG];
#pragma unroll
      for (int g = 0; g < NG; g++) fetch_bin(r1, bi1 + g, bx, by, ox, oy, ns[g], ne[g]);
      // candidate i of the group: slot gs[g] + i - c[g - 1] for the bin g
      // whose running count c[g] first exceeds i
      int c[NG];
#pragma unroll
      for (int g = 0; g < NG; g++) c[g] = (g ? c[g - 1] : 0) + (ge[g] - gs[g]);
      const int nt = c[NG - 1];
      auto slot = [&](int i) {
        int sl = gs[0] + i;
#pragma unroll
        for (int g = 1; g < NG; g++)
          if (i >= c[g - 1]) sl = gs[g] + (i - c[g - 1]);
        return sl;
      };
      double qx0 = 0, qx1 = 0, qy0 = 0, qy1 = 0;
      for (int i = 0; i < nt; i++) {
        const int t = i & 1;
        const int s = slot(i);
        if (t == 0) {  // the next two candidates of the group, loads in flight together
          const int s1 = slot(min(i + 1, nt - 1));
          qx0 = gld(a.x, s);
          qy0 = gld(a.y, s);
          qx1 = gld(a.x, s1);
          qy1 = gld(a.y, s1);
        }
        double qx = t == 0 ? qx0 : qx1;
        double qy = t == 0 ? qy0 : qy1;
        if (s != (int)k) {
          wk.candidates++;
          Row<T> r3;
          r3.nx = (T)(qx - px);
          r3.ny = (T)(qy - py);
          T sq = r3.nx * r3.nx + r3.ny * r3.ny;
          r3.s = sq * (T)0.5;
          if (!(sq * ((T)1 - (T)8 * u) > (T)4 * R2)) {
            cqx = qx - px;
            cqy = qy - py;
            clip(r3, s);
            if (why || n == 0) return;
          }
        }
      }
      r = r1;
      bi = bi1;
#pragma unroll
      for (int g = 0; g < NG; g++) {
        gs[g] = ns[g];
        ge[g] = ne[g];
      }
      if (bi == 0) {  // ring r - 1 done: stop when ring r is out of reach
        double dmin = (r - 1) * a.bw + edge;
        if (r > rmax || dmin * dmin > 4.0 * (double)R2 * 1.00001) return;
      }
    }
  }

  // The octagon of a point with span Sq (walls at distance Sq along the
  // axes, |x| + |y| = Dq on the diagonals) holds the disc of radius
  // r = min(Sq, Dq / sqrt 2) about the point.  Cell vertex v lies on the
  // bisector of p and the point, so its distance from the point is |v|:
  // true when the bound on |v|^2 is below r^2 (the float products below
  // round up by at most 2^-23 relative, which the factor 0.99999 covers).
  TRIME_D static bool within_inradius(const VRec<T> &v, float Sq) {
    if (!(Sq > 0.0f)) return false;
    const float Dq = 1.41421356f * Sq;
    const float r2 = fminf(Sq * Sq, 0.5f * (Dq * Dq)) * 0.99999f;
    return vert_r2(v.x, v.y, v.e) < (T)r2;
  }

  // Is cell vertex j (circumcentre of p, q and `other`) inside the octagon
  // of the point in slot q?  1 inside, 0 outside; may set why.  Nearly
  // every vertex is decided by the inradius alone; the walls decide the
  // rest.
  TRIME_D int inside_octagon(int j, int q, int other) {
    const T u = U<T>::v;
    VRec<T> v = P[j][tid];
    float Sq = gld(a.span, q), Dq = 1.41421356f * Sq;
    if (within_inradius(v, Sq)) return 1;
    T E = (T)v.e;
    double qxd = gld(a.x, q), qyd = gld(a.y, q);
    T qx = (T)(qxd - px), qy = (T)(qyd - py);
    T cx = v.x - qx, cy = v.y - qy;
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
          // in the frame of q: bisector(q, p), bisector(q, other), wall w of q
          if (exact_cut(a, (int)k, other, -1 - w, gld(a.id, q), qxd, qyd, Sq, Dq, ec) > 0) return 0;
        } else {
          int s64 = sizeof(T) == 4 ? oct_margin64(j, qxd, qyd, Sq, Dq, w) : 0;
          if (s64 > 0) return 0;
          if (s64 == 0) {
            why = WHY_AND;
            return 0;
          }
        }
      }
    }
    return 1;
  }

  TRIME_D bool valid_triangle(int s1, int s2) {
    return valid_triangle_at(gld(a.id, s1), gld(a.x, s1), gld(a.y, s1), gld(a.id, s2), gld(a.x, s2),
                             gld(a.y, s2));
  }
  // Tests 1-3 of the triangle of p and the points with ids i1, i2 at (x1, y1),
  // (x2, y2), its vertices taken in increasing id order.
  TRIME_D bool valid_triangle_at(int i1, double x1, double y1, int i2, double x2, double y2) {
    int i0 = pid;
    double x0 = px, y0 = py;
    if (i0 > i1) { int t = i0; i0 = i1; i1 = t; double w = x0; x0 = x1; x1 = w; w = y0; y0 = y1; y1 = w; }
    if (i1 > i2) { int t = i1; i1 = i2; i2 = t; double w = x1; x1 = x2; x2 = w; w = y1; y1 = y2; y2 = w; }
    if (i0 > i1) { int t = i0; i0 = i1; i1 = t; double w = x0; x0 = x1; x1 = w; w = y0; y0 = y1; y1 = w; }
    return tri_valid<G>(a, x0, y0, x1, y1, x2, y2);
  }

  TRIME_D void write_cell() {
    int cap = a.cell_cap;
    if (n > cap) {
      gst(a.cell_n, (int64_t)pid, -1);
      return;
    }
    int s = 0, best = 0x7fffffff;
    for (int j = 0; j < n; j++) {
      int c = con(j);
      int v = c >= 0 ? gld(a.id, c) : c;
      if (v < best) {
        best = v;
        s = j;
      }
    }
    for (int t = 0; t < n; t++) {
      int c = con((s + t) % n);
      gst(a.cell_cons, (int64_t)pid * cap + t, c >= 0 ? gld(a.id, c) : c);
    }
    gst(a.cell_n, (int64_t)pid, n);
  }

  // Weighted centroid (relative to p) at quadrature level L >= 1: the fan
  // triangles (p, v_t, v_t+1) bisected L - 1 times, one midpoint sample of
  // rho = mu^-2 per leaf.  getv(t, x, y) yields vertex t in V arithmetic.
  // Below QK bisections a leaf is reached by its bit path from the fan
  // triangle; deeper levels walk subtrees of QK bisections depth first, so
  // each bisection is done once.  Leaves are summed in the same order
  // either way.
  static constexpr int QK = 3;

  // The leaf geometry and weights are in V; the sums are FP64 in both
  // precisions: an FP32 sum over the hundreds of leaves of a large boundary
  // cell (up to the octagon, 5h) would move its centroid by more than the
  // 1e-5 h the FP32 mode allows.
  template <class V, class GetV>
  TRIME_D void level_centroid(int L, V fxf, V fyf, int cx0, int cy0, GetV &getv, V &cx, V &cy) {
    double sw = 0, swx = 0, swy = 0;
    const V idx = (V)a.inv_dx, idy = (V)a.inv_dy;
    const G *mu = (const G *)a.mu;
    const int nxc = a.nx - 2, nyc = a.ny - 2;
    int64_t last = -1;  // the four node values of the last grid cell are kept
    V m00 = 0, m10 = 0, m01 = 0, m11 = 0;
    auto leaf = [&](V x0, V y0, V x1, V y1, V x2, V y2) {
      V A = (V)0.5 * ((x1 - x0) * (y2 - y0) - (y1 - y0) * (x2 - x0));
      V gx = (x0 + x1 + x2) * (V)(1.0 / 3.0), gy = (y0 + y1 + y2) * (V)(1.0 / 3.0);
      // mu at p + g: bilinear in its cell (cells clamped to the grid)
      V fx = fxf + gx * idx, fy = fyf + gy * idy;
      V flx = floor(fx), fly = floor(fy);
      // the leaf lies within the octagon of p: its cell offset is a few
      // cells, so the sums stay in int (p's cell index is below nx, ny)
      int ci = cx0 + sat_int(flx), cj = cy0 + sat_int(fly);
      V tx = fx - flx, ty = fy - fly;
      if (ci < 0) { ci = 0; tx = 0; }
      if (ci > nxc) { ci = nxc; tx = 1; }
      if (cj < 0) { cj = 0; ty = 0; }
      if (cj > nyc) { cj = nyc; ty = 1; }
      int64_t n0 = (int64_t)cj * a.nx + ci;
      if (n0 != last) {
        m00 = (V)gld(mu, n0);
        m10 = (V)gld(mu, n0 + 1);
        m01 = (V)gld(mu, n0 + a.nx);
        m11 = (V)gld(mu, n0 + a.nx + 1);
        last = n0;
      }
      V m = (m00 * ((V)1 - tx) + m10 * tx) * ((V)1 - ty) + (m01 * ((V)1 - tx) + m11 * tx) * ty;
      const double w = (double)(A * recip<V>(m * m));
      sw += w;
      swx += w * (double)gx;
      swy += w * (double)gy;
    };
    const int D = L - 1;
    if constexpr (BLOCK == 1 || BLOCK == 8) {
      // one polygon per wavefront (BLOCK 1) or per group of 8 lanes (BLOCK
      // 8): leaf i of the n 2^D leaves goes to lane i mod g of the group
      // (bit path from its fan triangle); the partial sums meet in a
      // fixed-order tree at the group's first lane and are broadcast
      constexpr int g = BLOCK == 1 ? 64 : 8;
      const int lane = threadIdx.x & (g - 1);
      const int64_t total = (int64_t)n << D;
      for (int64_t i = lane; i < total; i += g) {
        int t = (int)(i >> D);
        int64_t b = i & (((int64_t)1 << D) - 1);
        V bx, by, cx_, cy_;
        getv(t, bx, by);
        getv(t + 1 == n ? 0 : t + 1, cx_, cy_);
        V x0 = 0, y0 = 0, x1 = bx, y1 = by, x2 = cx_, y2 = cy_;
        for (int d = D - 1; d >= 0; d--) {
          int e;
          V mx, my;
          longest_edge(x0, y0, x1, y1, x2, y2, e, mx, my);
          take_child(e, (int)((b >> d) & 1), mx, my, x0, y0, x1, y1, x2, y2);
        }
        leaf(x0, y0, x1, y1, x2, y2);
      }
      for (int off = g / 2; off > 0; off >>= 1) {
        sw += __shfl_down(sw, off, g);
        swx += __shfl_down(swx, off, g);
        swy += __shfl_down(swy, off, g);
      }
      sw = __shfl(sw, 0, g);
      swx = __shfl(swx, 0, g);
      swy = __shfl(swy, 0, g);
      wk.leaves += n << D;
      const double inv = 1.0 / sw;
      cx = (V)(swx * inv);
      cy = (V)(swy * inv);
      return;
    }
    V vx0, vy0, ax, ay;
    getv(0, vx0, vy0);
    ax = vx0;
    ay = vy0;
    for (int t = 0; t < n; t++) {
      V bx, by;
      if (t + 1 == n) {
        bx = vx0;
        by = vy0;
      } else {
        getv(t + 1, bx, by);
      }
      const int top = D < QK ? D : D - QK;  // bisections by bit path
      const int nb = 1 << top;
      for (int b = 0; b < nb; b++) {
        V x0 = 0, y0 = 0, x1 = ax, y1 = ay, x2 = bx, y2 = by;
        for (int d = top - 1; d >= 0; d--) {
          int e;
          V mx, my;
          longest_edge(x0, y0, x1, y1, x2, y2, e, mx, my);
          take_child(e, (b >> d) & 1, mx, my, x0, y0, x1, y1, x2, y2);
        }
        if (D < QK)
          leaf(x0, y0, x1, y1, x2, y2);
        else
          subtree<QK>(x0, y0, x1, y1, x2, y2, leaf);
      }
      ax = bx;
      ay = by;
    }
    wk.leaves += n << D;
    const double inv = 1.0 / sw;
    cx = (V)(swx * inv);
    cy = (V)(swy * inv);
  }

  // The adaptive level loop of the CVD target (Sec. 4.2 II) in V arithmetic.
  // BAND (FP32): false when a level decision lies within the error bound of
  // the two centroids compared; the caller then redoes it in FP64.
  template <class V, bool BAND, class GetV>
  TRIME_D bool cvd_levels(double h, double dp, GetV &getv, double &xnew, double &ynew, int &cap_hit,
                          V vtx_err = 0) {
    const V u = U<V>::v;
    V A = 0;
    {
      V x0, y0, xa, ya;
      getv(0, x0, y0);
      xa = x0;
      ya = y0;
      for (int j = 0; j < n; j++) {
        V xb, yb;
        if (j + 1 == n) {
          xb = x0;
          yb = y0;
        } else {
          getv(j + 1, xb, yb);
        }
        A += (V)0.5 * (xa * yb - ya * xb);
        xa = xb;
        ya = yb;
      }
    }
    double eps = fmax((dp < 0 ? h : dp) / h, a.prm.fac_end);
    V E = (V)(sqrt((double)A) * eps);
    double fx0 = (px - a.gx0) * a.inv_dx, fy0 = (py - a.gy0) * a.inv_dy;
    const int cx0 = sat_int(floor(fx0)), cy0 = sat_int(floor(fy0));  // p's cell: 0 <= fx0 < nx - 1
    V fxf = (V)(fx0 - (double)cx0), fyf = (V)(fy0 - (double)cy0);
    V R = sqrt((V)R2);
    V c0x = 0, c0y = 0, c1x = 0, c1y = 0;
    V err0 = 0;  // error bound of the previous level's centroid
    for (int L = 1;; L++) {
      level_centroid<V>(L, fxf, fyf, cx0, cy0, getv, c1x, c1y);
      V ex_ = c0x - c1x, ey_ = c0y - c1y;
      V d2 = ex_ * ex_ + ey_ * ey_;
      if constexpr (BAND) {
        // centroid error: the vertices' own error bounds, vertices and
        // weights (~32u R) plus the sums (u R per leaf term), for both
        // levels compared
        V err1 = (V)2 * vtx_err + ((V)32 + (V)2 * (V)(n << (L - 1))) * u * R;
        V dd = err0 + err1;
        V lo = fmax(E - dd, (V)0), hi = E + dd;
        if (d2 >= lo * lo && d2 <= hi * hi) return false;
        err0 = err1;
      }
      if (d2 < E * E) break;
      if (L >= a.prm.cvd_max_level) {
        cap_hit = 1;
        break;
      }
      c0x = c1x;
      c0y = c1y;
    }
    xnew = px + (double)c1x;
    ynew = py + (double)c1y;
    return true;
  }

  // CVD target of p (Sec. 4.2 II).  An FP32 level decision within its error
  // bound sends the point to the FP64 replay (WHY_LEVEL).
  TRIME_D void cvd_target(double h, double dp, double &xnew, double &ynew, int &cap_hit) {
    xnew = px;
    ynew = py;
    if (n == 0) return;
    auto getT = [&](int t, T &x, T &y) {
      VRec<T> v = P[t][tid];
      x = v.x;
      y = v.y;
    };
    constexpr bool band = !EXACT && sizeof(T) == 4;
    T emax = 0;
    if constexpr (band) {
      // the centroid moves by up to a few times the largest vertex error.
      // The vertices are rounded FP64 intersections: e is 7u|v| (rounding
      // and the cut test's allowance) plus the FP64 bound, which only a
      // nearly singular pair of rows makes large; such cells take the FP64
      // centroid pass (1e-6 h of excess keeps the centroid well inside the
      // 1e-5 h of the FP32 mode)
      const T u = U<T>::v;
      T excess = 0;
      for (int j = 0; j < n; j++) {
        VRec<T> v = P[j][tid];
        emax = fmax(emax, (T)v.e);
        excess = fmax(excess, (T)v.e - (T)7.0001 * u * fmax(fabs(v.x), fabs(v.y)));
      }
      if ((double)excess > 1e-6 * h) {
        why = WHY_PREC;
        return;
      }
    }
    if (!cvd_levels<T, band>(h, dp, getT, xnew, ynew, cap_hit, emax)) why = WHY_LEVEL;
  }

  // CVD target (Sec. 4.2 II) and treatment (Sec. 4.3) of p; false when an
  // FP32 decision lies within its error bound (why = WHY_LEVEL / WHY_TREAT).
  TRIME_D bool target_and_treat(double &xf, double &yf, uint8_t &cf, int &cap_hit, TreatCount &tc) {
    GCell cell;
    double tx, ty;
    locate(a, px, py, cell, tx, ty);
    double h = (double)cell_h(a, cell);
    double xnew, ynew;
    cvd_target(h, gld(a.dprev, k), xnew, ynew, cap_hit);
    if (why) return false;
    double band = (!EXACT && sizeof(T) == 4) ? 1e-6 * h : 0.0;
    bool unsure = false;
    treat<G>(a, px, py, gld(a.cat, k), xnew, ynew, band, xf, yf, cf, unsure, tc);
    // with band 0 (FP64) the comparisons as evaluated are the decisions
    if (unsure && band > 0.0) {
      why = WHY_TREAT;
      return false;
    }
    return true;
  }

  TRIME_D void write_cvd(double xf, double yf, uint8_t cf) {
    gst(a.xn, k, xf);
    gst(a.yn, k, yf);
    gst(a.catn, k, cf);
    gst(a.dprevn, k, sqrt((xf - px) * (xf - px) + (yf - py) * (yf - py)));
  }

  // The FP64 centroid pass of one deferred point: its cell's constraints
  // (entry cb of the deferred queue) give the FP64 vertices, then the CVD
  // target and the treatment run in FP64.
  // lead: the lane that writes the result and counts the work (one point
  // per wavefront: every lane runs the pass, the leaves spread over them)
  TRIME_D void centroid_replay(LaneStats &st, int64_t cb, bool lead = true) {
    pid = gld(a.id, k);
    px = gld(a.x, k);
    py = gld(a.y, k);
    S = gld(a.span, k);
    D = 1.41421356f * S;
    n = gld(a.cq_cons, cb);
    for (int j = 0; j < n; j++) P[j][tid].c = gld(a.cq_cons, cb + 1 + j);
    bool bad = false;
    for (int j = 0; j < n; j++) {
      double vx, vy;
      float E;
      if (!vertex64(j, vx, vy, E)) bad = true;
      P[j][tid].x = vx;
      P[j][tid].y = vy;
      P[j][tid].e = E;
    }
    double xf = px, yf = py;
    uint8_t cf = gld(a.cat, k);
    int cap_hit = 0;
    TreatCount tc;
    if (bad || !target_and_treat(xf, yf, cf, cap_hit, tc)) {  // cannot happen in FP64: keep p
      atomicOr(&a.counters[CNT_ERR], ERR_POLY_CAP);
      xf = px;
      yf = py;
      cf = gld(a.cat, k);
    }
    if (!lead) return;
    write_cvd(xf, yf, cf);
    st.newton_fail += tc.newton_fail();
    st.trace_fail += tc.trace_fail();
    st.cap_hits += cap_hit;
    st.leaves += wk.leaves;
  }

  // Quality of the valid triangle (p, jin, jout) (Eq. 10-11) into the lane
  // statistics and the beta histogram.
  TRIME_D void tri_quality(LaneStats &st, int *hist, int jin, int jout) const {
    st.nvalid++;
    double x1 = gld(a.x, jin), y1 = gld(a.y, jin), x2 = gld(a.x, jout), y2 = gld(a.y, jout);
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
    const int bin = beta_bin(be);
    atomicAdd(&hist[bin], 1);
  }

  // Everything after the cell for the wavefront-per-point kernel: every lane
  // holds the same lane state; lane j takes the octagon and validity tests
  // of vertex j and commits its triangle, the quadrature leaves are spread
  // over the lanes, and lane 0 writes the per-point outputs.  The same
  // decisions and outputs as finish().
  TRIME_D bool finish_wave(int lane, LaneStats &st, int *hist) {
    static_assert(BLOCK == 1 && VMAX <= 64, "one polygon per wavefront, at most one vertex per lane");
    if constexpr (MODE == MODE_CELLS) {
      if (lane == 0) {
        write_cell();
        if (n == 0) st.empty++;
        st.candidates += wk.candidates;
        st.margins += wk.margins;
        st.cuts += wk.cuts;
      }
      return true;
    } else {
      bool ex = false, va = false;
      int jin = -1, jout = -1;
      if (lane < n) {
        jin = con(lane == 0 ? n - 1 : lane - 1);
        jout = con(lane);
        bool test = jin >= 0 && jout >= 0;
        if constexpr (MODE == MODE_CVD) {  // only the triangles p owns are emitted
          if (test) test = pid < gld(a.id, jin) && pid < gld(a.id, jout);
        }
        if (test) {
          int e = inside_octagon(lane, jin, jout);
          if (!why && e) e = inside_octagon(lane, jout, jin);
          if (!why && e) {
            ex = true;
            va = valid_triangle(jin, jout);
          }
        }
      }
      if (__ballot(why != 0)) {  // an FP64-undecided octagon test: the exact stage takes the point
        why = WHY_AND;
        return false;
      }
      const uint64_t valid = __ballot(va);
      double xf = px, yf = py;
      uint8_t cf = 0;
      int cap_hit = 0;
      TreatCount tc;
      if constexpr (MODE == MODE_CVD) target_and_treat(xf, yf, cf, cap_hit, tc);  // FP64: cannot defer
      // triangles: lane j owns the one at vertex j when p has the smallest id
      bool own = ex && pid < gld(a.id, jin) && pid < gld(a.id, jout);
      const uint64_t owners = __ballot(own);
      const int nt_all = __popcll(owners);
      int64_t tbase = k * TRIME_TRI_PER_POINT;
      if (own) {
        int nt = __popcll(owners & ((1ull << lane) - 1ull));
        if (nt < TRIME_TRI_PER_POINT) {
          gst(a.tri, (tbase + nt) * 3 + 0, (int32_t)k);
          gst(a.tri, (tbase + nt) * 3 + 1, jin);
          gst(a.tri, (tbase + nt) * 3 + 2, jout);
          gst(a.tri_valid, tbase + nt, (uint8_t)va);
        } else {
          atomicOr(&a.counters[CNT_ERR], ERR_TRI_CAP);
        }
        st.ntri++;
        if (va) tri_quality(st, hist, jin, jout);
      }
      if (lane == 0) gst(a.tri_n, k, nt_all < TRIME_TRI_PER_POINT ? nt_all : TRIME_TRI_PER_POINT);
      if constexpr (MODE == MODE_EXTRACT) {
        // adjacency: edge j kept when a valid triangle sits at vertex j or
        // j + 1; lane j writes it at its rank by slot
        int jn = (lane + 1 >= n) ? 0 : lane + 1;
        bool keep = lane < n && jout >= 0 && (va || ((valid >> jn) & 1ull));
        const uint64_t kept = __ballot(keep);
        const int cnt = __popcll(kept);
        const int md = a.max_deg;
        if (keep) {
          int rank = 0;
          for (uint64_t m = kept; m; m &= m - 1) {
            int i = __ffsll((unsigned long long)m) - 1;
            rank += con(i) < jout;
          }
          if (rank < md) gst(a.adj, (int64_t)rank * a.n + k, jout);
        }
        if (lane == 0) {
          if (cnt > md) atomicOr(&a.counters[CNT_ERR], ERR_DEG_CAP);
          gst(a.deg, k, cnt < md ? cnt : md);
        }
      }
      if (lane == 0) {
        if constexpr (MODE == MODE_CVD) {
          write_cvd(xf, yf, cf);
          st.newton_fail += tc.newton_fail();
          st.trace_fail += tc.trace_fail();
          st.cap_hits += cap_hit;
        }
        if (n == 0) st.empty++;
        st.candidates += wk.candidates;
        st.margins += wk.margins;
        st.cuts += wk.cuts;
        st.leaves += wk.leaves;
      }
      return true;
    }
  }

  // The neighbours of the point's previous cell (by id, through the slot
  // of each id in the current binning), clipped before the scan: they are
  // most of the neighbours of the new cell, so the polygon and its radius
  // are close to final when the scan starts, the scan's reach and stop tests
  // prune most bins, and later candidates rarely cut.  The cell does not
  // depend on the order of the cuts (every decision is exact); the scan still
  // visits every bin within reach.
  // The previous cell's neighbours first: the list the point wrote before
  // the last binning, at its slot then, its entries slots of that order
  // mapped to this one.  Any list gives the same cell (every cut is exact);
  // indices outside [0, n) (a list older than the last load or addition of
  // points) are skipped.
  TRIME_D void warm() {
    const T u = U<T>::v;
    const int64_t ko = gld(a.old_slot, k);
    if (ko < 0 || ko >= a.n) return;
    int m = gld(a.warm_n_prev, ko);
    m = m < 0 ? 0 : (m > TRIME_WARM ? TRIME_WARM : m);
    for (int t = 0; t < m; t++) {
      const int e = gld(a.warm_nb_prev, ko * TRIME_WARM + t);
      if (e < 0 || e >= a.n) continue;
      const int q = gld(a.new_slot, (int64_t)e);
      if (q < 0 || q >= a.n || q == (int)k) continue;
      const double qx = gld(a.x, q), qy = gld(a.y, q);
      Row<T> r3;
      r3.nx = (T)(qx - px);
      r3.ny = (T)(qy - py);
      T sq = r3.nx * r3.nx + r3.ny * r3.ny;
      r3.s = sq * (T)0.5;
      if (!(sq * ((T)1 - (T)8 * u) > (T)4 * R2)) {
        cqx = qx - px;
        cqy = qy - py;
        clip<false>(r3, q);
        if (why || n == 0) return;
      }
    }
  }

  // The slots of the cell's neighbours, for the point's next cell, at the
  // point's slot.
  TRIME_D void keep_neighbours() {
    int t = 0;
    for (int j = 0; j < n; j++) {
      const int c = con(j);
      if (c >= 0 && t < TRIME_WARM) gst(a.warm_nb, k * TRIME_WARM + t++, (int32_t)c);
    }
    gst(a.warm_n, k, t);
  }

  // Everything for point k; returns false when the point must be replayed.
  TRIME_D bool run(LaneStats &st, int *hist) {
    if (!begin()) return false;
    if constexpr (!EXACT) {
      if (a.warm_n) warm();
      if (why) return false;
    }
    scan();
    if (why) return false;
    if (!finish(st, hist)) return false;
    if constexpr (!EXACT) {
      if (a.warm_n) keep_neighbours();
    }
    return true;
  }

  // The point and its initial polygon; false when the point must leave.
  TRIME_D bool begin() {
    pid = gld(a.id, k);
    px = gld(a.x, k);
    py = gld(a.y, k);
    S = gld(a.span, k);
    D = 1.41421356f * S;
    if (!(S > 0.0f)) {  // off the grid
      why = WHY_BOX;
      return false;
    }
    init_polygon();
    return !why;
  }

  // The ring scan of a whole wavefront for one point: every lane holds the
  // same lane state and polygon (LDS writes of equal values), the candidates
  // of a ring are loaded and range-tested 64 at a time, one per lane, and the
  // ones in range are clipped in lane order by all lanes together.  The cell
  // does not depend on the clip order (every decision is exact).
  //
  // Candidates are range-tested against a bound per direction.  q cuts a
  // vertex v only if q . v > |q|^2 / 2, which needs v within 90 degrees of
  // q and |q|^2 < 4 |v|^2.  q lies within 22.5 degrees of the nearest of 8
  // directions, so the bound of that direction is the largest |v|^2 over
  // the vertices within 112.5 degrees of it (23 degrees are used, for
  // rounding in the choice of the direction).  For a point on the boundary,
  // whose cell reaches the octagon outside the shape, neighbours inside the
  // shape then meet the small inner part of the cell, not the octagon's
  // corners.
  TRIME_D static int sector8(T x, T y) {
    const T ax = fabs(x), ay = fabs(y), t = (T)0.41421356;  // tan 22.5 deg
    if (ay <= t * ax) return x >= 0 ? 0 : 4;
    if (ax <= t * ay) return y >= 0 ? 2 : 6;
    if (x >= 0) return y >= 0 ? 1 : 7;
    return y >= 0 ? 3 : 5;
  }

  TRIME_D void update_sectors(int lane, T *sh_ro) {
    if (lane < 8) {
      const T c = (T)0.70710678118654752;
      const T dx = lane == 0 ? (T)1 : (lane == 4 ? (T)-1 : (lane == 2 || lane == 6 ? (T)0 : (lane == 1 || lane == 7 ? c : -c)));
      const T dy = lane == 2 ? (T)1 : (lane == 6 ? (T)-1 : (lane == 0 || lane == 4 ? (T)0 : (lane == 1 || lane == 3 ? c : -c)));
      T best = 0;
      for (int j = 0; j < n; j++) {
        VRec<T> v = P[j][tid];
        T vn = sqrt(v.x * v.x + v.y * v.y);
        if (v.x * dx + v.y * dy >= (T)-0.39073113 * vn - (T)2 * (T)v.e) best = fmax(best, vert_r2(v.x, v.y, v.e));
      }
      sh_ro[lane] = fmin(best, R2);
    }
    __syncthreads();
  }

  TRIME_D void scan_wave(int lane, int *sh_s0, int *sh_incl, T *sh_ro) {
    const T u = U<T>::v;
    int bx, by;
    bin_of(a, px, py, bx, by);
    update_sectors(lane, sh_ro);
    double ox = px - (a.bx0 + bx * a.bw), oy = py - (a.by0 + by * a.bw);
    double edge = fmax(0.0, fmin(fmin(ox, a.bw - ox), fmin(oy, a.bw - oy)));
    const int rmax = max(a.nbx, a.nby);
    for (int r = 0;; r++) {
      if (r > 0) {
        double dmin = (r - 1) * a.bw + edge;
        if (r > rmax || dmin * dmin > 4.0 * (double)R2 * 1.00001) return;
      }
      const int nbr = r == 0 ? 1 : 8 * r;
      for (int b0 = 0; b0 < nbr; b0 += 64) {
        int bi = b0 + lane, s0 = 0, cnt = 0;
        if (bi < nbr) {
          int dx, dy;
          ring_bin(r, bi, dx, dy);
          int xx = bx + dx, yy = by + dy;
          if (xx >= 0 && yy >= 0 && xx < a.nbx && yy < a.nby) {
            uint32_t key = morton((uint32_t)xx, (uint32_t)yy);
            s0 = gld(a.bin_start, (int64_t)key);
            cnt = gld(a.bin_start, (int64_t)key + 1) - s0;
          }
        }
        int incl = cnt;
        for (int off = 1; off < 64; off <<= 1) {
          int y = __shfl_up(incl, off);
          if (lane >= off) incl += y;
        }
        const int total = __shfl(incl, 63);
        sh_s0[lane] = s0;
        sh_incl[lane] = incl;
        __syncthreads();
        for (int c0 = 0; c0 < total; c0 += 64) {
          int c = c0 + lane, sl = -1;
          bool pass = false;
          if (c < total) {
            int lo = 0, hi = 63;  // first bin with incl > c
            while (lo < hi) {
              int mid = (lo + hi) >> 1;
              if (sh_incl[mid] > c) hi = mid; else lo = mid + 1;
            }
            int first = lo > 0 ? sh_incl[lo - 1] : 0;
            sl = sh_s0[lo] + (c - first);
            if (sl != (int)k) {
              T nx = (T)(gld(a.x, sl) - px), ny = (T)(gld(a.y, sl) - py);
              T sq = nx * nx + ny * ny;
              pass = !(sq * ((T)1 - (T)8 * u) > (T)4 * sh_ro[sector8(nx, ny)]);
            }
          }
          wk.candidates += __popcll(__ballot(c < total && sl != (int)k));
          uint64_t m = __ballot(pass);
          while (m) {
            int j = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            int sj = __shfl(sl, j);
            Row<T> r3;
            r3.nx = (T)(gld(a.x, sj) - px);
            r3.ny = (T)(gld(a.y, sj) - py);
            T sq = r3.nx * r3.nx + r3.ny * r3.ny;
            r3.s = sq * (T)0.5;
            if (!(sq * ((T)1 - (T)8 * u) > (T)4 * sh_ro[sector8(r3.nx, r3.ny)])) {
              int cuts0 = wk.cuts;
              clip(r3, sj);
              if (why || n == 0) return;
              if (wk.cuts != cuts0) update_sectors(lane, sh_ro);
            }
          }
        }
        __syncthreads();
      }
    }
  }

  // Everything after the cell: decisions, CVD target and treatment, then
  // the commit of the outputs; false when the point must leave.
  // Bit j of nb: edge j of the polygon is a bisector (its constraint a
  // point, not a wall); of gt: a bisector of a point with a larger id than
  // p.  Small polygons issue every id load at once.
  TRIME_D void edge_masks(uint32_t &nb, uint32_t &gt) const {
    nb = 0;
    gt = 0;
    if constexpr (VMAX <= 16) {
      int ids[VMAX];
#pragma unroll
      for (int j = 0; j < VMAX; j++) {
        const int c = j < n ? con(j) : -1;
        ids[j] = gld(a.id, c >= 0 ? (int64_t)c : k);
        nb |= (uint32_t)(c >= 0) << j;
      }
#pragma unroll
      for (int j = 0; j < VMAX; j++) gt |= (uint32_t)(ids[j] > pid) << j;
      gt &= nb;
    } else {
      for (int j = 0; j < n; j++) {
        const int c = con(j);
        if (c < 0) continue;
        nb |= 1u << j;
        if (gld(a.id, c) > pid) gt |= 1u << j;
      }
    }
  }
  // Bit j: bit j - 1 of m (cyclically over the n edges); vertex j lies
  // between edges j - 1 and j.
  TRIME_D uint32_t prev_edge(uint32_t m) const {
    if (n <= 0) return 0u;
    const uint32_t full = n >= 32 ? 0xffffffffu : (1u << n) - 1u;
    return ((m << 1) | (m >> (n - 1))) & full;
  }

  TRIME_D bool finish(LaneStats &st, int *hist) {
    if constexpr (MODE == MODE_CELLS) {
      write_cell();
    } else {
      // ---- decisions: triangles at the VV vertices, validity.  A CVD step
      // emits only the triangles p owns (smallest id), so it tests only
      // those; extraction needs validity at every vertex (adjacency rows).
      // the vertices to test, as a mask, so that the tests below loop over
      // them only (a wavefront then runs as many trips as its lane with the
      // most such vertices, not as its largest polygon)
      uint32_t nb, gt;
      edge_masks(nb, gt);
      const uint32_t owned = gt & prev_edge(gt), test = MODE == MODE_CVD ? owned : nb & prev_edge(nb);
      uint32_t exists = 0, valid = 0;
      for (uint32_t m = test; m; m &= m - 1) {
        const int j = __ffs(m) - 1;
        int jin = con(j == 0 ? n - 1 : j - 1), jout = con(j);
        // every load of the vertex at once: the spans for the octagon tests,
        // ids and positions for Tests 1-3
        const float S1 = gld(a.span, jin), S2 = gld(a.span, jout);
        const int i1 = gld(a.id, jin), i2 = gld(a.id, jout);
        const double x1 = gld(a.x, jin), y1 = gld(a.y, jin), x2 = gld(a.x, jout), y2 = gld(a.y, jout);
        const VRec<T> v = P[j][tid];
        int e = within_inradius(v, S1) ? 1 : inside_octagon(j, jin, jout);
        if (why) return false;
        if (e) e = within_inradius(v, S2) ? 1 : inside_octagon(j, jout, jin);
        if (why) return false;
        if (!e) continue;
        exists |= 1u << j;
        if (valid_triangle_at(i1, x1, y1, i2, x2, y2)) valid |= 1u << j;
      }
      // ---- CVD target and treatment; an FP32 decision within its bound
      // defers them to the FP64 centroid pass (the cell is final)
      double xf = px, yf = py;
      uint8_t cf = 0;
      int cap_hit = 0;
      TreatCount tc;
      bool defer = false;
      if constexpr (MODE == MODE_CVD) {
        int leaves0 = wk.leaves;
        defer = !target_and_treat(xf, yf, cf, cap_hit, tc);
        if (defer) wk.leaves = leaves0;
      }
      // ---- commit: nothing below can send the point back
      int nt = 0;
      int64_t tbase = k * TRIME_TRI_PER_POINT;
      for (uint32_t m = exists & owned; m; m &= m - 1) {
        const int j = __ffs(m) - 1;
        int jin = con(j == 0 ? n - 1 : j - 1), jout = con(j);
        bool v = (valid >> j) & 1;
        if (nt < TRIME_TRI_PER_POINT) {
          gst(a.tri, (tbase + nt) * 3 + 0, (int32_t)k);
          gst(a.tri, (tbase + nt) * 3 + 1, jin);
          gst(a.tri, (tbase + nt) * 3 + 2, jout);
          gst(a.tri_valid, tbase + nt, (uint8_t)v);
        } else {
          atomicOr(&a.counters[CNT_ERR], ERR_TRI_CAP);
        }
        nt++;
        st.ntri++;
        if (v) {
          st.nvalid++;
          double x1 = gld(a.x, jin), y1 = gld(a.y, jin), x2 = gld(a.x, jout), y2 = gld(a.y, jout);
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
          const int bin = beta_bin(be);
          atomicAdd(&hist[bin], 1);
        }
      }
      gst(a.tri_n, k, nt < TRIME_TRI_PER_POINT ? nt : TRIME_TRI_PER_POINT);
      if constexpr (MODE == MODE_EXTRACT) {
        // adjacency row: edge j is kept when a valid triangle sits at one of
        // its two ends (vertices j and j + 1); sorted by slot in the unused
        // error-bound field of the polygon records
        int cnt = 0;
        for (int j = 0; j < n; j++) {
          int c = con(j);
          int jn = (j + 1 == n) ? 0 : j + 1;
          if (c < 0 || !(((valid >> j) & 1) || ((valid >> jn) & 1))) continue;
          int t = cnt++;
          while (t > 0 && __float_as_int(P[t - 1][tid].e) > c) {
            P[t][tid].e = P[t - 1][tid].e;
            t--;
          }
          P[t][tid].e = __int_as_float(c);
        }
        int md = a.max_deg;
        if (cnt > md) atomicOr(&a.counters[CNT_ERR], ERR_DEG_CAP);
        int w = cnt < md ? cnt : md;
        for (int t = 0; t < w; t++) gst(a.adj, (int64_t)t * a.n + k, __float_as_int(P[t][tid].e));
        gst(a.deg, k, w);
      }
      if constexpr (MODE == MODE_CVD) {
        if (defer && n >= CQ_STRIDE) {  // cannot happen: only fast-kernel lanes (n < CQ_STRIDE) defer
          atomicOr(&a.counters[CNT_ERR], ERR_POLY_CAP);
          defer = false;
          xf = px;
          yf = py;
          cf = gld(a.cat, k);
        }
        if (defer) {
          int w = atomicAdd(&a.counters[CNT_QUEUE3], 1);
          gst(a.queue3, (int64_t)w, (int32_t)k);
          int64_t cb = (int64_t)w * CQ_STRIDE;
          gst(a.cq_cons, cb, n);
          for (int j = 0; j < n; j++) gst(a.cq_cons, cb + 1 + j, con(j));
          atomicAdd(&a.counters[CNT_REASON + why], 1);
        } else {
          write_cvd(xf, yf, cf);
        }
        // the same fields on both paths (no per-path stores to the stats)
        int kept = defer ? 0 : 1;
        st.replays += 1 - kept;
        st.newton_fail += kept & tc.newton_fail();
        st.trace_fail += kept & tc.trace_fail();
        st.cap_hits += kept & cap_hit;
      }
    }
    if (n == 0) st.empty++;
    st.candidates += wk.candidates;
    st.margins += wk.margins;
    st.cuts += wk.cuts;
    st.leaves += wk.leaves;
    if (ec.calls) {
      st.exact_pts++;
      st.exact_calls += ec.calls;
      st.sos += ec.sos;
      if (ec.err) atomicOr(&a.counters[CNT_ERR], ERR_EXACT_CAP);
    }
    return true;
  }
};

// The quality sums of the point a replay kernel just finished, added on
// their own: which block replays which point follows the queue order, which
// varies from run to run, so a block's sum over its points would too.  One
// point per lane (g = 1) or per wavefront (g = 64: its triangles are spread
// over the lanes and summed in a fixed shuffle order, lane 0 adds them).
template <int g> TRIME_D void flush_point_quality(const KArgs &a, LaneStats &st) {
  double sa = st.sa, sb = st.sb, sq = st.sq, am = st.amax;
  if constexpr (g == 64) {
    for (int off = 32; off > 0; off >>= 1) {
      sa += __shfl_down(sa, off);
      sb += __shfl_down(sb, off);
      sq += __shfl_down(sq, off);
      am = fmax(am, __shfl_down(am, off));
    }
  }
  if (g == 1 || (threadIdx.x & 63) == 0) quality_add(a.stats, sa, sb, sq, am);
  st.sa = st.sb = st.sq = st.amax = 0;
}

// The lane statistics of one wavefront summed into lane 0 in a fixed
// shuffle order: the FP sums, the largest alpha and the counts.
struct WaveSums {
  double v[4];
  int iv[16];
};
TRIME_D WaveSums wave_sums(const LaneStats &st) {
  WaveSums r = {{st.sa, st.sb, st.sq, st.amax},
                {st.nq, st.ntri, st.nvalid, st.replays, st.exact_pts, st.exact_calls, st.sos, st.overflow,
                 st.empty, st.newton_fail, st.trace_fail, st.cap_hits, st.candidates, st.margins, st.cuts,
                 st.leaves}};
  for (int off = 32; off > 0; off >>= 1) {
    r.v[0] += __shfl_down(r.v[0], off);
    r.v[1] += __shfl_down(r.v[1], off);
    r.v[2] += __shfl_down(r.v[2], off);
    r.v[3] = fmax(r.v[3], __shfl_down(r.v[3], off));
#pragma unroll
    for (int q = 0; q < 16; q++) r.iv[q] += __shfl_down(r.iv[q], off);
  }
  return r;
}

// w += o: a block combines its wavefronts' sums in wavefront order.
TRIME_D void add_sums(WaveSums &w, const WaveSums &o) {
  w.v[0] += o.v[0];
  w.v[1] += o.v[1];
  w.v[2] += o.v[2];
  w.v[3] = fmax(w.v[3], o.v[3]);
#pragma unroll
  for (int q = 0; q < 16; q++) w.iv[q] += o.iv[q];
}

// One block's combined sums into the device stats (one thread).
TRIME_D void emit_sums(const KArgs &a, const WaveSums &w) {
  trime_stats *S = a.stats;
  typedef unsigned long long ull;
  if (w.iv[0]) {
    quality_add(S, w.v[0], w.v[1], w.v[2], w.v[3]);
    atomicAdd((ull *)&S->nq, (ull)w.iv[0]);
  }
  if (w.iv[1]) atomicAdd((ull *)&S->ntri, (ull)w.iv[1]);
  if (w.iv[2]) atomicAdd((ull *)&S->nvalid, (ull)w.iv[2]);
  if (w.iv[3]) atomicAdd((ull *)&S->fp64_replays, (ull)w.iv[3]);
  if (w.iv[4]) atomicAdd((ull *)&S->exact_points, (ull)w.iv[4]);
  if (w.iv[5]) atomicAdd((ull *)&S->exact_calls, (ull)w.iv[5]);
  if (w.iv[6]) atomicAdd((ull *)&S->sos_calls, (ull)w.iv[6]);
  if (w.iv[7]) atomicAdd((ull *)&S->overflow_points, (ull)w.iv[7]);
  if (w.iv[8]) atomicAdd((ull *)&S->empty_cells, (ull)w.iv[8]);
  if (w.iv[9]) atomicAdd((ull *)&S->newton_fail, (ull)w.iv[9]);
  if (w.iv[10]) atomicAdd((ull *)&S->trace_fail, (ull)w.iv[10]);
  if (w.iv[11]) atomicAdd((ull *)&S->level_cap_hits, (ull)w.iv[11]);
  if (w.iv[12]) atomicAdd((ull *)&S->work_candidates, (ull)w.iv[12]);
  if (w.iv[13]) atomicAdd((ull *)&S->work_margins, (ull)w.iv[13]);
  if (w.iv[14]) atomicAdd((ull *)&S->work_cuts, (ull)w.iv[14]);
  if (w.iv[15]) atomicAdd((ull *)&S->work_leaves, (ull)w.iv[15]);
}

// The block's beta histogram (complete after a barrier) into the stats.
template <int BLOCK> TRIME_D void emit_hist(const KArgs &a, const int *hist) {
  for (int b = threadIdx.x; b < 40; b += BLOCK)
    if (hist[b]) atomicAdd((unsigned long long *)&a.stats->hist_beta[b], (unsigned long long)hist[b]);
}

// Block reduction of the lane statistics into the device stats.
template <int BLOCK> TRIME_D void flush_stats(const KArgs &a, LaneStats &st, int *hist) {
  __shared__ WaveSums rs[BLOCK / 64];
  const WaveSums w = wave_sums(st);
  if ((threadIdx.x & 63) == 0) rs[threadIdx.x >> 6] = w;
  __syncthreads();
  if (threadIdx.x == 0) {
    WaveSums b = rs[0];
    for (int q = 1; q < BLOCK / 64; q++) add_sums(b, rs[q]);
    emit_sums(a, b);
  }
  emit_hist<BLOCK>(a, hist);
}

template <int BLOCK> TRIME_D void zero_hist(int *hist) {
  for (int b = threadIdx.x; b < 40; b += BLOCK) hist[b] = 0;
  __syncthreads();
}

TRIME_D void push(const KArgs &a, int which, int64_t k, int why) {
  int32_t *q = which == 2 ? a.queue2 : a.queue;
  int slot = atomicAdd(&a.counters[which == 2 ? CNT_QUEUE2 : CNT_QUEUE], 1);
  gst(q, (int64_t)slot, (int32_t)k);
  atomicAdd(&a.counters[CNT_REASON + why], 1);
}

// The part of the processing order a block takes.  Blocks are dispatched to
// the 8 XCDs (each with its own L2) in turn; here each XCD takes runs of C
// consecutive blocks (the state's XCD run, 8 by default, tuned), the runs
// going round the XCDs, so that neighbouring blocks, which read the same
// bins and positions, share an L2 while the work stays spread over the
// XCDs.  b: the block within its shape, p: its block in the launch (a batch
// puts shapes one after another), whose residue mod 8 names the XCD.  A
// bijection of [0, nb) for every C: the groups of 8 runs are counted from
// the launch's block 0, and blocks outside a whole group keep their place.
TRIME_D uint32_t xcd_block(uint32_t b, uint32_t nb, uint32_t p, uint32_t C) {
  if (C <= 1) return b;
  const uint32_t G = 8u * C;
  const uint32_t r = (p - b) % G;  // where the shape starts within a group
  const uint32_t s = b + r;        // position counted from that group's start
  const uint32_t g0 = s - s % G;
  if (g0 < r || g0 + G > nb + r) return b;  // a group cut by the shape's ends
  const uint32_t x = s & 7u, j = (s % G) >> 3;
  return g0 + x * C + j - r;
}

// Fast kernel: one point per lane, slots in the processing order.  Points it
// cannot finish (an undecided decision, a polygon beyond its capacity, the
// grid box within reach) go to the FP64 replay queue.
template <class T, class G, int MODE, int VMAX, int B> struct Cells {
  using Args = KArgs;
  static constexpr int BLOCK = B;
  // The point at position w of the processing order, its polygon in lane
  // slot `slot` of P.
  template <int PB>
  TRIME_D static void point(const KArgs &a, int64_t w, VRec<T> (&P)[VMAX][PB], int slot, LaneStats &st,
                            int *hist) {
    if (w < a.n && TRIME_HEAVY_WAVE && w < gld(a.counters, (int64_t)CNT_HEAVY)) {
      // points on the boundary (first in the order) scan the most bins: one
      // wavefront per point loads their candidates 64 at a time
      int64_t k = gld(a.order, w);
      push(a, 1, k, WHY_HEAVY);
    } else if (w < a.n) {
      int64_t k = gld(a.order, w);
      Lane<T, G, MODE, false, VMAX, PB> L(a, P, slot, k);
      if (!L.run(st, hist)) {
        push(a, 1, k, L.why);
        st.replays++;
        if (L.why == WHY_POLY) st.overflow++;
      }
    }
  }
  TRIME_D static void run(const KArgs &a, Blk blk) {
    if (cond_off(a)) return;
    __shared__ VRec<T> P[VMAX][B];
    __shared__ int hist[40];
    zero_hist<B>(hist);
    LaneStats st;
    point<B>(a, (int64_t)xcd_block(blk.id, blk.n, blockIdx.x, (uint32_t)a.xcd_run) * B + threadIdx.x, P, threadIdx.x,
             st, hist);
    flush_stats<B>(a, st, hist);
  }
  // The work of block blk by one wavefront (a block of 64 threads), 64 of
  // the block's points at a time, their statistics combined as the block
  // combines its wavefronts' (so the sums are the same).  The tile is
  // blk.id itself: the persistent kernel places its own work.
  struct WaveShm {
    VRec<T> P[VMAX][64];
    int hist[40];
  };
  TRIME_D static void run_wave(const KArgs &a, Blk blk, WaveShm &sh) {
    if (cond_off(a)) return;
    const int lane = threadIdx.x & 63;
    zero_hist<64>(sh.hist);
    WaveSums acc;
    for (int sub = 0; sub < B / 64; sub++) {
      LaneStats st;
      point<64>(a, (int64_t)blk.id * B + sub * 64 + lane, sh.P, lane, st, sh.hist);
      const WaveSums w = wave_sums(st);
      if (sub == 0)
        acc = w;
      else
        add_sums(acc, w);
    }
    if (lane == 0) emit_sums(a, acc);
    __syncthreads();
    emit_hist<64>(a, sh.hist);
  }
};

// The passes after the fast kernel, in one launch so that they overlap:
//  - blocks [0, wgrid): FP64 replay of the queue, one wavefront per point
//    (grid-stride): the ring scan, the tests, triangles and quadrature are
//    shared by the 64 lanes.  Points FP64 cannot decide go on to the exact
//    queue.
//  - the blocks after them (CVD): the deferred FP32 centroids, one
//    wavefront per point while there are few, a group of 8 lanes per point
//    when many: FP64 vertices from the stored constraints, FP64 CVD target
//    and treatment, the quadrature leaves spread over the lanes.  The cells
//    and triangles of these points were committed by the fast kernel.
// Deferred centroids up to this many take one wavefront each.
constexpr int64_t POST_WAVE_POINTS = 1024;

template <class G, int MODE, int VMAX> struct CellsPost {
  struct Args {
    KArgs a;
    int32_t wgrid;
  };
  static constexpr int BLOCK = 64;
  static constexpr int V = CQ_STRIDE - 1;
  struct Shm {
    VRec<double> P[VMAX][1];
    VRec<double> PC[V][8];
    int hist[40];
    int s0[64], incl[64];
    double ro[8];
  };
  TRIME_D static void run(const Args &A, Blk blk) {
    __shared__ Shm sh;
    body(A, blk, sh);
  }
  TRIME_D static void body(const Args &A, Blk blk, Shm &sh) {
    const KArgs &a = A.a;
    if (cond_off(a)) return;
    auto &P = sh.P;
    auto &PC = sh.PC;
    int *hist = sh.hist;
    zero_hist<64>(hist);
    LaneStats st;
    const int lane = threadIdx.x;
    const int64_t wg = A.wgrid;
    if ((int64_t)blk.id < wg) {
      int64_t nq = gld(a.counters, (int64_t)CNT_QUEUE);
      for (int64_t w = blk.id; w < nq; w += wg) {
        int64_t k = gld(a.queue, w);
        Lane<double, G, MODE, false, VMAX, 1> L(a, P, 0, k);
        bool ok = L.begin();
        if (ok) {
          L.scan_wave(lane, sh.s0, sh.incl, sh.ro);
          ok = !L.why;
        }
        if (ok) ok = L.finish_wave(lane, st, hist);
        if (!ok && lane == 0) push(a, 2, k, L.why);
        flush_point_quality<64>(a, st);
        __syncthreads();
      }
    } else if constexpr (MODE == MODE_CVD) {
      // deferred FP32 centroids: few of them, one point per wavefront (its
      // quadrature leaves spread over the lanes: latency); many, one point
      // per group of 8 lanes (throughput)
      const int64_t cb = (int64_t)blk.id - wg, cg = (int64_t)blk.n - wg;
      int64_t nq = gld(a.counters, (int64_t)CNT_QUEUE3);
      if (nq <= POST_WAVE_POINTS) {
        for (int64_t w = cb; w < nq; w += cg) {
          int64_t k = gld(a.queue3, w);
          Lane<double, G, MODE_CVD, false, VMAX, 1> L(a, P, 0, k);
          L.centroid_replay(st, w * CQ_STRIDE, lane == 0);
          __syncthreads();
        }
      } else {
        // the loop bound is uniform over the block: every group reaches the
        // shuffles of the quadrature together (idle groups on a dummy point)
        for (int64_t w0 = cb * 8; w0 < nq; w0 += cg * 8) {
          const int64_t w = w0 + (lane >> 3);
          const bool live = w < nq;
          int64_t k = gld(a.queue3, live ? w : w0);
          Lane<double, G, MODE_CVD, false, V, 8> L(a, PC, lane >> 3, k);
          L.centroid_replay(st, (live ? w : w0) * CQ_STRIDE, live && (lane & 7) == 0);
          __syncthreads();
        }
      }
    }
    flush_stats<64>(a, st, hist);
  }
};

// Exact replay of the second queue.
template <class G, int MODE, int VMAX, int B> struct CellsExact {
  using Args = KArgs;
  static constexpr int BLOCK = B;
  TRIME_D static void run(const KArgs &a, Blk blk) {
    if (cond_off(a)) return;
    __shared__ VRec<double> P[VMAX][B];
    __shared__ int hist[40];
    body(a, blk, P, hist);
  }
  // P: the polygon records, in LDS or (the persistent kernel) in the
  // calling wavefront's slice of device memory.
  TRIME_D static void body(const KArgs &a, Blk blk, VRec<double> (&P)[VMAX][B], int *hist) {
    if (cond_off(a)) return;
    zero_hist<B>(hist);
    LaneStats st;
    int64_t nq = gld(a.counters, (int64_t)CNT_QUEUE2);
    for (int64_t w = (int64_t)blk.id * B + threadIdx.x; w < nq; w += (int64_t)blk.n * B) {
      int64_t k = gld(a.queue2, w);
      Lane<double, G, MODE, true, VMAX, B> L(a, P, threadIdx.x, k);
      const bool ok = L.run(st, hist);
      flush_point_quality<1>(a, st);
      if (!ok) {  // beyond the polygon capacity, or off the grid: keep the point
        st.overflow++;
        atomicOr(&a.counters[CNT_ERR], ERR_POLY_CAP);
        if constexpr (MODE == MODE_CVD) {
          gst(a.xn, k, gld(a.x, k));
          gst(a.yn, k, gld(a.y, k));
          gst(a.catn, k, gld(a.cat, k));
          gst(a.dprevn, k, 0.0);
        }
        if constexpr (MODE == MODE_EXTRACT) gst(a.deg, k, 0);
        if constexpr (MODE != MODE_CELLS) gst(a.tri_n, k, 0);
        if constexpr (MODE == MODE_CELLS) gst(a.cell_n, (int64_t)gld(a.id, k), -1);
      }
    }
    flush_stats<B>(a, st, hist);
  }
};

// Shapes of the cell kernels as the launchers use them.
// Lanes (points) per block of the fast kernel.  CVD in FP32: 256, whose
// 45 KB of polygon records let three blocks share a CU, still three
// wavefronts per SIMD (the VGPR limit); at holes20 the CVD iterations ran
// 1.5% faster than with 128 over 40 iterations (192: 0.2% slower than 256,
// 384: 58% slower, 64: 12% slower).  Everything else: 128.  The extraction
// of DistMesh steps ran 4-9% slower with 256 (ellipses, the star batch),
// and FP64, held at two wavefronts per SIMD by its 24-byte records, 1.5%
// slower.
#ifndef TRIME_FAST_BLOCK_CVD32
#define TRIME_FAST_BLOCK_CVD32 256
#endif
template <class T, int MODE> constexpr int fast_block() {
  return (sizeof(T) == 4 && MODE == MODE_CVD) ? TRIME_FAST_BLOCK_CVD32 : 128;
}
#ifndef TRIME_FAST_VMAX
#define TRIME_FAST_VMAX 11
#endif
constexpr int FAST_VMAX = TRIME_FAST_VMAX;  // polygon capacity of the fast kernel
constexpr int REPLAY_BLOCK = 64;
constexpr int REPLAY_VMAX = 32;
constexpr int WAVE_VMAX = 64;
constexpr int WAVE_GRID = TRIME_HEAVY_WAVE ? 4096 : 1024;
constexpr int CENTROID_GRID = 4096;  // blocks for the deferred centroids (8 points each per round)
static_assert(FAST_VMAX < CQ_STRIDE, "a deferred cell must fit its queue entry");

// kinds (persistent batch kernel): the shapes the launchers use
template <class T, class G, int MODE, int B> struct KindOf<Cells<T, G, MODE, FAST_VMAX, B>> {
  static constexpr uint32_t code = kcode(KF_CELLS, is_dbl<T>(), is_dbl<G>(), MODE);
};
template <class G, int MODE> struct KindOf<CellsPost<G, MODE, WAVE_VMAX>> {
  static constexpr uint32_t code = kcode(KF_POST, false, is_dbl<G>(), MODE);
};
template <class G, int MODE> struct KindOf<CellsExact<G, MODE, REPLAY_VMAX, REPLAY_BLOCK>> {
  static constexpr uint32_t code = kcode(KF_EXACT, false, is_dbl<G>(), MODE);
};

}  // namespace trime
