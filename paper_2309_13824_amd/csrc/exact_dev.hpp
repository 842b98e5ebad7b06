// Exact sign of a cut predicate by floating-point expansion arithmetic
// (J. R. Shewchuk, "Adaptive precision floating-point arithmetic and fast
// robust geometric predicates", 1997): Two-Sum, Two-Product (via FMA),
// Grow-Expansion, Scale-Expansion and Compress, with zero elimination.
// Used only by the FP64 replay kernel, for the rare decisions that the FP64
// error bound cannot settle; symbolic perturbation (Edelsbrunner and Mücke,
// 1990) resolves exact zeros.
#pragma once
#include "trime_dev.hpp"

namespace trime {
namespace ex {

constexpr int CAP = 64;

TRIME_D void two_sum(double a, double b, double &x, double &y) {
  x = a + b;
  double bv = x - a;
  double av = x - bv;
  double br = b - bv;
  double ar = a - av;
  y = ar + br;
}

TRIME_D void two_prod(double a, double b, double &x, double &y) {
  x = a * b;
  y = fma(a, b, -x);
}

// h = e + b; h may alias e.  Returns the length (>= 1).
TRIME_D int grow(const double *e, int ne, double b, double *h) {
  double q = b;
  int hn = 0;
  for (int i = 0; i < ne; i++) {
    double qn, hh;
    two_sum(q, e[i], qn, hh);
    q = qn;
    if (hh != 0.0) h[hn++] = hh;
  }
  if (q != 0.0 || hn == 0) h[hn++] = q;
  return hn;
}

// In-place compression of a nonoverlapping expansion (increasing magnitude).
TRIME_D int compress(double *e, int n) {
  if (n <= 1) return n;
  double h[CAP];
  int bottom = n - 1;
  double Q = e[bottom];
  for (int i = n - 2; i >= 0; i--) {
    double Qn, q;
    two_sum(Q, e[i], Qn, q);
    if (q != 0.0) {
      h[bottom--] = Qn;
      Q = q;
    } else {
      Q = Qn;
    }
  }
  int top = 0;
  for (int i = bottom + 1; i < n; i++) {
    double Qn, q;
    two_sum(h[i], Q, Qn, q);
    if (q != 0.0) e[top++] = q;
    Q = Qn;
  }
  e[top] = Q;
  return top + 1;
}

// h = e + f (h must not alias f).
TRIME_D int sum(const double *e, int ne, const double *f, int nf, double *h, int *err) {
  for (int i = 0; i < ne; i++) h[i] = e[i];
  int hn = ne;
  for (int j = 0; j < nf; j++) {
    if (hn + 1 > CAP) {
      *err = 1;
      return hn;
    }
    hn = grow(h, hn, f[j], h);
  }
  return compress(h, hn);
}

// h = e * b
TRIME_D int scale(const double *e, int ne, double b, double *h, int *err) {
  if (ne == 0 || b == 0.0) return 0;
  if (2 * ne > CAP) {
    *err = 1;
    return 0;
  }
  double Q, hh;
  int hn = 0;
  two_prod(e[0], b, Q, hh);
  if (hh != 0.0) h[hn++] = hh;
  for (int i = 1; i < ne; i++) {
    double p1, p0, s;
    two_prod(e[i], b, p1, p0);
    two_sum(Q, p0, s, hh);
    if (hh != 0.0) h[hn++] = hh;
    two_sum(p1, s, Q, hh);
    if (hh != 0.0) h[hn++] = hh;
  }
  if (Q != 0.0 || hn == 0) h[hn++] = Q;
  return hn;
}

// h = e * f (h must not alias e or f)
TRIME_D int mul(const double *e, int ne, const double *f, int nf, double *h, int *err) {
  double t[CAP], acc[CAP];
  int an = 0;
  for (int j = 0; j < nf; j++) {
    int tn = scale(e, ne, f[j], t, err);
    an = sum(t, tn, acc, an, h, err);
    for (int k = 0; k < an; k++) acc[k] = h[k];
  }
  for (int k = 0; k < an; k++) h[k] = acc[k];
  return an;
}

TRIME_D int sign(const double *e, int n) {
  for (int k = n - 1; k >= 0; k--)
    if (e[k] != 0.0) return e[k] > 0 ? 1 : -1;
  return 0;
}

TRIME_D int negate(double *e, int n) {
  for (int k = 0; k < n; k++) e[k] = -e[k];
  return n;
}

// exact a - b
TRIME_D int diff(double a, double b, double *h) {
  double x, y;
  two_sum(a, -b, x, y);
  int n = 0;
  if (y != 0.0) h[n++] = y;
  if (x != 0.0 || n == 0) h[n++] = x;
  return n;
}

// A constraint of a cell in exact form, in the frame of the generator p:
// kept side n . u <= s, u = x - p.
struct XRow {
  int kind;  // 0 bisector with point id, 1 wall
  int id;
  double nx[2], ny[2];
  int nnx, nny;
  double s[CAP];
  int ns;
};

// Bisector of p and q: n = q - p, s = |n|^2 / 2.
TRIME_D void bisector(XRow &r, int id, double qx, double qy, double px, double py, int *err) {
  r.kind = 0;
  r.id = id;
  r.nnx = diff(qx, px, r.nx);
  r.nny = diff(qy, py, r.ny);
  double a[CAP], b[CAP];
  int na = mul(r.nx, r.nnx, r.nx, r.nnx, a, err);
  int nb = mul(r.ny, r.nny, r.ny, r.nny, b, err);
  r.ns = sum(a, na, b, nb, r.s, err);
  for (int k = 0; k < r.ns; k++) r.s[k] *= 0.5;  // exact halving
}

// Fixed wall: normal (wx, wy) in {0, +-1}^2; offset s given exactly as the
// expansion s0 (an octagon offset S or D) or, for a box wall through the
// coordinate c along the axis of the normal, s = n . (c - p).
TRIME_D void wall(XRow &r, int wx, int wy, bool box, double s0, double c, double px, double py) {
  r.kind = 1;
  r.id = -1;
  r.nnx = 0;
  r.nny = 0;
  if (wx) r.nx[r.nnx++] = (double)wx;
  if (wy) r.ny[r.nny++] = (double)wy;
  if (!box) {
    r.ns = 1;
    r.s[0] = s0;
  } else {
    r.ns = wx ? diff(c, px, r.s) : diff(c, py, r.s);
    if ((wx ? wx : wy) < 0) negate(r.s, r.ns);
  }
}

// det [n_a; n_b] exactly
TRIME_D int cross(const XRow &a, const XRow &b, double *h, int *err) {
  double t1[CAP], t2[CAP];
  int n1 = mul(a.nx, a.nnx, b.ny, b.nny, t1, err);
  int n2 = mul(a.ny, a.nny, b.nx, b.nnx, t2, err);
  negate(t2, n2);
  return sum(t1, n1, t2, n2, h, err);
}

// Sign of the margin of r3 at the vertex r1 ∩ r2 in the frame of point pid:
// +1 cut (the vertex lies strictly outside r3's kept side), -1 kept.
// The 3x3 determinant det3 = [n_k, s_k] equals C3 (s3 - n3 . v) with C3 the
// determinant of the first two normals, so sign(m) = -sign(det3) sign(C3).
// Exact zeros: each bisector offset carries (eps_p - eps_q)/2 with a larger
// infinitesimal eps for a smaller id; d det3 / d eps_q = -C_k / 2 and
// d det3 / d eps_p = sum of C_k / 2 over the bisector rows.  An exact zero of
// fixed walls only is not a cut.
TRIME_D int margin_sign(const XRow *r1, const XRow *r2, const XRow *r3, int pid, int *err,
                        int *sos) {
  double C1[CAP], C2[CAP], C3[CAP], t[CAP], d[CAP], d2[CAP];
  int n1 = cross(*r2, *r3, C1, err);
  int n2 = cross(*r3, *r1, C2, err);
  int n3 = cross(*r1, *r2, C3, err);
  int s3 = sign(C3, n3);
  if (s3 == 0) return -1;
  int nd = mul(r1->s, r1->ns, C1, n1, d, err);
  int nt = mul(r2->s, r2->ns, C2, n2, t, err);
  nd = sum(d, nd, t, nt, d2, err);
  nt = mul(r3->s, r3->ns, C3, n3, t, err);
  nd = sum(d2, nd, t, nt, d, err);
  int sdet = sign(d, nd);
  if (sdet == 0) {
    const XRow *rows[3] = {r1, r2, r3};
    const double *cof[3] = {C1, C2, C3};
    const int cn[3] = {n1, n2, n3};
    int ids[4], sg[4], nt2 = 0;
    double cp[CAP], tmp[CAP];
    int ncp = 0;
    bool any = false;
    for (int k = 0; k < 3; k++) {
      if (rows[k]->kind != 0) continue;
      any = true;
      ncp = sum(cp, ncp, cof[k], cn[k], tmp, err);
      for (int q = 0; q < ncp; q++) cp[q] = tmp[q];
      ids[nt2] = rows[k]->id;
      sg[nt2] = -sign(cof[k], cn[k]);
      nt2++;
    }
    if (!any) return -1;
    ids[nt2] = pid;
    sg[nt2] = sign(cp, ncp);
    nt2++;
    *sos = 1;
    // the smallest id with a nonzero coefficient decides
    int best = -1;
    for (int k = 0; k < nt2; k++)
      if (sg[k] != 0 && (best < 0 || ids[k] < ids[best])) best = k;
    if (best < 0) return -1;
    sdet = sg[best];
  }
  return (-sdet * s3) > 0 ? 1 : -1;
}

}  // namespace ex
}  // namespace trime
