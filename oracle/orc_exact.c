/*
 * Exact arithmetic for the oracle's combinatorial predicates (test
 * infrastructure only).
 *
 * The paper computes every Voronoi cell independently by half-plane cuts
 * (Sec. 2.1) and notes that floating-point error can make neighbouring cells
 * disagree near points equidistant from four generators.  The oracle instead
 * takes every cut decision exactly: a double-precision evaluation with a
 * rigorous error bound, and, when the bound cannot decide, the same
 * determinant in exact binary big-float arithmetic (each double is an
 * integer times a power of two, so sums and products of them are exact).
 * Exact zeros are resolved by Simulation of Simplicity (Edelsbrunner and
 * Mücke, 1990) applied to infinitesimal power weights eps_id, where a smaller
 * point id carries a larger weight.  This makes the cell of every point the
 * exact cell of one fixed, generic (perturbed) configuration, so all cells
 * agree with one another and with the Delaunay triangulation.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "orc_internal.h"

/* ---------------- binary big-float: value = sign * M * 2^exp ---------------- */
#define BF_MAXL 160 /* 5120-bit magnitudes */

typedef struct {
  int sign; /* -1, 0, +1 */
  int exp;
  int n;    /* limbs in use */
  uint32_t m[BF_MAXL];
} bf;

static void bf_die(const char *what) {
  fprintf(stderr, "oracle exact arithmetic: %s\n", what);
  abort();
}

static void bf_norm(bf *a) {
  while (a->n > 0 && a->m[a->n - 1] == 0) a->n--;
  if (a->n == 0) {
    a->sign = 0;
    a->exp = 0;
    return;
  }
  int k = 0;
  while (a->m[k] == 0) k++;
  if (k) {
    memmove(a->m, a->m + k, (size_t)(a->n - k) * 4);
    a->n -= k;
    a->exp += 32 * k;
  }
}

static void bf_zero(bf *a) {
  a->sign = 0;
  a->exp = 0;
  a->n = 0;
}

static void bf_set_d(bf *a, double d) {
  if (!isfinite(d)) bf_die("non-finite input");
  if (d == 0.0) {
    bf_zero(a);
    return;
  }
  int e;
  double f = frexp(fabs(d), &e); /* f in [0.5, 1) */
  uint64_t mant = (uint64_t)ldexp(f, 53);
  a->sign = d < 0 ? -1 : 1;
  a->exp = e - 53;
  a->m[0] = (uint32_t)mant;
  a->m[1] = (uint32_t)(mant >> 32);
  a->n = 2;
  bf_norm(a);
}

/* out = in << s (bits); returns limb count */
static int mag_shl(uint32_t *out, const uint32_t *in, int n, int s) {
  int q = s >> 5, r = s & 31;
  if (n + q + 1 > BF_MAXL) bf_die("magnitude overflow in shift");
  for (int k = 0; k < q; k++) out[k] = 0;
  uint32_t prev = 0;
  for (int k = 0; k < n; k++) {
    uint32_t cur = in[k];
    out[k + q] = r ? (cur << r) | (prev >> (32 - r)) : cur;
    prev = cur;
  }
  out[n + q] = r ? prev >> (32 - r) : 0;
  return n + q + 1;
}

static int mag_cmp(const uint32_t *a, int na, const uint32_t *b, int nb) {
  while (na > 0 && a[na - 1] == 0) na--;
  while (nb > 0 && b[nb - 1] == 0) nb--;
  if (na != nb) return na > nb ? 1 : -1;
  for (int k = na - 1; k >= 0; k--)
    if (a[k] != b[k]) return a[k] > b[k] ? 1 : -1;
  return 0;
}

static int mag_add(uint32_t *out, const uint32_t *a, int na, const uint32_t *b, int nb) {
  int n = na > nb ? na : nb;
  if (n + 1 > BF_MAXL) bf_die("magnitude overflow in add");
  uint64_t c = 0;
  for (int k = 0; k < n; k++) {
    uint64_t t = c + (k < na ? a[k] : 0) + (k < nb ? b[k] : 0);
    out[k] = (uint32_t)t;
    c = t >> 32;
  }
  out[n] = (uint32_t)c;
  return n + 1;
}

/* a >= b */
static int mag_sub(uint32_t *out, const uint32_t *a, int na, const uint32_t *b, int nb) {
  int64_t br = 0;
  for (int k = 0; k < na; k++) {
    int64_t t = (int64_t)a[k] - (k < nb ? b[k] : 0) - br;
    br = t < 0;
    out[k] = (uint32_t)(t + (br << 32));
  }
  return na;
}

static void bf_add(bf *r, const bf *a, const bf *b) {
  if (a->sign == 0) {
    if (r != b) *r = *b;
    return;
  }
  if (b->sign == 0) {
    if (r != a) *r = *a;
    return;
  }
  uint32_t A[BF_MAXL], B[BF_MAXL];
  int e = a->exp < b->exp ? a->exp : b->exp;
  int na = mag_shl(A, a->m, a->n, a->exp - e);
  int nb = mag_shl(B, b->m, b->n, b->exp - e);
  int sa = a->sign, sb = b->sign;
  if (sa == sb) {
    r->n = mag_add(r->m, A, na, B, nb);
    r->sign = sa;
  } else {
    int c = mag_cmp(A, na, B, nb);
    if (c == 0) {
      bf_zero(r);
      return;
    }
    if (c > 0) {
      r->n = mag_sub(r->m, A, na, B, nb);
      r->sign = sa;
    } else {
      r->n = mag_sub(r->m, B, nb, A, na);
      r->sign = sb;
    }
  }
  r->exp = e;
  bf_norm(r);
}

static void bf_neg(bf *r, const bf *a) {
  if (r != a) *r = *a;
  r->sign = -r->sign;
}

static void bf_sub(bf *r, const bf *a, const bf *b) {
  bf nb;
  bf_neg(&nb, b);
  bf_add(r, a, &nb);
}

static void bf_mul(bf *r, const bf *a, const bf *b) {
  if (a->sign == 0 || b->sign == 0) {
    bf_zero(r);
    return;
  }
  int n = a->n + b->n;
  if (n > BF_MAXL) bf_die("magnitude overflow in mul");
  uint32_t R[BF_MAXL];
  memset(R, 0, sizeof(uint32_t) * (size_t)n);
  for (int i = 0; i < a->n; i++) {
    uint64_t c = 0;
    for (int j = 0; j < b->n; j++) {
      uint64_t t = (uint64_t)a->m[i] * b->m[j] + R[i + j] + c;
      R[i + j] = (uint32_t)t;
      c = t >> 32;
    }
    R[i + b->n] = (uint32_t)c;
  }
  r->sign = a->sign * b->sign;
  r->exp = a->exp + b->exp;
  r->n = n;
  memcpy(r->m, R, sizeof(uint32_t) * (size_t)n);
  bf_norm(r);
}

/* ---------------- rows in exact and floating-point form ---------------- */

void orc_bis_row(orc_row *r, int64_t qid, double qx, double qy) {
  memset(r, 0, sizeof *r);
  r->kind = 0;
  r->qid = qid;
  r->qx = qx;
  r->qy = qy;
}

/* Octagon walls 0..7 (outward normals at 0, 45, ..., 315 degrees; offsets S
   on the axis walls and D on the diagonal ones) and the box walls 8..11
   (x <= bx1, y <= by1, x >= bx0, y >= by0). */
void orc_wall_row(orc_row *r, int w, float S, float D, double bx0, double by0, double bx1,
                  double by1) {
  static const int NX[8] = {1, 1, 0, -1, -1, -1, 0, 1};
  static const int NY[8] = {0, 1, 1, 1, 0, -1, -1, -1};
  memset(r, 0, sizeof *r);
  r->kind = 1;
  if (w < 8) {
    r->wnx = NX[w];
    r->wny = NY[w];
    r->wbox = 0;
    r->wc = (w & 1) ? (double)D : (double)S;
  } else {
    r->wbox = 1;
    switch (w) {
      case 8: r->wnx = 1; r->wny = 0; r->wpx = bx1; r->wpy = 0; break;
      case 9: r->wnx = 0; r->wny = 1; r->wpx = 0; r->wpy = by1; break;
      case 10: r->wnx = -1; r->wny = 0; r->wpx = bx0; r->wpy = 0; break;
      default: r->wnx = 0; r->wny = -1; r->wpx = 0; r->wpy = by0; break;
    }
  }
}

void orc_row_fp(const orc_row *r, double px, double py, double *nx, double *ny, double *s) {
  if (r->kind == 0) {
    *nx = r->qx - px;
    *ny = r->qy - py;
    *s = (*nx * *nx + *ny * *ny) * 0.5;
  } else {
    *nx = r->wnx;
    *ny = r->wny;
    if (!r->wbox)
      *s = r->wc;
    else
      *s = r->wnx != 0 ? r->wnx * (r->wpx - px) : r->wny * (r->wpy - py);
  }
}

static void row_bf(const orc_row *r, double px, double py, bf *nx, bf *ny, bf *s) {
  bf a, b;
  if (r->kind == 0) {
    bf_set_d(&a, r->qx);
    bf_set_d(&b, px);
    bf_sub(nx, &a, &b);
    bf_set_d(&a, r->qy);
    bf_set_d(&b, py);
    bf_sub(ny, &a, &b);
    bf t1, t2;
    bf_mul(&t1, nx, nx);
    bf_mul(&t2, ny, ny);
    bf_add(s, &t1, &t2);
    if (s->sign) s->exp -= 1; /* exact halving */
  } else {
    bf_set_d(nx, r->wnx);
    bf_set_d(ny, r->wny);
    if (!r->wbox) {
      bf_set_d(s, r->wc);
    } else if (r->wnx != 0) {
      bf_set_d(&a, r->wpx);
      bf_set_d(&b, px);
      bf_sub(s, &a, &b);
      if (r->wnx < 0) bf_neg(s, s);
    } else {
      bf_set_d(&a, r->wpy);
      bf_set_d(&b, py);
      bf_sub(s, &a, &b);
      if (r->wny < 0) bf_neg(s, s);
    }
  }
}

/* 2x2 determinant  a*d - b*c  exactly */
static void bf_det2(bf *r, const bf *a, const bf *b, const bf *c, const bf *d) {
  bf t1, t2;
  bf_mul(&t1, a, d);
  bf_mul(&t2, b, c);
  bf_sub(r, &t1, &t2);
}

/*
 * With rows (n_k, s_k), k = 1..3, the vertex v of rows 1, 2 and the margin
 * m = n_3 . v - s_3 satisfy  det3 = C3 * (s_3 - n_3 . v), where det3 is the
 * 3x3 determinant [n_k, s_k] and C_k are the cofactors of its last column
 * (C3 = det[n_1; n_2]).  Hence sign(m) = -sign(det3) * sign(C3).
 * Each bisector offset carries (eps_p - eps_q)/2, so
 *   d det3 / d eps_p = sum over bisector rows of C_k / 2,
 *   d det3 / d eps_q = -C_k / 2 for the bisector row k with point q.
 */
int orc_pred_rows(const orc_row *r1, const orc_row *r2, const orc_row *r3, double px,
                  double py, int64_t pid, int *used_exact, int *used_sos) {
  const double u = ldexp(1.0, -53);
  double n1x, n1y, s1, n2x, n2y, s2, n3x, n3y, s3;
  orc_row_fp(r1, px, py, &n1x, &n1y, &s1);
  orc_row_fp(r2, px, py, &n2x, &n2y, &s2);
  orc_row_fp(r3, px, py, &n3x, &n3y, &s3);
  double C1 = n2x * n3y - n2y * n3x;
  double C2 = n3x * n1y - n3y * n1x;
  double C3 = n1x * n2y - n1y * n2x;
  double det = s1 * C1 + s2 * C2 + s3 * C3;
  double P = fabs(s1) * (fabs(n2x * n3y) + fabs(n2y * n3x)) +
             fabs(s2) * (fabs(n3x * n1y) + fabs(n3y * n1x)) +
             fabs(s3) * (fabs(n1x * n2y) + fabs(n1y * n2x));
  double P3 = fabs(n1x * n2y) + fabs(n1y * n2x);
  /* inputs carry relative error <= 4u (the squared offsets), each product
     and sum adds one rounding; 64u is a generous rigorous bound. */
  if (fabs(det) > 64.0 * u * P && fabs(C3) > 16.0 * u * P3) {
    double m_sign = -(det > 0 ? 1.0 : -1.0) * (C3 > 0 ? 1.0 : -1.0);
    return m_sign > 0 ? 1 : -1;
  }
  if (used_exact) *used_exact = 1;
  bf N1x, N1y, S1, N2x, N2y, S2, N3x, N3y, S3;
  row_bf(r1, px, py, &N1x, &N1y, &S1);
  row_bf(r2, px, py, &N2x, &N2y, &S2);
  row_bf(r3, px, py, &N3x, &N3y, &S3);
  bf E1, E2, E3, t, D;
  bf_det2(&E1, &N2x, &N2y, &N3x, &N3y);
  bf_det2(&E2, &N3x, &N3y, &N1x, &N1y);
  bf_det2(&E3, &N1x, &N1y, &N2x, &N2y);
  if (E3.sign == 0) return -1; /* parallel pair: no vertex; never cut */
  bf_mul(&D, &S1, &E1);
  bf_mul(&t, &S2, &E2);
  bf_add(&D, &D, &t);
  bf_mul(&t, &S3, &E3);
  bf_add(&D, &D, &t);
  int sdet = D.sign;
  if (sdet == 0) {
    /* symbolic perturbation: collect (id, coefficient sign) */
    const orc_row *rows[3] = {r1, r2, r3};
    const bf *cof[3] = {&E1, &E2, &E3};
    int64_t ids[4];
    int sg[4];
    int nt = 0;
    bf cp;
    bf_zero(&cp);
    int any_bis = 0;
    for (int k = 0; k < 3; k++) {
      if (rows[k]->kind != 0) continue;
      any_bis = 1;
      bf_add(&cp, &cp, cof[k]);
      ids[nt] = rows[k]->qid;
      sg[nt] = -cof[k]->sign;
      nt++;
    }
    if (!any_bis) return -1; /* fixed walls only: exact zero is not a cut */
    ids[nt] = pid;
    sg[nt] = cp.sign;
    nt++;
    /* smallest id first */
    for (int a = 0; a < nt; a++)
      for (int b = a + 1; b < nt; b++)
        if (ids[b] < ids[a]) {
          int64_t ti = ids[a];
          ids[a] = ids[b];
          ids[b] = ti;
          int ts = sg[a];
          sg[a] = sg[b];
          sg[b] = ts;
        }
    if (used_sos) *used_sos = 1;
    for (int a = 0; a < nt; a++)
      if (sg[a] != 0) {
        sdet = sg[a];
        break;
      }
    if (sdet == 0) return -1;
  }
  return (-sdet * E3.sign) > 0 ? 1 : -1;
}

/* Exact incircle sign: > 0 when d lies inside the circle through a, b, c
   taken counter-clockwise.  Used by the brute-force pins. */
int orc_incircle_sign(double ax, double ay, double bx, double by, double cx, double cy,
                      double dx, double dy) {
  bf X[3], Y[3], Z[3], t1, t2, D;
  double px[3] = {ax, bx, cx}, py[3] = {ay, by, cy};
  bf Dx, Dy;
  bf_set_d(&Dx, dx);
  bf_set_d(&Dy, dy);
  for (int k = 0; k < 3; k++) {
    bf a;
    bf_set_d(&a, px[k]);
    bf_sub(&X[k], &a, &Dx);
    bf_set_d(&a, py[k]);
    bf_sub(&Y[k], &a, &Dy);
    bf_mul(&t1, &X[k], &X[k]);
    bf_mul(&t2, &Y[k], &Y[k]);
    bf_add(&Z[k], &t1, &t2);
  }
  /* det [X Y Z] by the first column */
  bf m0, m1, m2;
  bf_det2(&m0, &Y[1], &Z[1], &Y[2], &Z[2]);
  bf_det2(&m1, &Y[0], &Z[0], &Y[2], &Z[2]);
  bf_det2(&m2, &Y[0], &Z[0], &Y[1], &Z[1]);
  bf_mul(&D, &X[0], &m0);
  bf_mul(&t1, &X[1], &m1);
  bf_sub(&D, &D, &t1);
  bf_mul(&t1, &X[2], &m2);
  bf_add(&D, &D, &t1);
  return D.sign;
}
