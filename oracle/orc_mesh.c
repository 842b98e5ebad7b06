/*
 * Oracle: Procedure I (Sec. 2.1, Sec. 4.1) -- bounded Voronoi cells by
 * half-plane cuts, Delaunay triangles from the cells, and the three validity
 * tests; mesh quality (Eq. 10-11).  Test infrastructure only.
 *
 * Cell of point i (Sec. 4.1): start from an octagon of span S = fac_voro*h_i
 * around p_i and cut it by the bisector of every neighbour.  Readings:
 *  - "span S" is the apothem: |u_x|, |u_y| <= S and |u_x| + |u_y| <= D with
 *    D = fl32(fl32(sqrt 2) * S), S = fl32(fac_voro * h_cell) in float, h_cell
 *    the float h of the grid cell holding p_i;
 *  - the cell is also clipped by the grid's bounding box (the container);
 *  - every cut decision is exact (orc_exact.c);
 *  - neighbours are taken in order of distance and the scan stops once the
 *    next one is farther than twice the largest vertex distance: such a
 *    point q satisfies q.v - |q|^2/2 < 0 for every vertex v, so it cannot cut.
 *
 * Triangles (Sec. 1.1, Sec. 4.1): every cell vertex formed by the bisectors
 * of two neighbours j, k is the circumcentre of (i, j, k).  Reading: the
 * triangle exists when that circumcentre is a vertex of all three bounded
 * cells (it is inside the octagons of j and k as well); the smallest id owns
 * it and stores it counter-clockwise, owner first.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "orc_internal.h"

#define ORC_MAXV 256

typedef struct {
  const orc_grid *g;
  const orc_params *prm;
  int64_t n;
  const double *x, *y;
  double bx0, by0, bx1, by1;
  /* bucket grid for neighbour search (plain uniform buckets) */
  int bnx, bny;
  double bw;
  int64_t *bstart; /* bnx*bny + 1 */
  int64_t *bitems;
} octx;

static int point_span(const octx *c, double px, double py, float *S, float *D) {
  int64_t cell;
  double tx, ty;
  if (!orc_locate(c->g, px, py, &cell, &tx, &ty)) return 0;
  float h = c->g->hcell[cell];
  *S = (float)c->prm->fac_voro * h;
  *D = 1.41421356f * *S;
  return 1;
}

static void make_row(const octx *c, float S, float D, int32_t con, orc_row *r) {
  if (con >= 0)
    orc_bis_row(r, con, c->x[con], c->y[con]);
  else
    orc_wall_row(r, -1 - con, S, D, c->bx0, c->by0, c->bx1, c->by1);
}

static int pred(const octx *c, int64_t pid, double px, double py, float S, float D, int32_t c1,
                int32_t c2, int32_t c3, orc_counters *cnt) {
  orc_row r1, r2, r3;
  make_row(c, S, D, c1, &r1);
  make_row(c, S, D, c2, &r2);
  make_row(c, S, D, c3, &r3);
  int ue = 0, us = 0;
  int s = orc_pred_rows(&r1, &r2, &r3, px, py, pid, &ue, &us);
  if (cnt) {
    cnt->clip_tests++;
    cnt->exact_calls += ue;
    cnt->sos_calls += us;
  }
  return s;
}

static void vertex_xy(const octx *c, double px, double py, float S, float D, int32_t c1,
                      int32_t c2, double *vx, double *vy) {
  orc_row r1, r2;
  make_row(c, S, D, c1, &r1);
  make_row(c, S, D, c2, &r2);
  double n1x, n1y, s1, n2x, n2y, s2;
  orc_row_fp(&r1, px, py, &n1x, &n1y, &s1);
  orc_row_fp(&r2, px, py, &n2x, &n2y, &s2);
  double det = n1x * n2y - n1y * n2x;
  *vx = (s1 * n2y - s2 * n1y) / det;
  *vy = (n1x * s2 - n2x * s1) / det;
}

/* Cut the polygon (CCW edge constraints) by constraint con. */
static int clip(const octx *c, int64_t pid, double px, double py, float S, float D,
                int32_t *cons, int n, int32_t con, orc_counters *cnt) {
  int cut[ORC_MAXV];
  int ncut = 0;
  for (int k = 0; k < n; k++) {
    cut[k] = pred(c, pid, px, py, S, D, cons[(k - 1 + n) % n], cons[k], con, cnt) > 0;
    ncut += cut[k];
  }
  if (ncut == 0) return n;
  if (cnt) cnt->cuts++;
  if (ncut == n) return 0;
  int k0 = -1, k1 = -1, starts = 0;
  for (int k = 0; k < n; k++) {
    if (cut[k] && !cut[(k - 1 + n) % n]) {
      k0 = k;
      starts++;
    }
    if (cut[k] && !cut[(k + 1) % n]) k1 = k;
  }
  if (starts != 1) {
    fprintf(stderr, "oracle: non-contiguous cut run (point %lld)\n", (long long)pid);
    abort();
  }
  int32_t out[ORC_MAXV];
  int m = 0;
  out[m++] = con;
  for (int t = k1;; t = (t + 1) % n) {
    out[m++] = cons[t];
    if (t == (k0 - 1 + n) % n) break;
  }
  if (m > ORC_MAXV - 2) {
    fprintf(stderr, "oracle: polygon capacity exceeded\n");
    abort();
  }
  memcpy(cons, out, sizeof(int32_t) * (size_t)m);
  return m;
}

static double poly_rmax2(const octx *c, double px, double py, float S, float D,
                         const int32_t *cons, int n) {
  double r2 = 0.0;
  for (int k = 0; k < n; k++) {
    double vx, vy;
    vertex_xy(c, px, py, S, D, cons[(k - 1 + n) % n], cons[k], &vx, &vy);
    double t = vx * vx + vy * vy;
    if (t > r2) r2 = t;
  }
  return r2;
}

/* Octagon of point i clipped by the box. */
static int initial_polygon(const octx *c, int64_t i, double px, double py, float S, float D,
                           int32_t *cons, orc_counters *cnt) {
  int n = 8;
  for (int w = 0; w < 8; w++) cons[w] = -1 - w;
  for (int w = 8; w < 12; w++) {
    n = clip(c, i, px, py, S, D, cons, n, -1 - w, cnt);
    if (n == 0) return 0;
  }
  return n;
}

typedef struct {
  double d2;
  int64_t id;
} cand;

static int cand_cmp(const void *a, const void *b) {
  const cand *x = a, *y = b;
  if (x->d2 < y->d2) return -1;
  if (x->d2 > y->d2) return 1;
  return (x->id > y->id) - (x->id < y->id);
}

static void octx_init(octx *c, const orc_grid *g, const orc_params *prm, int64_t n,
                      const double *x, const double *y, int buckets) {
  memset(c, 0, sizeof *c);
  c->g = g;
  c->prm = prm;
  c->n = n;
  c->x = x;
  c->y = y;
  c->bx0 = g->x0;
  c->by0 = g->y0;
  c->bx1 = g->x0 + (g->nx - 1) * g->dx;
  c->by1 = g->y0 + (g->ny - 1) * g->dy;
  if (!buckets) return;
  double W = c->bx1 - c->bx0, Hh = c->by1 - c->by0;
  double w = sqrt(W * Hh / (double)(n > 0 ? n : 1)) * 2.0;
  if (!(w > 0)) w = W;
  c->bw = w;
  c->bnx = (int)(W / w) + 1;
  c->bny = (int)(Hh / w) + 1;
  int64_t nb = (int64_t)c->bnx * c->bny;
  c->bstart = calloc((size_t)nb + 1, sizeof(int64_t));
  c->bitems = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t *key = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  for (int64_t i = 0; i < n; i++) {
    int bx = (int)floor((x[i] - c->bx0) / w), by = (int)floor((y[i] - c->by0) / w);
    if (bx < 0) bx = 0;
    if (by < 0) by = 0;
    if (bx >= c->bnx) bx = c->bnx - 1;
    if (by >= c->bny) by = c->bny - 1;
    key[i] = (int64_t)by * c->bnx + bx;
    c->bstart[key[i] + 1]++;
  }
  for (int64_t b = 0; b < nb; b++) c->bstart[b + 1] += c->bstart[b];
  int64_t *fill = malloc(sizeof(int64_t) * (size_t)nb);
  memcpy(fill, c->bstart, sizeof(int64_t) * (size_t)nb);
  for (int64_t i = 0; i < n; i++) c->bitems[fill[key[i]]++] = i;
  free(fill);
  free(key);
}

static void octx_free(octx *c) {
  free(c->bstart);
  free(c->bitems);
}

/* The cell of point i.  all_pairs: scan every point, no stopping radius. */
static int cell_of(const octx *c, int64_t i, int32_t *cons, int all_pairs, orc_counters *cnt) {
  double px = c->x[i], py = c->y[i];
  float S, D;
  if (!point_span(c, px, py, &S, &D)) return -2;
  int n = initial_polygon(c, i, px, py, S, D, cons, cnt);
  if (n == 0) return 0;
  double r0 = 2.0 * sqrt(poly_rmax2(c, px, py, S, D, cons, n)) * 1.001;
  cand *cl = NULL;
  int64_t nc = 0, capc = 0;
  if (all_pairs) {
    capc = c->n;
    cl = malloc(sizeof(cand) * (size_t)(capc > 0 ? capc : 1));
    for (int64_t j = 0; j < c->n; j++) {
      if (j == i) continue;
      double dx = c->x[j] - px, dy = c->y[j] - py;
      cl[nc].d2 = dx * dx + dy * dy;
      cl[nc].id = j;
      nc++;
    }
  } else {
    int bx0 = (int)floor((px - r0 - c->bx0) / c->bw), bx1 = (int)floor((px + r0 - c->bx0) / c->bw);
    int by0 = (int)floor((py - r0 - c->by0) / c->bw), by1 = (int)floor((py + r0 - c->by0) / c->bw);
    if (bx0 < 0) bx0 = 0;
    if (by0 < 0) by0 = 0;
    if (bx1 >= c->bnx) bx1 = c->bnx - 1;
    if (by1 >= c->bny) by1 = c->bny - 1;
    capc = 64;
    cl = malloc(sizeof(cand) * (size_t)capc);
    for (int by = by0; by <= by1; by++)
      for (int bx = bx0; bx <= bx1; bx++) {
        int64_t b = (int64_t)by * c->bnx + bx;
        for (int64_t t = c->bstart[b]; t < c->bstart[b + 1]; t++) {
          int64_t j = c->bitems[t];
          if (j == i) continue;
          double dx = c->x[j] - px, dy = c->y[j] - py;
          double d2 = dx * dx + dy * dy;
          if (d2 > r0 * r0) continue;
          if (nc == capc) {
            capc *= 2;
            cl = realloc(cl, sizeof(cand) * (size_t)capc);
          }
          cl[nc].d2 = d2;
          cl[nc].id = j;
          nc++;
        }
      }
  }
  qsort(cl, (size_t)nc, sizeof(cand), cand_cmp);
  double rmax2 = poly_rmax2(c, px, py, S, D, cons, n);
  for (int64_t t = 0; t < nc; t++) {
    if (cnt) cnt->candidates++;
    if (!all_pairs && cl[t].d2 > 4.0 * rmax2 * 1.002) break;
    int m = clip(c, i, px, py, S, D, cons, n, (int32_t)cl[t].id, cnt);
    if (m == 0) {
      n = 0;
      break;
    }
    if (m != n || m != 0) {
      n = m;
      rmax2 = poly_rmax2(c, px, py, S, D, cons, n);
    }
  }
  free(cl);
  if (n == 0 && cnt) cnt->empty_cells++;
  return n;
}

struct orc_cellctx {
  octx c;
};

orc_cellctx *orc_cellctx_new(const orc_grid *g, const orc_params *prm, int64_t n,
                             const double *x, const double *y) {
  orc_cellctx *cc = malloc(sizeof *cc);
  octx_init(&cc->c, g, prm, n, x, y, 1);
  return cc;
}

void orc_cellctx_free(orc_cellctx *cc) {
  octx_free(&cc->c);
  free(cc);
}

int orc_cellctx_cell(const orc_cellctx *cc, int64_t i, int32_t *cons, double *vx, double *vy,
                     int cap, orc_counters *cnt) {
  const octx *c = &cc->c;
  int32_t poly[ORC_MAXV];
  int m = cell_of(c, i, poly, 0, cnt);
  if (m > cap) return -1;
  if (m < 0) return m;
  float S = 0, D = 0;
  point_span(c, c->x[i], c->y[i], &S, &D);
  for (int k = 0; k < m; k++) {
    cons[k] = poly[k];
    if (vx && vy)
      vertex_xy(c, c->x[i], c->y[i], S, D, poly[(k - 1 + m) % m], poly[k], &vx[k], &vy[k]);
  }
  return m;
}

int orc_cell(const orc_grid *g, const orc_params *prm, int64_t n, const double *x,
             const double *y, int64_t i, int32_t *cons, double *vx, double *vy, int cap,
             orc_counters *cnt) {
  orc_cellctx *cc = orc_cellctx_new(g, prm, n, x, y);
  int m = orc_cellctx_cell(cc, i, cons, vx, vy, cap, cnt);
  orc_cellctx_free(cc);
  return m;
}

static void canon_store(const int32_t *poly, int m, int32_t *dst) {
  int s = 0;
  for (int k = 1; k < m; k++)
    if (poly[k] < poly[s]) s = k;
  for (int k = 0; k < m; k++) dst[k] = poly[(s + k) % m];
}

static int cells_all_impl(const orc_grid *g, const orc_params *prm, int64_t n, const double *x,
                          const double *y, int32_t *cons, int32_t *ncons, int cap, int all_pairs,
                          int nthreads, orc_counters *cnt) {
  octx c;
  octx_init(&c, g, prm, n, x, y, !all_pairs);
  int err = 0;
  orc_counters tot;
  memset(&tot, 0, sizeof tot);
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
  {
    orc_counters loc;
    memset(&loc, 0, sizeof loc);
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
      int32_t poly[ORC_MAXV];
      int m = cell_of(&c, i, poly, all_pairs, &loc);
      if (m < 0 || m > cap) {
#pragma omp atomic write
        err = 1;
        ncons[i] = -1;
        continue;
      }
      ncons[i] = m;
      canon_store(poly, m, cons + (size_t)i * cap);
    }
#pragma omp critical
    {
      int64_t *a = (int64_t *)&tot, *b = (int64_t *)&loc;
      for (size_t k = 0; k < sizeof(orc_counters) / sizeof(int64_t); k++) a[k] += b[k];
    }
  }
  if (cnt) {
    int64_t *a = (int64_t *)cnt, *b = (int64_t *)&tot;
    for (size_t k = 0; k < sizeof(orc_counters) / sizeof(int64_t); k++) a[k] += b[k];
  }
  octx_free(&c);
  return err ? -1 : 0;
}

int orc_cells_all(const orc_grid *g, const orc_params *prm, int64_t n, const double *x,
                  const double *y, int32_t *cons, int32_t *ncons, int cap, int nthreads,
                  orc_counters *cnt) {
  return cells_all_impl(g, prm, n, x, y, cons, ncons, cap, 0, nthreads, cnt);
}

int orc_cells_all_pairs(const orc_grid *g, const orc_params *prm, int64_t n, const double *x,
                        const double *y, int32_t *cons, int32_t *ncons, int cap) {
  return cells_all_impl(g, prm, n, x, y, cons, ncons, cap, 1, 1, NULL);
}

/* Is the circumcentre of (j, a, b) inside the octagon of j?  Evaluated in
   j's frame with the same exact predicate as the cuts. */
static int inside_octagon(const octx *c, int64_t j, int64_t a, int64_t b, orc_counters *cnt) {
  double px = c->x[j], py = c->y[j];
  float S, D;
  if (!point_span(c, px, py, &S, &D)) return 0;
  for (int w = 0; w < 8; w++)
    if (pred(c, j, px, py, S, D, (int32_t)a, (int32_t)b, -1 - w, cnt) > 0) return 0;
  return 1;
}

int orc_predicate(const orc_grid *g, const orc_params *prm, const double *x, const double *y,
                  int64_t i, int32_t c1, int32_t c2, int32_t c3, int *used_exact) {
  octx c;
  octx_init(&c, g, prm, 0, x, y, 0);
  float S, D;
  if (!point_span(&c, x[i], y[i], &S, &D)) return 0;
  orc_row r1, r2, r3;
  make_row(&c, S, D, c1, &r1);
  make_row(&c, S, D, c2, &r2);
  make_row(&c, S, D, c3, &r3);
  return orc_pred_rows(&r1, &r2, &r3, x[i], y[i], i, used_exact, NULL);
}

/* ---- validity: Procedure I's check, Sec. 4.1 Tests 1-3 ---- */

static double bilin(const orc_grid *g, const double *f, int64_t cell, double tx, double ty) {
  int64_t ci = cell % (g->nx - 1), cj = cell / (g->nx - 1);
  size_t n0 = (size_t)cj * g->nx + (size_t)ci;
  double f00 = f[n0], f10 = f[n0 + 1], f01 = f[n0 + g->nx], f11 = f[n0 + g->nx + 1];
  return (f00 * (1.0 - tx) + f10 * tx) * (1.0 - ty) + (f01 * (1.0 - tx) + f11 * tx) * ty;
}

double orc_sdf_at(const orc_grid *g, double x, double y, int *on_grid) {
  int64_t cell;
  double tx, ty;
  if (!orc_locate(g, x, y, &cell, &tx, &ty)) {
    *on_grid = 0;
    return INFINITY;
  }
  *on_grid = 1;
  return bilin(g, g->sdf, cell, tx, ty);
}

static double geps_of(const orc_grid *g, const orc_params *prm, int64_t cell) {
  return prm->fac_geps * fmin((double)g->hcell[cell], g->h_avg);
}

int orc_triangle_valid(const orc_grid *g, const orc_params *prm, const double *x,
                       const double *y, int32_t a, int32_t b, int32_t c) {
  int32_t t;
  if (a > b) { t = a; a = b; b = t; }
  if (b > c) { t = b; b = c; c = t; }
  if (a > b) { t = a; a = b; b = t; }
  int64_t cell;
  double tx, ty;
  /* Test 1: centroid */
  double gx = ((x[a] + x[b]) + x[c]) / 3.0, gy = ((y[a] + y[b]) + y[c]) / 3.0;
  if (!orc_locate(g, gx, gy, &cell, &tx, &ty)) return 0;
  uint8_t ct = g->cat[cell];
  if (ct == ORC_CAT_INNER) return 1;
  if (ct == ORC_CAT_OUTER) return 0;
  if (bilin(g, g->sdf, cell, tx, ty) > geps_of(g, prm, cell)) return 0;
  /* Test 2: edge midpoints inside or on the boundary */
  int32_t pa[3] = {a, b, a}, pb[3] = {b, c, c};
  int count = 0;
  for (int e = 0; e < 3; e++) {
    double mx = (x[pa[e]] + x[pb[e]]) * 0.5, my = (y[pa[e]] + y[pb[e]]) * 0.5;
    if (!orc_locate(g, mx, my, &cell, &tx, &ty)) continue;
    uint8_t cm = g->cat[cell];
    if (cm == ORC_CAT_INNER)
      count++;
    else if (cm == ORC_CAT_BOUNDARY && bilin(g, g->sdf, cell, tx, ty) <= geps_of(g, prm, cell))
      count++;
  }
  if (count >= 2) return 1;
  if (count == 0 || prm->test2_mode == 1) return 0;
  /* Test 3: circumcentre */
  double bx = x[b] - x[a], by = y[b] - y[a], qx = x[c] - x[a], qy = y[c] - y[a];
  double d = 2.0 * (bx * qy - by * qx);
  if (d == 0.0) return 0;
  double b2 = bx * bx + by * by, q2 = qx * qx + qy * qy;
  double ux = (qy * b2 - by * q2) / d, uy = (bx * q2 - qx * b2) / d;
  double R = sqrt(ux * ux + uy * uy);
  double ccx = x[a] + ux, ccy = y[a] + uy;
  if (!orc_locate(g, ccx, ccy, &cell, &tx, &ty)) return 0;
  double s = bilin(g, g->sdf, cell, tx, ty);
  return fabs(s) / R <= prm->T_tria;
}

static int i64cmp(const void *a, const void *b) {
  int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
  return (x > y) - (x < y);
}

#define ORC_TRI_PER_POINT 64

int orc_triangulate(const orc_grid *g, const orc_params *prm, int64_t n, const double *x,
                    const double *y, int32_t *tri, uint8_t *valid, int64_t tri_cap,
                    int64_t *ntri, int64_t *rowptr, int32_t *col, int64_t adj_cap,
                    int64_t *nadj, int nthreads, orc_counters *cnt) {
  octx c;
  octx_init(&c, g, prm, n, x, y, 1);
  int32_t *own = malloc(sizeof(int32_t) * 2 * (size_t)ORC_TRI_PER_POINT * (size_t)(n > 0 ? n : 1));
  int32_t *nown = calloc((size_t)(n > 0 ? n : 1), sizeof(int32_t));
  int err = 0;
  orc_counters tot;
  memset(&tot, 0, sizeof tot);
#pragma omp parallel num_threads(nthreads > 0 ? nthreads : 1)
  {
    orc_counters loc;
    memset(&loc, 0, sizeof loc);
#pragma omp for schedule(dynamic, 64)
    for (int64_t i = 0; i < n; i++) {
      int32_t poly[ORC_MAXV];
      int m = cell_of(&c, i, poly, 0, &loc);
      if (m < 0) {
#pragma omp atomic write
        err = 1;
        continue;
      }
      int k = 0;
      for (int t = 0; t < m; t++) {
        int32_t j = poly[(t - 1 + m) % m], l = poly[t];
        if (j < 0 || l < 0 || !(i < j && i < l)) continue;
        if (!inside_octagon(&c, j, i, l, &loc) || !inside_octagon(&c, l, i, j, &loc)) continue;
        if (k == ORC_TRI_PER_POINT) {
#pragma omp atomic write
          err = 1;
          break;
        }
        own[((size_t)i * ORC_TRI_PER_POINT + k) * 2] = j;
        own[((size_t)i * ORC_TRI_PER_POINT + k) * 2 + 1] = l;
        k++;
      }
      nown[i] = k;
    }
#pragma omp critical
    {
      int64_t *a = (int64_t *)&tot, *b = (int64_t *)&loc;
      for (size_t k = 0; k < sizeof(orc_counters) / sizeof(int64_t); k++) a[k] += b[k];
    }
  }
  if (cnt) {
    int64_t *a = (int64_t *)cnt, *b = (int64_t *)&tot;
    for (size_t k = 0; k < sizeof(orc_counters) / sizeof(int64_t); k++) a[k] += b[k];
  }
  octx_free(&c);
  if (err) {
    free(own);
    free(nown);
    return -2;
  }
  int64_t T = 0;
  for (int64_t i = 0; i < n; i++) T += nown[i];
  *ntri = T;
  if (T > tri_cap) {
    free(own);
    free(nown);
    *nadj = -1;
    return -1;
  }
  int64_t t = 0;
  for (int64_t i = 0; i < n; i++)
    for (int k = 0; k < nown[i]; k++, t++) {
      tri[3 * t] = (int32_t)i;
      tri[3 * t + 1] = own[((size_t)i * ORC_TRI_PER_POINT + k) * 2];
      tri[3 * t + 2] = own[((size_t)i * ORC_TRI_PER_POINT + k) * 2 + 1];
    }
  free(own);
  free(nown);
#pragma omp parallel for num_threads(nthreads > 0 ? nthreads : 1) schedule(static)
  for (int64_t q = 0; q < T; q++)
    valid[q] = (uint8_t)orc_triangle_valid(g, prm, x, y, tri[3 * q], tri[3 * q + 1], tri[3 * q + 2]);
  /* adjacency: unique edges of valid triangles, symmetric, rows sorted */
  int64_t *deg = calloc((size_t)n + 1, sizeof(int64_t));
  for (int64_t q = 0; q < T; q++)
    if (valid[q])
      for (int e = 0; e < 3; e++) {
        deg[tri[3 * q + e]] += 2; /* both other vertices */
      }
  int64_t tot_slots = 0;
  for (int64_t i = 0; i < n; i++) tot_slots += deg[i];
  int32_t *tmp = malloc(sizeof(int32_t) * (size_t)(tot_slots > 0 ? tot_slots : 1));
  int64_t *st = malloc(sizeof(int64_t) * ((size_t)n + 1));
  st[0] = 0;
  for (int64_t i = 0; i < n; i++) st[i + 1] = st[i] + deg[i];
  int64_t *fill = calloc((size_t)n + 1, sizeof(int64_t));
  for (int64_t q = 0; q < T; q++)
    if (valid[q])
      for (int e = 0; e < 3; e++) {
        int32_t v = tri[3 * q + e];
        tmp[st[v] + fill[v]++] = tri[3 * q + (e + 1) % 3];
        tmp[st[v] + fill[v]++] = tri[3 * q + (e + 2) % 3];
      }
  int64_t A = 0;
  for (int64_t i = 0; i < n; i++) {
    int32_t *r = tmp + st[i];
    int64_t dn = deg[i];
    qsort(r, (size_t)dn, sizeof(int32_t), i64cmp);
    int64_t u = 0;
    for (int64_t k = 0; k < dn; k++)
      if (k == 0 || r[k] != r[k - 1]) r[u++] = r[k];
    deg[i] = u;
    A += u;
  }
  *nadj = A;
  if (A > adj_cap) {
    free(tmp);
    free(st);
    free(fill);
    free(deg);
    return -1;
  }
  int64_t o = 0;
  for (int64_t i = 0; i < n; i++) {
    rowptr[i] = o;
    for (int64_t k = 0; k < deg[i]; k++) col[o++] = tmp[st[i] + k];
  }
  rowptr[n] = o;
  free(tmp);
  free(st);
  free(fill);
  free(deg);
  return 0;
}

/* ---- mesh quality, Eq. 10-11 ---- */

void orc_triangle_quality(double ax, double ay, double bx, double by, double cx, double cy,
                          double *alpha, double *beta) {
  double l0 = sqrt((bx - ax) * (bx - ax) + (by - ay) * (by - ay));
  double l1 = sqrt((cx - bx) * (cx - bx) + (cy - by) * (cy - by));
  double l2 = sqrt((ax - cx) * (ax - cx) + (ay - cy) * (ay - cy));
  double A2 = fabs((bx - ax) * (cy - ay) - (by - ay) * (cx - ax)); /* twice the area */
  /* R = l0 l1 l2 / (2 A2), r_in = A2 / (l0 + l1 + l2), alpha = R / (2 r_in) */
  *alpha = (l0 * l1 * l2) * (l0 + l1 + l2) / (4.0 * A2 * A2);
  double lmax = fmax(l0, fmax(l1, l2)), lmin = fmin(l0, fmin(l1, l2));
  *beta = lmax / lmin;
}

void orc_quality(const double *x, const double *y, const int32_t *tri, const uint8_t *valid,
                 int64_t ntri, orc_stats *st) {
  memset(st, 0, sizeof *st);
  double sa = 0, sb = 0, sq = 0, amax = 0;
  int64_t cnt = 0;
  for (int64_t q = 0; q < ntri; q++) {
    if (valid && !valid[q]) continue;
    int32_t a = tri[3 * q], b = tri[3 * q + 1], c = tri[3 * q + 2];
    double al, be;
    orc_triangle_quality(x[a], y[a], x[b], y[b], x[c], y[c], &al, &be);
    sa += sqrt(al);
    sb += sqrt(be);
    sq += 1.0 / al;
    if (al > amax) amax = al;
    /* 40 bins of width 0.05 from beta = 1, the last one open; the bin is
       chosen before converting, since beta has no upper bound (a valid
       triangle can have an edge many orders shorter than the others) */
    double fb = floor((be - 1.0) / 2.0 * 40.0);
    int bin = 39;
    if (fb < 39.0) bin = fb > 0.0 ? (int)fb : 0;
    st->hist_beta[bin] += 1.0;
    cnt++;
  }
  st->ntri = cnt;
  if (cnt) {
    st->half_mean_alpha = (sa / cnt) * (sa / cnt);
    st->half_mean_beta = (sb / cnt) * (sb / cnt);
    st->max_alpha = amax;
    st->min_q = 1.0 / amax;
    st->mean_q = sq / cnt;
    for (int k = 0; k < 40; k++) st->hist_beta[k] /= (double)cnt;
  }
}
