/* Internal declarations of the CPU oracle (test infrastructure only). */
#ifndef ORC_INTERNAL_H
#define ORC_INTERNAL_H
#include "orc.h"

/* One constraint of a cell, in the frame of the generator p:
   a bisector with point q (kind 0) or a fixed wall (kind 1).
   The kept side is  n . u <= s  with u = x - p.
   Bisector:  n = q - p,  s = |n|^2 / 2   (+ symbolic weights, see orc_exact.c)
   Wall:      n = (wnx, wny) in {0, +-1}^2,  s = wc  (octagon, exact float)
              or s = wnx*(wpx - px) + wny*(wpy - py)  (box wall through (wpx, wpy)) */
typedef struct {
  int kind;          /* 0 bisector, 1 wall                                   */
  int64_t qid;       /* bisector: point id                                    */
  double qx, qy;     /* bisector: absolute position of q                      */
  double wnx, wny;   /* wall normal                                           */
  int wbox;          /* wall: 0 octagon (s = wc), 1 box (s through wpx, wpy)  */
  double wc, wpx, wpy;
} orc_row;

/* Exact sign of the margin of r3 at the vertex r1 ∩ r2, frame point (px, py)
   with id pid: +1 when the vertex lies strictly on the cut side of r3, -1
   otherwise.  Exact zeros with a bisector involved are resolved by symbolic
   perturbation; an exact zero between fixed walls counts as not cut. */
int orc_pred_rows(const orc_row *r1, const orc_row *r2, const orc_row *r3, double px,
                  double py, int64_t pid, int *used_exact, int *used_sos);

/* Rows of the octagon / box walls of a point. */
void orc_wall_row(orc_row *r, int w, float S, float D, double bx0, double by0, double bx1,
                  double by1);
void orc_bis_row(orc_row *r, int64_t qid, double qx, double qy);
/* Floating-point (n, s) of a row relative to p; used for vertex coordinates. */
void orc_row_fp(const orc_row *r, double px, double py, double *nx, double *ny, double *s);

/* Reusable neighbour-search context for per-cell queries. */
typedef struct orc_cellctx orc_cellctx;
orc_cellctx *orc_cellctx_new(const orc_grid *g, const orc_params *prm, int64_t n,
                             const double *x, const double *y);
void orc_cellctx_free(orc_cellctx *c);
/* Cell of point i with vertex coordinates relative to p_i (see orc_cell). */
int orc_cellctx_cell(const orc_cellctx *c, int64_t i, int32_t *cons, double *vx, double *vy,
                     int cap, orc_counters *cnt);
int orc_cvd_centroid_ctx(const orc_cellctx *cc, const orc_grid *g, const orc_params *prm,
                         const double *x, const double *y, int64_t i, double dprev, double *cx,
                         double *cy, double *area, orc_counters *cnt);

#endif
