/*
 * Plain CPU oracle for the per-iteration hot path of the TriMe++ meshers
 * (Lu & Rycroft, "TriMe++: Multi-threaded triangular meshing in two
 * dimensions", arXiv 2309.13824).
 *
 * TEST INFRASTRUCTURE ONLY.  This library defines what the GPU path must
 * compute; it is slow on purpose, evaluates every floating-point quantity in
 * FP64 and every combinatorial predicate exactly (FP64 filter, then exact
 * big-float arithmetic, then symbolic perturbation for exact ties).  Only the
 * test-suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load it.  It shares no code, header, table or helper with the GPU library.
 *
 * Every function names the passage of the paper it follows.  Where the paper
 * is silent or ambiguous, the reading taken is stated at the function it
 * affects.
 */
#ifndef ORC_H
#define ORC_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- geometry (Sec. 3.1: analytic SDF and set operations) ---------------- */
enum { ORC_OP_INIT = 0, ORC_OP_UNION = 1, ORC_OP_DIFF = 2, ORC_OP_INTERSECT = 3 };
enum { ORC_PRIM_DISK = 0, ORC_PRIM_BOX = 1, ORC_PRIM_ELLIPSE = 2, ORC_PRIM_POLYGON = 3, ORC_PRIM_SEGMENTS = 4 };

typedef struct {
  int32_t op, kind;
  /* DISK: cx, cy, r.  BOX: x0, y0, x1, y1.  ELLIPSE: cx, cy, a, b, phi.
     POLYGON: vertices in poly[voff .. voff+nv) as (x, y) pairs, any winding.
     SEGMENTS: a closed clockwise loop of line segments through poly[voff ..
     voff+nv) (Sec. 3.2): distance to the nearest segment, sign from its
     inward normal (orc_segments_sdf). */
  double p[6];
  int32_t voff, nv;
} orc_prim;

/* Signed distance to a closed clockwise loop of nv >= 3 segments, segment k
   from v_k to v_(k+1 mod nv) (Sec. 3.2).  The magnitude is the distance to
   the nearest segment (the closest point p* = a + t (b - a), t clamped to
   [0, 1]); equal distances go to the lower segment index.  The inward
   normal of a segment is its direction turned clockwise by 90 degrees (the
   interior lies to the right of a clockwise loop), unit length; when p* is
   an end point the normal is the mean of the unit normals of the two
   segments that meet there.  The sign is negative (inside) when
   (p - p*) . n > 0, else positive.  Brute force over every segment.  If
   seg_out is not null it receives the nearest segment's index. */
double orc_segments_sdf(const double *v, int32_t nv, double x, double y, int32_t *seg_out);

/* ---- sizing field (Sec. 3.3-3.4, Eq. 9) ---------------------------------- */
enum {
  ORC_SZ_UNIFORM = 0,     /* mu = 1                                          */
  ORC_SZ_ABS_SDF = 1,     /* mu = a0 + a1*|sdf(x)|                           */
  ORC_SZ_GAUSS_RHO = 2,   /* rho = a0 + a1*sum_k exp(-|x-c_k|^2/s2); mu = rho^-1/2 */
  ORC_SZ_HOLE_RAMP = 3,   /* mu = 1 + (a0-1)*min(d_H(x)/a1, 1), d_H = distance to
                             the nearest primitive listed in holes[]           */
  ORC_SZ_AUTO = 4         /* automatic (Eq. 8): mu = min_s K |s - x| + lfs(s),
                             K = a0, s the ncent points of cent, lfs given    */
};
typedef struct {
  int32_t kind;
  double a0, a1, s2;
  int32_t ncent;
  const double *cent;     /* ncent (x, y) pairs                               */
  int32_t nholes;
  const int32_t *holes;   /* indices into the primitive list                   */
  const double *lfs;      /* AUTO: lfs of each of the ncent points             */
} orc_sizing;

/* ---- automatic sizing (Sec. 3.3, Eq. 8; App. A) -------------------------- */
/* Boundary points (App. A), in primitive order: a disk or an ellipse at
   m = max(3, floor(2 pi r / d_s) + 1) equal steps of its angle parameter
   (r the larger semi-axis), (r cos t, r sin t) about its centre (an
   ellipse's (a cos t, b sin t) turned by phi); a box as the clockwise loop
   (x0,y0) (x0,y1) (x1,y1) (x1,y0), a polygon or a segment loop through its
   vertices: every vertex, then floor(L / d_s) points splitting each segment
   of length L > d_s evenly.  A point is kept when the geometry's signed
   distance there is at most geps in magnitude (the parts of each boundary
   that bound the whole geometry).  Returns the count (the first cap points
   are written). */
int64_t orc_boundary_points(const orc_prim *prims, int32_t nprims, const double *poly, double d_s, double geps,
                            double *out, int64_t cap);
/* App. A trimming of boundary points, in place: sweeps over the points in
   index order until one changes nothing.  Point i (not removed, not done)
   takes its closest other remaining point p* whose midpoint m with it lies
   on the boundary (distance to the nearest segment of the SEGMENTS loops at
   most geps), the nearest first, ties to the lower index.  With none, or p*
   at least d_s away, point i is done; otherwise p* is removed and point i
   moves to m.  Returns the count of the remaining points, compacted in
   order. */
int64_t orc_trim_boundary(const orc_prim *prims, int32_t nprims, const double *poly, double d_s, double geps,
                          double *pts, int64_t n);
/* Medial-axis approximating points: for each point s, its Voronoi cell among
   all points (every other point's bisector, in index order, clipping the box
   [box0, box2] x [box1, box3]); v1 = the farthest cell vertex, added unless
   it lies on the box (it then stands for a vertex at infinity); v2 = the
   farthest cell vertex not on the box with (v2 - s) . (v1 - s) < 0, added if
   there is one.  Returns the count (first cap points written). */
int64_t orc_medial_points(const double *s, int64_t ns, const double box[4], double *out, int64_t cap);
/* keep[i] = at least n_thres other medial points within r_nei of point i. */
int64_t orc_trim_medial(const double *m, int64_t nm, double r_nei, int32_t n_thres, uint8_t *keep);
/* lfs(s) = distance to the nearest kept medial point (inf when none). */
void orc_lfs(const double *s, int64_t ns, const double *m, int64_t nm, const uint8_t *keep, double *lfs);
/* mu(x, y) = min over s of K |s - (x, y)| + lfs(s) (Eq. 8). */
double orc_auto_mu(const double *s, const double *lfs, int64_t ns, double K, double x, double y);

/* ---- the geometry grid (Sec. 3.2, Sec. 3.7) ------------------------------ */
enum { ORC_CAT_OUTER = 0, ORC_CAT_INNER = 1, ORC_CAT_BOUNDARY = 2 };

typedef struct {
  int32_t nx, ny;          /* nodes; cells are (nx-1) x (ny-1)                 */
  double x0, y0, dx, dy;   /* node (i, j) sits at (x0 + i*dx, y0 + j*dy)       */
  double inv_dx, inv_dy;   /* 1/dx, 1/dy (double division)                     */
  const double *sdf;       /* nx*ny, row-major (j*nx + i)                      */
  const double *mu;        /* nx*ny                                            */
  const uint8_t *cat;      /* (nx-1)*(ny-1) cell categories                    */
  const float *hcell;      /* (nx-1)*(ny-1) local desired edge length h_i      */
  double h_avg;            /* mean h over inner + selected boundary cells      */
} orc_grid;

/* Control parameters (Table 8 defaults; k and dt from the DistMesh method the
   paper builds on, which Table 8 leaves open). */
typedef struct {
  double fac_F;        /* 1.2   Eq. 3                                         */
  double fac_voro;     /* 5     span of the octagon, Sec. 4.1                 */
  double fac_pt;       /* 0.4   movement cap, Sec. 3.7                        */
  double fac_retria;   /* 0.1   re-triangulation threshold, Sec. 3.7          */
  double fac_end;      /* 0.001 Sec. 3.7 / Sec. 4.2                           */
  double fac_geps;     /* 0.01  Sec. 3.7                                      */
  double T_tria;       /* 0.4   Test 3, Sec. 4.1                              */
  double alpha_hat;    /* 1     damping, Eq. 14                               */
  int32_t T_newton;    /* 10    Newton step cap, Sec. 4.3                     */
  double k_spring;     /* 1     Eq. 2                                         */
  double dt;           /* 0.2   Eq. 5                                         */
  int32_t cvd_max_level;   /* 12  quadrature level cap                       */
  int32_t trace_max_steps; /* 64  sphere-tracing step cap                    */
  int32_t trace_bisect;    /* 8   sphere-tracing overshoot bisections         */
  int32_t test2_mode;      /* 0: count==1 goes to Test 3; 1: count<=1 invalid */
} orc_params;

typedef struct {
  int64_t candidates;    /* distance tests of neighbour candidates            */
  int64_t clip_tests;    /* vertex-vs-half-plane predicate evaluations        */
  int64_t cuts;          /* half-planes that removed at least one vertex      */
  int64_t exact_calls;   /* predicate evaluations that needed exact arithmetic */
  int64_t sos_calls;     /* exact zeros resolved by symbolic perturbation     */
  int64_t quad_points;   /* CVD quadrature points evaluated                   */
  int64_t level_cap_hits;
  int64_t newton_fail;
  int64_t trace_fail;
  int64_t empty_cells;
} orc_counters;

void orc_default_params(orc_params *p);

/* ---- setup (Sec. 3.1-3.3, Sec. 3.7) -------------------------------------- */
/* Fills sdf/mu nodes (rounded to float when dtype_bytes == 4), the cell
   categories, per-cell h and h_avg.  Returns 0 on success. */
int orc_grid_build(const orc_prim *prims, int32_t nprims, const double *poly,
                   const orc_sizing *sz, int32_t nx, int32_t ny, double x0, double y0,
                   double dx, double dy, int32_t dtype_bytes, int64_t n_total,
                   double *sdf, double *mu, uint8_t *cat, float *hcell,
                   double *h_avg, double *H);
/* Exact analytic SDF of the CSG geometry at one point (no grid). */
double orc_sdf_eval(const orc_prim *prims, int32_t nprims, const double *poly,
                    double x, double y);

/* ---- grid lookups --------------------------------------------------------- */
void orc_grid_init(orc_grid *g, int32_t nx, int32_t ny, double x0, double y0,
                   double dx, double dy, const double *sdf, const double *mu,
                   const uint8_t *cat, const float *hcell, double h_avg);
/* 1 if (x, y) lies in a grid cell; *cell = row-major cell index. */
int orc_locate(const orc_grid *g, double x, double y, int64_t *cell, double *tx, double *ty);
double orc_sdf_at(const orc_grid *g, double x, double y, int *on_grid);

/* ---- Procedure I: bounded Voronoi cells (Sec. 2.1, Sec. 4.1) ------------- */
/* Cell of point i as a CCW list of edge constraints: >= 0 a neighbour id,
   -1-w a wall (w = 0..7 octagon walls, 8..11 box walls).  Returns the number
   of edges (0 for an empty cell, -1 if more than cap). */
int orc_cell(const orc_grid *g, const orc_params *prm, int64_t n, const double *x,
             const double *y, int64_t i, int32_t *cons, double *vx, double *vy, int cap,
             orc_counters *cnt);
/* All cells, canonically rotated (smallest constraint first); rows of cap. */
int orc_cells_all(const orc_grid *g, const orc_params *prm, int64_t n, const double *x,
                  const double *y, int32_t *cons, int32_t *ncons, int cap, int nthreads,
                  orc_counters *cnt);
/* Same, by brute force over all points (no neighbour search, no stopping
   radius): the reference for the binned search. */
int orc_cells_all_pairs(const orc_grid *g, const orc_params *prm, int64_t n, const double *x,
                        const double *y, int32_t *cons, int32_t *ncons, int cap);

/* Delaunay extraction + Tests 1-3 (Proc. I, Sec. 4.1).  Writes the owned
   triangles (CCW, min id first) and their validity, then the symmetric
   adjacency of valid triangles (rows sorted by id).  tri_cap / adj_cap bound
   the outputs; returns 0, or -1 on capacity overflow (*ntri / *nadj then hold
   the required sizes). */
int orc_triangulate(const orc_grid *g, const orc_params *prm, int64_t n, const double *x,
                    const double *y, int32_t *tri, uint8_t *valid, int64_t tri_cap,
                    int64_t *ntri, int64_t *rowptr, int32_t *col, int64_t adj_cap,
                    int64_t *nadj, int nthreads, orc_counters *cnt);
/* Validity of one triangle (Tests 1-3) given its three vertex ids. */
int orc_triangle_valid(const orc_grid *g, const orc_params *prm, const double *x,
                       const double *y, int32_t a, int32_t b, int32_t c);

/* ---- DistMesh step (Sec. 2.2, Eq. 2-5, Alg. 1) --------------------------- */
/* fac_mu over the unique edges of the adjacency (Eq. 3). */
double orc_fac_mu(const orc_grid *g, int64_t n, const double *x, const double *y,
                  const int64_t *rowptr, const int32_t *col, double *sum_l2, double *sum_mu2);
/* One force update + treatment.  Writes new positions and categories and
   returns the number of points whose movement since the last triangulation
   exceeds fac_retria*h (the re-triangulation flag is this count > 0). */
int64_t orc_dm_step(const orc_grid *g, const orc_params *prm, int64_t n, const double *x,
                    const double *y, const uint8_t *cat, const int64_t *rowptr,
                    const int32_t *col, const double *xl, const double *yl, double *xn,
                    double *yn, uint8_t *catn, double *fac_mu_out, orc_counters *cnt);

/* ---- CVD step (Sec. 2.3, Eq. 6, Alg. 2, Sec. 4.2 II) --------------------- */
/* One Lloyd update with adaptive quadrature + treatment.  dprev is the
   previous movement of each point (input), dprevn receives the new one. */
int orc_cvd_step(const orc_grid *g, const orc_params *prm, int64_t n, const double *x,
                 const double *y, const uint8_t *cat, const double *dprev, double *xn,
                 double *yn, uint8_t *catn, double *dprevn, int32_t *levels, int nthreads,
                 orc_counters *cnt);
/* Centroid of one cell (relative to the generator) and the level used. */
int orc_cvd_centroid(const orc_grid *g, const orc_params *prm, int64_t n, const double *x,
                     const double *y, int64_t i, double dprev, double *cx, double *cy,
                     double *area, orc_counters *cnt);

/* ---- point treatment (Sec. 4.3, Eq. 12-14) ------------------------------- */
void orc_treat(const orc_grid *g, const orc_params *prm, double xo, double yo, uint8_t cat_old,
               double xnew, double ynew, double *xf, double *yf, uint8_t *catf,
               orc_counters *cnt);
uint8_t orc_point_category(const orc_grid *g, const orc_params *prm, double x, double y);
void orc_point_categories(const orc_grid *g, const orc_params *prm, int64_t n, const double *x,
                          const double *y, uint8_t *out);

/* ---- mesh quality (Sec. 3.6, Eq. 10-11) ---------------------------------- */
typedef struct {
  int64_t ntri;
  double min_q, mean_q, half_mean_alpha, half_mean_beta, max_alpha;
  double hist_beta[40];   /* beta in [1, 3), 40 bins, normalised             */
} orc_stats;
void orc_quality(const double *x, const double *y, const int32_t *tri, const uint8_t *valid,
                 int64_t ntri, orc_stats *st);
void orc_triangle_quality(double ax, double ay, double bx, double by, double cx, double cy,
                          double *alpha, double *beta);

/* ---- exact predicate exposed for the pins -------------------------------- */
/* Sign (+1 cut / -1 kept) of the margin of constraint c3 at the vertex of
   constraints c1, c2 of point i's cell (ids as in orc_cell). */
int orc_predicate(const orc_grid *g, const orc_params *prm, const double *x, const double *y,
                  int64_t i, int32_t c1, int32_t c2, int32_t c3, int *used_exact);
/* Exact sign of the 2-D incircle determinant of points a, b, c, d. */
int orc_incircle_sign(double ax, double ay, double bx, double by, double cx, double cy,
                      double dx, double dy);

#ifdef __cplusplus
}
#endif
#endif
