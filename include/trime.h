/*
 * trime.h -- C ABI of the MI355X (gfx950) library for the per-iteration hot
 * path of the TriMe++ iterative meshers (Lu & Rycroft, "TriMe++:
 * Multi-threaded triangular meshing in two dimensions", arXiv 2309.13824).
 *
 * One meshing iteration (Alg. 1 DistMesh, Alg. 2 CVD, Sec. 4.2 III hybrid):
 *   bin the points (Voro++ block grid, Sec. 6 example)  -> trime_bin_points
 *   bounded Voronoi cell of every point (Sec. 2.1, 4.1)  -> trime_voronoi_cells
 *   Delaunay triangles + validity tests (Proc. I, 4.1)   -> trime_delaunay_extract
 *   DistMesh force step / CVD centroid step + treatment -> trime_step_dm,
 *   (Eq. 2-5, Eq. 6, Sec. 4.2, Sec. 4.3)                    trime_step_cvd,
 *                                                          trime_step_hybrid
 * with the geometry grid built once by trime_sdf_grid_build (Sec. 3.1-3.3,
 * 3.7).
 *
 * Conventions
 *  - Every function returns a trime_status.  Argument errors are detected on
 *    the host before anything is launched.  Device-side conditions (capacity
 *    overflow, FP64 fallbacks, projection failures) are counted in the
 *    device trime_stats of the state; trime_stats_check() turns a host copy
 *    of it into a status.
 *  - Ownership: the caller allocates and frees all device memory.  A state
 *    lives in one caller-allocated device workspace sized by
 *    trime_state_workspace_bytes(); the library keeps no pointer after a
 *    call returns, allocates no device memory in any call except
 *    trime_sdf_grid_build (setup: one temporary buffer for the primitive
 *    list, the candidate lists of SEGMENTS primitives and of automatic
 *    sizing) and trime_auto_sizing (its scratch), and never synchronises
 *    except in trime_state_bind (setup: reads the grid scalars),
 *    trime_sdf_grid_build with SEGMENTS primitives or automatic sizing,
 *    trime_auto_sizing, trime_stats_read, trime_autotune (tuning),
 *    trime_add_points and trime_run_growing.
 *  - Streams: `stream` is a hipStream_t (passed as void*); 0 is the null
 *    stream.  All work is enqueued on it in order.
 *  - Layouts: structure of arrays.  Positions are float64 x[n], y[n] in both
 *    precision modes, indexed by point id (0..n-1).  Triangles are int32
 *    (a, b, c) counter-clockwise with the smallest id first.  Adjacency rows
 *    are sorted by id.  Grid arrays are row-major, node (i, j) at
 *    j*nx + i, cell (i, j) at j*(nx-1) + i.
 *  - Precision: TRIME_FP64 evaluates everything in FP64 ("plain FP64");
 *    TRIME_FP32 evaluates cells, quadrature and forces in FP32 and replays a
 *    point in FP64 whenever one of its decisions falls within the stated
 *    FP32 error bound.  In both modes cut decisions that FP64 cannot settle
 *    are taken exactly (expansion arithmetic) with symbolic tie-breaking, so
 *    the combinatorial output does not depend on precision, order or tuning.
 */
#ifndef TRIME_H
#define TRIME_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TRIME_OK = 0,
  TRIME_EINVAL = 1,       /* bad argument (null pointer, bad size, bad enum)   */
  TRIME_EUNSUPPORTED = 2, /* valid request this build does not implement       */
  TRIME_ECAPACITY = 3,    /* an output or workspace is too small               */
  TRIME_EHIP = 4,         /* HIP runtime error; see trime_last_error()         */
  TRIME_EDEGENERATE = 5   /* coincident points were found (results complete)   */
} trime_status;

enum { TRIME_FP64 = 0, TRIME_FP32 = 1 };
enum { TRIME_CAT_OUTER = 0, TRIME_CAT_INNER = 1, TRIME_CAT_BOUNDARY = 2 };

/* ---- geometry and sizing input (Sec. 3.1, 3.3, Eq. 9) -------------------- */
enum { TRIME_OP_INIT = 0, TRIME_OP_UNION = 1, TRIME_OP_DIFF = 2, TRIME_OP_INTERSECT = 3 };
enum { TRIME_PRIM_DISK = 0, TRIME_PRIM_BOX = 1, TRIME_PRIM_ELLIPSE = 2, TRIME_PRIM_POLYGON = 3,
       TRIME_PRIM_SEGMENTS = 4 };

/* One analytic primitive of the constructive geometry.  Parameters p:
   DISK (cx, cy, r); BOX (x0, y0, x1, y1); ELLIPSE (cx, cy, a, b, phi);
   POLYGON: vertices poly[voff .. voff+nv) of trime_geometry.poly (distance
   to the nearest edge, inside by crossing number).
   SEGMENTS: line-segment input (Sec. 3.2), a closed clockwise loop of the
   nv >= 3 segments poly[voff + k] -> poly[voff + (k + 1) mod nv].  The
   distance is to the nearest segment (equal distances: the lower index), at
   the closest point p* = a + t (b - a), t clamped to [0, 1].  The inward
   normal n is the segment's direction turned clockwise by 90 degrees (unit
   length), or at an end point the mean of the two segments' unit normals;
   the value is negative (inside) when (p - p*) . n > 0.  The grid build
   finds each node's nearest segment in per-cell candidate lists that it
   builds first (device memory it allocates and frees, and one stream
   synchronisation per level of the list hierarchy).  The running
   sdf s is combined with the primitive's t by op: INIT s = t, UNION min(s, t),
   DIFF max(s, -t), INTERSECT max(s, t) (Sec. 3.1 set operations). */
typedef struct {
  int32_t op, kind;
  double p[6];
  int32_t voff, nv;
} trime_prim;

typedef struct {
  int32_t nprims;
  const trime_prim *prims; /* host memory, nprims entries                     */
  int32_t npoly;
  const double *poly;      /* host memory, npoly (x, y) pairs                 */
} trime_geometry;

enum {
  TRIME_SZ_UNIFORM = 0,   /* mu = 1                                          */
  TRIME_SZ_ABS_SDF = 1,   /* mu = a0 + a1 |sdf|                              */
  TRIME_SZ_GAUSS_RHO = 2, /* rho = a0 + a1 sum_k exp(-|x - c_k|^2 / s2), mu = rho^-1/2 */
  TRIME_SZ_HOLE_RAMP = 3, /* mu = 1 + (a0 - 1) min(d_H / a1, 1), d_H = distance to
                             the nearest primitive listed in holes              */
  TRIME_SZ_AUTO = 4       /* automatic (Sec. 3.3, Eq. 8): mu(x) = min over the
                             boundary points s of K |x - s| + lfs(s), K = a0;
                             see trime_auto_sizing                             */
};
typedef struct {
  int32_t kind;
  double a0, a1, s2;
  int32_t ncent;
  const double *cent;   /* host, ncent (x, y) pairs                         */
  int32_t nholes;
  const int32_t *holes; /* host, indices into the primitive list            */
  int32_t n_thres;      /* AUTO: medial points need this many neighbours (0 -> 3) */
  double fac_nei;       /* AUTO: neighbour radius fac_nei n_thres d_s (0 -> 2)   */
  double fac_geps;      /* AUTO: on-boundary tolerance of the boundary-point
                           trimming, fac_geps min(dx, dy) (0 -> 0.01)         */
} trime_sizing;

/* Vertex-centred node grid: node (i, j) at (x0 + i dx, y0 + j dy).  Node
   values are float64 (dtype_bytes 8) or float32 (4). */
typedef struct {
  int32_t nx, ny;
  double x0, y0, dx, dy;
  int32_t dtype_bytes;
} trime_grid;

/* Scalars of the geometry grid (Sec. 3.7), written to device memory. */
typedef struct {
  double H;        /* h_cell = mu_cell * H                                  */
  double h_avg;    /* mean h over inner + selected boundary cells           */
  double area_sel; /* area of the selected cells                            */
  int64_t n_sel;   /* number of selected cells                              */
} trime_grid_scalars;

/* Control parameters: Table 8 defaults (k_spring and dt, left open there, are
   the DistMesh defaults 1 and 0.2). */
typedef struct {
  double fac_F, fac_voro, fac_pt, fac_retria, fac_end, fac_geps, T_tria, alpha_hat;
  int32_t T_newton;
  double k_spring, dt;
  int32_t cvd_max_level;   /* quadrature level cap (12)                    */
  int32_t trace_max_steps; /* sphere-tracing step cap (64)                  */
  int32_t trace_bisect;    /* sphere-tracing overshoot bisections (8)       */
  int32_t test2_mode;      /* 0: one midpoint inside -> Test 3; 1: invalid  */
} trime_params;

/* Control block of an adaptive run (trime_step_adaptive), kept on the
   device with the statistics.  Iterations are numbered from 0 within the
   run. */
enum { TRIME_STOP_NONE = 0, TRIME_STOP_QUALITY = 1, TRIME_STOP_MOVEMENT = 2 };
typedef struct {
  int32_t method;      /* method of the next iteration (TRIME_METHOD_*)      */
  int32_t stopped;     /* 1 once a termination test held                    */
  int32_t iters;       /* iterations run (the stopping one included)        */
  int32_t switch_iter; /* iteration whose statistics switched DistMesh to CVD, -1 */
  int32_t stop_iter;   /* iteration whose statistics ended the run, -1      */
  int32_t reason;      /* TRIME_STOP_*                                      */
  int32_t moving;      /* an inner point moved >= fac_end*h in the iteration */
  int32_t have_prev;   /* prev holds the statistics of the previous iteration */
  int32_t growing;     /* points are still to be added (trime_run_growing)  */
  int32_t add_request; /* the iteration just run asks for new points        */
  int32_t gate[8];     /* per-iteration kernel gates (internal)             */
  double prev[3];      /* M_1/2(alpha), M_1/2(beta), max alpha: previous    */
  double last[3];      /* the same, iteration just run                      */
  double rel[3];       /* their relative changes (-1 when not defined)      */
} trime_adapt_ctl;

/* Device-side counters and statistics of a state (read with trime_stats_read). */
typedef struct {
  int64_t fp64_replays;    /* points recomputed in FP64 after an uncertain FP32 decision */
  int64_t exact_points;    /* points whose cell needed the exact stage        */
  int64_t exact_calls;     /* exact predicate evaluations                     */
  int64_t sos_calls;       /* exact zeros resolved by symbolic perturbation   */
  int64_t overflow_points; /* cells beyond the polygon / row capacity         */
  int64_t newton_fail, trace_fail, level_cap_hits, empty_cells;
  int64_t ntri;            /* owned triangles of the last extraction          */
  int64_t nvalid;          /* of which valid                                  */
  int64_t moved;           /* points beyond fac_retria*h since last triangulation */
  int64_t triangulations;  /* extractions run by the step functions           */
  int64_t iterations;
  int32_t retri_flag;      /* re-triangulate before the next DistMesh step    */
  int32_t error;           /* nonzero: a capacity or internal error occurred  */
  double sum_l2, sum_mu2, fac_mu; /* Eq. 3 of the last DistMesh force step     */
  /* mesh quality of the nq valid triangles of the last extraction or quality
     pass (Eq. 10-11): sums of sqrt(alpha), sqrt(beta) and q = 1/alpha, with
     alpha = R_circ / (2 r_in) and beta = l_max / l_min of each triangle.  The
     device accumulates the sums exactly in quality_acc; trime_stats_read
     fills these four and the finished values below from it. */
  double sum_sqrt_alpha, sum_sqrt_beta, sum_q, max_alpha;
  int64_t nq;
  int64_t hist_beta[40];   /* beta in [1, 3), 40 bins, last bin open           */
  /* work of the cell passes that produced the committed results, since the
     last load: neighbours tested against the search range, vertex margins
     evaluated, polygon cuts, quadrature leaf triangles (Sec. 4.2 II) */
  int64_t work_candidates, work_margins, work_cuts, work_leaves;
  trime_adapt_ctl adapt;   /* the last adaptive run                           */
  /* Eq. 11 with p = 1/2 and the quality criteria of Sec. 6, finished from the
     exact sums (0 when nq = 0): M_1/2(alpha) = (sum_sqrt_alpha / nq)^2,
     M_1/2(beta) = (sum_sqrt_beta / nq)^2, mean q = sum_q / nq, min q =
     1 / max_alpha.  The adaptive runs take their decisions on the same values,
     computed the same way on the device. */
  double half_mean_alpha, half_mean_beta, mean_q, min_q;
  /* internal: 128-bit fixed-point sums (units of 2^-52; low word first) of
     sqrt(alpha), sqrt(beta) and q.  Each contribution (a block's or a
     replayed point's partial sum, in a fixed order) is truncated to the unit,
     and integer addition does not depend on the order in which the blocks
     finish, so identical inputs give bit-identical statistics. */
  uint64_t quality_acc[6];
} trime_stats;

/* Per-point arrays of a state are kept in "slot" order: the order of the
   last binning (points sorted by bin, then by their previous slot; the
   first binning after a load orders them by id).  Positional arrays are
   double-buffered per step, order arrays per binning. */
typedef struct {
  double *x, *y;  /* positions                                            */
  double *dprev;  /* previous movement (CVD error bound, Sec. 4.2)        */
  uint8_t *cat;   /* point category (Sec. 3.5)                            */
} trime_posbuf;

typedef struct {
  int32_t *id;    /* point id of each slot                                */
  float *span;    /* octagon span S of each point (Sec. 4.1)              */
  double *xl, *yl;/* positions at the last triangulation (Alg. 1)         */
} trime_ordbuf;

/* Triangles are kept per owner slot: up to TRIME_TRI_PER_POINT each (the
   owner, the smallest id, can own every triangle around it). */
#define TRIME_TRI_PER_POINT 16

/* A meshing state: configuration set by the caller, device buffers laid out
   by trime_state_bind in one caller-allocated workspace. */
typedef struct {
  /* -- configuration (caller) -- */
  int64_t n;               /* number of points, 1 .. 2^30                    */
  int32_t precision;       /* TRIME_FP64 or TRIME_FP32                       */
  int32_t max_deg;         /* adjacency row capacity (0 -> 16)               */
  double bin_density;      /* mean points per bin (0 -> 3.3, Sec. 6 example) */
  trime_grid grid;
  const void *sdf;         /* device node grids from trime_sdf_grid_build    */
  const void *mu;
  const uint8_t *cat_grid; /* device, (nx-1)(ny-1)                           */
  const float *hcell;      /* device, (nx-1)(ny-1)                           */
  const trime_grid_scalars *scal; /* device                                   */
  trime_params params;
  /* -- laid out by trime_state_bind (device pointers into the workspace) -- */
  trime_posbuf pos[2];
  trime_ordbuf ord[2];
  int32_t cur_pos, cur_ord; /* current buffers                              */
  int32_t *adj;            /* max_deg * n, column-major rows of slots        */
  int32_t *deg;            /* n                                              */
  int32_t *tri;            /* 3 * TRIME_TRI_PER_POINT * n, owner slot major  */
  uint8_t *tri_valid;      /* TRIME_TRI_PER_POINT * n                        */
  int32_t *tri_n;          /* n: owned triangles per slot                    */
  int32_t *perm;           /* n + 1: binning scratch (the points of each bin,
                              then the scan of the processing-order flags)  */
  int32_t *key;            /* n: bin key of each point (binning scratch)     */
  int32_t *rank;           /* n: binning scratch (rank in the bin, then the
                              processing-order flag of each slot)           */
  int32_t *order;          /* n: slots in the order the cell kernels take them
                              (points on the boundary first, they cost most) */
  int32_t *bin_start;      /* nkeys + 1                                      */
  int32_t *bin_fill;       /* nkeys                                          */
  int32_t *scan_tmp;       /* scan block sums                                */
  int32_t *queue;          /* 3(n+1) + 16n: points replayed in FP64, exactly,
                              and FP32 cells whose centroid is redone in FP64 */
  int32_t *counters;       /* small device counters                          */
  double *partials;        /* per-block partial sums                         */
  trime_stats *stats;      /* device                                         */
  /* bin grid (Morton-ordered square bins over the node grid's box) */
  int32_t nbx, nby, lbits;
  double bx0, by0, bw;
  double area_sel;         /* host copy of scal->area_sel                    */
  int64_t nkeys;
  /* optional hipEvent_t pair (caller-owned, may be null): recorded just
     before and after the fused cell kernel of each extraction / CVD step */
  void *ev_cells[2];
  /* -- point addition (Sec. 3.6) -- */
  int64_t n_cap;           /* caller: capacity for added points (0 -> n); the
                              workspace is laid out for n_cap points       */
  double h_scale;          /* set by trime_state_bind and trime_add_points:
                              every h of the grid is read times
                              sqrt(n_grid / n) (Sec. 3.7: the desired edge
                              length of N points over the same region goes
                              as 1/sqrt(N))                                  */
  int64_t nkeys_cap;       /* bin keys the workspace holds (set by bind)    */
  int64_t n_grid;          /* caller: the point count the grid was built for
                              (n_total of trime_sdf_grid_build; 0 -> n, set
                              by bind)                                      */
  /* the neighbours of each point's last cell, which the point's next cell
     clips first: in the buffer set of the slot order they were written in,
     by slot, as slots of that order (laid out by bind, cleared by load) */
  int32_t *warm_n[2];      /* n_cap each: count (0: none)                   */
  int32_t *warm_nb[2];     /* TRIME_WARM * n_cap each: neighbour slots      */
  int32_t *old_slot;       /* n_cap: each slot's slot before the last binning */
  int32_t *new_slot;       /* n_cap: the slot each previous slot went to    */
  /* -- placement (tuning only: results do not depend on it) -- */
  int32_t xcd_run;         /* caller, 0..256: blocks of the fused cell kernel
                              that one XCD (one L2) takes in a row, the runs
                              going round the 8 XCDs (0: 8; 1: the
                              hardware's own round robin); trime_autotune
                              picks it                                      */
} trime_state;

/* neighbours kept per point for the next cell */
#define TRIME_WARM 12

/* A fixed hybrid schedule: segments (method, iterations) run in order. */
enum { TRIME_METHOD_DM = 0, TRIME_METHOD_CVD = 1,
       TRIME_METHOD_DM_ALWAYS = 2 /* trime_batch_create only: DistMesh re-triangulating every iteration */ };
typedef struct {
  int32_t nseg;
  const int32_t *method;   /* host, nseg                                     */
  const int32_t *iters;    /* host, nseg                                     */
} trime_schedule;

/* Cells written by trime_voronoi_cells: for each point id the CCW list of
   edge constraints (>= 0 neighbour id; -1-w wall w, w = 0..7 octagon walls
   at outward normals 0, 45, .., 315 degrees, 8..11 box walls x <= x1,
   y <= y1, x >= x0, y >= y0), rotated to start at its smallest entry. */
typedef struct {
  int32_t cap;      /* entries per point                                     */
  int32_t *cons;    /* device, n * cap                                       */
  int32_t *ncons;   /* device, n (-1: more than cap)                         */
} trime_cells;

/* ------------------------------------------------------------------------ */
const char *trime_last_error(void);
const char *trime_version(void);
void trime_default_params(trime_params *p);

/* Geometry grid (Sec. 3.1-3.3, Sec. 3.7).  Fills sdf and mu at the nodes
   (dtype of grid), the cell categories (boundary when |sdf(mid)| <= cell
   diagonal, else inner when sdf(mid) < 0, else outer; mid value = mean of the
   4 corner nodes), h_cell = mu_cell * H with mu_cell the mean of the corner
   mu nodes and H = sqrt(dx dy sum_sel mu_cell^-2 / n_total) over the
   selected cells (inner, and boundary with sdf(mid) <= 0.5 min(dx, dy)), and
   the scalars.  All outputs are device pointers sized by the grid. */
trime_status trime_sdf_grid_build(const trime_geometry *g, const trime_sizing *sz,
                                  const trime_grid *grid, int64_t n_total, void *d_sdf,
                                  void *d_mu, uint8_t *d_cat, float *d_hcell,
                                  trime_grid_scalars *d_scal, void *stream);

/* trime_sdf_grid_build for callers that cannot allocate device memory (code
   under HIP graph capture, tight serving loops, harnesses that forbid
   hipMalloc): the same grids, bit for bit, with the primitive list, polygon
   vertices, density centres, hole indices and the partial sums of H in a
   static device array of 6 MiB that each GPU holds until the process ends,
   instead of a temporary allocation.  It calls no allocating routine (the
   host arrays are copied with hipMemcpyAsync).  Every call on a GPU shares
   that array, so calls that overlap on one GPU race; serialise them (one
   stream, or an event between them).  Errors: as trime_sdf_grid_build;
   TRIME_EUNSUPPORTED for SEGMENTS primitives and automatic sizing (their
   candidate lists need allocations); TRIME_ECAPACITY when the primitive
   list, vertices, centres, holes and one pair of doubles per 256 grid cells
   need more than the 6 MiB (a grid of 8192^2 nodes takes 4 MiB). */
trime_status trime_sdf_grid_build_noalloc(const trime_geometry *g, const trime_sizing *sz,
                                          const trime_grid *grid, int64_t n_total, void *d_sdf,
                                          void *d_mu, uint8_t *d_cat, float *d_hcell,
                                          trime_grid_scalars *d_scal, void *stream);

/* Size of the device workspace of a configured state (bytes, 256-aligned).
   TRIME_EINVAL for n outside 1 .. 2^30, a bad precision or grid, or missing
   grid arrays; reads the grid scalars from the device. */
trime_status trime_state_workspace_bytes(const trime_state *st, size_t *bytes);
/* Lays the state's buffers out in d_ws (>= workspace bytes).  Synchronous:
   reads the grid scalars from the device. */
trime_status trime_state_bind(trime_state *st, void *d_ws, size_t bytes, void *stream);
/* Copies positions (device, by id) into the state (slot = id until the first
   binning), sets categories (Sec. 3.5), d_prev = -1 (the first CVD
   iteration uses h) and clears the stats.  Positions belong inside the
   grid's box: a point outside it has no cell, is kept where it is by every
   step, and sets trime_stats.error. */
trime_status trime_state_load(trime_state *st, const double *d_x, const double *d_y, void *stream);
/* Current positions and categories, scattered back to id order (device). */
trime_status trime_export_points(const trime_state *st, double *d_x, double *d_y, uint8_t *d_cat,
                                 void *stream);
/* Owned triangles of the last extraction as ids (CCW, smallest id first),
   with validity; rows in owner-slot order.  d_tri: 3*cap int32, d_valid: cap
   bytes; *d_count receives the number (device int64). */
trime_status trime_export_triangles(const trime_state *st, int32_t *d_tri, uint8_t *d_valid,
                                    int64_t cap, int64_t *d_count, void *stream);
/* Adjacency of the valid triangles by id: rows of max_deg entries (id-major,
   d_col[i*max_deg + t]) sorted by id, d_deg[i] entries each. */
trime_status trime_export_adjacency(const trime_state *st, int32_t *d_deg, int32_t *d_col,
                                    void *stream);

/* Sorts the points into Morton-ordered bins of the bin grid (the Voro++
   container blocks of the paper's example code): new slot order by
   (bin key, previous slot); the first binning after a load orders each bin
   by id.  Permutes every per-point array into it, sets the positions
   of the last triangulation to the current ones and the span S of every
   point (Sec. 4.1: S = fac_voro * h of the point's cell). */
trime_status trime_bin_points(trime_state *st, void *stream);

/* Bounded Voronoi cell of every point (Sec. 2.1, Sec. 4.1): the octagon
   |u_x|, |u_y| <= S, |u_x| + |u_y| <= fl32(fl32(sqrt 2) S) around the point,
   clipped by the node grid's box and by the bisector of every neighbour.
   Needs trime_bin_points first.  Writes `out` (must be non-null). */
trime_status trime_voronoi_cells(trime_state *st, const trime_cells *out, void *stream);

/* Delaunay triangles of the cells (Proc. I): the circumcentre of a cell
   vertex between the bisectors of neighbours j, k yields triangle (i, j, k)
   when it is a vertex of all three cells; the smallest id owns it.  Runs
   Tests 1-3 on every triangle and keeps the owned triangles with their
   validity and the adjacency of the valid triangles (slot form; see the
   export functions), and their quality statistics.  Needs trime_bin_points
   first. */
trime_status trime_delaunay_extract(trime_state *st, void *stream);

/* n_iter DistMesh iterations (Alg. 1): re-triangulate (bin + extract) when
   the flag is set (always on the first iteration of the call when
   `fresh` != 0), Eq. 3 scaling, spring forces (Eq. 2), forward Euler (Eq. 5)
   and treatment (Sec. 4.3); the flag is set when a point moved more than
   fac_retria*h since the last triangulation.  always_retriangulate != 0
   triangulates every iteration.  The flag is read on the device (binning
   and extraction are launched every iteration and do their work only when
   it is raised), so the call makes no host reads and can be captured in a
   HIP graph. */
trime_status trime_step_dm(trime_state *st, int32_t n_iter, int32_t fresh,
                           int32_t always_retriangulate, void *stream);
/* n_iter CVD iterations (Alg. 2): bin, cells, adaptive-quadrature centroid
   with rho = mu^-2 (Sec. 4.2 II), treatment; triangles and quality stats of
   every iteration's cells. */
trime_status trime_step_cvd(trime_state *st, int32_t n_iter, void *stream);
/* A fixed schedule of DistMesh and CVD segments (Sec. 2.4, 4.2 III). */
trime_status trime_step_hybrid(trime_state *st, const trime_schedule *sch, void *stream);

/* ---- adaptive runs ---------------------------------------------------------
   Termination on mesh quality or small movement (Sec. 6, thresholds in
   Table 8) and the quality-driven switch of hybrid meshing from DistMesh to
   CVD (Sec. 4.2, hybrid meshing).  Each iteration measures the mesh it works
   on: the valid triangles of its triangulation (DistMesh keeps the last one
   until a point has moved more than fac_retria*h, Alg. 1) at the positions
   the iteration starts from: M_1/2(alpha), M_1/2(beta) (Eq. 10-11) and max
   alpha.  After the update, with r the relative change of each against the
   previous iteration:
   - mode TRIME_ADAPT_HYBRID, DistMesh phase: the next iterations are CVD
     when r(M_1/2 alpha) < t_switch;
   - otherwise the run stops when r(M_1/2 alpha) < t_quality, r(M_1/2 beta)
     < t_quality and r(max alpha) < t_amax (TRIME_STOP_QUALITY), else when
     no inner point (category at the start of the iteration) moved by
     fac_end*h or more, h of the cell it started in (TRIME_STOP_MOVEMENT).
   The first iteration has no previous statistics: only the movement test can
   end it.  DistMesh iterations run in flag mode and triangulate on the first
   iteration of the run.
   All decisions are taken on the device: the call enqueues max_iter
   iterations whose kernels check the control block (in stats->adapt) and do
   nothing once the run has stopped, apart from carrying the positions over,
   so it makes no host reads and can be captured in a HIP graph.  Read the
   outcome with trime_stats_read.  Errors: TRIME_EINVAL for a null or unbound
   state, a null cfg, an unknown mode, max_iter < 0 or a negative or NaN
   threshold. */
enum { TRIME_ADAPT_DM = 0, TRIME_ADAPT_CVD = 1, TRIME_ADAPT_HYBRID = 2 };
typedef struct {
  int32_t mode;        /* TRIME_ADAPT_*                                      */
  int32_t max_iter;    /* iterations enqueued                                */
  double t_quality;    /* T_end_quality (Table 8: 0.001)                     */
  double t_amax;       /* T_end_alpha_max (Table 8: 0.005)                   */
  double t_switch;     /* T_switch_quality (Table 8: 0.0015)                 */
} trime_adaptive;
trime_status trime_step_adaptive(trime_state *st, const trime_adaptive *cfg, void *stream);

/* ---- point addition (Sec. 3.6) ---------------------------------------------
   trime_add_points appends n_add points to a state: the centroids of the
   n_add valid triangles of the stored triangulation (as the last extraction,
   DistMesh triangulation or CVD step left it) with the largest ratio of
   circumradius to the local desired edge length h, at the current positions:
   h of the grid cell holding the centroid (clamped to the grid), with the
   state's h_scale.  Ties in the ratio go to the smaller (owner id, second id)
   of the triangle (owner: its smallest id, first in CCW order), so the
   selection is unique.  The circumradius is
   sqrt(|ab|^2 |bc|^2 |ca|^2) / (2 |(b - a) x (c - a)|), the centroid
   ((x_a + x_b) + x_c) / 3, in FP64.  The new points take the ids n, n + 1,
   ... in the order of (owner id, second id) of their triangles, d_prev = -1,
   and the category (Sec. 3.5) and octagon span of their position under the
   new h_scale = sqrt(n_grid / (n + n_add)) (Sec. 3.7), which the state
   takes.  Afterwards the adjacency is stale and the next DistMesh iteration
   of an adaptive run re-triangulates (stats->retri_flag = 1, have_prev = 0).
   The call synchronises the stream.  Errors: TRIME_EINVAL for n_add < 0,
   n + n_add > n_cap or more points than valid triangles; TRIME_ECAPACITY
   when the valid triangles outnumber the key buffer (max_deg n_cap / 4
   keys, 4 n_cap for max_deg 16). */
trime_status trime_add_points(trime_state *st, int64_t n_add, void *stream);

/* An adaptive run with point addition (Sec. 3.6): the state starts with its
   current n points (fac_init N_total of them in the paper; the grid is built
   for N_total = n_grid points, so h is read times sqrt(n_grid / n)) and
   grows to n_total <= n_cap.  While n < n_total an iteration whose relative
   changes of M_1/2(alpha) and M_1/2(beta) are both below t_add adds
   min(floor(fac_add n), n_total - n) points with trime_add_points, h_scale
   becoming sqrt(n_grid / n) for the new n; the switch and the termination
   tests of trime_step_adaptive apply once all points are in.  The run reads
   the control block after every iteration (synchronising; not for graph
   capture) and returns once the run has stopped or after max_iter
   iterations; read the outcome with trime_stats_read.  Errors: as
   trime_step_adaptive and trime_add_points, and TRIME_EINVAL for n_total
   outside [n, n_cap], a negative t_add or fac_add <= 0. */
typedef struct {
  trime_adaptive base;  /* mode, max_iter and the Table 8 thresholds      */
  int64_t n_total;      /* N_total                                        */
  double t_add;         /* T_add_quality (Table 8: 0.002)                 */
  double fac_add;       /* fac_add (Table 8: 0.6)                         */
} trime_growing;
trime_status trime_run_growing(trime_state *st, const trime_growing *cfg, void *stream);

/* ---- automatic sizing (Sec. 3.3, Eq. 8; App. A) ----------------------------
   The steps of TRIME_SZ_AUTO, which trime_sdf_grid_build runs before its
   node pass (mu at the nodes, h from it as for every sizing):
   - boundary points S (App. A), in primitive order, d_s = a1 min(dx, dy)
     (fac_s in App. A): a disk or an ellipse at m = max(3, floor(2 pi r /
     d_s) + 1) equal steps of its angle parameter (r its larger semi-axis);
     a box as the clockwise loop (x0,y0) (x0,y1) (x1,y1) (x1,y0), a polygon
     or a segment loop through its vertices: each vertex, then on a segment
     of length L > d_s the floor(L / d_s) points that split it evenly; of
     these, the points where the geometry's signed distance is within
     geps = fac_geps min(dx, dy) (the parts that bound the whole shape);
   - their trimming (App. A): sweeps over S in index order until one changes
     nothing; a point (not removed, not done) takes its closest remaining
     point p* whose midpoint m with it lies on the boundary (the geometry's
     signed distance within geps; the nearest first, ties to the lower
     index); with none, or p* at least d_s away, the point is done,
     otherwise p* is removed and the point moves to m (serial, on the host);
   - medial-axis approximating points: the Voronoi cell of each s among S,
     clipped to the grid's box grown by its width and height on every side;
     v1 = its farthest vertex, kept unless a box edge meets it (then it
     stands for a vertex at infinity), v2 = its farthest vertex without a box
     edge in the open half plane (v - s) . (v1 - s) < 0, if any; in the order
     of S, v1 before v2 (a cell that reaches 254 vertices while it is
     clipped gives none);
   - trimming: a medial point is kept when at least n_thres other medial
     points lie within r_nei = fac_nei n_thres d_s;
   - lfs(s) = the distance to the nearest kept medial point;
   - mu(x) = min over s of K |x - s| + lfs(s), K = a0, at the grid nodes.
   trime_auto_sizing runs the first four on the device and returns S
   (d_pts, s_cap points), the medial points (d_medial, m_cap points) with
   their keep flags, and lfs (d_lfs, s_cap entries); *ns_out and *nm_out
   receive the counts.  Synchronises the stream; allocates and frees device
   scratch.  Errors: TRIME_EINVAL for a bad primitive, a sizing kind other
   than AUTO, a1 <= 0, a0 < 0 or no kept medial point; TRIME_ECAPACITY when s_cap < |S| or
   m_cap < 2 |S| (the counts known so far are written). */
trime_status trime_auto_sizing(const trime_geometry *geo, const trime_sizing *sz, const trime_grid *grid,
                               double *d_pts, int64_t s_cap, int64_t *ns_out, double *d_medial, uint8_t *d_keep,
                               int64_t m_cap, int64_t *nm_out, double *d_lfs, void *stream);

/* Mesh quality of the state's valid triangles (Eq. 10-11) into stats. */
trime_status trime_quality(trime_state *st, void *stream);

/* Copies the device stats to host memory (synchronises the stream) and
   finishes the quality fields there: the sums from quality_acc, then
   M_1/2(alpha), M_1/2(beta), mean q and min q (Eq. 10-11). */
trime_status trime_stats_read(const trime_state *st, trime_stats *host, void *stream);
trime_status trime_stats_check(const trime_stats *host);

/* ---- batches of shapes in one graph ----------------------------------------
   Many shapes of uneven size are meshed by one HIP graph launch: the graph
   holds n_iter iterations (method TRIME_METHOD_DM: Alg. 1 DistMesh in flag
   mode; TRIME_METHOD_CVD: Alg. 2) of
   every state, the states spread round-robin over nstreams concurrent
   branches, so small shapes fill the GPU together.  n_iter must be even (the
   double-buffered arrays then return to the same buffers and the graph can
   be launched again for the next n_iter iterations).  Creation captures on
   `stream`, which must not be the null stream; it creates nstreams-1 side
   streams (default priority) and nstreams events and instantiates the
   graph: setup, not the hot path.  The states must be bound and loaded, and
   must not request timing events.  trime_graph_destroy frees everything
   the graph owns; the states stay the caller's. */
typedef struct trime_graph trime_graph;
trime_status trime_batch_graph_create(trime_state *const *states, int32_t nstates, int32_t method,
                                      int32_t n_iter, int32_t nstreams, trime_graph **out, void *stream);
trime_status trime_graph_launch(trime_graph *g, void *stream);
trime_status trime_graph_destroy(trime_graph *g);

/* ---- batches of shapes, one launch per kernel --------------------------------
   The batched launch of many shapes: trime_batch_create records one period
   of the chosen method (two iterations, after which every buffer swap is
   back where it started) for every state without launching anything, and
   merges the records kernel by kernel.  trime_batch_run then issues each
   kernel of an iteration once for all shapes: each block finds its shape in
   a table of per-shape arguments (binary search over the per-shape block
   offsets) and runs the same code on that shape's buffers.  Each shape's
   results equal running it alone with trime_step_dm (flag mode, fresh = 0;
   method TRIME_METHOD_DM_ALWAYS: always_retriangulate = 1) or
   trime_step_cvd; its statistics stay in its own state.
   - states: bound and loaded, no timing events, all with the same precision
     and grid dtype (they must record the same sequence of kernels); they
     must stay bound to the same workspaces while the batch exists, and
     their buffer parity must be the one they had at creation when the batch
     runs (runs of an even number of iterations keep it).
   - Ownership: the library allocates the argument tables in device memory
     at creation (synchronising) and frees them in trime_batch_destroy.
   - trime_batch_run enqueues n_iter (even) iterations on the stream; it
     makes no host reads and can be captured in a HIP graph.
   Errors: TRIME_EINVAL for bad arguments or states whose kernel sequences
   differ; TRIME_EHIP for a failed allocation or copy. */
typedef struct trime_batch trime_batch;
trime_status trime_batch_create(trime_state *const *states, int32_t nstates, int32_t method, trime_batch **out);
trime_status trime_batch_run(trime_batch *b, int32_t n_iter, void *stream);
trime_status trime_batch_destroy(trime_batch *b);

/* ---- persistent batches -------------------------------------------------------
   Switched off by default: unless the library is built with
   TRIME_PERSIST_ENABLE, trime_batch_make_persistent returns TRIME_EINVAL and
   leaves the batch as it was (on MI355X a launch of the persistent kernel
   has not completed; the CPU emulation of the library builds it in and
   checks it against the shapes run alone).
   trime_batch_make_persistent switches a batch to one launch per
   trime_batch_run for all its iterations: a persistent kernel (blocks of one
   wavefront, as many as the device holds at once) takes work items from a
   queue, in the role of the paper's dynamically scheduled threads (Sec. 5)
   spread over the shapes.  An item is one kernel of the recorded period for
   one shape and a chunk of that kernel's blocks, each run by the wavefront
   in a form that computes what the block computes (the same sums in the
   same order); items are handed out period by period, kernel by kernel,
   larger shapes first, and an item starts when its shape has finished every
   item before it, so shapes move through their kernels independently
   instead of all shapes waiting at every kernel boundary.  Each shape's
   results (positions, categories, triangles, statistics) are bit-identical
   to the one-launch-per-kernel batch's.
   - tiles_cells: blocks of the fast cell kernel (128 points each) per item;
     tiles_other: blocks per item of the other bulk kernels (the replay
     queues take one block per item).  Both in [1, 4096].
   - Ownership: allocates its tables, per-shape counters and the exact
     stage's polygons (48 KiB per block of the kernel) in device memory at
     this call (synchronising); trime_batch_destroy frees them.
   - A persistent trime_batch_run enqueues a counter-clearing fill kernel and
     the one launch: no host reads, capturable in a HIP graph.  Runs of one
     batch on streams that overlap race.
   - A run still waiting 20 s after its launch started (a fault of the
     schedule, never expected) stops: the remaining items are skipped and
     the value 32 is ORed into the error field of the stats of a shape that
     waited.
   Errors: TRIME_EINVAL for a null or already persistent batch, tiles out of
   range, a batch whose kernels have no persistent form, or more work items
   than one launch counts (trime_batch_run: run fewer iterations per call);
   TRIME_EHIP for a failed query, allocation or copy. */
trime_status trime_batch_make_persistent(trime_batch *b, int32_t tiles_cells, int32_t tiles_other);


/* ---- autotuner (tuning only) ------------------------------------------------
   Two settings change the speed and not the results.  The bin size sets how
   many neighbours a cell scans and how far, and the slot order; the XCD run
   (trime_state.xcd_run) sets which L2 serves which block of the fused cell
   kernel.  The combinatorial results depend on neither: every cut decision
   is exact, so cells, triangles, validity and adjacency are the same for
   every bin size.  Floating-point results depend on the bin size only
   through rounding: a cell's vertex list starts at a vertex that follows the
   order in which the neighbours were clipped, which sets the order of the
   centroid and quality sums, so positions after a CVD step and the quality
   sums agree across bin sizes to rounding (within the precision mode's
   tolerance), not bit for bit; the XCD run moves whole blocks between L2s
   and changes nothing (bit-identical).  trime_autotune times n_iter CVD
   iterations (Alg. 2) from the positions (d_x, d_y) for every candidate
   pair (density, XCD run): densities[nd] in points per bin, xcd_runs[nr]
   (null or nr = 0: the state's own xcd_run only).  It leaves the state
   bound to d_ws with the fastest pair and loaded with (d_x, d_y), and
   returns the pair in best_density and best_run (best_run may be null).
   d_ws must hold trime_autotune_workspace_bytes() bytes (the largest layout
   of the densities).  Synchronises the stream once per candidate; creates
   and destroys two HIP events; allocates no device memory.  ms_out (host,
   nd * max(nr, 1) entries, density-major, may be null) receives each
   candidate's time per iteration. */
trime_status trime_autotune_workspace_bytes(const trime_state *st, const double *densities, int32_t nd,
                                            size_t *bytes);
trime_status trime_autotune(trime_state *st, void *d_ws, size_t bytes, const double *d_x, const double *d_y,
                            const double *densities, int32_t nd, const int32_t *xcd_runs, int32_t nr,
                            int32_t n_iter, double *best_density, int32_t *best_run, float *ms_out, void *stream);

#ifdef __cplusplus
}
#endif
#endif
