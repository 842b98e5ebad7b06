// Runs meshing iterations of the library, built for the CPU stand-in of the
// HIP runtime, on one case file, with every buffer of the state in an
// allocation of its own (so that AddressSanitizer reports any access beyond
// one), and checks the queue counters against their capacities after every
// kernel launch.  Test infrastructure.
//
//   run_case IN OUT
// IN: int64 n; int32 nx, ny; double x0, y0, dx, dy; int32 dtype_bytes,
//     precision; double bin_density; int32 iters, method (1 CVD, 0 DM,
//     2 and 3 the persistent batch, 4 one binning, the cells and one
//     extraction with their exports);
//     then sdf and mu (nx ny values of dtype), cat ((nx-1)(ny-1) bytes),
//     hcell ((nx-1)(ny-1) float), the scalars (4 doubles: H, h_avg,
//     area_sel, n_sel), x and y (n doubles each).
// OUT: per iteration x, y (n doubles each) and cat (n bytes) by id, then the
//     trime_stats struct and the largest queue counts seen (3 int64).
//     Method 4 writes instead: the cells (ncons, n int32; cons, n * 64
//     int32), the triangle count (int64), the triangles (3 * count int32) and
//     their validity (count bytes), max_deg (int32), the adjacency (deg, n
//     int32; col, n * max_deg int32), then the stats and queue counts.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "trime.h"

namespace trime {
size_t scan_tmp_ints(int64_t n);
int dm_partials(int64_t n);
}
namespace emu {
extern void (*after_launch)();
extern long parks, blocks_waited;
}

static trime_state S;
static std::vector<trime_state *> all_states;  // every state whose queues are checked
static int64_t max_q[3] = {0, 0, 0};
static int nchecks = 0;

static void *alloc(size_t bytes) {
  void *p = malloc(bytes ? bytes : 1);
  memset(p, 0xA5, bytes ? bytes : 1);  // no buffer starts out zeroed by chance
  return p;
}

// queue counters (counters[0], [4], [5]): FP64 replay, exact, deferred
// centroids; each queue holds n + 1 entries
static void check_queues() {
  for (trime_state *T : all_states) {
    const int32_t *c = T->counters;
    const int32_t q[3] = {c[0], c[4], c[5]};
    for (int k = 0; k < 3; k++) {
      if (q[k] < 0 || q[k] > T->n + 1) {
        fprintf(stderr, "queue %d holds %d entries, capacity %lld\n", k, q[k], (long long)T->n + 1);
        abort();
      }
      if (q[k] > max_q[k]) max_q[k] = q[k];
    }
  }
  nchecks++;
}

static void read_all(FILE *f, void *p, size_t bytes) {
  if (bytes && fread(p, 1, bytes, f) != bytes) {
    fprintf(stderr, "short input\n");
    exit(2);
  }
}

#define OK(x)                                                               \
  do {                                                                      \
    trime_status e_ = (x);                                                  \
    if (e_) {                                                               \
      fprintf(stderr, "%s failed: %d %s\n", #x, (int)e_, trime_last_error()); \
      exit(3);                                                              \
    }                                                                       \
  } while (0)

// A state on the case's grid with every buffer in an allocation of its own,
// of the size the layout gives it.
static void setup(trime_state &T, int64_t n, int32_t prec, double dens, int32_t nx, int32_t ny, double x0,
                  double y0, double dx, double dy, int32_t dtb, void *sdf, void *mu, uint8_t *cat, float *hcell,
                  trime_grid_scalars *scal) {
  memset(&T, 0, sizeof T);
  T.n = n;
  T.precision = prec;
  T.max_deg = 16;
  T.bin_density = dens;
  T.grid.nx = nx;
  T.grid.ny = ny;
  T.grid.x0 = x0;
  T.grid.y0 = y0;
  T.grid.dx = dx;
  T.grid.dy = dy;
  T.grid.dtype_bytes = dtb;
  T.sdf = sdf;
  T.mu = mu;
  T.cat_grid = cat;
  T.hcell = hcell;
  T.scal = scal;
  trime_default_params(&T.params);
  size_t ws = 0;
  OK(trime_state_workspace_bytes(&T, &ws));
  void *wsp = alloc(ws);
  OK(trime_state_bind(&T, wsp, ws, nullptr));
  // every buffer in an allocation of its own, of the size the layout gives it
  const int64_t nkeys = T.nkeys_cap > T.nkeys ? T.nkeys_cap : T.nkeys;
  const int64_t md = T.max_deg;
  for (int b = 0; b < 2; b++) {
    T.pos[b].x = (double *)alloc(8 * n);
    T.pos[b].y = (double *)alloc(8 * n);
    T.pos[b].dprev = (double *)alloc(8 * n);
    T.pos[b].cat = (uint8_t *)alloc(n);
    T.ord[b].id = (int32_t *)alloc(4 * n);
    T.ord[b].span = (float *)alloc(4 * n);
    T.ord[b].xl = (double *)alloc(8 * n);
    T.ord[b].yl = (double *)alloc(8 * n);
  }
  T.adj = (int32_t *)alloc(4 * md * n);
  T.deg = (int32_t *)alloc(4 * n);
  T.tri = (int32_t *)alloc(4 * 3 * TRIME_TRI_PER_POINT * n);
  T.tri_valid = (uint8_t *)alloc(TRIME_TRI_PER_POINT * n);
  T.tri_n = (int32_t *)alloc(4 * (n + 1));
  T.perm = (int32_t *)alloc(4 * (n + 1));
  T.key = (int32_t *)alloc(4 * n);
  T.rank = (int32_t *)alloc(4 * n);
  T.order = (int32_t *)alloc(4 * n);
  T.bin_start = (int32_t *)alloc(4 * (nkeys + 1));
  T.bin_fill = (int32_t *)alloc(4 * nkeys);
  T.scan_tmp = (int32_t *)alloc(4 * (trime::scan_tmp_ints(nkeys > n ? nkeys : n) + 1));
  T.queue = (int32_t *)alloc(4 * (3 * (n + 1) + 16 * n + 512));
  T.counters = (int32_t *)alloc(4 * 32);
  const int64_t np = trime::dm_partials(n);
  T.partials = (double *)alloc(8 * 2 * (np > 1 ? np : 1));
  T.stats = (trime_stats *)alloc(sizeof(trime_stats));
  for (int b = 0; b < 2; b++) {
    T.warm_n[b] = (int32_t *)alloc(4 * n);
    T.warm_nb[b] = (int32_t *)alloc(4 * TRIME_WARM * n);
  }
  T.old_slot = (int32_t *)alloc(4 * n);
  T.new_slot = (int32_t *)alloc(4 * n);
  memset(T.counters, 0, 4 * 32);

  all_states.push_back(&T);
}

// Method 2 (DistMesh) or 3 (CVD): a persistent batch of two shapes on the
// case's grid, the n points and the first n / 3 of them, against the same
// shapes run alone; after every two iterations each shape's positions,
// categories and statistics must be bit-identical.  OUT receives, per two
// iterations, the first shape's x, y (n doubles each) and cat by id.
static int run_persistent(bool cvd, int iters, const char *outp, int64_t n, double *x, double *y, int32_t prec,
                          double dens, int32_t nx, int32_t ny, double x0, double y0, double dx, double dy,
                          int32_t dtb, void *sdf, void *mu, uint8_t *cat, float *hcell, trime_grid_scalars *scal) {
  static trime_state B[2], R[2];
  const int64_t ns[2] = {n, n / 3};
  for (int k = 0; k < 2; k++) {
    setup(B[k], ns[k], prec, dens, nx, ny, x0, y0, dx, dy, dtb, sdf, mu, cat, hcell, scal);
    setup(R[k], ns[k], prec, dens, nx, ny, x0, y0, dx, dy, dtb, sdf, mu, cat, hcell, scal);
    OK(trime_state_load(&B[k], x, y, nullptr));
    OK(trime_state_load(&R[k], x, y, nullptr));
  }
  trime_state *bs[2] = {&B[0], &B[1]};
  trime_batch *b = nullptr;
  OK(trime_batch_create(bs, 2, cvd ? TRIME_METHOD_CVD : TRIME_METHOD_DM, &b));
  OK(trime_batch_make_persistent(b, 1, 2));
  FILE *out = fopen(outp, "wb");
  std::vector<double> ax(n), ay(n), rx(n), ry(n);
  std::vector<uint8_t> ac(n), rc(n);
  for (int it = 0; it + 2 <= iters; it += 2) {
    OK(trime_batch_run(b, 2, nullptr));
    for (int k = 0; k < 2; k++) {
      if (cvd)
        OK(trime_step_cvd(&R[k], 2, nullptr));
      else
        OK(trime_step_dm(&R[k], 2, 0, 0, nullptr));
      OK(trime_export_points(&B[k], ax.data(), ay.data(), ac.data(), nullptr));
      OK(trime_export_points(&R[k], rx.data(), ry.data(), rc.data(), nullptr));
      const size_t m = (size_t)ns[k];
      if (memcmp(ax.data(), rx.data(), 8 * m) || memcmp(ay.data(), ry.data(), 8 * m) ||
          memcmp(ac.data(), rc.data(), m)) {
        fprintf(stderr, "shape %d: positions after iteration %d differ from the shape run alone\n", k, it + 2);
        return 4;
      }
      trime_stats sa, sr;
      OK(trime_stats_read(&B[k], &sa, nullptr));
      OK(trime_stats_read(&R[k], &sr, nullptr));
      if (memcmp(&sa, &sr, sizeof sa)) {
        fprintf(stderr, "shape %d: statistics after iteration %d differ from the shape run alone\n", k, it + 2);
        return 5;
      }
      if (sa.error) {
        fprintf(stderr, "shape %d: error %d\n", k, sa.error);
        return 6;
      }
    }
    OK(trime_export_points(&B[0], ax.data(), ay.data(), ac.data(), nullptr));
    fwrite(ax.data(), 8, n, out);
    fwrite(ay.data(), 8, n, out);
    fwrite(ac.data(), 1, n, out);
    fprintf(stderr, "iterations %d-%d equal\n", it + 1, it + 2);
  }
  fclose(out);
  OK(trime_batch_destroy(b));
  fprintf(stderr, "ok: %d launches checked, persistent batch equal to the shapes alone; %ld parked threads (sleeps "
          "and fences), %ld turns to another block\n", nchecks, emu::parks, emu::blocks_waited);
  return 0;
}

int main(int argc, char **argv) {
  if (argc != 3) return 2;
  FILE *in = fopen(argv[1], "rb");
  if (!in) return 2;
  int64_t n;
  int32_t nx, ny, dtb, prec, iters, method;
  double x0, y0, dx, dy, dens;
  read_all(in, &n, 8);
  read_all(in, &nx, 4);
  read_all(in, &ny, 4);
  read_all(in, &x0, 8);
  read_all(in, &y0, 8);
  read_all(in, &dx, 8);
  read_all(in, &dy, 8);
  read_all(in, &dtb, 4);
  read_all(in, &prec, 4);
  read_all(in, &dens, 8);
  read_all(in, &iters, 4);
  read_all(in, &method, 4);
  const size_t nn = (size_t)nx * ny, nc = (size_t)(nx - 1) * (ny - 1);
  void *sdf = alloc(nn * dtb), *mu = alloc(nn * dtb);
  uint8_t *cat = (uint8_t *)alloc(nc);
  float *hcell = (float *)alloc(nc * 4);
  trime_grid_scalars *scal = (trime_grid_scalars *)alloc(sizeof(trime_grid_scalars));
  double sc[4];
  double *x = (double *)alloc(8 * n), *y = (double *)alloc(8 * n);
  read_all(in, sdf, nn * dtb);
  read_all(in, mu, nn * dtb);
  read_all(in, cat, nc);
  read_all(in, hcell, nc * 4);
  read_all(in, sc, sizeof sc);
  read_all(in, x, 8 * n);
  read_all(in, y, 8 * n);
  fclose(in);
  scal->H = sc[0];
  scal->h_avg = sc[1];
  scal->area_sel = sc[2];
  scal->n_sel = (int64_t)sc[3];

  setup(S, n, prec, dens, nx, ny, x0, y0, dx, dy, dtb, sdf, mu, cat, hcell, scal);
  emu::after_launch = check_queues;

  double *ex = (double *)alloc(8 * n), *ey = (double *)alloc(8 * n);
  uint8_t *ec = (uint8_t *)alloc(n);
  OK(trime_state_load(&S, x, y, nullptr));
  if (method == 2 || method == 3) return run_persistent(method == 3, iters, argv[2], n, x, y, prec, dens, nx, ny, x0, y0, dx, dy,
                                         dtb, sdf, mu, cat, hcell, scal);
  FILE *out = fopen(argv[2], "wb");
  if (method == 4) {
    const int32_t cap = 64;
    int32_t *cons = (int32_t *)alloc(4 * (size_t)n * cap), *ncons = (int32_t *)alloc(4 * n);
    const trime_cells cells = {cap, cons, ncons};
    OK(trime_bin_points(&S, nullptr));
    OK(trime_voronoi_cells(&S, &cells, nullptr));
    OK(trime_delaunay_extract(&S, nullptr));
    const int64_t tcap = (int64_t)n * TRIME_TRI_PER_POINT;
    int32_t *tri = (int32_t *)alloc(12 * tcap);
    uint8_t *valid = (uint8_t *)alloc(tcap);
    int64_t *count = (int64_t *)alloc(8);
    OK(trime_export_triangles(&S, tri, valid, tcap, count, nullptr));
    const int32_t md = S.max_deg;
    int32_t *deg = (int32_t *)alloc(4 * n), *col = (int32_t *)alloc(4 * (size_t)n * md);
    OK(trime_export_adjacency(&S, deg, col, nullptr));
    fwrite(ncons, 4, n, out);
    fwrite(cons, 4, (size_t)n * cap, out);
    fwrite(count, 8, 1, out);
    fwrite(tri, 4, 3 * (size_t)*count, out);
    fwrite(valid, 1, (size_t)*count, out);
    fwrite(&md, 4, 1, out);
    fwrite(deg, 4, n, out);
    fwrite(col, 4, (size_t)n * md, out);
    iters = 0;
  }
  for (int it = 0; it < iters; it++) {
    if (method == 1)
      OK(trime_step_cvd(&S, 1, nullptr));
    else
      OK(trime_step_dm(&S, 1, it == 0, 1, nullptr));
    OK(trime_export_points(&S, ex, ey, ec, nullptr));
    fwrite(ex, 8, n, out);
    fwrite(ey, 8, n, out);
    fwrite(ec, 1, n, out);
    fprintf(stderr, "iteration %d done (queues so far: %lld %lld %lld)\n", it + 1, (long long)max_q[0],
            (long long)max_q[1], (long long)max_q[2]);
  }
  trime_stats st;
  OK(trime_stats_read(&S, &st, nullptr));
  fwrite(&st, sizeof st, 1, out);
  fwrite(max_q, 8, 3, out);
  fclose(out);
  fprintf(stderr, "ok: %d launches checked, exact points %lld, replays %lld, error %d\n", nchecks,
          (long long)st.exact_points, (long long)st.fp64_replays, st.error);
  return 0;
}
