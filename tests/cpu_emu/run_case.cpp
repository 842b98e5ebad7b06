// Runs meshing iterations of the library, built for the CPU stand-in of the
// HIP runtime, on one case file, with every buffer of the state in an
// allocation of its own (so that AddressSanitizer reports any access beyond
// one), and checks the queue counters against their capacities after every
// kernel launch.  Test infrastructure.
//
//   run_case IN OUT
// IN: int64 n; int32 nx, ny; double x0, y0, dx, dy; int32 dtype_bytes,
//     precision; double bin_density; int32 iters, method (1 CVD, 0 DM);
//     then sdf and mu (nx ny values of dtype), cat ((nx-1)(ny-1) bytes),
//     hcell ((nx-1)(ny-1) float), the scalars (4 doubles: H, h_avg,
//     area_sel, n_sel), x and y (n doubles each).
// OUT: per iteration x, y (n doubles each) and cat (n bytes) by id, then the
//     trime_stats struct and the largest queue counts seen (3 int64).
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
}

static trime_state S;
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
  const int32_t *c = S.counters;
  const int32_t q[3] = {c[0], c[4], c[5]};
  for (int k = 0; k < 3; k++) {
    if (q[k] < 0 || q[k] > S.n + 1) {
      fprintf(stderr, "queue %d holds %d entries, capacity %lld\n", k, q[k], (long long)S.n + 1);
      abort();
    }
    if (q[k] > max_q[k]) max_q[k] = q[k];
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

  memset(&S, 0, sizeof S);
  S.n = n;
  S.precision = prec;
  S.max_deg = 16;
  S.bin_density = dens;
  S.grid.nx = nx;
  S.grid.ny = ny;
  S.grid.x0 = x0;
  S.grid.y0 = y0;
  S.grid.dx = dx;
  S.grid.dy = dy;
  S.grid.dtype_bytes = dtb;
  S.sdf = sdf;
  S.mu = mu;
  S.cat_grid = cat;
  S.hcell = hcell;
  S.scal = scal;
  trime_default_params(&S.params);
  size_t ws = 0;
  OK(trime_state_workspace_bytes(&S, &ws));
  void *wsp = alloc(ws);
  OK(trime_state_bind(&S, wsp, ws, nullptr));
  // every buffer in an allocation of its own, of the size the layout gives it
  const int64_t nkeys = S.nkeys_cap > S.nkeys ? S.nkeys_cap : S.nkeys;
  const int64_t md = S.max_deg;
  for (int b = 0; b < 2; b++) {
    S.pos[b].x = (double *)alloc(8 * n);
    S.pos[b].y = (double *)alloc(8 * n);
    S.pos[b].dprev = (double *)alloc(8 * n);
    S.pos[b].cat = (uint8_t *)alloc(n);
    S.ord[b].id = (int32_t *)alloc(4 * n);
    S.ord[b].span = (float *)alloc(4 * n);
    S.ord[b].xl = (double *)alloc(8 * n);
    S.ord[b].yl = (double *)alloc(8 * n);
  }
  S.adj = (int32_t *)alloc(4 * md * n);
  S.deg = (int32_t *)alloc(4 * n);
  S.tri = (int32_t *)alloc(4 * 3 * TRIME_TRI_PER_POINT * n);
  S.tri_valid = (uint8_t *)alloc(TRIME_TRI_PER_POINT * n);
  S.tri_n = (int32_t *)alloc(4 * (n + 1));
  S.perm = (int32_t *)alloc(4 * (n + 1));
  S.key = (int32_t *)alloc(4 * n);
  S.rank = (int32_t *)alloc(4 * n);
  S.order = (int32_t *)alloc(4 * n);
  S.bin_start = (int32_t *)alloc(4 * (nkeys + 1));
  S.bin_fill = (int32_t *)alloc(4 * nkeys);
  S.scan_tmp = (int32_t *)alloc(4 * (trime::scan_tmp_ints(nkeys > n ? nkeys : n) + 1));
  S.queue = (int32_t *)alloc(4 * (3 * (n + 1) + 16 * n + 512));
  S.counters = (int32_t *)alloc(4 * 32);
  const int64_t np = trime::dm_partials(n);
  S.partials = (double *)alloc(8 * 2 * (np > 1 ? np : 1));
  S.stats = (trime_stats *)alloc(sizeof(trime_stats));
#ifdef TRIME_WARM
  S.warm_n = (int32_t *)alloc(4 * n);
  S.warm_id = (int32_t *)alloc(4 * TRIME_WARM * n);
  S.slot_of_id = (int32_t *)alloc(4 * n);
#endif
  memset(S.counters, 0, 4 * 32);
  emu::after_launch = check_queues;

  double *ex = (double *)alloc(8 * n), *ey = (double *)alloc(8 * n);
  uint8_t *ec = (uint8_t *)alloc(n);
  OK(trime_state_load(&S, x, y, nullptr));
  FILE *out = fopen(argv[2], "wb");
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
