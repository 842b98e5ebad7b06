// Adaptive runs: termination on mesh quality or small movement (Sec. 6,
// thresholds in Table 8) and the quality-driven switch of hybrid meshing
// from DistMesh to CVD (Sec. 4.2, hybrid meshing), decided on the device.
//
// The host enqueues every iteration of the run; a one-thread kernel before
// each iteration turns the control block (stats->adapt) into gates, and each
// kernel of the iteration returns at once when its gate is zero.  After the
// update a grid pass raises `moving` when an inner point moved by fac_end*h
// or more, and a one-thread kernel compares the iteration's quality with the
// previous one and decides.
#include "launch.hpp"

namespace trime {

__global__ void k_adapt_init(KArgs a, int method) {
  trime_adapt_ctl *c = &a.stats->adapt;
  c->method = method;
  c->stopped = 0;
  c->iters = 0;
  c->switch_iter = -1;
  c->stop_iter = -1;
  c->reason = TRIME_STOP_NONE;
  c->moving = 0;
  c->have_prev = 0;
  c->growing = 0;
  c->add_request = 0;
  for (int g = 0; g < 8; g++) c->gate[g] = 0;
  for (int q = 0; q < 3; q++) {
    c->prev[q] = 0.0;
    c->last[q] = 0.0;
    c->rel[q] = -1.0;
  }
  a.stats->retri_flag = 1;  // DistMesh triangulates on the first iteration
}

__global__ void k_adapt_pre(KArgs a) {
  trime_adapt_ctl *c = &a.stats->adapt;
  const int run = !c->stopped;
  const int dm = run && c->method == TRIME_METHOD_DM;
  const int cvd = run && c->method == TRIME_METHOD_CVD;
  const int retri = a.stats->retri_flag != 0;
  c->gate[G_BIN] = cvd || (dm && retri);
  c->gate[G_DMTRI] = dm && retri;
  c->gate[G_DMQ] = dm && !retri;
  c->gate[G_CVD] = cvd;
  c->gate[G_DM] = dm;
  c->gate[G_COPY] = !run;
  c->gate[G_RUN] = run;
  c->moving = 0;
}

// Inner points (category at the start of the iteration) that moved by
// fac_end*h or more, h of the cell they started in.
__global__ __launch_bounds__(256) void k_adapt_move(KArgs a) {
  if (cond_off(a)) return;
  int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool mv = false;
  if (k < a.n && a.cat[k] == TRIME_CAT_INNER) {
    double x = a.x[k], y = a.y[k];
    GCell cell;
    double tx, ty;
    if (locate(a, x, y, cell, tx, ty)) {
      double dx = a.xn[k] - x, dy = a.yn[k] - y;
      mv = sqrt(dx * dx + dy * dy) >= a.prm.fac_end * (double)cell_h(a, cell);
    }
  }
  if (__ballot(mv) && (threadIdx.x & 63) == 0) atomicOr(&a.stats->adapt.moving, 1);
}

// Positions, movements and categories carried over unchanged (the run has
// stopped; the host still swaps the buffers every iteration).
__global__ __launch_bounds__(256) void k_adapt_copy(KArgs a) {
  if (cond_off(a)) return;
  int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= a.n) return;
  a.xn[k] = a.x[k];
  a.yn[k] = a.y[k];
  a.dprevn[k] = a.dprev[k];
  a.catn[k] = a.cat[k];
}

// The decisions after iteration c->iters (one thread).  While points are
// still to be added (Sec. 3.6) the only decision is whether to add them:
// both half-mean changes below t_add; switch and termination wait.
__global__ void k_adapt_post(KArgs a, int hybrid, double t_quality, double t_amax, double t_switch, double t_add) {
  trime_adapt_ctl *c = &a.stats->adapt;
  if (c->stopped) return;
  trime_stats *S = a.stats;
  const int it = c->iters++;
  const bool have = S->nq > 0;
  quality_finish(S);  // the values trime_stats_read reports
  double cur[3] = {0.0, 0.0, 0.0};
  if (have) {
    cur[0] = S->half_mean_alpha;
    cur[1] = S->half_mean_beta;
    cur[2] = S->max_alpha;
  }
  bool rel_ok = have && c->have_prev && c->prev[0] > 0.0 && c->prev[1] > 0.0 && c->prev[2] > 0.0;
  for (int q = 0; q < 3; q++) {
    c->last[q] = cur[q];
    c->rel[q] = rel_ok ? fabs(cur[q] - c->prev[q]) / c->prev[q] : -1.0;
  }
  c->add_request = 0;
  if (c->growing) {
    if (rel_ok && c->rel[0] < t_add && c->rel[1] < t_add) c->add_request = 1;
  } else if (hybrid && c->method == TRIME_METHOD_DM) {
    if (rel_ok && c->rel[0] < t_switch) {
      c->method = TRIME_METHOD_CVD;
      c->switch_iter = it;
    }
  } else if (rel_ok && c->rel[0] < t_quality && c->rel[1] < t_quality && c->rel[2] < t_amax) {
    c->stopped = 1;
    c->reason = TRIME_STOP_QUALITY;
    c->stop_iter = it;
  } else if (!c->moving) {
    c->stopped = 1;
    c->reason = TRIME_STOP_MOVEMENT;
    c->stop_iter = it;
  }
  for (int q = 0; q < 3; q++) c->prev[q] = cur[q];
  c->have_prev = have ? 1 : 0;
}

void launch_adapt_init(const KArgs &a, int method, hipStream_t s) {
  hipLaunchKernelGGL(k_adapt_init, dim3(1), dim3(1), 0, s, a, method);
}

void launch_adapt_pre(const KArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_adapt_pre, dim3(1), dim3(1), 0, s, a);
}

const int32_t *adapt_gate(const trime_state *st, int g) { return &st->stats->adapt.gate[g]; }

void launch_adapt_end(const KArgs &a, int hybrid, double t_quality, double t_amax, double t_switch,
                      double t_add, hipStream_t s) {
  int nb = (int)((a.n + 255) / 256);
  if (nb) {
    KArgs c = a;
    c.cond = &a.stats->adapt.gate[G_COPY];
    hipLaunchKernelGGL(k_adapt_copy, dim3(nb), dim3(256), 0, s, c);
    c.cond = &a.stats->adapt.gate[G_RUN];
    hipLaunchKernelGGL(k_adapt_move, dim3(nb), dim3(256), 0, s, c);
  }
  hipLaunchKernelGGL(k_adapt_post, dim3(1), dim3(1), 0, s, a, hybrid, t_quality, t_amax, t_switch, t_add);
}

}  // namespace trime
