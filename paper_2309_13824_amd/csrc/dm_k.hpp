// The DistMesh step's kernels (Sec. 2.2, Alg. 1, Eq. 2-5) and the small
// state kernels of an iteration; launchers in dm.hip.
#pragma once
#include "geom_dev.hpp"
#include "launch.hpp"

namespace trime {

constexpr int DM_BLOCK = 256;

template <class G> struct DmSums {
  using Args = KArgs;
  static constexpr int BLOCK = DM_BLOCK;
  TRIME_D static void run(const KArgs &a, Blk blk);
  TRIME_D static void run_wave(const KArgs &a, Blk blk);
  TRIME_D static void lane_sums(const KArgs &a, int64_t k, double &l2, double &m2);
};
// sum l^2 and sum mu(m)^2 over the edges (k, j > k) of point k
template <class G> TRIME_D void DmSums<G>::lane_sums(const KArgs &a, int64_t k, double &l2, double &m2) {
  l2 = 0.0;
  m2 = 0.0;
  if (k < a.n) {
    double px = a.x[k], py = a.y[k];
    int d = a.deg[k];
    for (int t = 0; t < d; t++) {
      int j = a.adj[(int64_t)t * a.n + k];
      if (j <= k) continue;
      double qx = a.x[j], qy = a.y[j];
      double dx = px - qx, dy = py - qy;
      double m = mu_clamped<G>(a, (px + qx) * 0.5, (py + qy) * 0.5);
      l2 += dx * dx + dy * dy;
      m2 += m * m;
    }
  }
}
template <class G> TRIME_D void DmSums<G>::run(const KArgs &a, Blk blk) {
  if (cond_off(a)) return;
  __shared__ double s1[DM_BLOCK / 64], s2[DM_BLOCK / 64];
  double l2, m2;
  lane_sums(a, (int64_t)blk.id * DM_BLOCK + threadIdx.x, l2, m2);
  for (int off = 32; off > 0; off >>= 1) {
    l2 += __shfl_down(l2, off);
    m2 += __shfl_down(m2, off);
  }
  int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  if (lane == 0) {
    s1[w] = l2;
    s2[w] = m2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double A = 0, B = 0;
    for (int q = 0; q < DM_BLOCK / 64; q++) {
      A += s1[q];
      B += s2[q];
    }
    a.partials[2 * blk.id] = A;
    a.partials[2 * blk.id + 1] = B;
  }
}
// The block's partial by one wavefront: its four wavefronts' sums one after
// the other, added in the block's order.
template <class G> TRIME_D void DmSums<G>::run_wave(const KArgs &a, Blk blk) {
  if (cond_off(a)) return;
  const int lane = threadIdx.x & 63;
  double A = 0, B = 0;
  for (int w = 0; w < DM_BLOCK / 64; w++) {
    double l2, m2;
    lane_sums(a, (int64_t)blk.id * DM_BLOCK + w * 64 + lane, l2, m2);
    for (int off = 32; off > 0; off >>= 1) {
      l2 += __shfl_down(l2, off);
      m2 += __shfl_down(m2, off);
    }
    A += l2;
    B += m2;
  }
  if (lane == 0) {
    a.partials[2 * blk.id] = A;
    a.partials[2 * blk.id + 1] = B;
  }
}

struct DmFinal {
  struct Args {
    KArgs a;
    int32_t nparts;
  };
  static constexpr int BLOCK = 256;
  TRIME_D static void run(const Args &A_, Blk blk);
  TRIME_D static void run_wave(const Args &A_, Blk blk);
};
TRIME_D void DmFinal::run(const Args &A_, Blk) {
  const KArgs &a = A_.a;
  const int nparts = A_.nparts;
  if (cond_off(a)) return;
  __shared__ double s1[256], s2[256];
  double A = 0, B = 0;
  for (int q = threadIdx.x; q < nparts; q += 256) {
    A += a.partials[2 * q];
    B += a.partials[2 * q + 1];
  }
  s1[threadIdx.x] = A;
  s2[threadIdx.x] = B;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      s1[threadIdx.x] += s1[threadIdx.x + w];
      s2[threadIdx.x] += s2[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.stats->sum_l2 = s1[0];
    a.stats->sum_mu2 = s2[0];
    a.stats->fac_mu = s2[0] > 0 ? sqrt(s1[0] / s2[0]) : 0.0;
  }
}
// The same tree by one wavefront: lane L holds the sums of threads L,
// L + 64, L + 128 and L + 192; the steps 128 and 64 add them in registers,
// the steps 32 ... 1 across lanes, every addition the block's.
TRIME_D void DmFinal::run_wave(const Args &A_, Blk) {
  const KArgs &a = A_.a;
  const int nparts = A_.nparts;
  if (cond_off(a)) return;
  const int lane = threadIdx.x & 63;
  double A[4], B[4];
#pragma unroll
  for (int j = 0; j < 4; j++) {
    A[j] = 0;
    B[j] = 0;
    for (int q = lane + 64 * j; q < nparts; q += 256) {
      A[j] += a.partials[2 * q];
      B[j] += a.partials[2 * q + 1];
    }
  }
  A[0] += A[2];
  B[0] += B[2];
  A[1] += A[3];
  B[1] += B[3];
  A[0] += A[1];
  B[0] += B[1];
  double sa = A[0], sb = B[0];
  for (int w = 32; w > 0; w >>= 1) {
    const double oa = __shfl_down(sa, w), ob = __shfl_down(sb, w);
    if (lane < w) {
      sa += oa;
      sb += ob;
    }
  }
  if (lane == 0) {
    a.stats->sum_l2 = sa;
    a.stats->sum_mu2 = sb;
    a.stats->fac_mu = sb > 0 ? sqrt(sa / sb) : 0.0;
  }
}

// Force, forward Euler, treatment and the large-movement test of one point.
// T is the precision of the force arithmetic; returns false when a decision
// fell within the FP32 band (replay in FP64).
template <class T, class G>
TRIME_D bool dm_point(const KArgs &a, int64_t k, int &moved, TreatCount &tc) {
  double px = a.x[k], py = a.y[k];
  double fac_mu = a.stats->fac_mu;
  T l0s = (T)(a.prm.fac_F * fac_mu);
  T Fx = 0, Fy = 0;
  int d = a.deg[k];
  for (int t = 0; t < d; t++) {
    int j = a.adj[(int64_t)t * a.n + k];
    double qx = a.x[j], qy = a.y[j];
    T dx = (T)(px - qx), dy = (T)(py - qy);
    T l = sqrt(dx * dx + dy * dy);
    if (l == (T)0) continue;
    T m = (T)mu_clamped<G>(a, (px + qx) * 0.5, (py + qy) * 0.5);
    T l0 = m * l0s;
    T f = l < l0 ? (T)a.prm.k_spring * (l0 - l) : (T)0;
    T w = f / l;
    Fx += w * dx;
    Fy += w * dy;
  }
  double xnew = px + a.prm.dt * (double)Fx, ynew = py + a.prm.dt * (double)Fy;
  GCell cell;
  double tx, ty;
  double band = 0.0;
  if (sizeof(T) == 4 && locate(a, px, py, cell, tx, ty)) band = 1e-6 * (double)cell_h(a, cell);
  double xf, yf;
  uint8_t cf;
  bool unsure = false;
  treat<G>(a, px, py, a.cat[k], xnew, ynew, band, xf, yf, cf, unsure, tc);
  moved = 0;
  if (locate(a, xf, yf, cell, tx, ty)) {
    double h = a.prm.fac_retria * (double)cell_h(a, cell);
    double ex = xf - a.xl[k], ey = yf - a.yl[k];
    double r2 = ex * ex + ey * ey;
    if (sizeof(T) == 4 && fabs(r2 - h * h) <= 1e-5 * h * h) unsure = true;
    moved = r2 > h * h;
  }
  if (unsure) return false;
  a.xn[k] = xf;
  a.yn[k] = yf;
  a.catn[k] = cf;
  a.dprevn[k] = sqrt((xf - px) * (xf - px) + (yf - py) * (yf - py));
  return true;
}

template <class T, class G> struct DmForce {
  using Args = KArgs;
  static constexpr int BLOCK = DM_BLOCK;
  TRIME_D static void run(const KArgs &a, Blk blk) { body(a, blk, threadIdx.x); }
  TRIME_D static void body(const KArgs &a, Blk blk, int t);
};
template <class T, class G> TRIME_D void DmForce<T, G>::body(const KArgs &a, Blk blk, int t) {
  if (cond_off(a)) return;
  int64_t k = (int64_t)blk.id * DM_BLOCK + t;
  int moved = 0, replay = 0;
  TreatCount tc;
  if (k < a.n) {
    if (!dm_point<T, G>(a, k, moved, tc)) {
      int q = atomicAdd(&a.counters[CNT_QUEUE], 1);
      a.queue[q] = (int)k;
      replay = 1;
      moved = 0;
      tc.fail = 0;
    }
  }
  int nf = tc.newton_fail(), tf = tc.trace_fail();
  for (int off = 32; off > 0; off >>= 1) {
    moved += __shfl_down(moved, off);
    replay += __shfl_down(replay, off);
    nf += __shfl_down(nf, off);
    tf += __shfl_down(tf, off);
  }
  if ((t & 63) == 0) {
    if (moved) atomicAdd((unsigned long long *)&a.stats->moved, (unsigned long long)moved);
    if (replay) atomicAdd((unsigned long long *)&a.stats->fp64_replays, (unsigned long long)replay);
    if (nf) atomicAdd((unsigned long long *)&a.stats->newton_fail, (unsigned long long)nf);
    if (tf) atomicAdd((unsigned long long *)&a.stats->trace_fail, (unsigned long long)tf);
  }
}

template <class G> struct DmForceReplay {
  using Args = KArgs;
  static constexpr int BLOCK = DM_BLOCK;
  TRIME_D static void run(const KArgs &a, Blk blk) { body(a, blk, threadIdx.x); }
  TRIME_D static void body(const KArgs &a, Blk blk, int t);
};
template <class G> TRIME_D void DmForceReplay<G>::body(const KArgs &a, Blk blk, int t) {
  if (cond_off(a)) return;
  int nq = a.counters[CNT_QUEUE];
  for (int w = blk.id * DM_BLOCK + t; w < nq; w += blk.n * DM_BLOCK) {
    int64_t k = a.queue[w];
    int moved = 0;
    TreatCount tc;
    dm_point<double, G>(a, k, moved, tc);
    if (moved) atomicAdd((unsigned long long *)&a.stats->moved, 1ull);
    if (tc.newton_fail()) atomicAdd((unsigned long long *)&a.stats->newton_fail, 1ull);
    if (tc.trace_fail()) atomicAdd((unsigned long long *)&a.stats->trace_fail, 1ull);
  }
}

struct DmFlag {
  using Args = KArgs;
  static constexpr int BLOCK = 64;
  TRIME_D static void run(const KArgs &a, Blk) {
    if (cond_off(a) || threadIdx.x != 0) return;
    a.stats->retri_flag = a.stats->moved > 0 ? 1 : 0;
    a.stats->iterations++;
  }
};

// Sets the re-triangulation flag (the first iteration of a segment, or
// every iteration when asked to).
struct SetFlag {
  using Args = KArgs;
  static constexpr int BLOCK = 64;
  TRIME_D static void run(const KArgs &a, Blk) {
    if (threadIdx.x == 0) a.stats->retri_flag = 1;
  }
};

struct DmBegin {
  using Args = KArgs;
  static constexpr int BLOCK = 64;
  TRIME_D static void run(const KArgs &a, Blk) {
    if (cond_off(a) || threadIdx.x != 0) return;
    a.stats->moved = 0;
    a.counters[CNT_QUEUE] = 0;
  }
};

// Clears the quality part of the stats (before an extraction / quality pass).
struct StatsReset {
  struct Args {
    KArgs a;
    int32_t full;
  };
  static constexpr int BLOCK = 64;
  TRIME_D static void run(const Args &A, Blk);
};
TRIME_D void StatsReset::run(const Args &A, Blk) {
  if (cond_off(A.a)) return;
  stats_reset(A.a, A.full, threadIdx.x);
}

// Copies the error bits of the counters into the stats and counts an
// extraction.
struct FinishExtract {
  using Args = KArgs;
  static constexpr int BLOCK = 64;
  TRIME_D static void run(const KArgs &a, Blk) {
    if (cond_off(a) || threadIdx.x != 0) return;
    a.stats->error |= a.counters[CNT_ERR];
    a.stats->triangulations++;
    a.counters[CNT_QUEUE] = 0;
  }
};

// kinds (persistent batch kernel)
template <class G> struct KindOf<DmSums<G>> { static constexpr uint32_t code = kcode(KF_DMSUMS, false, is_dbl<G>()); };
template <> struct KindOf<DmFinal> { static constexpr uint32_t code = kcode(KF_DMFINAL); };
template <class T, class G> struct KindOf<DmForce<T, G>> {
  static constexpr uint32_t code = kcode(KF_DMFORCE, is_dbl<T>(), is_dbl<G>());
};
template <class G> struct KindOf<DmForceReplay<G>> {
  static constexpr uint32_t code = kcode(KF_DMREPLAY, false, is_dbl<G>());
};
template <> struct KindOf<DmFlag> { static constexpr uint32_t code = kcode(KF_DMFLAG); };
template <> struct KindOf<SetFlag> { static constexpr uint32_t code = kcode(KF_SETFLAG); };
template <> struct KindOf<DmBegin> { static constexpr uint32_t code = kcode(KF_DMBEGIN); };
template <> struct KindOf<StatsReset> { static constexpr uint32_t code = kcode(KF_STATSRESET); };
template <> struct KindOf<FinishExtract> { static constexpr uint32_t code = kcode(KF_FINISH); };

}  // namespace trime
