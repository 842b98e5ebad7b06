// DistMesh step (Sec. 2.2, Alg. 1, Eq. 2-5) and state helper kernels.
//
// The paper scatters each edge force to both end points with atomics
// (Sec. 5).  Here every point gathers over its own adjacency row instead:
// the force of an edge is computed from the same inputs at both ends (the
// midpoint (p_i + p_j)/2 and |p_i - p_j| are symmetric in i and j), so the
// two ends see exactly opposite forces and no atomics are needed.
// fac_mu (Eq. 3) is an ordered two-level reduction of sum l^2 and
// sum mu(m)^2 over the unique edges (j > i), accumulated in FP64.
#include "dm_k.hpp"

namespace trime {

void launch_set_flag(const KArgs &a, hipStream_t s) { launch<SetFlag>(a, 1, s); }

template <class G> static void launch_dm_g(const KArgs &a, hipStream_t s) {
  const uint32_t nb = (uint32_t)((a.n + DM_BLOCK - 1) / DM_BLOCK);
  launch<DmBegin>(a, 1, s);
  launch<DmSums<G>>(a, nb, s);
  launch<DmFinal>(DmFinal::Args{a, (int32_t)nb}, 1, s);
  if (a.precision == TRIME_FP32)
    launch<DmForce<float, G>>(a, nb, s);
  else
    launch<DmForce<double, G>>(a, nb, s);
  // the replay queue holds the few points an FP32 decision left open
  const int64_t nr = a.n / 16384;
  launch<DmForceReplay<G>>(a, (uint32_t)(nr < 2 ? 2 : (nr > 64 ? 64 : nr)), s);
  launch<DmFlag>(a, 1, s);
}

void launch_dm(const KArgs &a, int grid_bytes, hipStream_t s) {
  if (grid_bytes == 4)
    launch_dm_g<float>(a, s);
  else
    launch_dm_g<double>(a, s);
}

int dm_partials(int64_t n) { return (int)((n + DM_BLOCK - 1) / DM_BLOCK); }

// ------------------------------------------------------------ helpers ----


template <class G> __global__ void k_load(KArgs a, LoadArgs l) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n) return;
  double x = l.xin[k], y = l.yin[k];
  l.x[k] = x;
  l.y[k] = y;
  l.xl[k] = x;
  l.yl[k] = y;
  l.dprev[k] = -1.0;
  l.id[k] = (int)k;
  a.order[k] = (int)k;
  l.span[k] = span_at(a, x, y);
  bool unsure = false;
  l.cat[k] = point_category<G>(a, x, y, 0.0, unsure);
}

void launch_load(const KArgs &a, const LoadArgs &l, int grid_bytes, hipStream_t s) {
  int nb = (int)((a.n + 255) / 256);
  if (!nb) return;
  if (grid_bytes == 4)
    hipLaunchKernelGGL(k_load<float>, dim3(nb), dim3(256), 0, s, a, l);
  else
    hipLaunchKernelGGL(k_load<double>, dim3(nb), dim3(256), 0, s, a, l);
}

__global__ void k_export_points(KArgs a, double *xo, double *yo, uint8_t *co) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n) return;
  int i = a.id[k];
  if (xo) xo[i] = a.x[k];
  if (yo) yo[i] = a.y[k];
  if (co) co[i] = a.cat[k];
}

void launch_export_points(const KArgs &a, double *xo, double *yo, uint8_t *co, hipStream_t s) {
  int nb = (int)((a.n + 255) / 256);
  if (nb) hipLaunchKernelGGL(k_export_points, dim3(nb), dim3(256), 0, s, a, xo, yo, co);
}

// Triangles: offsets = exclusive scan of tri_n (slot order), then ids.
__global__ void k_export_tri(KArgs a, const int32_t *off, int32_t *out, uint8_t *valid, int64_t cap,
                             int64_t *count) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0 && count) *count = off[a.n];
  if (k >= a.n) return;
  int o = off[k];
  for (int t = 0; t < a.tri_n[k]; t++) {
    int64_t q = o + t;
    if (q >= cap) return;
    int64_t b = (k * TRIME_TRI_PER_POINT + t) * 3;
    out[3 * q + 0] = a.id[a.tri[b + 0]];
    out[3 * q + 1] = a.id[a.tri[b + 1]];
    out[3 * q + 2] = a.id[a.tri[b + 2]];
    valid[q] = a.tri_valid[k * TRIME_TRI_PER_POINT + t];
  }
}

void launch_export_tri(const KArgs &a, int32_t *off, int32_t *scan_tmp, int32_t *out,
                       uint8_t *valid, int64_t cap, int64_t *count, hipStream_t s) {
  scan_i32(a.tri_n, off, a.n, scan_tmp, s);
  int nb = (int)((a.n + 255) / 256);
  if (nb) hipLaunchKernelGGL(k_export_tri, dim3(nb), dim3(256), 0, s, a, off, out, valid, cap, count);
}

// Adjacency rows translated to ids and sorted, id-major.
__global__ void k_export_adj(KArgs a, int32_t *deg_o, int32_t *col_o) {
  int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.n) return;
  int i = a.id[k];
  int d = a.deg[k];
  int md = a.max_deg;
  int32_t *row = col_o + (int64_t)i * md;
  for (int t = 0; t < d; t++) {
    int v = a.id[a.adj[(int64_t)t * a.n + k]];
    int u = t;
    while (u > 0 && row[u - 1] > v) {
      row[u] = row[u - 1];
      u--;
    }
    row[u] = v;
  }
  deg_o[i] = d;
}

void launch_export_adj(const KArgs &a, int32_t *deg_o, int32_t *col_o, hipStream_t s) {
  int nb = (int)((a.n + 255) / 256);
  if (nb) hipLaunchKernelGGL(k_export_adj, dim3(nb), dim3(256), 0, s, a, deg_o, col_o);
}

// Quality of the stored valid triangles with the current positions.
__global__ __launch_bounds__(256) void k_quality(KArgs a) {
  if (cond_off(a)) return;
  __shared__ int hist[40];
  for (int b = threadIdx.x; b < 40; b += 256) hist[b] = 0;
  __syncthreads();
  int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double sa = 0, sb = 0, sq = 0, amax = 0;
  int nq = 0;
  if (k < a.n) {
    for (int t = 0; t < a.tri_n[k]; t++) {
      if (!a.tri_valid[k * TRIME_TRI_PER_POINT + t]) continue;
      int64_t b = (k * TRIME_TRI_PER_POINT + t) * 3;
      int s0 = a.tri[b], s1 = a.tri[b + 1], s2 = a.tri[b + 2];
      double ax = a.x[s0], ay = a.y[s0], bx = a.x[s1], by = a.y[s1], cx = a.x[s2], cy = a.y[s2];
      double l0 = sqrt((bx - ax) * (bx - ax) + (by - ay) * (by - ay));
      double l1 = sqrt((cx - bx) * (cx - bx) + (cy - by) * (cy - by));
      double l2 = sqrt((ax - cx) * (ax - cx) + (ay - cy) * (ay - cy));
      double A2 = fabs((bx - ax) * (cy - ay) - (by - ay) * (cx - ax));
      double al = (l0 * l1 * l2) * (l0 + l1 + l2) / (4.0 * A2 * A2);
      double be = fmax(l0, fmax(l1, l2)) / fmin(l0, fmin(l1, l2));
      sa += sqrt(al);
      sb += sqrt(be);
      sq += 1.0 / al;
      amax = fmax(amax, al);
      nq++;
      const int bin = beta_bin(be);
      atomicAdd(&hist[bin], 1);
    }
  }
  for (int off = 32; off > 0; off >>= 1) {
    sa += __shfl_down(sa, off);
    sb += __shfl_down(sb, off);
    sq += __shfl_down(sq, off);
    amax = fmax(amax, __shfl_down(amax, off));
    nq += __shfl_down(nq, off);
  }
  if ((threadIdx.x & 63) == 0 && nq) {  // one wavefront's 64 slots, summed in a fixed order
    quality_add(a.stats, sa, sb, sq, amax);
    atomicAdd((unsigned long long *)&a.stats->nq, (unsigned long long)nq);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < 40; b += 256)
    if (hist[b]) atomicAdd((unsigned long long *)&a.stats->hist_beta[b], (unsigned long long)hist[b]);
}

void launch_stats_reset(const KArgs &a, int full, hipStream_t s) {
  launch<StatsReset>(StatsReset::Args{a, full}, 1, s);
}

void launch_quality(const KArgs &a, hipStream_t s) {
  int nb = (int)((a.n + 255) / 256);
  launch<StatsReset>(StatsReset::Args{a, 0}, 1, s);
  if (nb) hipLaunchKernelGGL(k_quality, dim3(nb), dim3(256), 0, s, a);
}

void launch_finish_extract(const KArgs &a, hipStream_t s) { launch<FinishExtract>(a, 1, s); }

}  // namespace trime
