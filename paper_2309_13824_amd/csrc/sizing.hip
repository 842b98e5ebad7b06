// Automatic sizing field (Sec. 3.3, Eq. 8) on the GPU: medial-axis
// approximating points from the Voronoi cells of the boundary points, their
// trimming by neighbour count, the local feature size of every boundary
// point, and the candidate lists for mu(x) = min over s of K |x - s| + lfs(s).
//
// Each boundary point's Voronoi cell is clipped from a box by the bisector
// of every other point, in index order, so the cells (and the poles taken
// from them) are the same polygons, vertex for vertex, that a serial
// brute-force construction produces.
#include "segsdf_dev.hpp"

namespace trime {

const char *lfs_field_build(const double *d_s, const double *d_lfs, int64_t ns, double K, double bx0, double by0,
                            double bx1, double by1, double target, LfsField *F, std::vector<void *> &allocs,
                            hipStream_t s);

constexpr int PV = 256;  // vertices of a cell (the clip gives up at PV - 2)

// One wavefront per boundary point i; the polygon lives in LDS.  The lanes
// test 64 bisectors at a time against the current polygon and the first
// that cuts it (in index order) is applied, cooperatively: the sequence of
// effective clips, and every operation of each, is that of clipping by all
// points in index order.  Poles then as for a serial construction: v1 = the
// farthest vertex (a medial point unless a box edge meets it: it then
// stands for a vertex at infinity), v2 = the farthest vertex without a box
// edge in the open half plane opposite v1.
__global__ __launch_bounds__(64) void k_medial(const double *s, int64_t ns, const double *box, double *cand,
                                               uint8_t *flags) {
  __shared__ double X[2][PV], Y[2][PV], V[PV];
  __shared__ int32_t E[2][PV];
  __shared__ int cnt_sh[64];
  const int64_t i = blockIdx.x;
  const int lane = threadIdx.x;
  const double sx = s[2 * i], sy = s[2 * i + 1];
  int cur = 0, n = 4;
  if (lane == 0) {
    X[0][0] = box[0], Y[0][0] = box[1], E[0][0] = -1;
    X[0][1] = box[2], Y[0][1] = box[1], E[0][1] = -1;
    X[0][2] = box[2], Y[0][2] = box[3], E[0][2] = -1;
    X[0][3] = box[0], Y[0][3] = box[3], E[0][3] = -1;
  }
  __syncthreads();
  bool overflow = false;
  int64_t j0 = 0;
  while (j0 < ns && !overflow) {
    // does bisector j = j0 + lane cut the current polygon?
    const int64_t j = j0 + lane;
    bool cut = false;
    if (j < ns && j != i) {
      const double tx = s[2 * j], ty = s[2 * j + 1];
      if (!(tx == sx && ty == sy)) {
        const double nx = tx - sx, ny = ty - sy, mx = 0.5 * (sx + tx), my = 0.5 * (sy + ty);
        for (int k = 0; k < n && !cut; k++) cut = (X[cur][k] - mx) * nx + (Y[cur][k] - my) * ny > 0;
      }
    }
    const uint64_t mask = __ballot(cut);
    if (!mask) {
      j0 += 64;
      continue;
    }
    const int64_t jc = j0 + __ffsll((unsigned long long)mask) - 1;
    const double tx = s[2 * jc], ty = s[2 * jc + 1];
    const double nx = tx - sx, ny = ty - sy, mx = 0.5 * (sx + tx), my = 0.5 * (sy + ty);
    for (int k = lane; k < n; k += 64) V[k] = (X[cur][k] - mx) * nx + (Y[cur][k] - my) * ny;
    __syncthreads();
    // emit, per vertex k in order: the vertex if inside, then the crossing
    // of edge k if it crosses
    int base = 0;
    for (int k0 = 0; k0 < n; k0 += 64) {
      const int k = k0 + lane;
      int c = 0;
      bool in0 = false, in1 = false;
      if (k < n) {
        const int k1 = k + 1 == n ? 0 : k + 1;
        in0 = V[k] <= 0;
        in1 = V[k1] <= 0;
        c = (in0 ? 1 : 0) + (in0 != in1 ? 1 : 0);
      }
      cnt_sh[lane] = c;
      __syncthreads();
      int before = 0, total = 0;
      for (int q = 0; q < 64; q++) {
        before += q < lane ? cnt_sh[q] : 0;
        total += cnt_sh[q];
      }
      int o = base + before;
      const int nxt = cur ^ 1;
      if (k < n && base + total <= PV) {
        const int k1 = k + 1 == n ? 0 : k + 1;
        if (in0) {
          X[nxt][o] = X[cur][k], Y[nxt][o] = Y[cur][k], E[nxt][o] = E[cur][k];
          o++;
        }
        if (in0 != in1) {
          const double t = V[k] / (V[k] - V[k1]);
          X[nxt][o] = X[cur][k] + t * (X[cur][k1] - X[cur][k]);
          Y[nxt][o] = Y[cur][k] + t * (Y[cur][k1] - Y[cur][k]);
          E[nxt][o] = in0 ? (int32_t)jc : E[cur][k];
        }
      }
      base += total;
      __syncthreads();
    }
    overflow = base >= PV - 2;
    n = base;
    cur ^= 1;
    j0 = jc + 1;
  }
  if (lane != 0) return;
  uint8_t f = 0;
  if (!overflow && n >= 3) {
    int b1 = -1;
    double d1 = -1.0;
    for (int k = 0; k < n; k++) {
      const double d = (X[cur][k] - sx) * (X[cur][k] - sx) + (Y[cur][k] - sy) * (Y[cur][k] - sy);
      if (d > d1) d1 = d, b1 = k;
    }
    const double ux = X[cur][b1] - sx, uy = Y[cur][b1] - sy;
    if (E[cur][b1] >= 0 && E[cur][b1 == 0 ? n - 1 : b1 - 1] >= 0) {
      f |= 1;
      cand[4 * i] = X[cur][b1];
      cand[4 * i + 1] = Y[cur][b1];
    }
    int b2 = -1;
    double d2 = -1.0;
    for (int k = 0; k < n; k++) {
      const bool real = E[cur][k] >= 0 && E[cur][k == 0 ? n - 1 : k - 1] >= 0;
      if (!real || (X[cur][k] - sx) * ux + (Y[cur][k] - sy) * uy >= 0) continue;
      const double d = (X[cur][k] - sx) * (X[cur][k] - sx) + (Y[cur][k] - sy) * (Y[cur][k] - sy);
      if (d > d2) d2 = d, b2 = k;
    }
    if (b2 >= 0) {
      f |= 2;
      cand[4 * i + 2] = X[cur][b2];
      cand[4 * i + 3] = Y[cur][b2];
    }
  }
  flags[i] = f;
}

__global__ __launch_bounds__(256) void k_medial_count(const uint8_t *flags, int64_t ns, int32_t *cnt) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < ns) cnt[i] = (flags[i] & 1) + ((flags[i] >> 1) & 1);
}

// Medial points in the order of their boundary points (v1 before v2).
__global__ __launch_bounds__(256) void k_medial_compact(const double *cand, const uint8_t *flags, const int32_t *off,
                                                        int64_t ns, double *medial) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= ns) return;
  int64_t o = off[i];
  if (flags[i] & 1) {
    medial[2 * o] = cand[4 * i];
    medial[2 * o + 1] = cand[4 * i + 1];
    o++;
  }
  if (flags[i] & 2) {
    medial[2 * o] = cand[4 * i + 2];
    medial[2 * o + 1] = cand[4 * i + 3];
  }
}

// keep[i]: at least n_thres other medial points within r_nei (squared
// distances against r_nei^2).
__global__ __launch_bounds__(256) void k_medial_trim(const double *m, int64_t nm, double r2, int n_thres,
                                                     uint8_t *keep, int32_t *kept) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = i < nm;
  const double mx = live ? m[2 * i] : 0.0, my = live ? m[2 * i + 1] : 0.0;
  int64_t c = 0;
  for (int64_t j = 0; j < nm; j++) {
    const double dx = m[2 * j] - mx, dy = m[2 * j + 1] - my;
    c += (j != i && dx * dx + dy * dy <= r2) ? 1 : 0;
  }
  if (!live) return;
  keep[i] = c >= n_thres;
  if (c >= n_thres) atomicAdd(kept, 1);
}

// lfs(s_i): the distance to the nearest kept medial point.
__global__ __launch_bounds__(256) void k_lfs(const double *s, int64_t ns, const double *m, int64_t nm,
                                             const uint8_t *keep, double *lfs) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const bool live = i < ns;
  const double sx = live ? s[2 * i] : 0.0, sy = live ? s[2 * i + 1] : 0.0;
  double best = INFINITY;
  for (int64_t j = 0; j < nm; j++) {
    if (!keep[j]) continue;
    const double dx = m[2 * j] - sx, dy = m[2 * j + 1] - sy;
    const double d = sqrt(dx * dx + dy * dy);
    if (d < best) best = d;
  }
  if (live) lfs[i] = best;
}

static unsigned blocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b > 0 ? (n + b - 1) / b : 1); }

const char *auto_sizing_build(const double *d_s, int64_t ns, const double box[4], const double gbox[4],
                              double r_nei, int n_thres, double K, double target, double *medial, uint8_t *keep,
                              double *lfs, int64_t *nm_host, LfsField *F, std::vector<void *> &allocs,
                              hipStream_t s) {
  double *cand = nullptr, *d_box = nullptr;
  uint8_t *flags = nullptr;
  int32_t *cnt = nullptr, *off = nullptr, *tmp = nullptr, *counters = nullptr;
  if (hipMallocAsync((void **)&cand, sizeof(double) * 4 * (size_t)ns, s) != hipSuccess ||
      hipMallocAsync((void **)&d_box, sizeof(double) * 4, s) != hipSuccess ||
      hipMallocAsync((void **)&flags, (size_t)ns, s) != hipSuccess ||
      hipMallocAsync((void **)&cnt, sizeof(int32_t) * (size_t)ns, s) != hipSuccess ||
      hipMallocAsync((void **)&off, sizeof(int32_t) * (size_t)(ns + 1), s) != hipSuccess ||
      hipMallocAsync((void **)&tmp, sizeof(int32_t) * (scan_tmp_ints(ns) + 1), s) != hipSuccess ||
      hipMallocAsync((void **)&counters, sizeof(int32_t) * 2, s) != hipSuccess)
    return "automatic sizing: allocation";
  for (void *p : {(void *)cand, (void *)d_box, (void *)flags, (void *)cnt, (void *)off, (void *)tmp,
                  (void *)counters})
    allocs.push_back(p);
  if (hipMemcpyAsync(d_box, box, sizeof(double) * 4, hipMemcpyHostToDevice, s) != hipSuccess)
    return "automatic sizing: copy the box";
  launch_fill_i32(counters, 2, 0, s);
  hipLaunchKernelGGL(k_medial, dim3((unsigned)ns), dim3(64), 0, s, d_s, ns, (const double *)d_box, cand, flags);
  hipLaunchKernelGGL(k_medial_count, dim3(blocks(ns, 256)), dim3(256), 0, s, (const uint8_t *)flags, ns, cnt);
  scan_i32(cnt, off, ns, tmp, s);
  hipLaunchKernelGGL(k_medial_compact, dim3(blocks(ns, 256)), dim3(256), 0, s, (const double *)cand,
                     (const uint8_t *)flags, (const int32_t *)off, ns, medial);
  int32_t nm = 0;
  if (hipMemcpyAsync(&nm, off + ns, sizeof nm, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return "automatic sizing: read the medial point count";
  *nm_host = nm;
  hipLaunchKernelGGL(k_medial_trim, dim3(blocks(nm, 256)), dim3(256), 0, s, (const double *)medial, (int64_t)nm,
                     r_nei * r_nei, n_thres, keep, counters + 1);
  hipLaunchKernelGGL(k_lfs, dim3(blocks(ns, 256)), dim3(256), 0, s, d_s, ns, (const double *)medial, (int64_t)nm,
                     (const uint8_t *)keep, lfs);
  int32_t kept = 0;
  if (hipMemcpyAsync(&kept, counters + 1, sizeof kept, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return "automatic sizing: read the kept count";
  if (kept == 0) return "automatic sizing: no medial point survives the trimming";
  if (!F) return nullptr;
  return lfs_field_build(d_s, lfs, ns, K, gbox[0], gbox[1], gbox[2], gbox[3], target, F, allocs, s);
}

}  // namespace trime
