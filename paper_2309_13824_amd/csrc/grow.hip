// Point addition (Sec. 3.6): new points at the centroids of the triangles
// with the largest ratio of circumradius to the local desired edge length.
//
// Every valid triangle gets a 128-bit key: the FP64 bits of its ratio (a
// positive double orders as its bits), then the complement of (owner id,
// second id), so that equal ratios rank the smaller ids first and no two
// keys are equal.  A radix select over the 16 key bytes, most significant
// first, finds the n_add-th largest key K; the triangles with key >= K are
// the selection.  The new points take ids in the order of (owner id, second
// id): a count per owner id, an exclusive scan over the ids, and a rank by
// second id within each owner's (at most 16) triangles.
#include "geom_dev.hpp"
#include "launch.hpp"

namespace trime {

struct Key128 {
  uint64_t hi, lo;
};

// Circumradius over h of triangle t of owner slot k, and its centroid;
// h_sel: the h scale the selection uses (the write kernel runs with the
// scale after the addition in its arguments).
TRIME_D Key128 tri_key(const KArgs &a, int64_t k, int t, double h_sel, double &gx, double &gy) {
  const int64_t b = (k * TRIME_TRI_PER_POINT + t) * 3;
  const int s0 = a.tri[b], s1 = a.tri[b + 1], s2 = a.tri[b + 2];
  const double xa = a.x[s0], ya = a.y[s0], xb = a.x[s1], yb = a.y[s1], xc = a.x[s2], yc = a.y[s2];
  const double d1x = xb - xa, d1y = yb - ya, d2x = xc - xa, d2y = yc - ya;
  const double cross = d1x * d2y - d1y * d2x;
  const double la2 = d1x * d1x + d1y * d1y;
  const double lb2 = (xc - xb) * (xc - xb) + (yc - yb) * (yc - yb);
  const double lc2 = d2x * d2x + d2y * d2y;
  const double R = sqrt(la2 * lb2 * lc2) / (2.0 * fabs(cross));
  gx = ((xa + xb) + xc) / 3.0;
  gy = ((ya + yb) + yc) / 3.0;
  // the cell holding the centroid, clamped to the grid
  double fx = floor((gx - a.gx0) * a.inv_dx), fy = floor((gy - a.gy0) * a.inv_dy);
  fx = fmin(fmax(fx, 0.0), (double)(a.nx - 2));
  fy = fmin(fmax(fy, 0.0), (double)(a.ny - 2));
  const float h0 = gld(a.hcell, (int64_t)fy * (a.nx - 1) + (int64_t)fx);
  const float h = h_sel == 1.0 ? h0 : (float)((double)h0 * h_sel);  // as cell_h
  const double ratio = R / (double)h;
  Key128 key;
  key.hi = (uint64_t)__double_as_longlong(ratio);
  key.lo = ~(((uint64_t)(uint32_t)a.id[s0] << 32) | (uint64_t)(uint32_t)a.id[s1]);
  return key;
}

TRIME_D bool key_ge(const Key128 &x, const Key128 &y) { return x.hi > y.hi || (x.hi == y.hi && x.lo >= y.lo); }

// Byte d (0 = most significant) of a key.
TRIME_D uint32_t key_byte(const Key128 &x, int d) {
  return d < 8 ? (uint32_t)(x.hi >> (56 - 8 * d)) & 255u : (uint32_t)(x.lo >> (120 - 8 * d)) & 255u;
}

struct SelState {
  Key128 prefix;      // the bytes found so far
  int64_t remaining;  // keys still to take at or below the prefix
  int32_t hist[256];
};

// Valid triangles of each owner slot.
__global__ __launch_bounds__(256) void k_grow_count(KArgs a, int32_t *cnt) {
  int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= a.n) return;
  int c = 0, nt = a.tri_n[k];
  for (int t = 0; t < nt; t++) c += a.tri_valid[k * TRIME_TRI_PER_POINT + t] ? 1 : 0;
  cnt[k] = c;
}

__global__ __launch_bounds__(256) void k_grow_keys(KArgs a, const int32_t *off, Key128 *keys) {
  int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= a.n) return;
  int64_t w = off[k];
  int nt = a.tri_n[k];
  for (int t = 0; t < nt; t++) {
    if (!a.tri_valid[k * TRIME_TRI_PER_POINT + t]) continue;
    double gx, gy;
    keys[w++] = tri_key(a, k, t, a.h_scale, gx, gy);
  }
}

// Histogram of byte d over the keys that carry the prefix's first d bytes.
__global__ __launch_bounds__(256) void k_grow_hist(const Key128 *keys, int64_t nk, SelState *sel, int d) {
  __shared__ int h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const Key128 p = sel->prefix;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < nk; i += (int64_t)gridDim.x * 256) {
    const Key128 x = keys[i];
    bool match = true;
    for (int e = 0; e < d; e++) match = match && key_byte(x, e) == key_byte(p, e);
    if (match) atomicAdd(&h[key_byte(x, d)], 1);
  }
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&sel->hist[threadIdx.x], h[threadIdx.x]);
}

// Byte d of the n_add-th largest key: from the top, the first digit whose
// count reaches the keys still to take (one thread).
__global__ void k_grow_pick(SelState *sel, int d) {
  if (threadIdx.x != 0) return;
  int64_t above = 0;
  int digit = 0;
  for (int v = 255; v >= 0; v--) {
    int64_t c = sel->hist[v];
    if (above + c >= sel->remaining) {
      digit = v;
      break;
    }
    above += c;
  }
  sel->remaining -= above;
  if (d < 8)
    sel->prefix.hi |= (uint64_t)digit << (56 - 8 * d);
  else
    sel->prefix.lo |= (uint64_t)digit << (120 - 8 * d);
  for (int v = 0; v < 256; v++) sel->hist[v] = 0;
}

__global__ void k_grow_init(SelState *sel, int64_t n_add) {
  if (threadIdx.x != 0) return;
  sel->prefix.hi = 0;
  sel->prefix.lo = 0;
  sel->remaining = n_add;
  for (int v = 0; v < 256; v++) sel->hist[v] = 0;
}

// Selected triangles per owner id (ids are a permutation of 0..n-1).
__global__ __launch_bounds__(256) void k_grow_mark(KArgs a, const SelState *sel, int32_t *cnt_id) {
  int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= a.n) return;
  const Key128 K = sel->prefix;
  int c = 0, nt = a.tri_n[k];
  for (int t = 0; t < nt; t++) {
    if (!a.tri_valid[k * TRIME_TRI_PER_POINT + t]) continue;
    double gx, gy;
    if (key_ge(tri_key(a, k, t, a.h_scale, gx, gy), K)) c++;
  }
  cnt_id[a.id[k]] = c;
}

// The new points: owner slot k writes its selected triangles' centroids at
// the slots n + base[id] + rank, rank by second id; ids equal their slots.
// The arguments carry the h scale after the addition (categories, spans);
// h_sel is the one the selection used.
template <class G>
__global__ __launch_bounds__(256) void k_grow_write(KArgs a, double h_sel, const SelState *sel, const int32_t *base,
                                                    double *x, double *y, double *dprev, uint8_t *cat, int32_t *id,
                                                    float *span, double *xl, double *yl) {
  int64_t k = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (k >= a.n) return;
  const Key128 K = sel->prefix;
  int nt = a.tri_n[k];
  int sec[TRIME_TRI_PER_POINT];
  double cx[TRIME_TRI_PER_POINT], cy[TRIME_TRI_PER_POINT];
  int m = 0;
  for (int t = 0; t < nt && t < TRIME_TRI_PER_POINT; t++) {
    if (!a.tri_valid[k * TRIME_TRI_PER_POINT + t]) continue;
    double gx, gy;
    if (!key_ge(tri_key(a, k, t, h_sel, gx, gy), K)) continue;
    int s1 = a.tri[(k * TRIME_TRI_PER_POINT + t) * 3 + 1];
    int v = a.id[s1];
    int j = m++;
    while (j > 0 && sec[j - 1] > v) {
      sec[j] = sec[j - 1];
      cx[j] = cx[j - 1];
      cy[j] = cy[j - 1];
      j--;
    }
    sec[j] = v;
    cx[j] = gx;
    cy[j] = gy;
  }
  const int64_t b0 = a.n + base[a.id[k]];
  for (int r = 0; r < m; r++) {
    const int64_t s = b0 + r;
    x[s] = cx[r];
    y[s] = cy[r];
    xl[s] = cx[r];
    yl[s] = cy[r];
    dprev[s] = -1.0;
    id[s] = (int32_t)s;
    bool unsure = false;
    cat[s] = point_category<G>(a, cx[r], cy[r], 0.0, unsure);
    span[s] = span_at(a, cx[r], cy[r]);
  }
}

// The control block around an addition: whether points are still to come,
// and after one, no previous statistics and a DistMesh re-triangulation.
__global__ void k_grow_state(KArgs a, int growing, int added) {
  if (threadIdx.x != 0) return;
  a.stats->adapt.growing = growing;
  a.stats->adapt.add_request = 0;
  if (added) {
    a.stats->adapt.have_prev = 0;
    a.stats->retri_flag = 1;
  }
}

// Steps of a point addition, in the order the library enqueues them.
void launch_grow_count(const KArgs &a, int32_t *cnt, hipStream_t s) {
  int nb = (int)((a.n + 255) / 256);
  if (nb) hipLaunchKernelGGL(k_grow_count, dim3(nb), dim3(256), 0, s, a, cnt);
}

void launch_grow_select(const KArgs &a, const int32_t *off, void *keys, int64_t nk, void *sel, int64_t n_add,
                        hipStream_t s) {
  int nb = (int)((a.n + 255) / 256);
  if (nb) hipLaunchKernelGGL(k_grow_keys, dim3(nb), dim3(256), 0, s, a, off, (Key128 *)keys);
  hipLaunchKernelGGL(k_grow_init, dim3(1), dim3(64), 0, s, (SelState *)sel, n_add);
  int hb = (int)((nk + 255) / 256);
  hb = hb < 1 ? 1 : (hb > 1024 ? 1024 : hb);
  for (int d = 0; d < 16; d++) {
    hipLaunchKernelGGL(k_grow_hist, dim3(hb), dim3(256), 0, s, (const Key128 *)keys, nk, (SelState *)sel, d);
    hipLaunchKernelGGL(k_grow_pick, dim3(1), dim3(64), 0, s, (SelState *)sel, d);
  }
}

void launch_grow_mark(const KArgs &a, const void *sel, int32_t *cnt_id, hipStream_t s) {
  int nb = (int)((a.n + 255) / 256);
  if (nb) hipLaunchKernelGGL(k_grow_mark, dim3(nb), dim3(256), 0, s, a, (const SelState *)sel, cnt_id);
}

void launch_grow_write(const KArgs &a, double h_sel, int grid_bytes, const void *sel, const int32_t *base, double *x,
                       double *y, double *dprev, uint8_t *cat, int32_t *id, float *span, double *xl, double *yl,
                       hipStream_t s) {
  int nb = (int)((a.n + 255) / 256);
  if (!nb) return;
  if (grid_bytes == 4)
    hipLaunchKernelGGL(k_grow_write<float>, dim3(nb), dim3(256), 0, s, a, h_sel, (const SelState *)sel, base, x, y,
                       dprev, cat, id, span, xl, yl);
  else
    hipLaunchKernelGGL(k_grow_write<double>, dim3(nb), dim3(256), 0, s, a, h_sel, (const SelState *)sel, base, x, y,
                       dprev, cat, id, span, xl, yl);
}

void launch_grow_state(const KArgs &a, int growing, int added, hipStream_t s) {
  hipLaunchKernelGGL(k_grow_state, dim3(1), dim3(64), 0, s, a, growing, added);
}

size_t grow_key_bytes() { return sizeof(Key128); }
size_t grow_sel_bytes() { return sizeof(SelState); }

}  // namespace trime
