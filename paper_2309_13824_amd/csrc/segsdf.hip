// Signed distance to a closed clockwise loop of line segments (Sec. 3.2).
//
// The magnitude at a node is the distance to the nearest segment (equal
// distances go to the lower segment index); the sign comes from the inward
// normal at the closest point: the segment's own (its direction turned
// clockwise by 90 degrees), or at an end point the mean of the two segments'
// normals.  (p - p*) . n > 0 means inside, negative distance.
//
// The paper finds the nearest segment of a point by walking a lattice of
// segment cells outwards ring by ring and then checking every cell within
// the bounding circle of the first non-empty ring.  A node k cells from the
// boundary costs O(k^2) cells that way, which at millions of nodes deep
// inside a shape dominates.  Here the same bound works on whole cells: a
// segment can be the nearest one for some point of a cell only if its
// distance to the cell's centre is at most the nearest distance at the
// centre plus the cell's diameter (two triangle inequalities).  A hierarchy
// of cell grids, each cell filtering its parent's candidate list with that
// bound, leaves every node a short list that contains its nearest segment,
// so the result equals the brute-force minimum bit for bit.
#include "segsdf_dev.hpp"

namespace trime {

// ------------------------------------------------------ candidate build --

struct SegLevelArgs {
  const double *v;
  int nv;
  // parent grid: F x F children per parent cell, the same origin
  int pnx;
  const int32_t *pstart, *pcand;
  int F, cnx, cny;
  double x0, y0, cw, ch;
  int32_t *cnt;                 // count pass: per child cell
  const int32_t *cstart;        // fill pass
  int32_t *ccand;
};

constexpr int SB = 256;

__device__ double block_min(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
  for (int w = SB / 2; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sh[threadIdx.x] = fmin(sh[threadIdx.x], sh[threadIdx.x + w]);
    __syncthreads();
  }
  double r = sh[0];
  __syncthreads();
  return r;
}

// Nearest distance at the child's centre over the parent's list, and the
// filter bound; the child's parent range in [ps, pe).
__device__ double child_bound(const SegLevelArgs &A, int64_t c, double &cx, double &cy, int32_t &ps, int32_t &pe,
                              double *sh) {
  const int ci = (int)(c % A.cnx), cj = (int)(c / A.cnx);
  const int64_t p = (int64_t)(cj / A.F) * A.pnx + ci / A.F;
  ps = A.pstart[p];
  pe = A.pstart[p + 1];
  cx = A.x0 + ((double)ci + 0.5) * A.cw;
  cy = A.y0 + ((double)cj + 0.5) * A.ch;
  double dmin = INFINITY;
  for (int32_t i = ps + threadIdx.x; i < pe; i += SB) {
    double t;
    dmin = fmin(dmin, seg_dist_t(A.v, A.nv, A.pcand[i], cx, cy, t));
  }
  dmin = block_min(dmin, sh);
  // a segment nearest to some point within r of the centre lies within
  // dmin + 2r of the centre; the factor covers rounding of the distances
  const double r = 0.5 * sqrt(A.cw * A.cw + A.ch * A.ch);
  return (dmin + 2.0 * r) * (1.0 + 1e-9);
}

__global__ __launch_bounds__(SB) void k_seg_count(SegLevelArgs A) {
  __shared__ double sh[SB];
  __shared__ int cnt_sh;
  const int64_t c = blockIdx.x;
  double cx, cy;
  int32_t ps, pe;
  const double bound = child_bound(A, c, cx, cy, ps, pe, sh);
  if (threadIdx.x == 0) cnt_sh = 0;
  __syncthreads();
  int n = 0;
  for (int32_t i = ps + threadIdx.x; i < pe; i += SB) {
    double t;
    n += seg_dist_t(A.v, A.nv, A.pcand[i], cx, cy, t) <= bound ? 1 : 0;
  }
  if (n) atomicAdd(&cnt_sh, n);
  __syncthreads();
  if (threadIdx.x == 0) A.cnt[c] = cnt_sh;
}

// The kept candidates in the parent's order (ascending segment index).
__global__ __launch_bounds__(SB) void k_seg_fill(SegLevelArgs A) {
  __shared__ double sh[SB];
  __shared__ int wsum[SB / 64];
  const int64_t c = blockIdx.x;
  double cx, cy;
  int32_t ps, pe;
  const double bound = child_bound(A, c, cx, cy, ps, pe, sh);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int32_t out = A.cstart[c];
  const int32_t end = A.cstart[c + 1];  // the count pass kept as many
  for (int32_t base = ps; base < pe; base += SB) {
    const int32_t i = base + threadIdx.x;
    double t;
    const bool keep = i < pe && seg_dist_t(A.v, A.nv, A.pcand[i], cx, cy, t) <= bound;
    const uint64_t m = __ballot(keep);
    if (lane == 0) wsum[w] = __popcll(m);
    __syncthreads();
    int before = 0, total = 0;
    for (int q = 0; q < SB / 64; q++) {
      before += q < w ? wsum[q] : 0;
      total += wsum[q];
    }
    const int32_t o = out + before + __popcll(m & ((1ull << lane) - 1ull));
    if (keep && o < end) A.ccand[o] = A.pcand[i];
    out += total;
    __syncthreads();
  }
}

__global__ void k_seg_iota(int32_t *p, int n, int32_t *start) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = i;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    start[0] = 0;
    start[1] = n;
  }
}

// Builds the candidate hierarchy of one loop (device vertices d_v) over the
// box [bx0, bx1] x [by0, by1], down to cells of about `target` on a side.
// Allocations go to `allocs` (freed by the caller after the grid build).
const char *seg_tree_build(const double *d_v, int nv, double bx0, double by0, double bx1, double by1,
                           double target, SegTree *T, std::vector<void *> &allocs, hipStream_t s) {
  const int F = 8;
  const double W = bx1 - bx0, H = by1 - by0;
  int levels = 1;
  while (levels < 3 && fmax(W, H) / pow((double)F, levels) > target) levels++;
  int32_t *start = nullptr, *cand = nullptr;
  if (hipMallocAsync((void **)&start, 2 * sizeof(int32_t), s) != hipSuccess) return "segment lattice: allocation";
  allocs.push_back(start);
  if (hipMallocAsync((void **)&cand, sizeof(int32_t) * (size_t)nv, s) != hipSuccess)
    return "segment lattice: allocation";
  allocs.push_back(cand);
  hipLaunchKernelGGL(k_seg_iota, dim3((nv + 255) / 256 < 1024 ? (nv + 255) / 256 : 1024), dim3(256), 0, s, cand, nv,
                     start);
  int pnx = 1;
  for (int l = 1; l <= levels; l++) {
    const int cnx = pnx * F;
    const int64_t nc = (int64_t)cnx * cnx;
    SegLevelArgs A;
    A.v = d_v;
    A.nv = nv;
    A.pnx = pnx;
    A.pstart = start;
    A.pcand = cand;
    A.F = F;
    A.cnx = cnx;
    A.cny = cnx;
    A.x0 = bx0;
    A.y0 = by0;
    A.cw = W / cnx;
    A.ch = H / cnx;
    int32_t *cnt = nullptr, *cstart = nullptr;
    if (hipMallocAsync((void **)&cnt, sizeof(int32_t) * (size_t)nc, s) != hipSuccess ||
        hipMallocAsync((void **)&cstart, sizeof(int32_t) * (size_t)(nc + 1), s) != hipSuccess)
      return "segment lattice: allocation";
    allocs.push_back(cnt);
    allocs.push_back(cstart);
    int32_t *tmp = nullptr;
    if (hipMallocAsync((void **)&tmp, sizeof(int32_t) * (scan_tmp_ints(nc) + 1), s) != hipSuccess)
      return "segment lattice: allocation";
    allocs.push_back(tmp);
    A.cnt = cnt;
    A.cstart = cstart;
    A.ccand = nullptr;
    hipLaunchKernelGGL(k_seg_count, dim3((unsigned)nc), dim3(SB), 0, s, A);
    scan_i32(cnt, cstart, nc, tmp, s);
    int32_t total = 0;
    if (hipMemcpyAsync(&total, cstart + nc, sizeof total, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return "segment lattice: read candidate count";
    if (total < 0) return "segment lattice: more than 2^31 candidates";
    int32_t *ccand = nullptr;
    if (hipMallocAsync((void **)&ccand, sizeof(int32_t) * (size_t)(total > 0 ? total : 1), s) != hipSuccess)
      return "segment lattice: allocation";
    allocs.push_back(ccand);
    A.ccand = ccand;
    hipLaunchKernelGGL(k_seg_fill, dim3((unsigned)nc), dim3(SB), 0, s, A);
    start = cstart;
    cand = ccand;
    pnx = cnx;
  }
  T->v = d_v;
  T->nv = nv;
  T->nx = pnx;
  T->ny = pnx;
  T->x0 = bx0;
  T->y0 = by0;
  T->cw = W / pnx;
  T->ch = H / pnx;
  T->start = start;
  T->cand = cand;
  return nullptr;
}

}  // namespace trime
