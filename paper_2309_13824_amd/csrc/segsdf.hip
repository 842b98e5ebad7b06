// Candidate lists over cell grids, for the nearest segment of a clockwise
// segment loop (Sec. 3.2) and for the automatic sizing field (Eq. 8).
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

template <class M> struct LevelArgs {
  M metric;
  // parent grid: F x F children per parent cell, the same origin
  int pnx;
  const int32_t *pstart, *pcand;
  int F, cnx, cny;
  double x0, y0, cw, ch;
  int32_t *cnt;           // count pass: per child cell
  const int32_t *cstart;  // fill pass
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

// The minimum at the child's centre over the parent's list, and the filter
// bound: an item that gives the minimum somewhere within r of the centre has
// a value there at most the minimum plus slack(r); the factor covers rounding.
template <class M>
__device__ double child_bound(const LevelArgs<M> &A, int64_t c, double &cx, double &cy, int32_t &ps, int32_t &pe,
                              double *sh) {
  const int ci = (int)(c % A.cnx), cj = (int)(c / A.cnx);
  const int64_t p = (int64_t)(cj / A.F) * A.pnx + ci / A.F;
  ps = A.pstart[p];
  pe = A.pstart[p + 1];
  cx = A.x0 + ((double)ci + 0.5) * A.cw;
  cy = A.y0 + ((double)cj + 0.5) * A.ch;
  double vmin = INFINITY;
  for (int32_t i = ps + threadIdx.x; i < pe; i += SB) vmin = fmin(vmin, A.metric.value(A.pcand[i], cx, cy));
  vmin = block_min(vmin, sh);
  const double r = 0.5 * sqrt(A.cw * A.cw + A.ch * A.ch);
  return (vmin + A.metric.slack(r)) * (1.0 + 1e-9);
}

template <class M> __global__ __launch_bounds__(SB) void k_cand_count(LevelArgs<M> A) {
  __shared__ double sh[SB];
  __shared__ int cnt_sh;
  const int64_t c = blockIdx.x;
  double cx, cy;
  int32_t ps, pe;
  const double bound = child_bound(A, c, cx, cy, ps, pe, sh);
  if (threadIdx.x == 0) cnt_sh = 0;
  __syncthreads();
  int n = 0;
  for (int32_t i = ps + threadIdx.x; i < pe; i += SB) n += A.metric.value(A.pcand[i], cx, cy) <= bound ? 1 : 0;
  if (n) atomicAdd(&cnt_sh, n);
  __syncthreads();
  if (threadIdx.x == 0) A.cnt[c] = cnt_sh;
}

// The kept candidates in the parent's order (ascending).
template <class M> __global__ __launch_bounds__(SB) void k_cand_fill(LevelArgs<M> A) {
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
    const bool keep = i < pe && A.metric.value(A.pcand[i], cx, cy) <= bound;
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

__global__ void k_cand_iota(int32_t *p, int n, int32_t *start) {
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = i;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    start[0] = 0;
    start[1] = n;
  }
}

// Builds the candidate hierarchy of n items over the box [bx0, bx1] x
// [by0, by1]: up to three levels of 8 x 8 refinement, down to cells of about
// `target` on a side.  Allocations go to `allocs` (freed by the caller).
template <class M>
static const char *cand_build(const M &metric, int n, double bx0, double by0, double bx1, double by1, double target,
                              CandGrid *G, std::vector<void *> &allocs, hipStream_t s) {
  const int F = 8;
  const double W = bx1 - bx0, H = by1 - by0;
  int levels = 1;
  while (levels < 3 && fmax(W, H) / pow((double)F, levels) > target) levels++;
  int32_t *start = nullptr, *cand = nullptr;
  if (hipMallocAsync((void **)&start, 2 * sizeof(int32_t), s) != hipSuccess) return "candidate lists: allocation";
  allocs.push_back(start);
  if (hipMallocAsync((void **)&cand, sizeof(int32_t) * (size_t)(n > 0 ? n : 1), s) != hipSuccess)
    return "candidate lists: allocation";
  allocs.push_back(cand);
  const int ib = (n + 255) / 256;
  hipLaunchKernelGGL(k_cand_iota, dim3(ib < 1 ? 1 : (ib > 1024 ? 1024 : ib)), dim3(256), 0, s, cand, n, start);
  int pnx = 1;
  for (int l = 1; l <= levels; l++) {
    const int cnx = pnx * F;
    const int64_t nc = (int64_t)cnx * cnx;
    LevelArgs<M> A;
    A.metric = metric;
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
    int32_t *cnt = nullptr, *cstart = nullptr, *tmp = nullptr;
    if (hipMallocAsync((void **)&cnt, sizeof(int32_t) * (size_t)nc, s) != hipSuccess ||
        hipMallocAsync((void **)&cstart, sizeof(int32_t) * (size_t)(nc + 1), s) != hipSuccess ||
        hipMallocAsync((void **)&tmp, sizeof(int32_t) * (scan_tmp_ints(nc) + 1), s) != hipSuccess)
      return "candidate lists: allocation";
    allocs.push_back(cnt);
    allocs.push_back(cstart);
    allocs.push_back(tmp);
    A.cnt = cnt;
    A.cstart = cstart;
    A.ccand = nullptr;
    hipLaunchKernelGGL(k_cand_count<M>, dim3((unsigned)nc), dim3(SB), 0, s, A);
    scan_i32(cnt, cstart, nc, tmp, s);
    int32_t total = 0;
    if (hipMemcpyAsync(&total, cstart + nc, sizeof total, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return "candidate lists: read the candidate count";
    if (total < 0) return "candidate lists: more than 2^31 candidates";
    int32_t *ccand = nullptr;
    if (hipMallocAsync((void **)&ccand, sizeof(int32_t) * (size_t)(total > 0 ? total : 1), s) != hipSuccess)
      return "candidate lists: allocation";
    allocs.push_back(ccand);
    A.ccand = ccand;
    hipLaunchKernelGGL(k_cand_fill<M>, dim3((unsigned)nc), dim3(SB), 0, s, A);
    start = cstart;
    cand = ccand;
    pnx = cnx;
  }
  G->nx = pnx;
  G->ny = pnx;
  G->x0 = bx0;
  G->y0 = by0;
  G->cw = W / pnx;
  G->ch = H / pnx;
  G->start = start;
  G->cand = cand;
  return nullptr;
}

const char *seg_tree_build(const double *d_v, int nv, double bx0, double by0, double bx1, double by1,
                           double target, SegTree *T, std::vector<void *> &allocs, hipStream_t s) {
  T->v = d_v;
  T->nv = nv;
  return cand_build(SegMetric{d_v, nv}, nv, bx0, by0, bx1, by1, target, &T->g, allocs, s);
}

const char *lfs_field_build(const double *d_s, const double *d_lfs, int64_t ns, double K, double bx0, double by0,
                            double bx1, double by1, double target, LfsField *F, std::vector<void *> &allocs,
                            hipStream_t s) {
  F->s = d_s;
  F->lfs = d_lfs;
  F->ns = ns;
  F->K = K;
  return cand_build(LfsMetric{d_s, d_lfs, K}, (int)ns, bx0, by0, bx1, by1, target, &F->g, allocs, s);
}

}  // namespace trime
