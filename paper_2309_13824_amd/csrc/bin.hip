// Launchers of the binning kernels (the kernels themselves: bin_k.hpp).
#include "bin_k.hpp"

namespace trime {

__global__ void k_fill_i32(int32_t *p, int64_t n, int32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

// Exclusive scan of in[0..n) into out[0..n], out[n] = total; skipped when
// cond is set and *cond == 0.
void scan_i32(const int32_t *in, int32_t *out, int64_t n, int32_t *tmp, hipStream_t s,
              const int32_t *cond) {
  int64_t nt = (n + SCAN_TILE - 1) / SCAN_TILE;
  if (nt == 0) nt = 1;
  ScanArgs A{in, out, n, nt, tmp, cond};
  launch<ScanTiles>(A, (uint32_t)nt, s);
  if (nt <= SCAN_FEW_TILES) {
    launch<ScanAddFew>(A, (uint32_t)nt, s);
    return;
  }
  launch<ScanSums>(A, 1, s);
  launch<ScanAdd>(A, (uint32_t)nt, s);
}

size_t scan_tmp_ints(int64_t n) { return (size_t)((n + SCAN_TILE - 1) / SCAN_TILE) + 2; }

void launch_bin(const KArgs &a, const GatherArgs &g, int64_t nkeys, int32_t *scan_tmp,
                hipStream_t s, int32_t reset) {
  const int B = 256;
  const uint32_t nb = (uint32_t)((a.n + B - 1) / B);
  // the fill is grid-stride: a grid that grows with the bin count, at most 1024
  const int64_t nf0 = (nkeys + 4 * B - 1) / (4 * B);
  const uint32_t nf = (uint32_t)(nf0 < 1024 ? nf0 : 1024);
  launch<FillCond>(FillCond::Args{a, a.bin_fill, nkeys, reset}, nf, s);
  launch<BinKeys>(a, nb, s);
  scan_i32(a.bin_fill, a.bin_start, nkeys, scan_tmp, s, a.cond);
  launch<BinScatter>(a, nb, s);
  launch<BinPlace>(BinPlace::Args{a, g}, nb, s);
  // the processing order from the flags in rank[]
  const int64_t nt = a.n > 0 ? (a.n + SCAN_TILE - 1) / SCAN_TILE : 1;
  if (nt <= SCAN_FEW_TILES) {
    const ScanArgs A{a.rank, a.perm, a.n, nt, scan_tmp, a.cond};
    launch<ScanTiles>(A, (uint32_t)nt, s);
    launch<OrderAdd>(OrderAdd::Args{a, A}, (uint32_t)nt, s);
  } else {
    scan_i32(a.rank, a.perm, a.n, scan_tmp, s, a.cond);
    launch<OrderScatter>(a, nb, s);
  }
}

// p[i] = i (grid-stride).
__global__ void k_iota_i32(int32_t *p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = (int32_t)i;
}

void launch_iota_i32(int32_t *p, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(k_iota_i32, dim3(256), dim3(256), 0, s, p, n);
}

void launch_fill_i32(int32_t *p, int64_t n, int32_t v, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_i32, dim3(256), dim3(256), 0, s, p, n, v);
}

}  // namespace trime
