// Launchers of the cell kernels (the kernels themselves: cells_k.hpp).
#include "cells_k.hpp"

namespace trime {

// ------------------------------------------------------------ launchers --
static int64_t clamp64(int64_t v, int64_t lo, int64_t hi) { return v < lo ? lo : (v > hi ? hi : v); }

// The queue passes get grids that grow with the point count (their queues
// hold a small fraction of the points), up to the sizes that fill the chip.
template <class T, class G, int MODE> static void launch_mode(const KArgs &a, hipStream_t s) {
  constexpr int FB = fast_block<T, MODE>();
  const uint32_t nb = (uint32_t)((a.n + FB - 1) / FB);
  const bool rec = g_launch_log != nullptr;
  if (a.ev0 && !rec) (void)hipEventRecord((hipEvent_t)a.ev0, s);
  launch<Cells<T, G, MODE, FAST_VMAX, FB>>(a, nb, s);
  if (a.ev1 && !rec) (void)hipEventRecord((hipEvent_t)a.ev1, s);
  const int wgrid = (int)clamp64(a.n / 512, 8, WAVE_GRID);
  const int cgrid = (MODE == MODE_CVD && sizeof(T) == 4) ? (int)clamp64(a.n / 128, 4, CENTROID_GRID) : 0;
  using Post = CellsPost<G, MODE, WAVE_VMAX>;
  launch<Post>(typename Post::Args{a, wgrid}, (uint32_t)(wgrid + cgrid), s);
  launch<CellsExact<G, MODE, REPLAY_VMAX, REPLAY_BLOCK>>(a, (uint32_t)clamp64(a.n / 8192, 2, 64), s);
}

template <class G> static void launch_g(const KArgs &a, int mode, hipStream_t s) {
  if (a.precision == TRIME_FP32) {
    if (mode == MODE_CELLS) launch_mode<float, G, MODE_CELLS>(a, s);
    else if (mode == MODE_EXTRACT) launch_mode<float, G, MODE_EXTRACT>(a, s);
    else launch_mode<float, G, MODE_CVD>(a, s);
  } else {
    if (mode == MODE_CELLS) launch_mode<double, G, MODE_CELLS>(a, s);
    else if (mode == MODE_EXTRACT) launch_mode<double, G, MODE_EXTRACT>(a, s);
    else launch_mode<double, G, MODE_CVD>(a, s);
  }
}

void launch_cells(const KArgs &a, int mode, int grid_bytes, hipStream_t s) {
  if (grid_bytes == 4)
    launch_g<float>(a, mode, s);
  else
    launch_g<double>(a, mode, s);
}

}  // namespace trime
