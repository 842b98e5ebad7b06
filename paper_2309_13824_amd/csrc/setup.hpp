// Setup-side declarations: the geometry grid build, segment loops, boundary
// points and the automatic sizing field (grid.hip, segsdf.hip, sizing.hip,
// boundary.hip and the ABI).
#pragma once
#include <vector>

#include "launch.hpp"

namespace trime {

// Candidate lists over a cell grid (segsdf.hip): cell c lists, in ascending
// order, every item that can give the minimum of a Lipschitz function
// family for some point of the cell.
struct CandGrid {
  int nx, ny;
  double x0, y0, cw, ch;
  const int32_t *start, *cand;
};

// A closed segment loop and its candidate lists (the nearest segment).
struct SegTree {
  const double *v;  // device vertices of the loop
  int nv;
  CandGrid g;
};

// Automatic sizing (Eq. 8): boundary points s with lfs(s), and candidate
// lists for min over s of K |x - s| + lfs(s).
struct LfsField {
  const double *s, *lfs;
  int64_t ns;
  double K;
  CandGrid g;
};

// Geometry for the grid build (device copies of the primitive lists).
struct GridPrims {
  int nprims;
  const trime_prim *prims;
  const double *poly;
  const SegTree *segs;  // per primitive (device); used by SEGMENTS only
  LfsField auto_mu;     // automatic sizing
  trime_sizing sz;  // cent / holes point into device memory
  const double *cent;
  const int32_t *holes;
  int nx, ny;
  double x0, y0, dx, dy;
  int64_t n_total;
};

int64_t grid_partials(int nx, int ny);
const char *seg_tree_build(const double *d_v, int nv, double bx0, double by0, double bx1, double by1,
                           double target, SegTree *T, std::vector<void *> &allocs, hipStream_t s);
// boundary points of the geometry (boundary.hip, host): the dense set of
// App. A (each primitive's boundary sampled, the points within geps of the
// whole geometry's boundary kept) and its trimming
double geometry_sdf(const trime_geometry *geo, double x, double y);
std::vector<double> boundary_points(const trime_geometry *geo, double d_s, double geps);
std::vector<double> trim_boundary(const trime_geometry *geo, double d_s, double geps, const std::vector<double> &in);
// automatic sizing (sizing.hip): medial points of the ns device boundary
// points from their Voronoi cells clipped to box (written to medial, room
// for 2 ns points, compacted in order; count to *nm_host), their keep
// flags, lfs, and (F not null) the candidate lists of the field over gbox
const char *auto_sizing_build(const double *d_s, int64_t ns, const double box[4], const double gbox[4],
                              double r_nei, int n_thres, double K, double target, double *medial, uint8_t *keep,
                              double *lfs, int64_t *nm_host, LfsField *F, std::vector<void *> &allocs,
                              hipStream_t s);
void launch_grid_build(const GridPrims &g, int dtype_bytes, void *sdf, void *mu, uint8_t *cat,
                       float *hcell, trime_grid_scalars *scal, double *part, hipStream_t s);

}  // namespace trime
