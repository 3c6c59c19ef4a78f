// Internal declarations of the adjoint (vjp.hip) of the HOPE right-hand side.
#pragma once

#include "hope_internal.hpp"

namespace hope {

// Arguments of the adjoint (vjp.hip)
// G^T rows (interior cells) per block of the LDS-staged transpose: one
// workgroup of 256 lanes, 16 per cell; at most kGtCap distinct ghost cells
// per block (48 KB of LDS)
constexpr int kGtCells = 16;
constexpr int kGtCap = 2048;

struct VjpArgs {
  const double* tab;
  const int32_t* itab;
  GridScalars gs;
  const double* q;
  const double* w;
  double* gq;
  double* T;       // point values of every cell, [NP][3][6n^2]
  double* Lam;     // their cotangents, same layout
  double* Dl;      // stencil cotangents of variables v0 .. v0+nv-1, [K^2][nv][6n^2] (on large grids
                   // over T, no longer read by then)
  double* gpad;    // padded cotangent, 3 x 6 x P x P
  // G^T by the interior cells that some ghost row reads (gt_rows of them)
  int32_t gt_rows;
  const int32_t* gt_cell;  // the interior cell of each row
  const int32_t* gt_ptr;   // rows + 1
  const int32_t* gt_row;   // padded offset (in one variable plane) of the ghost cell
  const int32_t* gt_ref;   // per entry: canonical value record | (frame code of the cell << 24)
                           // | (frame code of the ghost << 27), see GhostDev
  const GhostVal* gcval;   // canonical value records of the ghost map
  int64_t gt_nnz;
  // the LDS-staged transpose (gt_blocks = 0: the direct one), see hope_grid
  int32_t gt_blocks = 0, gt_umax = 0;
  const int32_t* gt_bptr = nullptr;
  const int32_t* gt_bsrc = nullptr;
  const uint16_t* gt_lidx = nullptr;
  const int32_t* gt_border = nullptr;
  TopoDev topo;            // bottom topography (null sbar: none)
  double* Lder;            // topography: cotangents of d(sqrtG phi_t)/dxi, /deta at the cell nodes,
                           // [2][m*m][6n^2]
  int v0 = 0, nv = 3;      // the variables of a kVjpWeno / kVjpGather launch
};
// whether the adjoint takes the stencil cotangents in groups of variables
// that fit in the point values' space (37 % less workspace at C360 WENO5);
// small grids take all three in one launch (third-size launches underfill
// the chip there: TPP11 C90 adjoint 0.435 -> 0.493 ms one by one)
inline bool vjp_grouped(int n) { return n >= 160; }
// variables per group: as many as have their stencil cotangents (k^2 per
// cell each) in the point values' space (3 (4m + m^2) per cell)
inline int vjp_group(int k, int m) {
  const int np3 = 3 * (4 * m + m * m);
  return 3 * k * k <= np3 ? 3 : (2 * k * k <= np3 ? 2 : 1);
}
// the adjoint's kernels in launch order (kVjpWeno and kVjpGather once per
// variable, in turn)
enum { kVjpTraces = 0, kVjpPoints, kVjpEdges, kVjpWeno, kVjpGather, kVjpGhostT, kVjpSteps };
int launch_vjp(int k, int weno, const VjpArgs& a, int step, void* stream);

}  // namespace hope
