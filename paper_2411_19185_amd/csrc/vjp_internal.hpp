// Internal declarations of the adjoint (vjp.hip) of the HOPE right-hand side.
#pragma once

#include "hope_internal.hpp"

namespace hope {

// Arguments of the adjoint (vjp.hip)
struct VjpArgs {
  const double* tab;
  const int32_t* itab;
  GridScalars gs;
  const double* q;
  const double* w;
  double* gq;
  double* T;       // point values of every cell, [NP][3][6n^2]
  double* Lam;     // their cotangents, same layout
  double* Dl;      // stencil cotangents: one variable [K^2][6n^2] (over T, no longer read by then),
                   // or all three [K^2][3][6n^2]
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
  TopoDev topo;            // bottom topography (null sbar: none)
  double* Lder;            // topography: cotangents of d(sqrtG phi_t)/dxi, /deta at the cell nodes,
                           // [2][m*m][6n^2]
  int var = -1;            // the variable of a kVjpWeno / kVjpGather launch (-1: all three)
};
// whether the adjoint takes the stencil cotangents one variable at a time
// (over the point values' space: 37 % less workspace at C360 WENO5 for
// about 2 % more time); small grids take all three in one launch, which
// measured 15 % faster at TPP11 C90 (launches a third the size underfill the
// chip there)
inline bool vjp_per_variable(int n) { return n >= 160; }
// the adjoint's kernels in launch order (kVjpWeno and kVjpGather once per
// variable, in turn)
enum { kVjpTraces = 0, kVjpPoints, kVjpEdges, kVjpWeno, kVjpGather, kVjpGhostT, kVjpSteps };
int launch_vjp(int k, int weno, const VjpArgs& a, int step, void* stream);

}  // namespace hope
