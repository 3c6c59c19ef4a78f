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
  double* T;       // point values of every cell, 6n^2 x NP x 3
  double* Lam;     // their cotangents, same layout
  double* Dl;      // WENO: stencil cotangents, 6n^2 x K^2 x 3
  double* gpad;    // padded cotangent, 3 x 6 x P x P
  const int32_t* gt_ptr;   // G^T by interior cell: 6n^2 + 1
  const int32_t* gt_row;   // padded offset of the ghost cell
  const double* gt_val;    // 5 x nnz, same component order as G
  int64_t gt_nnz;
};
// the adjoint's kernels in launch order
enum { kVjpTraces = 0, kVjpPoints, kVjpEdges, kVjpWeno, kVjpGather, kVjpGhostT, kVjpSteps };
int launch_vjp(int k, int weno, const VjpArgs& a, int step, void* stream);

}  // namespace hope
