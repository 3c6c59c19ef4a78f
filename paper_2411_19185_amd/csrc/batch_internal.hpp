// Internal declarations of the batched ensemble (batch.hip, batch_capi.cpp):
// members of one or several grids (uneven resolutions) advanced by one launch
// per kernel over all members.
#pragma once

#include "hope_internal.hpp"

namespace hope {

// One ensemble member, as the device sees it.  Offsets are in elements from
// the base pointers of a launch (states: q_all or one workspace state set;
// fields: the unpadded output).
struct BatchMember {
  const double* tab;        // the member's grid tables (shared by members of one grid)
  const int32_t* itab;
  const double* fcoef;      // this member's 6 x 3 Coriolis coefficients
  GridScalars gs;
  int64_t q_off;            // padded state [3][6][P][P]
  int64_t f_off;            // unpadded field [3][6][n][n]
  int64_t bt_off;           // panel-edge traces [24 n m][3]
  int32_t edge_begin;       // first flattened panel-edge side (multiple of 64)
  int32_t strip_w, seg_h, n_strips, n_segs;
  int32_t half;             // strip_w <= kHalfStrip: two strips per work item
  int32_t seam_block;       // first block of this member's records in the seam launch
  int64_t seam_off;         // segment seams at seam + seam_off (SeamLayout), or -1: none
};

// The members of one grid, for the ghost fill: rows of that grid's G are
// applied to all of its members while the row's entries are in registers.
struct BatchGrid {
  GhostDev g;
  int32_t row_begin;        // first flattened ghost row
  int32_t member_begin;     // into the member list grouped by grid
  int32_t member_count;
  int32_t P;
  // the LDS-staged fill: this grid's row blocks (as GhostDev.brow ..., at
  // most kHaloLdsCells cells each), the first in the launch's flattened list
  const int32_t* brow;
  const int32_t* bptr;
  const int32_t* bsrc;
  const uint32_t* lent;
  int32_t block_begin;
  int32_t blocks;
};

// One launch of a stage: q_{s+1} = ca q^n + cb q_s + cs * dt[member] * L(q_s)
// (cs alone when dt is null).
struct BatchStage {
  const double* in;         // base of the stage inputs (padded)
  const double* qn;         // base of q^n (padded) or null
  double* out;              // base of the outputs
  int32_t out_padded;       // 1: padded states at q_off, 0: fields at f_off
  double ca, cb, cs;
  const double* dt;         // per member, device, or null
  double* bt;               // base of the panel-edge trace scratch
  double* seam;             // base of the segment seams (or null)
};

// All enqueue on `stream`; return a hipError_t value.
// lanes: lanes per ghost row, halo_lanes(order) as in the single-grid fill
// with total_blocks > 0 the LDS-staged fill (each workgroup one row block of
// one grid, its members' cells staged kHaloLdsChunk members at a time; ucap:
// the longest cell list)
int launch_batch_fill_halo(const BatchGrid* grids, int n_grids, int total_rows, const int32_t* members_by_grid,
                           const BatchMember* members, double* base, int lanes, int total_blocks, int ucap,
                           void* stream);
// edge_member: the member of each block of 64 flattened panel-edge sides
int launch_batch_edge_traces(int k, int weno, const BatchMember* members, const int32_t* edge_member,
                             int total_edges, const double* in, double* bt, void* stream);
// the stage over all work items (one workgroup per item, or `blocks`
// persistent workgroups when 0 < blocks < n_items), then, with seam_blocks >
// 0, the segment seams of the members that have them (seam_member: the member
// of each block of 256 records; a member's records start on a block)
int launch_batch_stage(int k, int weno, const BatchMember* members, const int32_t* items, int n_items, int blocks,
                       const int32_t* seam_member, int seam_blocks, const BatchStage& st, void* stream);
constexpr int kSeamBlock = 256;

// members per ghost-fill pass (the accumulators of one pass live in
// registers): 8 measured 184 us per batched fill of the 64-member ensemble
// against 209 us for 16 (238 VGPRs, two wavefronts per SIMD) and 435 us for 32
#ifndef HOPE_HALO_CHUNK
#define HOPE_HALO_CHUNK 8
#endif
constexpr int kHaloChunk = HOPE_HALO_CHUNK;
// the LDS-staged batched fill stages kHaloLdsChunk members at a time, at most
// kHaloLdsCells cells per row block: 4 x 3 x 512 doubles = 48 KB of LDS per
// workgroup (a WENO5 ghost row reads up to 342 cells; rows that read more, from
// order 7, take the direct batched fill)
constexpr int kHaloLdsChunk = 4;
constexpr int kHaloLdsCells = 512;
// its workgroup size: kHaloLdsThreads / lanes rows per block (16 at 32 lanes).
// Neighbouring rows read mostly the same cells (at WENO5, blocks of 8 rows
// stage about 350 cells, blocks of 16 about 420), so twice the rows fit the
// same LDS and the CU holds twice the wavefronts
constexpr int kHaloLdsThreads = 512;

}  // namespace hope
