// Batched ensemble kernels (gfx950, FP64): one launch per kernel covers every
// member of an ensemble of uneven resolutions.  They run the same device
// bodies as the single-grid kernels (kernel_bodies.hpp), so a member's result
// is bitwise the one its own grid gives.
//
//  k_fill_halo_batch_lds  the same by row blocks, the cells a block reads
//                         staged in LDS for kHaloLdsChunk members at a time
//  k_fill_halo_batch      ghost fill g = G q (appendix (7.12)) of all members:
//                         one lane group per ghost row of a grid, applied to
//                         that grid's members while the row's entries sit in
//                         registers (G is read once per kHaloChunk members)
//  k_edge_traces_batch    panel-edge traces (3.26)-(3.29) of all members; each
//                         member's range is padded to 64 sides (whole
//                         wavefronts of lane groups)
//  k_stage_batch          the fused stage over a flattened list of work items
//                         (member, panel, strip, segment); with blocks < items
//                         it is persistent, each workgroup striding the list
//  k_stage_seams_batch    the segment seams of all members (WENO5, TPP9+)
#include <hip/hip_runtime.h>

#include "batch_internal.hpp"
#include "kernel_bodies.hpp"

namespace hope {

template <int LANES>
__global__ __launch_bounds__(256) void k_fill_halo_batch(const BatchGrid* __restrict__ grids, int n_grids,
                                                         int total_rows, const int32_t* __restrict__ mlist,
                                                         const BatchMember* __restrict__ mem,
                                                         double* __restrict__ base) {
  const int lb = xcd_block(blockIdx.x, gridDim.x);   // contiguous rows per L2 domain
  const int row = (int)((lb * (size_t)blockDim.x + threadIdx.x) / LANES);
  if (row >= total_rows) return;   // the whole lane group leaves together
  int gi = 0;
  while (gi + 1 < n_grids && grids[gi + 1].row_begin <= row) ++gi;
  const BatchGrid& bg = grids[gi];
  const GhostDev& g = bg.g;
  const int r = row - bg.row_begin;
  const int lane = threadIdx.x % LANES;
  const size_t plane = (size_t)6 * bg.P * bg.P;
  const int b = g.ptr[r], e = g.ptr[r + 1];
  const int d = g.dst[r];
  const int info = g.info[r];
  const GhostVal* cv = g.cval + (info & 0x0fffffff);
  for (int c0 = 0; c0 < bg.member_count; c0 += kHaloChunk) {
    const int cnt = min(kHaloChunk, bg.member_count - c0);
    double* qm[kHaloChunk];
#pragma unroll
    for (int t = 0; t < kHaloChunk; ++t) qm[t] = base + mem[mlist[bg.member_begin + c0 + min(t, cnt - 1)]].q_off;
    double acc[kHaloChunk][3];
#pragma unroll
    for (int t = 0; t < kHaloChunk; ++t) acc[t][0] = acc[t][1] = acc[t][2] = 0.0;
    for (int k = b + lane; k < e; k += LANES) {
      const GhostEnt en = g.ent[k];
      const int c = en.col;
      const int j = en.ce & 0x1fff, f = en.ce >> 13;
      const GhostVal cj = cv[j];
      const double v0 = cj.v[0];
      double w1, w2, w3, w4;   // the block rows acting on the cell's own frame
      frame_apply(f, cj.v[1], cj.v[2], w1, w2);
      frame_apply(f, cj.v[3], cj.v[4], w3, w4);
#pragma unroll
      for (int t = 0; t < kHaloChunk; ++t) {
        if (t < cnt) {
          const double* q = qm[t];
          const double a0 = q[c], a1 = q[plane + c], a2 = q[2 * plane + c];
          acc[t][0] = fma(v0, a0, acc[t][0]);
          acc[t][1] = fma(w1, a1, fma(w2, a2, acc[t][1]));
          acc[t][2] = fma(w3, a1, fma(w4, a2, acc[t][2]));
        }
      }
    }
#pragma unroll
    for (int t = 0; t < kHaloChunk; ++t) {
#pragma unroll
      for (int off = LANES / 2; off > 0; off >>= 1) {
        acc[t][0] += __shfl_xor(acc[t][0], off, LANES);
        acc[t][1] += __shfl_xor(acc[t][1], off, LANES);
        acc[t][2] += __shfl_xor(acc[t][2], off, LANES);
      }
      if (lane == 0 && t < cnt) {
        double* q = qm[t];
        double gu, gv;
        frame_apply(info >> 28, acc[t][1], acc[t][2], gu, gv);
        q[d] = acc[t][0];
        q[plane + d] = gu;
        q[2 * plane + d] = gv;
      }
    }
  }
}

// the batched fill by row blocks (BatchGrid.brow ...): workgroup lb takes one
// block of one grid; for each chunk of kHaloLdsChunk of that grid's members it
// stages their cells in LDS, then each row's lane group sums its entries from
// there, in the order of k_fill_halo_batch
template <int LANES>
__global__ __launch_bounds__(kHaloLdsThreads) void k_fill_halo_batch_lds(const BatchGrid* __restrict__ grids, int n_grids,
                                                             int total_blocks, int ucap,
                                                             const int32_t* __restrict__ mlist,
                                                             const BatchMember* __restrict__ mem,
                                                             double* __restrict__ base) {
  extern __shared__ double sq[];   // [kHaloLdsChunk][3][ucap]
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  if (lb >= total_blocks) return;   // the whole workgroup leaves together
  int gi = 0;
  while (gi + 1 < n_grids && grids[gi + 1].block_begin <= lb) ++gi;
  const BatchGrid& bg = grids[gi];
  const GhostDev& g = bg.g;
  const int b = lb - bg.block_begin;
  const int s0 = bg.bptr[b], U = bg.bptr[b + 1] - s0;
  const int row = bg.brow[b] + (int)threadIdx.x / LANES;
  const bool active = row < bg.brow[b + 1];   // uniform over a lane group
  const int lane = threadIdx.x % LANES;
  const size_t plane = (size_t)6 * bg.P * bg.P;
  const int kb = active ? g.ptr[row] : 0, ke = active ? g.ptr[row + 1] : 0;
  const int info = active ? g.info[row] : 0;
  const GhostVal* cv = g.cval + (info & 0x0fffffff);
  for (int c0 = 0; c0 < bg.member_count; c0 += kHaloLdsChunk) {
    const int cnt = min(kHaloLdsChunk, bg.member_count - c0);
    if (c0 > 0) __syncthreads();   // the previous chunk's LDS reads are done
    for (int x = threadIdx.x; x < cnt * U; x += blockDim.x) {
      const int t = x / U, u = x - t * U;
      const double* q = base + mem[mlist[bg.member_begin + c0 + t]].q_off;
      const int c = bg.bsrc[s0 + u];
      sq[(t * 3 + 0) * ucap + u] = q[c];
      sq[(t * 3 + 1) * ucap + u] = q[plane + c];
      sq[(t * 3 + 2) * ucap + u] = q[2 * plane + c];
    }
    __syncthreads();
    if (!active) continue;
    double acc[kHaloLdsChunk][3];
#pragma unroll
    for (int t = 0; t < kHaloLdsChunk; ++t) acc[t][0] = acc[t][1] = acc[t][2] = 0.0;
    for (int k = kb + lane; k < ke; k += LANES) {
      const uint32_t le = bg.lent[k];
      const int l = (int)(le >> 16), ce = (int)(le & 0xffffu);
      const int j = ce & 0x1fff, f = ce >> 13;
      const GhostVal cj = cv[j];
      const double v0 = cj.v[0];
      double w1, w2, w3, w4;   // the block rows acting on the cell's own frame
      frame_apply(f, cj.v[1], cj.v[2], w1, w2);
      frame_apply(f, cj.v[3], cj.v[4], w3, w4);
#pragma unroll
      for (int t = 0; t < kHaloLdsChunk; ++t) {
        if (t < cnt) {
          const double a0 = sq[(t * 3 + 0) * ucap + l], a1 = sq[(t * 3 + 1) * ucap + l],
                       a2 = sq[(t * 3 + 2) * ucap + l];
          acc[t][0] = fma(v0, a0, acc[t][0]);
          acc[t][1] = fma(w1, a1, fma(w2, a2, acc[t][1]));
          acc[t][2] = fma(w3, a1, fma(w4, a2, acc[t][2]));
        }
      }
    }
#pragma unroll
    for (int t = 0; t < kHaloLdsChunk; ++t) {
#pragma unroll
      for (int off = LANES / 2; off > 0; off >>= 1) {
        acc[t][0] += __shfl_xor(acc[t][0], off, LANES);
        acc[t][1] += __shfl_xor(acc[t][1], off, LANES);
        acc[t][2] += __shfl_xor(acc[t][2], off, LANES);
      }
      if (lane == 0 && t < cnt) {
        double* q = base + mem[mlist[bg.member_begin + c0 + t]].q_off;
        const int d = g.dst[row];
        double gu, gv;
        frame_apply(info >> 28, acc[t][1], acc[t][2], gu, gv);
        q[d] = acc[t][0];
        q[plane + d] = gu;
        q[2 * plane + d] = gv;
      }
    }
  }
}

template <int K, bool W, int M>
__global__ __launch_bounds__(64) void k_edge_traces_batch(const BatchMember* __restrict__ mem,
                                                           const int32_t* __restrict__ edge_member,
                                                           int total_edges, const double* __restrict__ in,
                                                           double* __restrict__ bt) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int idx = t / kEdgeLanes;   // one lane group per side
  if (idx >= total_edges) return;
  // every member's range starts on a multiple of 64 sides, so the member is
  // uniform over each wavefront
  const int mi = __builtin_amdgcn_readfirstlane(edge_member[idx / 64]);
  const BatchMember& bm = mem[mi];
  const int local = idx - bm.edge_begin;
  if (local >= 24 * bm.gs.n) return;   // the whole lane group leaves together
  edge_trace<K, W, M>((cdp)bm.tab, (cip)bm.itab, bm.gs, in + bm.q_off, bt + bm.bt_off, local, t % kEdgeLanes);
}

// the stage arguments of member mi in one launch
__device__ __forceinline__ StageArgs member_args(const BatchMember& bm, const BatchStage& S, int mi) {
  StageArgs A;
  A.q = S.in + bm.q_off;
  A.qn = S.qn ? S.qn + bm.q_off : nullptr;
  A.out = S.out + (S.out_padded ? bm.q_off : bm.f_off);
  A.bt = S.bt + bm.bt_off;
  A.ca = S.ca;
  A.cb = S.cb;
  A.cc = S.dt ? S.cs * S.dt[mi] : S.cs;
  A.out_padded = S.out_padded;
  A.strip_w = bm.strip_w;
  A.seg_h = bm.seg_h;
  A.n_strips = bm.n_strips;
  A.n_segs = bm.n_segs;
  A.half = bm.half;
  A.seam = (S.seam && bm.seam_off >= 0) ? S.seam + bm.seam_off : nullptr;
  return A;
}

// orders <= 5 fit 4 workgroups (3 wavefronts per SIMD) by LDS; the register
// allocation is held to that occupancy.  PERSIST: each workgroup strides the
// item list (fewer workgroups than items); else one item per workgroup, which
// keeps no loop state live across the stage body (no scratch at WENO5)
template <int K, bool W, int M, bool PERSIST>
__global__ __launch_bounds__(kStageThreads) __attribute__((amdgpu_waves_per_eu(K <= 5 ? 3 : 1))) void k_stage_batch(
    const BatchMember* __restrict__ mem, const int32_t* __restrict__ items, int n_items, BatchStage S) {
  __shared__ StageSmem<K, W, M> sm;
  auto run = [&](int it) {
    const int code = __builtin_amdgcn_readfirstlane(items[it]);
    const int mi = code >> 20, local = code & 0xFFFFF;
    const BatchMember& bm = mem[mi];
    const StageArgs A = member_args(bm, S, mi);
    stage_tile<K, W, M, false, kSeams<K, W, M>>(bm.tab, (cdp)bm.fcoef, bm.gs, A, local, sm);
  };
  if constexpr (PERSIST) {
    for (int it = blockIdx.x; it < n_items; it += gridDim.x) {
      if (it != (int)blockIdx.x) __syncthreads();   // the previous item's LDS reads are done
      run(it);
    }
  } else {
    run(blockIdx.x);   // the grid has exactly n_items workgroups
  }
}

// the segment seams of every member that has them: block b holds records
// (b - seam_block) 256 + thread of member seam_member[b]
template <int K, bool W, int M>
__global__ __launch_bounds__(kSeamBlock) void k_stage_seams_batch(const BatchMember* __restrict__ mem,
                                                                  const int32_t* __restrict__ seam_member,
                                                                  BatchStage S) {
  const int mi = __builtin_amdgcn_readfirstlane(seam_member[blockIdx.x]);
  const BatchMember& bm = mem[mi];
  const size_t idx = (size_t)(blockIdx.x - bm.seam_block) * kSeamBlock + threadIdx.x;
  if (idx >= (size_t)6 * (bm.n_segs - 1) * bm.gs.n) return;
  const StageArgs A = member_args(bm, S, mi);
  stage_seam<K, W, M>(bm.tab, bm.gs, A, idx);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
int launch_batch_fill_halo(const BatchGrid* grids, int n_grids, int total_rows, const int32_t* members_by_grid,
                           const BatchMember* members, double* base, int lanes, int total_blocks, int ucap,
                           void* stream) {
  if (total_rows == 0) return 0;
  const int threads = 256;
  if (lanes != 32 && lanes != 64) return (int)hipErrorInvalidValue;
  if (total_blocks > 0) {
    const int blocks = (total_blocks + kXcds - 1) / kXcds * kXcds;
    const size_t lds = (size_t)kHaloLdsChunk * 3 * ucap * sizeof(double);
    if (lanes == 64)
      hipLaunchKernelGGL(k_fill_halo_batch_lds<64>, dim3(blocks), dim3(kHaloLdsThreads), lds, (hipStream_t)stream,
                         grids, n_grids, total_blocks, ucap, members_by_grid, members, base);
    else
      hipLaunchKernelGGL(k_fill_halo_batch_lds<32>, dim3(blocks), dim3(kHaloLdsThreads), lds, (hipStream_t)stream,
                         grids, n_grids, total_blocks, ucap, members_by_grid, members, base);
    return (int)hipGetLastError();
  }
  int blocks = (int)(((size_t)total_rows * lanes + threads - 1) / threads);
  blocks = (blocks + kXcds - 1) / kXcds * kXcds;
  if (lanes == 64)
    hipLaunchKernelGGL(k_fill_halo_batch<64>, dim3(blocks), dim3(threads), 0, (hipStream_t)stream, grids, n_grids,
                       total_rows, members_by_grid, members, base);
  else
    hipLaunchKernelGGL(k_fill_halo_batch<32>, dim3(blocks), dim3(threads), 0, (hipStream_t)stream, grids, n_grids,
                       total_rows, members_by_grid, members, base);
  return (int)hipGetLastError();
}

template <int K, bool W, int M>
static int batch_edges_t(const BatchMember* members, const int32_t* edge_member, int total_edges, const double* in,
                         double* bt, void* stream) {
  hipLaunchKernelGGL((k_edge_traces_batch<K, W, M>), dim3((total_edges * kEdgeLanes + 63) / 64), dim3(64), 0,
                     (hipStream_t)stream, members, edge_member, total_edges, in, bt);
  return (int)hipGetLastError();
}

template <int K, bool W, int M>
static int batch_stage_t(const BatchMember* members, const int32_t* items, int n_items, int blocks,
                         const int32_t* seam_member, int seam_blocks, const BatchStage& st, void* stream) {
  if (blocks > 0 && blocks < n_items)
    hipLaunchKernelGGL((k_stage_batch<K, W, M, true>), dim3(blocks), dim3(kStageThreads), 0, (hipStream_t)stream,
                       members, items, n_items, st);
  else
    hipLaunchKernelGGL((k_stage_batch<K, W, M, false>), dim3(n_items), dim3(kStageThreads), 0, (hipStream_t)stream,
                       members, items, n_items, st);
  if constexpr (kSeams<K, W, M>) {
    if (seam_blocks > 0 && st.seam)
      hipLaunchKernelGGL((k_stage_seams_batch<K, W, M>), dim3(seam_blocks), dim3(kSeamBlock), 0,
                         (hipStream_t)stream, members, seam_member, st);
  }
  return (int)hipGetLastError();
}

#define HOPE_BATCH_DISPATCH(FN, ...)                  \
  do {                                                \
    if (!weno) {                                      \
      switch (k) {                                    \
        case 3: return FN<3, false, 2>(__VA_ARGS__);  \
        case 5: return FN<5, false, 3>(__VA_ARGS__);  \
        case 7: return FN<7, false, 4>(__VA_ARGS__);  \
        case 9: return FN<9, false, 5>(__VA_ARGS__);  \
        case 11: return FN<11, false, 6>(__VA_ARGS__);\
        case 13: return FN<13, false, 7>(__VA_ARGS__);\
      }                                               \
    } else {                                          \
      switch (k) {                                    \
        case 3: return FN<3, true, 2>(__VA_ARGS__);   \
        case 5: return FN<5, true, 3>(__VA_ARGS__);   \
      }                                               \
    }                                                 \
    return (int)hipErrorInvalidValue;                 \
  } while (0)

int launch_batch_edge_traces(int k, int weno, const BatchMember* members, const int32_t* edge_member,
                             int total_edges, const double* in, double* bt, void* stream) {
  if (total_edges == 0) return 0;
  HOPE_BATCH_DISPATCH(batch_edges_t, members, edge_member, total_edges, in, bt, stream);
}

int launch_batch_stage(int k, int weno, const BatchMember* members, const int32_t* items, int n_items, int blocks,
                       const int32_t* seam_member, int seam_blocks, const BatchStage& st, void* stream) {
  if (n_items == 0) return 0;
  HOPE_BATCH_DISPATCH(batch_stage_t, members, items, n_items, blocks, seam_member, seam_blocks, st, stream);
}

}  // namespace hope
