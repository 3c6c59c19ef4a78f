// HIP kernels (gfx950, FP64) of the HOPE right-hand side on one grid; the
// bodies they run are in kernel_bodies.hpp.
//
//  k_fill_halo     ghost cells g = G q (appendix (7.12)); halo_lanes(k) lanes per ghost row
//  k_fill_halo_lds the same by blocks of rows, the cells a block reads staged in LDS
//  k_edge_traces   at every panel-edge Gauss point, the neighbour panel's own
//                  trace, converted into this panel's variables (3.26)-(3.29);
//                  one group of kEdgeLanes lanes per panel-edge cell side
//  k_stage         fused reconstruction, LMARS, quadrature, sources, tendency
//                  and Runge-Kutta combination; one marching work item per
//                  workgroup (a strip, or two strips of <= 30 columns)
//  k_stage_seams   the flux through each internal segment boundary and the
//                  two rows beside it (segments of >= 2 rows)
//  k_combine       out = a x + b y + c z (the Runge-Kutta adjoint)
//  k_check_state   count of interior cells with a thickness that is not positive
//                  or a variable that is not finite
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>

#include "kernel_bodies.hpp"

namespace hope {

// ---------------------------------------------------------------------------
// Ghost fill
// ---------------------------------------------------------------------------
template <int LANES>
__global__ __launch_bounds__(256) void k_fill_halo(GhostDev g, double* __restrict__ q, int plane) {
  // each L2 domain takes a contiguous range of rows (the rows are ordered for it)
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  const int row = (int)((lb * (size_t)blockDim.x + threadIdx.x) / LANES);
  if (row >= g.rows) return;   // the whole lane group leaves together
  halo_row<LANES>(g, q, plane, row, threadIdx.x % LANES);
}

// the same, a block of rows per workgroup (GhostDev.brow): the interior cells
// the block reads are first copied to LDS (3 x umax doubles), then each row's
// lane group sums its entries from there, in the order of k_fill_halo
template <int LANES>
__global__ __launch_bounds__(fill_lds_threads(LANES)) void k_fill_halo_lds(GhostDev g, double* __restrict__ q, int plane) {
  extern __shared__ double sq[];
  const int b = xcd_block(blockIdx.x, gridDim.x);
  if (b >= g.blocks) return;   // the whole workgroup leaves together
  const int s0 = g.bptr[b], U = g.bptr[b + 1] - s0;
  const double* q1 = q + plane;
  const double* q2 = q + 2 * (size_t)plane;
  double* l0 = sq;
  double* l1 = sq + g.umax;
  double* l2 = sq + 2 * g.umax;
  for (int u = threadIdx.x; u < U; u += blockDim.x) {
    const int c = g.bsrc[s0 + u];
    l0[u] = q[c];
    l1[u] = q1[c];
    l2[u] = q2[c];
  }
  __syncthreads();
  const int row = g.brow[b] + (int)threadIdx.x / LANES;
  if (row >= g.brow[b + 1]) return;   // the whole lane group leaves together
  halo_row_from<LANES>(g, q, plane, row, threadIdx.x % LANES, [&](int k, int& ce, double& a0, double& a1, double& a2) {
    const uint32_t le = g.lent[k];
    const int l = (int)(le >> 16);
    ce = (int)(le & 0xffffu);
    a0 = l0[l];
    a1 = l1[l];
    a2 = l2[l];
  });
}

// ---------------------------------------------------------------------------
// Panel-edge traces: bt[((A*4+side)*n + t)*m + h][var], in A's variables
// ---------------------------------------------------------------------------
template <int K, bool W, int M, bool TP>
__global__ __launch_bounds__(64) void k_edge_traces(const double* __restrict__ tab_, const int32_t* __restrict__ itab_,
                                                     GridScalars gs, const double* __restrict__ q,
                                                     double* __restrict__ bt, TopoDev tp) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  const int idx = t / kEdgeLanes;
  if (idx >= 24 * gs.n) return;   // the whole lane group leaves together
  edge_trace<K, W, M, TP>((cdp)tab_, (cip)itab_, gs, q, bt, idx, t % kEdgeLanes, tp);
}

// ---------------------------------------------------------------------------
// Fused stage kernel: one work item per workgroup
// ---------------------------------------------------------------------------
// segment seams where kSeams (uses_seams on the host); WENO5 is held to
// three wavefronts per SIMD, the occupancy its workgroup's LDS allows (the
// seam stores would otherwise raise its allocation past it)

template <int K, bool W, int M, bool TP>
__global__ __launch_bounds__(kStageThreads) __attribute__((amdgpu_waves_per_eu((W && K == 5) ? 3 : 1))) void k_stage(
    const double* __restrict__ tab_, GridScalars gs, StageArgs A) {
  using C = Cfg<K, W, M>;
  __shared__ StageSmem<K, W, M, TP> sm;
  stage_tile<K, W, M, TP, kSeams<K, W, M>>(tab_, (cdp)tab_ + C::O.fcoef, gs, A, blockIdx.x, sm);
}

template <int K, bool W, int M, bool TP>
__global__ __launch_bounds__(256) void k_stage_seams(const double* __restrict__ tab_, GridScalars gs, StageArgs A,
                                                     size_t records) {
  const size_t idx = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= records) return;
  stage_seam<K, W, M, TP>(tab_, gs, A, idx);
}

// ---------------------------------------------------------------------------
// out = a x + b y + c z (unpadded fields; y, z may be null when b, c are 0)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_combine(size_t len, double* __restrict__ out, const double* x,
                                                  const double* y, const double* z, double a, double b, double c) {
  const size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= len) return;
  double v = a * x[k];
  if (y) v = fma(b, y[k], v);
  if (z) v = fma(c, z[k], v);
  out[k] = v;
}

int launch_combine(size_t len, double* out, const double* x, const double* y, const double* z, double a, double b,
                   double c, void* stream) {
  if (len == 0) return 0;
  hipLaunchKernelGGL(k_combine, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, (hipStream_t)stream, len, out, x,
                     y, z, a, b, c);
  return (int)hipGetLastError();
}

// ---------------------------------------------------------------------------
// Count of interior cells outside the system's domain (see launch_check_state)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_check_state(const double* __restrict__ q, int n, int r,
                                                      unsigned long long* __restrict__ bad) {
  const int P = n + 2 * r;
  const size_t nn = (size_t)n * n, cells = 6 * nn, plane = 6 * (size_t)P * P;
  unsigned long long cnt = 0;
  for (size_t c = (size_t)blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += (size_t)gridDim.x * blockDim.x) {
    const size_t f = c / nn, rem = c - f * nn;
    const size_t j = rem / n, i = rem - j * n;
    const size_t o = (f * P + j + r) * P + i + r;
    const double h = q[o], mu = q[o + plane], mv = q[o + 2 * plane];
    const bool ok = h > 0.0 && h <= DBL_MAX && fabs(mu) <= DBL_MAX && fabs(mv) <= DBL_MAX;
    cnt += ok ? 0 : 1;
  }
  if (cnt) atomicAdd(bad, cnt);
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
int launch_check_state(const double* q, int n, int r, unsigned long long* bad, void* stream) {
  const size_t cells = 6 * (size_t)n * n;
  const int blocks = (int)std::min<size_t>((cells + 255) / 256, 2048);
  hipLaunchKernelGGL(k_check_state, dim3(blocks), dim3(256), 0, (hipStream_t)stream, q, n, r, bad);
  return (int)hipGetLastError();
}

int launch_fill_halo(const GhostDev& g, double* q, int plane, int lanes, void* stream) {
  if (g.rows == 0) return 0;
  if (lanes != 32 && lanes != 64) return (int)hipErrorInvalidValue;
  const int threads = 256;
  if (g.blocks > 0) {
    const int blocks = (g.blocks + kXcds - 1) / kXcds * kXcds;
    const size_t lds = (size_t)3 * g.umax * sizeof(double);
    const dim3 t(fill_lds_threads(lanes));
    if (lanes == 64)
      hipLaunchKernelGGL(k_fill_halo_lds<64>, dim3(blocks), t, lds, (hipStream_t)stream, g, q, plane);
    else
      hipLaunchKernelGGL(k_fill_halo_lds<32>, dim3(blocks), t, lds, (hipStream_t)stream, g, q, plane);
    return (int)hipGetLastError();
  }
  int blocks = (int)(((size_t)g.rows * lanes + threads - 1) / threads);
  blocks = (blocks + kXcds - 1) / kXcds * kXcds;
  if (lanes == 64)
    hipLaunchKernelGGL(k_fill_halo<64>, dim3(blocks), dim3(threads), 0, (hipStream_t)stream, g, q, plane);
  else
    hipLaunchKernelGGL(k_fill_halo<32>, dim3(blocks), dim3(threads), 0, (hipStream_t)stream, g, q, plane);
  return (int)hipGetLastError();
}

template <int K, bool W, int M>
static int edge_traces_t(const double* tab, const int32_t* itab, const GridScalars& gs, const double* q, double* bt,
                         const TopoDev& tp, void* stream) {
  const int total = 24 * gs.n;
  const dim3 grid((total * kEdgeLanes + 63) / 64);
  if (tp.sbar)
    hipLaunchKernelGGL((k_edge_traces<K, W, M, true>), grid, dim3(64), 0, (hipStream_t)stream, tab, itab, gs, q, bt,
                       tp);
  else
    hipLaunchKernelGGL((k_edge_traces<K, W, M, false>), grid, dim3(64), 0, (hipStream_t)stream, tab, itab, gs, q, bt,
                       tp);
  return (int)hipGetLastError();
}

template <int K, bool W, int M>
static int stage_t(const double* tab, const GridScalars& gs, const StageArgs& a_in, void* stream, void* ev_start,
                   void* ev_stop) {
  StageArgs a = a_in;
  if constexpr (!kSeams<K, W, M>) a.seam = nullptr;   // the kernel is compiled without them
  const int items = stage_items(a.strip_w, a.n_strips, a.n_segs);
  const hipStream_t s = (hipStream_t)stream;
  const hipEvent_t e0 = (hipEvent_t)ev_start, e1 = (hipEvent_t)ev_stop;
  const bool seams = a.seam != nullptr;
  if (a.tp.sbar)
    hipExtLaunchKernelGGL((k_stage<K, W, M, true>), dim3(items), dim3(kStageThreads), 0, s, e0, seams ? nullptr : e1,
                          0, tab, gs, a);
  else
    hipExtLaunchKernelGGL((k_stage<K, W, M, false>), dim3(items), dim3(kStageThreads), 0, s, e0, seams ? nullptr : e1,
                          0, tab, gs, a);
  if constexpr (kSeams<K, W, M>) {
    if (seams) {
      const size_t records = (size_t)6 * (a.n_segs - 1) * gs.n;
      const dim3 grid((unsigned)((records + 255) / 256));
      if (a.tp.sbar)
        hipExtLaunchKernelGGL((k_stage_seams<K, W, M, true>), grid, dim3(256), 0, s, nullptr, e1, 0, tab, gs, a,
                              records);
      else
        hipExtLaunchKernelGGL((k_stage_seams<K, W, M, false>), grid, dim3(256), 0, s, nullptr, e1, 0, tab, gs, a,
                              records);
    }
  }
  return (int)hipGetLastError();
}

#define HOPE_DISPATCH(FN, ...)                                    \
  do {                                                            \
    if (!weno) {                                                  \
      switch (k) {                                                \
        case 3: return FN<3, false, 2>(__VA_ARGS__);              \
        case 5: return FN<5, false, 3>(__VA_ARGS__);              \
        case 7: return FN<7, false, 4>(__VA_ARGS__);              \
        case 9: return FN<9, false, 5>(__VA_ARGS__);              \
        case 11: return FN<11, false, 6>(__VA_ARGS__);            \
        case 13: return FN<13, false, 7>(__VA_ARGS__);            \
      }                                                           \
    } else {                                                      \
      switch (k) {                                                \
        case 3: return FN<3, true, 2>(__VA_ARGS__);               \
        case 5: return FN<5, true, 3>(__VA_ARGS__);               \
      }                                                           \
    }                                                             \
    return (int)hipErrorInvalidValue;                             \
  } while (0)

int launch_edge_traces(int k, int weno, const double* tab, const int32_t* itab, const GridScalars& gs,
                       const double* q, double* bt, const TopoDev& topo, void* stream) {
  HOPE_DISPATCH(edge_traces_t, tab, itab, gs, q, bt, topo, stream);
}

int launch_stage(int k, int weno, const double* tab, const int32_t* itab, const GridScalars& gs, const double* q,
                 const double* qn, double* out, int out_padded, double ca, double cb, double cc, const double* bt,
                 int strip_w, int seg_h, const TopoDev& topo, double* seam, void* stream, void* ev_start,
                 void* ev_stop) {
  (void)itab;
  StageArgs a;
  a.tp = topo;
  a.q = q;
  a.qn = qn;
  a.out = out;
  a.bt = bt;
  a.ca = ca;
  a.cb = cb;
  a.cc = cc;
  a.out_padded = out_padded;
  a.strip_w = strip_w;
  a.seg_h = seg_h;
  a.n_strips = (gs.n + strip_w - 1) / strip_w;
  a.n_segs = (gs.n + seg_h - 1) / seg_h;
  a.half = strip_w <= kHalfStrip;
  // seams only where the scratch is sized for them (segments of >= 2 rows,
  // >= 2 segments) and the kernel is compiled with them
  a.seam = has_seams(gs.n, seg_h) ? seam : nullptr;
  HOPE_DISPATCH(stage_t, tab, gs, a, stream, ev_start, ev_stop);
}

}  // namespace hope
