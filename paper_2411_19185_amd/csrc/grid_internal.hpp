// The grid object behind the opaque hope_grid handle, and host helpers
// shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>
#include <vector>

#include "hope.h"
#include "hope_internal.hpp"

struct hope_grid {
  hope::HostTables h;
  const double* tab = nullptr;     // all constant tables, see tab_offsets
  const int32_t* itab = nullptr;   // panel-edge map
  hope::GridScalars gs{};
  hope::GhostDev g{};
  hope::TopoDev topo{};            // bottom topography tables (null: none)
  std::vector<void*> allocs;
  size_t device_bytes = 0;
  unsigned long long* bad = nullptr;   // hope_check_state's counter
  mutable std::mutex check_mu;         // held by hope_check_state from clearing the counter to reading it
  int strip_w = 62, seg_h = 8;
  bool tables_cached = false;   // host tables read from a cache file
  // G^T by the interior cells some ghost row reads (adjoint of the ghost fill)
  int32_t gt_rows = 0;
  const int32_t* gt_cell = nullptr;
  const int32_t* gt_ptr = nullptr;
  const int32_t* gt_row = nullptr;
  const int32_t* gt_ref = nullptr;   // canonical value record and frame codes of each entry
  int64_t gt_nnz = 0;
  // blocks of kGtCells consecutive G^T rows for the LDS-staged transpose
  // (gt_blocks = 0: none): the distinct ghost cells block b reads are
  // gt_bsrc[gt_bptr[b] .. gt_bptr[b+1]), entry k's position in that list
  // gt_lidx[k], gt_umax the longest list; gt_border lists the blocks by the
  // mean index of the canonical value records they read (each L2 domain
  // takes a contiguous range of that list)
  int32_t gt_blocks = 0, gt_umax = 0;
  const int32_t* gt_bptr = nullptr;
  const int32_t* gt_bsrc = nullptr;
  const uint16_t* gt_lidx = nullptr;
  const int32_t* gt_border = nullptr;
  // optional per-kernel timing with HIP events on the launch stream
  bool timing = false;
  uint32_t timing_mask = 0;   // bit k: kernel index k is timed
  std::vector<hipEvent_t> pool;
  struct Rec { int kind; int a, b; };
  std::vector<Rec> recs;
  size_t used = 0;
};

namespace hope {
// Row blocks of an LDS-staged ghost fill (GhostDev.brow ...): consecutive
// device rows of a ghost map (CSR ptr over rows, ent = (col, ce) pairs, cols
// below cells), at most rb per block, closed early when the distinct interior
// cells they read would pass cap; lent packs each entry's ce with the position
// of its cell in its block's list.  Returns false (and leaves the vectors
// empty) when a row alone reads more than cap cells or an entry does not fit
// the packing.
struct FillBlocks {
  std::vector<int32_t> brow, bptr, bsrc;
  std::vector<uint32_t> lent;
  int umax = 0;
};
bool build_fill_blocks(int rows, const int32_t* ptr, const int32_t* ent, size_t cells, int rb, int cap,
                       FillBlocks& out);
// set the thread's error message and return the code
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
const char* last_error();
// Runge-Kutta stage coefficients: q_{s+1} = a_s q^n + b_s q_s + (cs_s dt) L(q_s)
void rk_coefs(int scheme, double a[3], double b[3], double cs[3]);
// strips of at most 62 columns, balanced over n
void balanced_strip(int n, int* strip_w, int* strips);
// one Runge-Kutta step of hope_rk_step with the workspace ws (stage states,
// then panel-edge traces); checks everything but the null pointers
int rk_step_ws(const hope_grid* G, double* q, double dt, int scheme, double* ws, size_t ws_bytes, void* stream);
// bytes of that workspace
size_t rk_workspace_bytes(const hope_grid* G);
// elements of the panel-edge trace scratch of one stage: 24 panel sides x n x m points x 3 variables
inline size_t trace_elems(const HostTables& h) { return 24 * (size_t)h.n * h.m * 3; }
// bytes of that scratch, rounded up to 256
inline size_t trace_bytes(const HostTables& h) { return (trace_elems(h) * sizeof(double) + 255) / 256 * 256; }
// whether the grid's stage uses segment seams: where a row's reconstruction
// is costly (WENO5, TPP9 and up).  At the cheaper orders the seam kernel and
// its stores cost more than the boundary rows they save (measured at C90:
// TPP3 0.072 -> 0.090, TPP5 0.108 -> 0.136, TPP7 0.186 -> 0.202 ms per RK
// step with seams; WENO5 C360 0.280 -> 0.242 and TPP11 C90 0.114 -> 0.082 ms
// per stage).
inline bool uses_seams(const HostTables& h) { return (h.weno && h.k == 5) || h.k >= 9; }
// bytes of one stage's scratch for segments of seg_h rows: the panel-edge
// traces, then (from byte trace_bytes) the segment seams, rounded up to 256
inline size_t stage_ws_bytes(const HostTables& h, int seg_h) {
  const size_t seams = uses_seams(h) ? seam_elems(h.n, h.m, seg_h) : 0;
  return trace_bytes(h) + (seams * sizeof(double) + 255) / 256 * 256;
}
}  // namespace hope
