// The grid object behind the opaque hope_grid handle, and host helpers
// shared by the C ABI translation units.
#pragma once
#include <hip/hip_runtime.h>

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
  std::vector<void*> allocs;
  size_t device_bytes = 0;
  double* bt = nullptr;      // panel-edge trace scratch, 24*n*m*3
  unsigned long long* bad = nullptr;   // hope_check_state's counter, after bt
  int strip_w = 62, seg_h = 8;
  bool tables_cached = false;   // host tables read from a cache file
  // G^T by the interior cells some ghost row reads (adjoint of the ghost fill)
  int32_t gt_rows = 0;
  const int32_t* gt_cell = nullptr;
  const int32_t* gt_ptr = nullptr;
  const int32_t* gt_row = nullptr;
  const int32_t* gt_ref = nullptr;   // canonical value record and frame codes of each entry
  int64_t gt_nnz = 0;
  // optional per-kernel timing with HIP events on the launch stream
  bool timing = false;
  uint32_t timing_mask = 0;   // bit k: kernel index k is timed
  std::vector<hipEvent_t> pool;
  struct Rec { int kind; int a, b; };
  std::vector<Rec> recs;
  size_t used = 0;
};

namespace hope {
// set the thread's error message and return the code
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
const char* last_error();
// Runge-Kutta stage coefficients: q_{s+1} = a_s q^n + b_s q_s + (cs_s dt) L(q_s)
void rk_coefs(int scheme, double a[3], double b[3], double cs[3]);
// strips of at most 62 columns, balanced over n
void balanced_strip(int n, int* strip_w, int* strips);
}  // namespace hope
