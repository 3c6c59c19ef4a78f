// Internal declarations shared by the host builder, the C ABI and the HIP
// kernels of the HOPE right-hand side.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace hope {

constexpr int kMaxOrder = 13;
constexpr int kMaxGauss = 7;
constexpr int kMaxPts = 4 * kMaxGauss + kMaxGauss * kMaxGauss;   // EQPs + CQPs of one cell
constexpr int kMaxSub = 9;                                          // WENO5 sub-stencils

// ---------------------------------------------------------------------------
// Host-side tables (built once per grid, long double inside, FP64 out)
// ---------------------------------------------------------------------------
struct HostTables {
  int n = 0, k = 0, r = 0, m = 0, P = 0, weno = 0, l = 0, s = 0;
  double radius = 0, omega = 0, tilt = 0, eps = 0, theta = 0;
  double delta = 0;
  // axis coordinates of one cell: [-1/2, +1/2, g_0 .. g_{m-1}]
  std::vector<double> gnode, gw;       // m
  std::vector<double> wc;              // (2+m) x k   centred TPP weights
  std::vector<double> wsub;            // l starts x (2+m) x l   sub-stencil weights
  std::vector<double> gp, gm, sp, sm;  // npts x s, npts x s, npts, npts
  std::vector<double> d1;              // (2+m) x l   1D linear weights d_s at each axis point
  std::vector<double> V;               // l starts x l x l   smoothness transform
  std::vector<double> lam;             // l x l   smoothness eigen-weights
  std::vector<double> Xe;              // n+1   X at cell edges
  std::vector<double> Xg;              // n x m X at Gauss nodes
  std::vector<double> sqe, sqg;        // sqrt(1 + X^2) at edges (n+1) and Gauss nodes (n x m)
  std::vector<double> fcoef;           // 6 x 3 Coriolis: f*delta = 2 Omega (c0 + cX X + cY Y)
  // ghost map, one row per ghost cell (same pattern for the 3 variables)
  std::vector<int32_t> g_dst;          // padded offset (within one variable plane) of the ghost
  std::vector<int32_t> g_ptr;          // row pointers
  std::vector<int32_t> g_col;          // padded offset of the interior cell
  std::vector<double> g_val;           // 5 x nnz: mass, C11, C12, C21, C22 (SoA)
  int ghost_sweeps = 0;
  // the same map in the form the ghost-fill kernels read: the cube's 24
  // rotations carry one quarter of panel 0's ghost ring (the canonical rows)
  // onto every ghost cell, so the values are stored once per canonical row
  // and every row keeps only its columns and a 16-bit reference per entry.
  // Rows are ordered for the L2 domains of the chip (see compress_ghost_map).
  std::vector<int32_t> z_dst;          // padded offset of the row's ghost
  std::vector<int32_t> z_info;         // start of its canonical row in z_cval | (output frame code << 28)
  std::vector<int32_t> z_ptr;          // row pointers
  std::vector<int32_t> z_ent;          // per entry: padded offset of the interior cell read (ascending in a
                                       // row), then entry within the canonical row | (frame code of the
                                       // cell's panel << 13)
  std::vector<double> z_cval;          // per canonical entry: mass, C11, C12, C21, C22, 0 (48 bytes)
  // panel-edge traces: for (panel A, side, t, h): the neighbour cell and point
  std::vector<int32_t> bt_cell;        // 6*4*n: padded offset of B's cell centre
  std::vector<int32_t> bt_side;        // 6*4*n: which side of B's cell (0 L,1 R,2 B,3 T)
  std::vector<int32_t> bt_rev;         // 6*4*n: 1 if the Gauss points run in reverse
  std::vector<double> bt_conv;         // 6*4*n*m*5: mass ratio, C11, C12, C21, C22
  std::string error;
};

// Coriolis coefficients of the 6 panels for a rotation axis tilted by tilt (18 values).
void coriolis_coefs(double tilt, double* out);

// d/dxi of the centred order-k weights at the 2+m axis points ((2+m) x k).
void derivative_weights(int k, int m, std::vector<double>& out);

// Bottom topography (section 2, (2.13)-(2.14)): the surface geopotential
// phi_s comes from a host function evaluated at unit vectors.
typedef void (*SurfaceFn)(int64_t count, const double* xyz, double* phis, void* user);
struct TopoHost {
  std::vector<double> sbar;   // 6 P P: cell averages of sqrtG phi_s; ghost cells: G applied to them
  std::vector<double> sx;     // 6 n (n+1) m: sqrtG phi_s at the x-edge Gauss points [p][j][edge i][h]
  std::vector<double> sy;     // 6 (n+1) n m: at the y-edge Gauss points [p][edge j][i][h]
  std::vector<double> sc;     // 6 n n m m: at the cell Gauss points [p][j][i][w (y node)][h (x node)]
};
// Builds the tables from the host ghost map of t (g_*, still present);
// returns 0 or a HOPE_ERR code with err set.
int build_topography(const HostTables& t, SurfaceFn fn, void* user, TopoHost& out, std::string& err);

// Builds every table; returns 0 on success, else a HOPE_ERR code with error set.
// ghost_iters: 0 for the fixed-point ghost map, N > 0 for N Jacobi sweeps from 0.
int build_tables(HostTables& t, int n, int k, int weno, double radius, double omega, double tilt,
                 double eps, double theta, int ghost_iters = 0);
// Identifies the build of the table code (cache files of other builds are ignored).
const char* tables_build_stamp();
// build_tables through an on-disk cache in dir (null or empty: no cache);
// *loaded tells whether the tables came from a cache file.
int build_tables_cached(HostTables& t, const char* dir, bool* loaded, int n, int k, int weno, double radius,
                        double omega, double tilt, double eps, double theta, int ghost_iters);

// ---------------------------------------------------------------------------
// All constant tables of a grid live in one FP64 buffer (and one int32
// buffer for the panel-edge map), so that a kernel carries one base pointer.
// Section offsets (in elements) depend on (order, scheme, n_gauss) for the
// fixed part and on n for the rest.
// ---------------------------------------------------------------------------
#if defined(__HIPCC__) || defined(__HIP__)
#define HOPE_HD __host__ __device__
#else
#define HOPE_HD
#endif

struct TabOffsets {
  int64_t wc, wd, wsub, gp, gm, sp, sm, d1, theta, V, lam, gw, fcoef, fixed;
  int64_t Xe, sqe, Xg, sqg, bt_conv, total;
  int64_t i_cell, i_side, i_rev, i_total;
};

HOPE_HD constexpr TabOffsets tab_offsets(int k, bool weno, int m, int n) {
  const int NA = 2 + m, NP = 4 * m + m * m, L = (k + 1) / 2, S = L * L;
  TabOffsets o{};
  o.wc = 0;
  o.wd = o.wc + NA * k;                 // derivative of the centred weights (topography)
  o.wsub = o.wd + NA * k;
  o.gp = o.wsub + (weno ? L * NA * L : 0);
  o.gm = o.gp + (weno ? NP * S : 0);
  o.sp = o.gm + (weno ? NP * S : 0);
  o.sm = o.sp + (weno ? NP : 0);
  o.d1 = o.sm + (weno ? NP : 0);
  o.theta = o.d1 + (weno ? NA * L : 0);
  o.V = o.theta + (weno ? 1 : 0);
  o.lam = o.V + (weno ? L * L * L : 0);
  o.gw = o.lam + (weno ? L * L : 0);
  o.fcoef = o.gw + m;
  o.fixed = o.fcoef + 18;
  o.Xe = o.fixed;
  o.sqe = o.Xe + (n + 1);
  o.Xg = o.sqe + (n + 1);
  o.sqg = o.Xg + (int64_t)n * m;
  o.bt_conv = o.sqg + (int64_t)n * m;
  o.total = o.bt_conv + 24LL * n * m * 5;
  o.i_cell = 0;
  o.i_side = 24LL * n;
  o.i_rev = 48LL * n;
  o.i_total = 72LL * n;
  return o;
}

// Axis points (0: -1/2, 1: +1/2, 2+h: Gauss node h) at which the 1D linear
// weights of genuine 2D WENO (tensor factors of gamma, (3.19)) have mixed
// signs: for order 5 the middle Gauss node (the cell centre); none for order
// 3.  Elsewhere every gamma of a point is positive and the split (3.20)-(3.21)
// reduces to the unsplit weights.  The host checks the computed weights
// against this rule when it builds a grid.
HOPE_HD constexpr bool weno_mixed_axis(int k, int m, int a) { return k == 5 && m % 2 == 1 && a == 2 + m / 2; }

// lanes that share one ghost row in the ghost-fill kernels: 32, or 64 from
// order 7 on, whose rows hold several hundred entries each (the single-grid
// and batched fills use the same count, so their sums agree bitwise)
HOPE_HD constexpr int halo_lanes(int k) { return k >= 7 ? 64 : 32; }

// workgroup size of the single grid's LDS-staged fill with `lanes` lanes per
// ghost row (fill_lds_threads(lanes) / lanes rows per block).  A block's
// staged cells grow far slower than its rows (neighbouring rows read mostly
// the same cells), so from order 7, where rows hold several hundred entries,
// blocks of 16 rows keep more wavefronts per CU for the same LDS; below, 8
// rows per block, since larger blocks leave CUs idle on small grids.  Each
// row's sums are the same whatever the block size.
HOPE_HD constexpr int fill_lds_threads(int lanes) { return lanes == 64 ? 1024 : 256; }

// Scalars every kernel needs.
struct GridScalars {
  double radius, omega2, eps, inv_delta;
  int n, P, r, m;
};

// Ghost map on the device in its rotation-compressed form (the z_* tables of
// HostTables).  A frame code f describes a cube rotation on one panel: the
// image of panel coordinates (X, Y) is (sx * (sw ? Y : X), sy * (sw ? X : Y))
// with sw = f & 1, sx = -1 if f & 2, sy = -1 if f & 4; contravariant momentum
// components map the same way.
struct alignas(8) GhostEnt {
  int32_t col;           // padded offset of the interior cell read
  int32_t ce;            // entry within the canonical row | (frame code << 13)
};
struct alignas(16) GhostVal {
  double v[6];           // mass, C11, C12, C21, C22, padding
};
struct GhostDev {
  const int32_t* dst;
  const int32_t* info;
  const int32_t* ptr;
  const GhostEnt* ent;
  const GhostVal* cval;
  int64_t nnz;           // entries of all rows
  int64_t cnnz;          // entries of the canonical rows
  int rows;
  // row blocks of the LDS-staged fill (blocks = 0: none): block b holds rows
  // brow[b] .. brow[b+1]-1, which read the interior cells bsrc[bptr[b] ..
  // bptr[b+1]) (offsets in variable 0 of the padded state, as GhostEnt.col);
  // lent[k] = entry k's ce (canonical value and frame code, 16 bits) | the
  // position of its cell in its block's list << 16; umax the longest list
  const int32_t* brow = nullptr;
  const int32_t* bptr = nullptr;
  const int32_t* bsrc = nullptr;
  const uint32_t* lent = nullptr;
  int blocks = 0;
  int umax = 0;
};

// Topography tables on the device (the TopoHost arrays); a null sbar means
// no topography.
struct TopoDev {
  const double* sbar = nullptr;
  const double* sx = nullptr;
  const double* sy = nullptr;
  const double* sc = nullptr;
};

// Strips of the fused stage of up to 30 columns (32 lanes with the two ring
// lanes) run two per workgroup, one in each half of its lanes, side by side
// over the same rows; wider strips take all 64 lanes.  Work items of a stage
// launch: (pair of strip columns, or strip column) x segment.
constexpr int kHalfStrip = 30;
inline int stage_items(int strip_w, int n_strips, int n_segs) {
  const int cols = 6 * n_strips;
  return (strip_w <= kHalfStrip ? (cols + 1) / 2 : cols) * n_segs;
}

// Segment seams.  Without them a segment reconstructs the top traces of the
// row below it and the bottom traces of the row above it, rows that the
// neighbouring segments reconstruct in full anyway.  With them (segments of
// at least 2 rows), the flux through each internal segment boundary e is
// left to the seam kernel: the segment below stores the top traces of row
// e-1 and that row's partial tendency (all but its top flux); the segment
// above stores the bottom traces of row e, the parts of row e's tendency
// other than its bottom flux (x-flux difference, sources) and its top flux.
// The seam kernel forms the boundary flux from the two traces with the same
// arithmetic and finishes both rows: results are bitwise those of the
// reconstructing path.  Record of panel p, boundary u (row e = u seg_h,
// 1 <= u < n_segs), column i: field f at seam[f NS + (p (n_segs-1) + u-1) n + i],
// NS = 6 (n_segs-1) n (neighbouring columns at neighbouring addresses).
struct SeamLayout {
  static constexpr int fields(int M) { return 6 * M + 11; }
  static constexpr int tt(int M, int h, int v) { return h * 3 + v; }            // top traces of row e-1
  static constexpr int tb(int M, int h, int v) { return 3 * M + h * 3 + v; }    // bottom traces of row e
  static constexpr int lo_acc(int M, int v) { return 6 * M + v; }               // row e-1 without its top flux
  static constexpr int hi_x(int M, int v) { return 6 * M + 3 + v; }             // row e: left minus right x flux
  static constexpr int hi_src(int M, int k) { return 6 * M + 6 + k; }           // row e: momentum sources
  static constexpr int hi_gt(int M, int v) { return 6 * M + 8 + v; }            // row e: its top flux
};
constexpr bool has_seams(int n, int seg_h) { return seg_h >= 2 && (n + seg_h - 1) / seg_h >= 2; }
constexpr size_t seam_elems(int n, int M, int seg_h) {
  return has_seams(n, seg_h) ? (size_t)SeamLayout::fields(M) * 6 * ((n + seg_h - 1) / seg_h - 1) * n : 0;
}

// Launchers implemented in kernels.hip.  All enqueue on `stream` and return a
// hipError_t value (0 on success).
// lanes: lanes per ghost row, halo_lanes(order)
int launch_fill_halo(const GhostDev& g, double* q, int plane, int lanes, void* stream);
// bad[0] += number of interior cells of the padded state q with variable 0 not
// positive and finite, or variables 1, 2 not finite; bad must be zeroed before
int launch_check_state(const double* q, int n, int r, unsigned long long* bad, void* stream);
int launch_combine(size_t len, double* out, const double* x, const double* y, const double* z, double a, double b,
                   double c, void* stream);
int launch_edge_traces(int k, int weno, const double* tab, const int32_t* itab, const GridScalars& gs,
                       const double* q, double* bt, const TopoDev& topo, void* stream);
// ev_start / ev_stop: null, or HIP events (hipEvent_t) that the launches
// record themselves (hipExtLaunchKernel): the start of the stage kernel and
// the end of the stage's last kernel, so that timing the stage adds no
// marker to the stream
int launch_stage(int k, int weno, const double* tab, const int32_t* itab, const GridScalars& gs,
                 const double* q, const double* qn, double* out, int out_padded, double ca, double cb, double cc,
                 const double* bt, int strip_w, int seg_h, const TopoDev& topo, double* seam, void* stream,
                 void* ev_start = nullptr, void* ev_stop = nullptr);

}  // namespace hope
