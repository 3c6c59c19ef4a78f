// C ABI of the HOPE right-hand side library (declared in include/hope.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <string>

#include "hope.h"
#include "grid_internal.hpp"
#include "vjp_internal.hpp"

using namespace hope;

namespace hope {
namespace {
thread_local std::string g_last_error;
}

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  return fail(HOPE_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e));
}

const char* last_error() { return g_last_error.c_str(); }
}  // namespace hope

namespace {
// kernels: 0 ghost fill, 1 edge traces, 2 stage
hipEvent_t next_event(hope_grid* G) {
  if (G->used == G->pool.size()) {
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    G->pool.push_back(e);
  }
  return G->pool[G->used++];
}

struct Timed {
  hope_grid* G;
  int kind;
  hipStream_t s;
  int a = -1;
  Timed(const hope_grid* g, int k, void* stream) : G(const_cast<hope_grid*>(g)), kind(k), s((hipStream_t)stream) {
    if (!G->timing || !((G->timing_mask >> kind) & 1u)) return;
    hipEvent_t e = next_event(G);
    if (!e) return;
    a = (int)G->used - 1;
    (void)hipEventRecord(e, s);
  }
  ~Timed() {
    if (a < 0) return;
    hipEvent_t e = next_event(G);
    if (!e) return;
    (void)hipEventRecord(e, s);
    G->recs.push_back({kind, a, (int)G->used - 1});
  }
};
// per-kernel timing whose two events the launches record themselves
// (launch_stage: hipExtLaunchKernel), so that timing adds no marker between
// kernels; off under stream capture
struct TimedLaunch {
  hope_grid* G;
  int kind;
  int a = -1, b = -1;
  hipEvent_t start = nullptr, stop = nullptr;
  TimedLaunch(const hope_grid* g, int k, void* stream) : G(const_cast<hope_grid*>(g)), kind(k) {
    if (!G->timing || !((G->timing_mask >> kind) & 1u)) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing((hipStream_t)stream, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    hipEvent_t e0 = next_event(G);
    if (!e0) return;
    const int i0 = (int)G->used - 1;
    hipEvent_t e1 = next_event(G);
    if (!e1) return;
    start = e0;
    stop = e1;
    a = i0;
    b = (int)G->used - 1;
  }
  // after a successful launch
  void done() {
    if (a >= 0) G->recs.push_back({kind, a, b});
  }
};
}  // namespace

// The grid's one mutable word: the counter of hope_check_state.  Every
// other scratch buffer of a call comes from the caller's workspace.
static int alloc_scratch(hope_grid* G) {
  const size_t bytes = 256;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) return hip_fail(e, "hipMalloc (check_state counter)");
  G->allocs.push_back(p);
  G->device_bytes += bytes;
  G->bad = static_cast<unsigned long long*>(p);
  return 0;
}

template <typename T>
static int upload(hope_grid* G, const std::vector<T>& v, const T** out) {
  *out = nullptr;
  if (v.empty()) return 0;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, v.size() * sizeof(T));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc");
  G->allocs.push_back(p);
  G->device_bytes += v.size() * sizeof(T);
  e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy");
  *out = static_cast<const T*>(p);
  return 0;
}

namespace hope {
bool build_fill_blocks(int rows, const int32_t* ptr, const int32_t* ent, size_t cells, int rb, int cap,
                       FillBlocks& out) {
  out = FillBlocks();
  if (rows == 0 || cap > 0xffff) return false;
  std::vector<int32_t> mark(cells, -1), seen(cells, -1), local(cells, 0);
  FillBlocks fb;
  fb.brow.push_back(0);
  fb.bptr.push_back(0);
  fb.lent.resize((size_t)ptr[rows]);
  int blk = 0, in_blk = 0, used = 0;
  for (int r = 0; r < rows; ++r) {
    int add = 0, distinct = 0;
    for (int32_t k = ptr[r]; k < ptr[r + 1]; ++k) {
      const int32_t c = ent[2 * (size_t)k], ce = ent[2 * (size_t)k + 1];
      if (c < 0 || (size_t)c >= cells || ce < 0 || ce > 0xffff) return false;
      if (seen[c] != r) {
        seen[c] = r;
        ++distinct;
        if (mark[c] != blk) ++add;
      }
    }
    if (distinct > cap) return false;
    if (in_blk > 0 && (in_blk == rb || used + add > cap)) {
      fb.brow.push_back(r);
      fb.bptr.push_back((int32_t)fb.bsrc.size());
      ++blk;
      in_blk = 0;
      used = 0;
    }
    for (int32_t k = ptr[r]; k < ptr[r + 1]; ++k) {
      const int32_t c = ent[2 * (size_t)k];
      if (mark[c] != blk) {
        mark[c] = blk;
        local[c] = used++;
        fb.bsrc.push_back(c);
      }
      fb.lent[k] = ((uint32_t)local[c] << 16) | (uint32_t)ent[2 * (size_t)k + 1];
    }
    fb.umax = std::max(fb.umax, used);
    ++in_blk;
  }
  fb.brow.push_back(rows);
  fb.bptr.push_back((int32_t)fb.bsrc.size());
  out = std::move(fb);
  return true;
}
}  // namespace hope

// The grid's own fill blocks: as many rows as one workgroup's lane groups take
// (fill_lds_threads / halo_lanes), at most 1024 cells (2048 from order 7) per block; without
// them (a row too long) the fill reads the state directly.
static int upload_fill_blocks(hope_grid* G) {
  const hope::HostTables& h = G->h;
  hope::FillBlocks fb;
  if (h.z_ptr.empty() ||
      !hope::build_fill_blocks((int)h.z_dst.size(), h.z_ptr.data(), h.z_ent.data(), (size_t)6 * h.P * h.P,
                               hope::fill_lds_threads(hope::halo_lanes(h.k)) / hope::halo_lanes(h.k),
                               h.k >= 7 ? 2048 : 1024, fb))
    return 0;
  hope::GhostDev& g = G->g;
  int e = upload(G, fb.brow, &g.brow);
  if (!e) e = upload(G, fb.bptr, &g.bptr);
  if (!e) e = upload(G, fb.bsrc, &g.bsrc);
  if (!e) e = upload(G, fb.lent, &g.lent);
  if (e) return e;
  g.blocks = (int)fb.brow.size() - 1;
  g.umax = fb.umax;
  return 0;
}

static void free_grid(hope_grid* G) {
  if (!G) return;
  for (hipEvent_t e : G->pool) (void)hipEventDestroy(e);
  for (void* p : G->allocs) (void)hipFree(p);
  delete G;
}

void hope::balanced_strip(int n, int* strip_w, int* strips) {
  *strips = (n + 61) / 62;
  *strip_w = (n + *strips - 1) / *strips;          // balance the strips
}

static void default_launch(hope_grid* G) {
  const int n = G->h.n;
  int sw, strips;
  balanced_strip(n, &sw, &strips);
  const bool seams = uses_seams(G->h);
  // half strips (<= kHalfStrip columns, 32 lanes each) when they leave fewer
  // lanes idle than full strips (64 lanes each), and with segment seams also
  // when they leave as many (twice the work items)
  const int hs = (n + kHalfStrip - 1) / kHalfStrip, hw = (n + hs - 1) / hs;
  if (sw > kHalfStrip && (32L * hs < 64L * strips || (seams && 32L * hs == 64L * strips))) {
    sw = hw;
    strips = hs;
  }
  G->strip_w = sw;
  int h;
  if (seams) {
    // short segments: with segment seams a boundary costs no reconstruction,
    // so the segments are 3 rows high where that still leaves about 4 work
    // items per workgroup slot of the chip (256 CUs x 4 resident workgroups
    // of the order-5 stage), else 2 (measured at C360 WENO5: (30, 3)
    // 0.242 ms, (30, 4) 0.244, (30, 2) 0.253, (60, 9) 0.30)
    h = 3;
    while (h > 2 && stage_items(sw, strips, (n + h - 1) / h) < 4000) --h;
  } else {
    // the tallest segments (fewest re-reconstructed boundary rows) that still
    // give about 1.4 work items per workgroup slot
    h = 12;
    while (h > 2 && stage_items(sw, strips, (n + h - 1) / h) < 1400) --h;
  }
  G->seg_h = std::min(h, n);
}

extern "C" {

const char* hope_last_error(void) { return last_error(); }

static int validate(const hope_grid_desc* desc) {
  if (desc->struct_size != (int32_t)sizeof(hope_grid_desc)) return fail(HOPE_ERR_INVALID, "struct_size mismatch");
  const int k = desc->order, n = desc->n;
  const int weno = desc->scheme;
  if (weno != HOPE_SCHEME_TPP && weno != HOPE_SCHEME_WENO) return fail(HOPE_ERR_INVALID, "bad scheme");
  if (k < 3 || k > kMaxOrder || k % 2 == 0) return fail(HOPE_ERR_UNSUPPORTED, "order must be odd, 3..13");
  if (weno && k > 5) return fail(HOPE_ERR_UNSUPPORTED, "WENO is built for orders 3 and 5");
  if (desc->n_gauss != 0 && desc->n_gauss != (k + 1) / 2)
    return fail(HOPE_ERR_UNSUPPORTED, "n_gauss must be (order+1)/2");
  if (n < k || n > 4096) return fail(HOPE_ERR_UNSUPPORTED, "n must satisfy order <= n <= 4096");
  if (!(desc->radius >= 0) || !std::isfinite(desc->axis_tilt) || !(desc->weno_eps >= 0))
    return fail(HOPE_ERR_INVALID, "bad physical parameter");
  if (desc->ghost_iters < 0 || desc->ghost_iters > 300)
    return fail(HOPE_ERR_INVALID, "ghost_iters must be 0 (fixed point) or 1..300 sweeps");
  return HOPE_OK;
}

int hope_grid_create(const hope_grid_desc* desc, hope_grid** out) {
  if (!desc || !out) return fail(HOPE_ERR_INVALID, "null argument");
  *out = nullptr;
  if (int v = validate(desc)) return v;
  const int k = desc->order, n = desc->n;
  const int weno = desc->scheme;
  const double radius = desc->radius > 0 ? desc->radius : 6.371e6;
  const double omega = desc->omega != 0 ? desc->omega : 7.292e-5;
  const double eps = desc->weno_eps > 0 ? desc->weno_eps : 1e-12;
  const double theta = desc->split_theta > 0 ? desc->split_theta : 3.0;
  hope_grid* G = new (std::nothrow) hope_grid;
  if (!G) return fail(HOPE_ERR_NOMEM, "host allocation");
  int st = 0;
  try {
    bool cached = false;
    st = build_tables_cached(G->h, desc->cache_dir, &cached, n, k, weno, radius, omega, desc->axis_tilt, eps, theta,
                             desc->ghost_iters);
    G->tables_cached = cached;
  } catch (const std::bad_alloc&) {
    free_grid(G);
    return fail(HOPE_ERR_NOMEM, "host allocation while building tables");
  }
  if (st) {
    std::string msg = G->h.error;
    free_grid(G);
    return fail(st, msg);
  }
  HostTables& h = G->h;
  {
    // pack the constant tables into one buffer (layout of tab_offsets)
    const TabOffsets O = tab_offsets(h.k, h.weno != 0, h.m, h.n);
    std::vector<double> tab(O.total, 0.0);
    auto put = [&](int64_t off, const std::vector<double>& v) { std::copy(v.begin(), v.end(), tab.begin() + off); };
    put(O.wc, h.wc);
    {
      std::vector<double> wd;
      derivative_weights(h.k, h.m, wd);
      put(O.wd, wd);
    }
    if (h.weno) {
      put(O.wsub, h.wsub);
      put(O.gp, h.gp);
      put(O.gm, h.gm);
      put(O.sp, h.sp);
      put(O.sm, h.sm);
      put(O.d1, h.d1);
      tab[O.theta] = h.theta;
      put(O.V, h.V);
      put(O.lam, h.lam);
    }
    put(O.gw, h.gw);
    put(O.fcoef, h.fcoef);
    put(O.Xe, h.Xe);
    put(O.sqe, h.sqe);
    put(O.Xg, h.Xg);
    put(O.sqg, h.sqg);
    put(O.bt_conv, h.bt_conv);
    std::vector<int32_t> itab(O.i_total, 0);
    std::copy(h.bt_cell.begin(), h.bt_cell.end(), itab.begin() + O.i_cell);
    std::copy(h.bt_side.begin(), h.bt_side.end(), itab.begin() + O.i_side);
    std::copy(h.bt_rev.begin(), h.bt_rev.end(), itab.begin() + O.i_rev);
    int e0 = upload(G, tab, &G->tab);
    if (!e0) e0 = upload(G, itab, &G->itab);
    if (e0) { free_grid(G); return e0; }
  }
  GridScalars& gsc = G->gs;
  gsc.radius = h.radius;
  gsc.omega2 = 2.0 * h.omega;
  gsc.eps = h.eps;
  gsc.inv_delta = 1.0 / h.delta;
  gsc.n = h.n;
  gsc.P = h.P;
  gsc.r = h.r;
  gsc.m = h.m;
  GhostDev& g = G->g;
  int e1 = upload(G, h.z_dst, &g.dst);
  if (!e1) e1 = upload(G, h.z_info, &g.info);
  if (!e1) e1 = upload(G, h.z_ptr, &g.ptr);
  const int32_t* ent = nullptr;
  const double* cval = nullptr;
  if (!e1) e1 = upload(G, h.z_ent, &ent);
  if (!e1) e1 = upload(G, h.z_cval, &cval);
  g.ent = reinterpret_cast<const GhostEnt*>(ent);       // device allocations are 256-byte aligned
  g.cval = reinterpret_cast<const GhostVal*>(cval);
  if (e1) { free_grid(G); return e1; }
  g.nnz = (int64_t)(h.z_ent.size() / 2);
  g.cnnz = (int64_t)(h.z_cval.size() / 6);
  g.rows = (int)h.z_dst.size();
  if (int eb = upload_fill_blocks(G)) { free_grid(G); return eb; }
  {
    // transpose of G, rows by interior cell (CSR over the cells it reads)
    const int n = h.n, P = h.P, r = h.r;
    const int cells = 6 * n * n;
    std::vector<int32_t> cnt(cells + 1, 0);
    auto cell_of = [&](int32_t off) {
      const int p = off / (P * P), jj = (off / P) % P - r, ii = off % P - r;
      return (p * n + jj) * n + ii;
    };
    for (int32_t col : h.g_col) cnt[cell_of(col) + 1]++;
    for (int c = 0; c < cells; ++c) cnt[c + 1] += cnt[c];
    const size_t nnz = h.g_col.size();
    std::vector<int32_t> rows(nnz), refs(nnz), fill(cnt.begin(), cnt.end() - 1);
    // each entry refers to the canonical value record of its G entry and
    // carries the two frame codes (the device rows hold the same entries in
    // the same column order)
    std::vector<int32_t> zrow(6 * (size_t)P * P, -1);
    for (size_t zr = 0; zr < h.z_dst.size(); ++zr) zrow[h.z_dst[zr]] = (int32_t)zr;
    for (size_t gr = 0; gr + 1 < h.g_ptr.size(); ++gr) {
      const int zr = zrow[h.g_dst[gr]];
      const int32_t info = h.z_info[zr], zb = h.z_ptr[zr];
      for (int32_t k = h.g_ptr[gr]; k < h.g_ptr[gr + 1]; ++k) {
        const int32_t col = h.z_ent[2 * (zb + (k - h.g_ptr[gr]))];
        const int32_t ce = h.z_ent[2 * (zb + (k - h.g_ptr[gr])) + 1];
        const int32_t rec = (info & 0x0fffffff) + (ce & 0x1fff);
        if (col != h.g_col[k] || rec >= (1 << 24)) {
          free_grid(G);
          return fail(HOPE_ERR_NUMERIC, "ghost map transpose: inconsistent rows");
        }
        const int c = cell_of(col);
        const int32_t pos = fill[c]++;
        rows[pos] = h.g_dst[gr];
        refs[pos] = rec | ((ce >> 13) << 24) | ((info >> 28) << 27);
      }
    }
    // keep only the cells some ghost row reads
    std::vector<int32_t> cptr(1, 0), ccell;
    for (int c = 0; c < cells; ++c)
      if (cnt[c + 1] > cnt[c]) {
        ccell.push_back(c);
        cptr.push_back(cnt[c + 1]);
      }
    G->gt_rows = (int32_t)ccell.size();
    int e2 = upload(G, cptr, &G->gt_ptr);
    if (!e2) e2 = upload(G, ccell, &G->gt_cell);
    if (!e2) e2 = upload(G, rows, &G->gt_row);
    if (!e2) e2 = upload(G, refs, &G->gt_ref);
    if (e2) { free_grid(G); return e2; }
    G->gt_nnz = (int64_t)nnz;
    // blocks of kGtCells rows of G^T with the distinct ghost cells they read
    // (kept only if every block fits kGtCap)
    {
      const int nrow = (int)ccell.size(), nblk = (nrow + kGtCells - 1) / kGtCells;
      std::vector<int32_t> bptr(1, 0), bsrc, mark(6 * (size_t)P * P, -1), local(6 * (size_t)P * P, 0);
      std::vector<uint16_t> lidx(nnz);
      bool ok = nrow > 0;
      int umax = 0;
      for (int b = 0; b < nblk && ok; ++b) {
        int used = 0;
        for (int32_t k = cptr[b * kGtCells]; k < cptr[std::min(nrow, (b + 1) * kGtCells)]; ++k) {
          const int32_t d = rows[k];
          if (mark[d] != b) {
            mark[d] = b;
            local[d] = used++;
            bsrc.push_back(d);
          }
          lidx[k] = (uint16_t)local[d];
        }
        if (used > kGtCap) ok = false;
        umax = std::max(umax, used);
        bptr.push_back((int32_t)bsrc.size());
      }
      if (ok) {
        int e3 = upload(G, bptr, &G->gt_bptr);
        if (!e3) e3 = upload(G, bsrc, &G->gt_bsrc);
        if (!e3) e3 = upload(G, lidx, &G->gt_lidx);
        // the blocks in order of the mean canonical record they read: the
        // records are shared by the 24 rotated images of a ghost row, so
        // blocks far apart on the cube read the same ones, and a contiguous
        // range of this list (one L2 domain's) reads a narrow band of them
        std::vector<double> key(nblk);
        for (int b = 0; b < nblk; ++b) {
          const int32_t lo = cptr[b * kGtCells], hi = cptr[std::min(nrow, (b + 1) * kGtCells)];
          double sum = 0;
          for (int32_t k = lo; k < hi; ++k) sum += (double)(refs[k] & 0xffffff);
          key[b] = sum / std::max(1, hi - lo);
        }
        std::vector<int32_t> order(nblk);
        for (int b = 0; b < nblk; ++b) order[b] = b;
        std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return key[x] < key[y]; });
        if (!e3) e3 = upload(G, order, &G->gt_border);
        if (e3) { free_grid(G); return e3; }
        G->gt_blocks = nblk;
        G->gt_umax = umax;
      }
    }
  }
  if (desc->surface_geopotential) {
    TopoHost th;
    std::string err;
    int et = 0;
    try {
      et = build_topography(h, desc->surface_geopotential, desc->surface_user, th, err);
    } catch (const std::bad_alloc&) {
      free_grid(G);
      return fail(HOPE_ERR_NOMEM, "host allocation while building the topography tables");
    }
    if (et) { free_grid(G); return fail(et, err); }
    int e4 = upload(G, th.sbar, &G->topo.sbar);
    if (!e4) e4 = upload(G, th.sx, &G->topo.sx);
    if (!e4) e4 = upload(G, th.sy, &G->topo.sy);
    if (!e4) e4 = upload(G, th.sc, &G->topo.sc);
    if (e4) { free_grid(G); return e4; }
  }
  int e3 = alloc_scratch(G);
  if (e3) { free_grid(G); return e3; }
  default_launch(G);
  hipError_t e;
  e = hipDeviceSynchronize();
  if (e != hipSuccess) { free_grid(G); return hip_fail(e, "hipDeviceSynchronize"); }
  // the device holds the ghost map and edge maps now; drop the host copies
  std::vector<int32_t>().swap(h.g_dst);
  std::vector<int32_t>().swap(h.g_ptr);
  std::vector<int32_t>().swap(h.g_col);
  std::vector<double>().swap(h.g_val);
  std::vector<int32_t>().swap(h.z_dst);
  std::vector<int32_t>().swap(h.z_info);
  std::vector<int32_t>().swap(h.z_ptr);
  std::vector<int32_t>().swap(h.z_ent);
  std::vector<double>().swap(h.z_cval);
  std::vector<double>().swap(h.bt_conv);
  *out = G;
  return HOPE_OK;
}

int hope_grid_derive(const hope_grid* base, double axis_tilt, hope_grid** out) {
  if (!base || !out) return fail(HOPE_ERR_INVALID, "null argument");
  *out = nullptr;
  if (!std::isfinite(axis_tilt)) return fail(HOPE_ERR_INVALID, "axis_tilt not finite");
  hope_grid* G = new (std::nothrow) hope_grid();
  if (!G) return fail(HOPE_ERR_NOMEM, "host allocation");
  // scalars and small tables of the base; the large device maps are shared
  const HostTables& b = base->h;
  HostTables& h = G->h;
  h.n = b.n; h.k = b.k; h.r = b.r; h.m = b.m; h.P = b.P; h.weno = b.weno; h.l = b.l; h.s = b.s;
  h.radius = b.radius; h.omega = b.omega; h.tilt = axis_tilt; h.eps = b.eps; h.theta = b.theta;
  h.delta = b.delta; h.ghost_sweeps = b.ghost_sweeps;
  h.fcoef.resize(18);
  coriolis_coefs(axis_tilt, h.fcoef.data());
  G->gs = base->gs;
  G->g = base->g;
  G->topo = base->topo;
  G->itab = base->itab;
  G->gt_rows = base->gt_rows;
  G->gt_cell = base->gt_cell;
  G->gt_ptr = base->gt_ptr;
  G->gt_row = base->gt_row;
  G->gt_ref = base->gt_ref;
  G->gt_blocks = base->gt_blocks;
  G->gt_umax = base->gt_umax;
  G->gt_bptr = base->gt_bptr;
  G->gt_bsrc = base->gt_bsrc;
  G->gt_lidx = base->gt_lidx;
  G->gt_border = base->gt_border;
  G->gt_nnz = base->gt_nnz;
  G->strip_w = base->strip_w;
  G->seg_h = base->seg_h;
  const TabOffsets O = tab_offsets(h.k, h.weno != 0, h.m, h.n);
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, sizeof(double) * O.total);
  if (e != hipSuccess) { free_grid(G); return hip_fail(e, "hipMalloc (derived tables)"); }
  G->allocs.push_back(p);
  G->device_bytes += sizeof(double) * O.total;
  e = hipMemcpy(p, base->tab, sizeof(double) * O.total, hipMemcpyDeviceToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(static_cast<double*>(p) + O.fcoef, h.fcoef.data(), 18 * sizeof(double), hipMemcpyHostToDevice);
  if (e != hipSuccess) { free_grid(G); return hip_fail(e, "hipMemcpy (derived tables)"); }
  G->tab = static_cast<const double*>(p);
  if (int e3 = alloc_scratch(G)) { free_grid(G); return e3; }
  e = hipDeviceSynchronize();
  if (e != hipSuccess) { free_grid(G); return hip_fail(e, "hipDeviceSynchronize"); }
  *out = G;
  return HOPE_OK;
}

void hope_grid_destroy(hope_grid* grid) {
  if (!grid) return;
  (void)hipDeviceSynchronize();
  free_grid(grid);
}

// adjoint scratch: point values T, their cotangents, the stencil cotangents
// (nD), padded cotangent, and with topography the cotangents of the mass
// derivatives at the cell nodes.  On large grids the stencil cotangents of a
// group of variables at a time (vjp_group: at most nT) reuse T's space: the
// point values are not read after the flux adjoints.
static size_t vjp_elems(const hope_grid* G, size_t* nT, size_t* nD, size_t* nG) {
  const HostTables& h = G->h;
  const size_t cells = 6ULL * h.n * h.n;
  const size_t np = 4 * h.m + h.m * h.m;
  *nT = cells * np * 3;
  *nD = vjp_grouped(h.n) ? 0 : cells * h.k * h.k * 3;
  *nG = 18ULL * h.P * h.P;
  const size_t nL = G->topo.sbar ? 2 * cells * h.m * h.m : 0;
  return 2 * *nT + *nD + *nG + nL;
}

int hope_grid_layout(const hope_grid* G, hope_layout* out) {
  if (!G || !out) return fail(HOPE_ERR_INVALID, "null argument");
  const HostTables& h = G->h;
  out->n = h.n;
  out->r = h.r;
  out->padded = h.P;
  out->n_gauss = h.m;
  out->state_elems = 18LL * h.P * h.P;
  out->interior_elems = 18LL * h.n * h.n;
  out->tendency_workspace_bytes = (int64_t)stage_ws_bytes(h, G->seg_h);
  out->rk_workspace_bytes = 2 * out->state_elems * (int64_t)sizeof(double) + out->tendency_workspace_bytes;
  {
    size_t nT, nD, nG;
    out->vjp_workspace_bytes = (int64_t)(vjp_elems(G, &nT, &nD, &nG) * sizeof(double));
  }
  out->rk_vjp_workspace_bytes = (2 * out->state_elems + 2 * out->interior_elems) * (int64_t)sizeof(double) +
                                std::max<int64_t>(out->vjp_workspace_bytes, out->tendency_workspace_bytes);
  out->ghost_cells = G->g.rows;
  out->ghost_nnz = G->g.nnz;
  out->device_bytes = (int64_t)G->device_bytes;
  out->ghost_sweeps = h.ghost_sweeps;
  out->tables_cached = G->tables_cached ? 1 : 0;
  out->fill_blocks = G->g.blocks;
  return HOPE_OK;
}

int hope_fill_halo(const hope_grid* G, double* q, void* stream) {
  if (!G || !q) return fail(HOPE_ERR_INVALID, "null argument");
  if (reinterpret_cast<uintptr_t>(q) % 8) return fail(HOPE_ERR_INVALID, "misaligned state");
  Timed tm(G, 0, stream);
  int e = launch_fill_halo(G->g, q, 6 * G->h.P * G->h.P, halo_lanes(G->h.k), stream);
  if (e) return hip_fail((hipError_t)e, "fill_halo launch");
  return HOPE_OK;
}

int hope_check_state(const hope_grid* G, const double* q, int64_t* n_bad, void* stream) {
  if (n_bad) *n_bad = 0;
  if (!G || !q) return fail(HOPE_ERR_INVALID, "null argument");
  if (reinterpret_cast<uintptr_t>(q) % 8) return fail(HOPE_ERR_INVALID, "misaligned state");
  hipStream_t s = (hipStream_t)stream;
  // the counter is the grid's: concurrent calls take turns (each ends with a
  // wait for its stream, so its counter use is over when it unlocks)
  std::lock_guard<std::mutex> lock(G->check_mu);
  hipError_t e = hipMemsetAsync(G->bad, 0, sizeof(unsigned long long), s);
  if (e != hipSuccess) return hip_fail(e, "check_state clear");
  int le = launch_check_state(q, G->h.n, G->h.r, G->bad, stream);
  if (le) return hip_fail((hipError_t)le, "check_state launch");
  unsigned long long count = 0;
  e = hipMemcpyAsync(&count, G->bad, sizeof(count), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "check_state read");
  if (n_bad) *n_bad = (int64_t)count;
  if (count) return fail(HOPE_ERR_NUMERIC, std::to_string(count) + " cells with a thickness that is not positive "
                                            "or a variable that is not finite");
  return HOPE_OK;
}

// one stage: ghost fill, panel-edge traces into bt (the caller's scratch of
// stage_ws_bytes: the traces, then the segment seams), fused stage kernel
// and, with seams, the seam kernel
static int run_stage(const hope_grid* G, double* q, const double* qn, double* out, int out_padded, double ca,
                     double cb, double cc, double* bt, void* stream) {
  int e;
  {
    Timed tm(G, 0, stream);
    e = launch_fill_halo(G->g, q, 6 * G->h.P * G->h.P, halo_lanes(G->h.k), stream);
  }
  if (e) return hip_fail((hipError_t)e, "fill_halo launch");
  {
    Timed tm(G, 1, stream);
    e = launch_edge_traces(G->h.k, G->h.weno, G->tab, G->itab, G->gs, q, bt, G->topo, stream);
  }
  if (e) return hip_fail((hipError_t)e, "edge_traces launch");
  {
    TimedLaunch tm(G, 2, stream);
    double* seam = uses_seams(G->h) ? bt + trace_bytes(G->h) / sizeof(double) : nullptr;
    e = launch_stage(G->h.k, G->h.weno, G->tab, G->itab, G->gs, q, qn, out, out_padded, ca, cb, cc, bt,
                     G->strip_w, G->seg_h, G->topo, seam, stream, tm.start, tm.stop);
    if (!e) tm.done();
  }
  if (e) return hip_fail((hipError_t)e, "stage launch");
  return HOPE_OK;
}

int hope_tendency(const hope_grid* G, double* q, double* dqdt, double* ws, size_t ws_bytes, void* stream) {
  if (!G || !q || !dqdt || !ws) return fail(HOPE_ERR_INVALID, "null argument");
  if (reinterpret_cast<uintptr_t>(q) % 8 || reinterpret_cast<uintptr_t>(dqdt) % 8 ||
      reinterpret_cast<uintptr_t>(ws) % 8)
    return fail(HOPE_ERR_INVALID, "misaligned buffer");
  if (ws_bytes < stage_ws_bytes(G->h, G->seg_h)) return fail(HOPE_ERR_INVALID, "workspace too small");
  return run_stage(G, q, nullptr, dqdt, 0, 0.0, 0.0, 1.0, ws, stream);
}

int hope_tendency_vjp(const hope_grid* G, double* q, const double* w, double* gq, double* ws, size_t ws_bytes,
                      void* stream) {
  if (!G || !q || !w || !gq || !ws) return fail(HOPE_ERR_INVALID, "null argument");
  if (reinterpret_cast<uintptr_t>(q) % 8 || reinterpret_cast<uintptr_t>(w) % 8 ||
      reinterpret_cast<uintptr_t>(gq) % 8 || reinterpret_cast<uintptr_t>(ws) % 8)
    return fail(HOPE_ERR_INVALID, "misaligned buffer");
  if (gq == w) return fail(HOPE_ERR_INVALID, "gq must not alias w");
  const HostTables& h = G->h;
  size_t nT, nD, nG;
  if (ws_bytes < vjp_elems(G, &nT, &nD, &nG) * sizeof(double)) return fail(HOPE_ERR_INVALID, "workspace too small");
  int e;
  {
    Timed tm(G, 0, stream);
    e = launch_fill_halo(G->g, q, 6 * h.P * h.P, halo_lanes(h.k), stream);
  }
  if (e) return hip_fail((hipError_t)e, "fill_halo launch");
  VjpArgs a;
  a.tab = G->tab;
  a.itab = G->itab;
  a.gs = G->gs;
  a.q = q;
  a.w = w;
  a.gq = gq;
  a.T = ws;
  a.Lam = ws + nT;
  a.Dl = vjp_grouped(h.n) ? ws : ws + 2 * nT;   // over T, or after T and its cotangents
  a.gpad = ws + 2 * nT + nD;
  a.gt_rows = G->gt_rows;
  a.gt_cell = G->gt_cell;
  a.gt_ptr = G->gt_ptr;
  a.gt_row = G->gt_row;
  a.gt_ref = G->gt_ref;
  a.gt_blocks = G->gt_blocks;
  a.gt_umax = G->gt_umax;
  a.gt_bptr = G->gt_bptr;
  a.gt_bsrc = G->gt_bsrc;
  a.gt_lidx = G->gt_lidx;
  a.gt_border = G->gt_border;
  a.gcval = G->g.cval;
  a.gt_nnz = G->gt_nnz;
  a.topo = G->topo;
  a.Lder = ws + 2 * nT + nD + nG;
  auto run = [&](int step) -> int {
    Timed tm(G, 3 + step, stream);
    return launch_vjp(h.k, h.weno, a, step, stream);
  };
  for (int step : {kVjpTraces, kVjpPoints, kVjpEdges})
    if ((e = run(step))) return hip_fail((hipError_t)e, "adjoint launch");
  // the stencil cotangents and the padded cotangent, a group of variables at
  // a time on large grids, all three at once on small ones
  const int group = vjp_grouped(h.n) ? vjp_group(h.k, h.m) : 3;
  for (int v0 = 0; v0 < 3; v0 += group) {
    a.v0 = v0;
    a.nv = std::min(group, 3 - v0);
    if ((e = run(kVjpWeno))) return hip_fail((hipError_t)e, "adjoint launch");
    if ((e = run(kVjpGather))) return hip_fail((hipError_t)e, "adjoint launch");
  }
  if ((e = run(kVjpGhostT))) return hip_fail((hipError_t)e, "adjoint launch");
  return HOPE_OK;
}

}  // extern "C"

// stage coefficients: q_{s+1} = a q_0 + b q_s + (cs dt) L(q_s)
void hope::rk_coefs(int scheme, double a[3], double b[3], double cs[3]) {
  if (scheme == HOPE_RK_SSP3) {
    a[0] = 0.0; b[0] = 1.0; cs[0] = 1.0;
    a[1] = 0.75; b[1] = 0.25; cs[1] = 0.25;
    a[2] = 1.0 / 3.0; b[2] = 2.0 / 3.0; cs[2] = 2.0 / 3.0;
  } else {
    a[0] = 0.0; b[0] = 1.0; cs[0] = 1.0 / 3.0;
    a[1] = 1.0; b[1] = 0.0; cs[1] = 0.5;
    a[2] = 1.0; b[2] = 0.0; cs[2] = 1.0;
  }
}

extern "C" {

int hope_rk_step_vjp(const hope_grid* G, double* q, double dt, int32_t scheme, const double* gout, double* gin,
                     double* ws, size_t ws_bytes, void* stream) {
  if (!G || !q || !gout || !gin || !ws) return fail(HOPE_ERR_INVALID, "null argument");
  if (scheme != HOPE_RK_SSP3 && scheme != HOPE_RK_WS3) return fail(HOPE_ERR_INVALID, "bad RK scheme");
  if (gin == gout) return fail(HOPE_ERR_INVALID, "gin must not alias gout");
  const size_t state = 18ULL * G->h.P * G->h.P, field = 18ULL * G->h.n * G->h.n;
  size_t nT, nD, nG;
  const size_t nv = vjp_elems(G, &nT, &nD, &nG);
  // the region after the two stage states and fields holds the adjoint's
  // scratch, and first the recomputed stages' traces and seams
  const size_t nr = std::max(nv, stage_ws_bytes(G->h, G->seg_h) / sizeof(double));
  if (ws_bytes < (2 * state + 2 * field + nr) * sizeof(double)) return fail(HOPE_ERR_INVALID, "workspace too small");
  if (reinterpret_cast<uintptr_t>(q) % 8 || reinterpret_cast<uintptr_t>(ws) % 8 ||
      reinterpret_cast<uintptr_t>(gout) % 8 || reinterpret_cast<uintptr_t>(gin) % 8)
    return fail(HOPE_ERR_INVALID, "misaligned buffer");
  if (!std::isfinite(dt)) return fail(HOPE_ERR_INVALID, "dt not finite");
  double a[3], b[3], c[3];
  rk_coefs(scheme, a, b, c);
  for (double& x : c) x *= dt;
  double* q1 = ws;
  double* q2 = ws + state;
  double* cur = ws + 2 * state;
  double* v = cur + field;
  double* vws = v + field;
  int st;
  // recompute the stage states (their panel-edge traces use the start of the
  // adjoint's scratch, which the reverse sweep overwrites only after them)
  if ((st = run_stage(G, q, nullptr, q1, 1, 0.0, b[0], c[0], vws, stream))) return st;
  if ((st = run_stage(G, q1, q, q2, 1, a[1], b[1], c[1], vws, stream))) return st;
  // reverse sweep: cur = dL/dq_{s+1}; gin accumulates dL/dq_0
  double* qs[3] = {q, q1, q2};
  int e = launch_combine(field, cur, gout, nullptr, nullptr, 1.0, 0.0, 0.0, stream);
  if (!e) e = launch_combine(field, gin, gout, nullptr, nullptr, 0.0, 0.0, 0.0, stream);
  if (e) return hip_fail((hipError_t)e, "combine launch");
  for (int s = 2; s >= 0; --s) {
    if ((st = hope_tendency_vjp(G, qs[s], cur, v, vws, nv * sizeof(double), stream))) return st;
    e = launch_combine(field, gin, gin, cur, nullptr, 1.0, a[s], 0.0, stream);         // gin += a_s cur
    if (!e) e = launch_combine(field, cur, cur, v, nullptr, b[s], c[s], 0.0, stream);  // cur = b_s cur + c_s v
    if (e) return hip_fail((hipError_t)e, "combine launch");
  }
  e = launch_combine(field, gin, gin, cur, nullptr, 1.0, 1.0, 0.0, stream);            // gin += cur (q_0 term)
  if (e) return hip_fail((hipError_t)e, "combine launch");
  return HOPE_OK;
}

int hope_rk_step(const hope_grid* G, double* q, double dt, int32_t scheme, double* ws, size_t ws_bytes,
                 void* stream) {
  if (!G || !q || !ws) return fail(HOPE_ERR_INVALID, "null argument");
  return rk_step_ws(G, q, dt, scheme, ws, ws_bytes, stream);
}

}  // extern "C"

size_t hope::rk_workspace_bytes(const hope_grid* G) {
  return 2 * 18ULL * G->h.P * G->h.P * sizeof(double) + stage_ws_bytes(G->h, G->seg_h);
}

int hope::rk_step_ws(const hope_grid* G, double* q, double dt, int scheme, double* ws, size_t ws_bytes,
                     void* stream) {
  if (scheme != HOPE_RK_SSP3 && scheme != HOPE_RK_WS3) return fail(HOPE_ERR_INVALID, "bad RK scheme");
  const size_t state = 18ULL * G->h.P * G->h.P;
  if (ws_bytes < 2 * state * sizeof(double) + stage_ws_bytes(G->h, G->seg_h))
    return fail(HOPE_ERR_INVALID, "workspace too small");
  if (reinterpret_cast<uintptr_t>(q) % 8 || reinterpret_cast<uintptr_t>(ws) % 8)
    return fail(HOPE_ERR_INVALID, "misaligned buffer");
  if (!std::isfinite(dt)) return fail(HOPE_ERR_INVALID, "dt not finite");
  double* w0 = ws;
  double* w1 = ws + state;
  double* bt = ws + 2 * state;
  double a[3], b[3], c[3];
  rk_coefs(scheme, a, b, c);
  for (double& x : c) x *= dt;
  int st;
  if ((st = run_stage(G, q, nullptr, w0, 1, a[0], b[0], c[0], bt, stream))) return st;
  if ((st = run_stage(G, w0, q, w1, 1, a[1], b[1], c[1], bt, stream))) return st;
  if ((st = run_stage(G, w1, q, q, 1, a[2], b[2], c[2], bt, stream))) return st;
  return HOPE_OK;
}

extern "C" {

int hope_grid_set_launch(hope_grid* G, int32_t strip_w, int32_t seg_h) {
  if (!G) return fail(HOPE_ERR_INVALID, "null argument");
  if (strip_w < 1 || strip_w > 62 || seg_h < 1 || seg_h > G->h.n)
    return fail(HOPE_ERR_INVALID, "launch shape out of range");
  G->strip_w = strip_w;
  G->seg_h = seg_h;
  return HOPE_OK;
}

int hope_grid_get_launch(const hope_grid* G, int32_t* strip_w, int32_t* seg_h) {
  if (!G || !strip_w || !seg_h) return fail(HOPE_ERR_INVALID, "null argument");
  *strip_w = G->strip_w;
  *seg_h = G->seg_h;
  return HOPE_OK;
}

int hope_grid_profile(hope_grid* G, int32_t enable) {
  if (!G) return fail(HOPE_ERR_INVALID, "null argument");
  const uint32_t all = (1u << (3 + kVjpSteps)) - 1u;
  uint32_t mask = 0;
  if (enable == 1) {
    mask = all;
  } else if (enable != 0) {
    if (!(enable & HOPE_PROFILE_SELECT) || ((uint32_t)enable & ~(uint32_t)HOPE_PROFILE_SELECT & ~all))
      return fail(HOPE_ERR_INVALID, "profile: 0, 1 or HOPE_PROFILE_SELECT | kernel bits");
    mask = (uint32_t)enable & all;
  }
  if (enable) {
    G->recs.clear();
    G->used = 0;
  }
  G->timing = enable != 0;
  G->timing_mask = mask;
  return HOPE_OK;
}

int hope_grid_profile_read(hope_grid* G, int32_t kernel, double* total_ms, int64_t* launches) {
  if (!G || !total_ms || !launches) return fail(HOPE_ERR_INVALID, "null argument");
  if (kernel < 0 || kernel > 2 + kVjpSteps) return fail(HOPE_ERR_INVALID, "bad kernel index");
  double tot = 0;
  int64_t cnt = 0;
  for (const auto& r : G->recs) {
    if (r.kind != kernel) continue;
    hipError_t e = hipEventSynchronize(G->pool[r.b]);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float ms = 0;
    e = hipEventElapsedTime(&ms, G->pool[r.a], G->pool[r.b]);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    tot += ms;
    ++cnt;
  }
  *total_ms = tot;
  *launches = cnt;
  return HOPE_OK;
}

int hope_inspect_ghost_map(const hope_grid_desc* desc, int64_t* rows, int64_t* nnz, int32_t* sweeps,
                           int32_t* dst, int32_t* ptr, int32_t* col, double* val) {
  if (!desc || !rows || !nnz) return fail(HOPE_ERR_INVALID, "null argument");
  if (int v = validate(desc)) return v;
  const int k = desc->order, n = desc->n;
  HostTables h;
  const double radius = desc->radius > 0 ? desc->radius : 6.371e6;
  int st = build_tables(h, n, k, desc->scheme, radius, 7.292e-5, 0.0, 1e-12, 3.0, desc->ghost_iters);
  if (st) return fail(st, h.error);
  *rows = (int64_t)h.g_dst.size();
  *nnz = (int64_t)h.g_col.size();
  if (sweeps) *sweeps = h.ghost_sweeps;
  if (dst) std::memcpy(dst, h.g_dst.data(), h.g_dst.size() * sizeof(int32_t));
  if (ptr) std::memcpy(ptr, h.g_ptr.data(), h.g_ptr.size() * sizeof(int32_t));
  if (col) std::memcpy(col, h.g_col.data(), h.g_col.size() * sizeof(int32_t));
  if (val) std::memcpy(val, h.g_val.data(), h.g_val.size() * sizeof(double));
  return HOPE_OK;
}

}  // extern "C"
