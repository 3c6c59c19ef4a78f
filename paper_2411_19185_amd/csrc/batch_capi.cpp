// C ABI of the batched ensemble (declared in include/hope.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "batch_internal.hpp"
#include "grid_internal.hpp"
#include "hope.h"

using namespace hope;

struct hope_batch {
  int n_members = 0, n_grids = 0, k = 0, weno = 0, m = 0;
  std::vector<const hope_grid*> member_grid;   // per member
  std::vector<const hope_grid*> grids;         // distinct grids, in order of first use
  std::vector<int64_t> q_off, f_off;           // per member
  int64_t state_elems = 0, field_elems = 0, bt_elems = 0;
  int total_rows = 0, total_edges = 0, n_items = 0, blocks = 0;
  int fill_blocks = 0, fill_ucap = 0;          // the LDS-staged fill (0: the direct one)
  std::vector<BatchMember> hmem;               // host copy of the member table
  BatchMember* mem = nullptr;
  BatchGrid* dgrids = nullptr;
  int32_t* mlist = nullptr;
  int32_t* edge_member = nullptr;              // member of each block of 64 panel-edge sides
  int32_t* items = nullptr;
  double* fcoef = nullptr;
  double* bt = nullptr;
  // segment seams (orders that use them): the buffer grows to what the launch
  // shapes need; seam_member gives the member of each block of the seam launch
  bool seams = false;
  double* seam = nullptr;
  size_t seam_cap = 0;
  int32_t* seam_member = nullptr;
  int seam_blocks = 0;
  std::vector<void*> allocs;
  // set once a stage has been recorded into a graph under stream capture: the
  // graph holds the work-item list and member table, so they stay fixed
  mutable bool captured = false;
};

namespace {

void free_batch(hope_batch* B) {
  if (!B) return;
  for (void* p : B->allocs) (void)hipFree(p);
  if (B->items) (void)hipFree(B->items);
  if (B->seam) (void)hipFree(B->seam);
  if (B->seam_member) (void)hipFree(B->seam_member);
  delete B;
}

template <typename T>
int upload_vec(hope_batch* B, const std::vector<T>& v, T** out) {
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(1, v.size()) * sizeof(T));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc (batch)");
  B->allocs.push_back(p);
  if (!v.empty()) {
    e = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy (batch)");
  }
  *out = static_cast<T*>(p);
  return HOPE_OK;
}

// work items (member << 20 | local item), costliest items first so that the
// tail of the launch is made of small ones
int build_items(hope_batch* B) {
  struct It { int64_t cost; int32_t code; };
  std::vector<It> its;
  for (int i = 0; i < B->n_members; ++i) {
    const BatchMember& bm = B->hmem[i];
    const int per = stage_items(bm.strip_w, bm.n_strips, bm.n_segs);
    if (per > (1 << 20)) return fail(HOPE_ERR_INVALID, "too many work items in one member");
    const int64_t cost = (int64_t)(bm.seg_h + 1) * (bm.half ? 64 : bm.strip_w + 2);
    for (int l = 0; l < per; ++l) its.push_back({cost, (int32_t)((i << 20) | l)});
  }
  std::stable_sort(its.begin(), its.end(), [](const It& a, const It& b) { return a.cost > b.cost; });
  std::vector<int32_t> codes(its.size());
  for (size_t t = 0; t < its.size(); ++t) codes[t] = its[t].code;
  if (B->items) (void)hipFree(B->items);
  B->items = nullptr;
  void* p = nullptr;
  hipError_t e = hipMalloc(&p, std::max<size_t>(1, codes.size()) * sizeof(int32_t));
  if (e != hipSuccess) return hip_fail(e, "hipMalloc (batch items)");
  B->items = static_cast<int32_t*>(p);
  if (!codes.empty()) {
    e = hipMemcpy(p, codes.data(), codes.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy (batch items)");
  }
  B->n_items = (int)codes.size();
  return HOPE_OK;
}

// the members' segment seams at their current launch shapes: offsets into
// the seam buffer (grown when needed) and the member of each block of 256
// records.  Run only when no queued work can still read the old ones.
int build_seams(hope_batch* B) {
  B->seam_blocks = 0;
  std::vector<int32_t> owner;
  size_t off = 0;
  for (int i = 0; i < B->n_members; ++i) {
    BatchMember& bm = B->hmem[i];
    bm.seam_off = -1;
    bm.seam_block = 0;
    if (!B->seams || !has_seams(bm.gs.n, bm.seg_h)) continue;
    bm.seam_off = (int64_t)off;
    bm.seam_block = (int32_t)owner.size();
    off += seam_elems(bm.gs.n, B->m, bm.seg_h);
    const size_t records = (size_t)6 * (bm.n_segs - 1) * bm.gs.n;
    owner.resize(owner.size() + (records + kSeamBlock - 1) / kSeamBlock, i);
  }
  auto none = [&](int status) {
    for (BatchMember& bm : B->hmem) bm.seam_off = -1;
    return status;
  };
  if (off > B->seam_cap) {
    if (B->seam) (void)hipFree(B->seam);
    B->seam = nullptr;
    B->seam_cap = 0;
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, off * sizeof(double));
    if (e != hipSuccess) return none(hip_fail(e, "hipMalloc (batch seams)"));
    B->seam = static_cast<double*>(p);
    B->seam_cap = off;
  }
  if (B->seam_member) (void)hipFree(B->seam_member);
  B->seam_member = nullptr;
  if (!owner.empty()) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, owner.size() * sizeof(int32_t));
    if (e != hipSuccess) return none(hip_fail(e, "hipMalloc (batch seam blocks)"));
    B->seam_member = static_cast<int32_t*>(p);
    e = hipMemcpy(p, owner.data(), owner.size() * sizeof(int32_t), hipMemcpyHostToDevice);
    if (e != hipSuccess) return none(hip_fail(e, "hipMemcpy (batch seam blocks)"));
  }
  B->seam_blocks = (int)owner.size();
  return HOPE_OK;
}

int upload_members(hope_batch* B) {
  hipError_t e = hipMemcpy(B->mem, B->hmem.data(), B->hmem.size() * sizeof(BatchMember), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy (batch members)");
  return HOPE_OK;
}

int batch_stage(const hope_batch* B, double* in, const double* qn, double* out, int out_padded, double ca,
                double cb, double cs, const double* dt, void* stream) {
  hipStreamCaptureStatus cs_status = hipStreamCaptureStatusNone;
  if (stream && hipStreamIsCapturing((hipStream_t)stream, &cs_status) == hipSuccess &&
      cs_status != hipStreamCaptureStatusNone)
    B->captured = true;
  int e = launch_batch_fill_halo(B->dgrids, B->n_grids, B->total_rows, B->mlist, B->mem, in, halo_lanes(B->k),
                                 B->fill_blocks, B->fill_ucap, stream);
  if (e) return hip_fail((hipError_t)e, "batch fill_halo launch");
  e = launch_batch_edge_traces(B->k, B->weno, B->mem, B->edge_member, B->total_edges, in, B->bt, stream);
  if (e) return hip_fail((hipError_t)e, "batch edge_traces launch");
  BatchStage st;
  st.in = in;
  st.qn = qn;
  st.out = out;
  st.out_padded = out_padded;
  st.ca = ca;
  st.cb = cb;
  st.cs = cs;
  st.dt = dt;
  st.bt = B->bt;
  st.seam = B->seam;
  e = launch_batch_stage(B->k, B->weno, B->mem, B->items, B->n_items, B->blocks, B->seam_member, B->seam_blocks, st,
                         stream);
  if (e) return hip_fail((hipError_t)e, "batch stage launch");
  return HOPE_OK;
}

bool misaligned(const void* p) { return reinterpret_cast<uintptr_t>(p) % 8 != 0; }

}  // namespace

extern "C" {

int hope_batch_create(const hope_grid* const* grids, int32_t n_members, const double* axis_tilt, hope_batch** out) {
  if (!grids || !out) return fail(HOPE_ERR_INVALID, "null argument");
  *out = nullptr;
  if (n_members < 1 || n_members > 2047) return fail(HOPE_ERR_INVALID, "n_members must be 1..2047");
  for (int i = 0; i < n_members; ++i) {
    if (!grids[i]) return fail(HOPE_ERR_INVALID, "null grid");
    if (grids[i]->h.k != grids[0]->h.k || grids[i]->h.weno != grids[0]->h.weno)
      return fail(HOPE_ERR_UNSUPPORTED, "all members must share order and scheme");
    if (grids[i]->topo.sbar) return fail(HOPE_ERR_UNSUPPORTED, "the batched kernels are built without topography");
    if (axis_tilt && !std::isfinite(axis_tilt[i])) return fail(HOPE_ERR_INVALID, "axis_tilt not finite");
  }
  hope_batch* B = new (std::nothrow) hope_batch();
  if (!B) return fail(HOPE_ERR_NOMEM, "host allocation");
  B->n_members = n_members;
  B->k = grids[0]->h.k;
  B->weno = grids[0]->h.weno;
  B->m = grids[0]->h.m;
  B->seams = uses_seams(grids[0]->h);
  B->member_grid.assign(grids, grids + n_members);
  std::vector<double> fco(18 * (size_t)n_members);
  int64_t qo = 0, fo = 0, bo = 0;
  int eb = 0;
  std::vector<int32_t> em;   // member of each block of 64 panel-edge sides
  B->hmem.resize(n_members);
  for (int i = 0; i < n_members; ++i) {
    const hope_grid* G = grids[i];
    if (std::find(B->grids.begin(), B->grids.end(), G) == B->grids.end()) B->grids.push_back(G);
    const int n = G->h.n, P = G->h.P;
    BatchMember& bm = B->hmem[i];
    bm.tab = G->tab;
    bm.itab = G->itab;
    bm.fcoef = nullptr;   // set after upload
    bm.gs = G->gs;
    bm.q_off = qo;
    bm.f_off = fo;
    bm.bt_off = bo;
    bm.edge_begin = eb;
    int sw, strips;
    balanced_strip(n, &sw, &strips);
    bm.strip_w = sw;
    bm.n_strips = strips;
    bm.seg_h = std::min(8, n);
    bm.n_segs = (n + bm.seg_h - 1) / bm.seg_h;
    bm.half = bm.strip_w <= kHalfStrip;
    B->q_off.push_back(qo);
    B->f_off.push_back(fo);
    qo += 18LL * P * P;
    fo += 18LL * n * n;
    bo += 24LL * n * B->m * 3;
    eb += ((24 * n + 63) / 64) * 64;
    em.resize(eb / 64, i);
    if (axis_tilt) coriolis_coefs(axis_tilt[i], &fco[18 * (size_t)i]);
    else std::copy(G->h.fcoef.begin(), G->h.fcoef.end(), fco.begin() + 18 * (size_t)i);
  }
  B->state_elems = qo;
  B->field_elems = fo;
  B->bt_elems = bo;
  B->total_edges = eb;
  // members grouped by grid, for the ghost fill
  std::vector<BatchGrid> bgs;
  std::vector<int32_t> ml;
  int rows = 0;
  for (const hope_grid* G : B->grids) {
    BatchGrid bg;
    bg.g = G->g;
    bg.row_begin = rows;
    bg.member_begin = (int32_t)ml.size();
    for (int i = 0; i < n_members; ++i)
      if (grids[i] == G) ml.push_back(i);
    bg.member_count = (int32_t)ml.size() - bg.member_begin;
    bg.P = G->h.P;
    bg.brow = bg.bptr = bg.bsrc = nullptr;
    bg.lent = nullptr;
    bg.block_begin = bg.blocks = 0;
    rows += G->g.rows;
    bgs.push_back(bg);
  }
  B->n_grids = (int)bgs.size();
  B->total_rows = rows;
  int st = HOPE_OK;
  {
    // row blocks of the LDS-staged fill for every grid, or none at all
    // (the grid keeps its ghost map on the device only: copied back here)
    std::vector<FillBlocks> fbs(B->grids.size());
    bool lds = true;
    for (size_t gi = 0; gi < B->grids.size() && lds; ++gi) {
      const hope_grid* G = B->grids[gi];
      const int grows = G->g.rows;
      std::vector<int32_t> ptr((size_t)grows + 1), ent(2 * (size_t)G->g.nnz);
      hipError_t e = hipMemcpy(ptr.data(), G->g.ptr, ptr.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
      if (e == hipSuccess)
        e = hipMemcpy(ent.data(), G->g.ent, ent.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
      if (e != hipSuccess) {
        st = hip_fail(e, "hipMemcpy (batch ghost map)");
        break;
      }
      lds = build_fill_blocks(grows, ptr.data(), ent.data(), (size_t)6 * G->h.P * G->h.P,
                              kHaloLdsThreads / halo_lanes(B->k), kHaloLdsCells, fbs[gi]);
    }
    if (st) lds = false;
    if (lds) {
      int nb = 0;
      for (size_t gi = 0; gi < B->grids.size() && !st; ++gi) {
        BatchGrid& bg = bgs[gi];
        st = upload_vec(B, fbs[gi].brow, const_cast<int32_t**>(&bg.brow));
        if (!st) st = upload_vec(B, fbs[gi].bptr, const_cast<int32_t**>(&bg.bptr));
        if (!st) st = upload_vec(B, fbs[gi].bsrc, const_cast<int32_t**>(&bg.bsrc));
        if (!st) st = upload_vec(B, fbs[gi].lent, const_cast<uint32_t**>(&bg.lent));
        bg.block_begin = nb;
        bg.blocks = (int32_t)fbs[gi].brow.size() - 1;
        nb += bg.blocks;
        B->fill_ucap = std::max(B->fill_ucap, fbs[gi].umax);
      }
      B->fill_blocks = nb;
    }
  }
  if (!st) st = upload_vec(B, fco, &B->fcoef);
  if (!st) st = upload_vec(B, bgs, &B->dgrids);
  if (!st) st = upload_vec(B, ml, &B->mlist);
  if (!st) st = upload_vec(B, em, &B->edge_member);
  if (!st) st = build_seams(B);
  if (!st) {
    for (int i = 0; i < n_members; ++i) B->hmem[i].fcoef = B->fcoef + 18 * (size_t)i;
    st = upload_vec(B, B->hmem, &B->mem);
  }
  if (!st) {
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, std::max<int64_t>(1, bo) * sizeof(double));
    if (e != hipSuccess) st = hip_fail(e, "hipMalloc (batch traces)");
    else {
      B->allocs.push_back(p);
      B->bt = static_cast<double*>(p);
    }
  }
  if (!st) st = build_items(B);
  if (st) {
    free_batch(B);
    return st;
  }
  *out = B;
  return HOPE_OK;
}

void hope_batch_destroy(hope_batch* batch) { free_batch(batch); }

int hope_batch_layout(const hope_batch* B, hope_batch_info* out, int64_t* state_offsets, int64_t* field_offsets) {
  if (!B || !out) return fail(HOPE_ERR_INVALID, "null argument");
  out->n_members = B->n_members;
  out->n_grids = B->n_grids;
  out->state_elems = B->state_elems;
  out->field_elems = B->field_elems;
  out->rk_workspace_bytes = 2 * B->state_elems * (int64_t)sizeof(double);
  out->items = B->n_items;
  out->blocks = B->blocks;
  out->ghost_rows = B->total_rows;
  out->fill_blocks = B->fill_blocks;
  for (int i = 0; i < B->n_members; ++i) {
    if (state_offsets) state_offsets[i] = B->q_off[i];
    if (field_offsets) field_offsets[i] = B->f_off[i];
  }
  return HOPE_OK;
}

int hope_batch_set_launch(hope_batch* B, const int32_t* strip_w, const int32_t* seg_h, int32_t blocks) {
  if (!B) return fail(HOPE_ERR_INVALID, "null argument");
  if (B->captured)
    return fail(HOPE_ERR_INVALID, "the launch shape of a batch is fixed once a stage has been captured in a graph "
                                  "(the graph refers to its work-item list)");
  if (blocks < 0) return fail(HOPE_ERR_INVALID, "blocks must be >= 0");
  for (int i = 0; i < B->n_members; ++i) {
    const int n = B->hmem[i].gs.n;
    const int sw = strip_w ? strip_w[i] : B->hmem[i].strip_w;
    const int sh = seg_h ? seg_h[i] : B->hmem[i].seg_h;
    if (sw < 1 || sw > 62 || sh < 1 || sh > n) return fail(HOPE_ERR_INVALID, "launch shape out of range");
  }
  for (int i = 0; i < B->n_members; ++i) {
    BatchMember& bm = B->hmem[i];
    const int n = bm.gs.n;
    if (strip_w) bm.strip_w = strip_w[i];
    if (seg_h) bm.seg_h = seg_h[i];
    bm.n_strips = (n + bm.strip_w - 1) / bm.strip_w;
    bm.n_segs = (n + bm.seg_h - 1) / bm.seg_h;
    bm.half = bm.strip_w <= kHalfStrip;
  }
  // work already queued on any stream may still read the member table and items
  hipError_t e0 = hipDeviceSynchronize();
  if (e0 != hipSuccess) return hip_fail(e0, "hipDeviceSynchronize");
  B->blocks = blocks;
  int st = build_seams(B);
  if (!st) st = upload_members(B);
  if (!st) st = build_items(B);
  if (st) return st;
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  return HOPE_OK;
}

int hope_batch_get_launch(const hope_batch* B, int32_t* strip_w, int32_t* seg_h, int32_t* blocks) {
  if (!B) return fail(HOPE_ERR_INVALID, "null argument");
  for (int i = 0; i < B->n_members; ++i) {
    if (strip_w) strip_w[i] = B->hmem[i].strip_w;
    if (seg_h) seg_h[i] = B->hmem[i].seg_h;
  }
  if (blocks) *blocks = B->blocks;
  return HOPE_OK;
}

int hope_batch_tendency(const hope_batch* B, double* q_all, double* dqdt_all, void* stream) {
  if (!B || !q_all || !dqdt_all) return fail(HOPE_ERR_INVALID, "null argument");
  if (misaligned(q_all) || misaligned(dqdt_all)) return fail(HOPE_ERR_INVALID, "misaligned buffer");
  return batch_stage(B, q_all, nullptr, dqdt_all, 0, 0.0, 0.0, 1.0, nullptr, stream);
}

int hope_batch_rk_stage(const hope_batch* B, int32_t stage, int32_t scheme, double* q_all, const double* dt,
                        double* ws, size_t ws_bytes, void* stream) {
  if (!B || !q_all || !dt || !ws) return fail(HOPE_ERR_INVALID, "null argument");
  if (scheme != HOPE_RK_SSP3 && scheme != HOPE_RK_WS3) return fail(HOPE_ERR_INVALID, "bad RK scheme");
  if (stage < 0 || stage > 2) return fail(HOPE_ERR_INVALID, "stage must be 0, 1 or 2");
  if (ws_bytes < 2 * (size_t)B->state_elems * sizeof(double)) return fail(HOPE_ERR_INVALID, "workspace too small");
  if (misaligned(q_all) || misaligned(dt) || misaligned(ws)) return fail(HOPE_ERR_INVALID, "misaligned buffer");
  double a[3], b[3], cs[3];
  rk_coefs(scheme, a, b, cs);
  double* w0 = ws;
  double* w1 = ws + B->state_elems;
  switch (stage) {
    case 0: return batch_stage(B, q_all, nullptr, w0, 1, a[0], b[0], cs[0], dt, stream);
    case 1: return batch_stage(B, w0, q_all, w1, 1, a[1], b[1], cs[1], dt, stream);
    default: return batch_stage(B, w1, q_all, q_all, 1, a[2], b[2], cs[2], dt, stream);
  }
}

int hope_batch_rk_step(const hope_batch* B, int32_t scheme, double* q_all, const double* dt, double* ws,
                       size_t ws_bytes, void* stream) {
  for (int s = 0; s < 3; ++s)
    if (int st = hope_batch_rk_stage(B, s, scheme, q_all, dt, ws, ws_bytes, stream)) return st;
  return HOPE_OK;
}

}  // extern "C"
