/*
 * hope.h -- C ABI of the MI355X (gfx950) implementation of the HOPE
 * shallow-water right-hand side on the gnomonic equiangular cubed sphere
 * (Zhou, "HOPE: an automatically differentiable high-order non-oscillatory
 * finite-volume shallow-water dynamic core", arXiv 2411.19185).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * State.  The prognostic variables are the cell averages, over the angular
 * coordinates dx dy, of q = (sqrtG phi, sqrtG phi u, sqrtG phi v) (eqs
 * (2.15)-(2.16)), phi = g h the geopotential, (u, v) contravariant winds in
 * rad/s, sqrtG of (2.8) including the radius squared.
 *
 * Panels are numbered 0..5 (the paper's 1..6, Figure 2.1).  Panel p maps the
 * point (X, Y) = (tan x, tan y), x, y in [-pi/4, pi/4], to the direction
 *   0: (1, X, Y)   1: (-X, 1, Y)   2: (-1, -X, Y)   3: (X, -1, Y)
 *   4: (-Y, X, 1)  5: (Y, X, -1)
 * (normalised), which satisfies (2.5) and reproduces J of (2.10)-(2.11).
 *
 * Padded layout.  A state buffer is FP64 [3][6][P][P] with P = n + 2r,
 * r = (order-1)/2, x fastest: element (var, panel, j, i) of interior cell
 * (i, j), 0 <= i, j < n, lives at ((var*6 + panel)*P + (j+r))*P + (i+r).
 * The outer r rings (corner blocks included, Figure 3.1b) are ghost cells.
 * Unpadded buffers (tendencies, cotangents) are FP64 [3][6][n][n].
 *
 * Ownership.  Every state, tendency, cotangent and workspace buffer is a
 * device allocation owned by the caller; hope_grid_layout gives the sizes.
 * The grid owns only its constant tables, allocated by hope_grid_create, and
 * no call allocates afterwards.  Every scratch buffer a call needs (the
 * panel-edge traces of a stage, the stage states of a Runge-Kutta step, the
 * adjoint's intermediates) comes from the workspace the caller passes, so a
 * grid is read-only once created: calls on one grid may run concurrently on
 * different streams, as long as each has its own state, output and workspace
 * buffers.  The exceptions are the calls that change the grid
 * (hope_grid_set_launch, hope_grid_profile), which must not overlap other
 * calls on it, and hope_check_state, whose concurrent calls take turns.
 *
 * Errors.  Every int-returning function returns HOPE_OK (0) or a negative
 * status; a thread-local message is available from hope_last_error().
 * Argument and launch errors are reported synchronously; faults inside a
 * kernel surface at the caller's next synchronisation of the stream.  No call
 * except hope_grid_create / hope_grid_destroy synchronises the device, and
 * hope_check_state, which waits for its stream.
 *
 * Streams are passed as void* holding a hipStream_t (NULL = null stream).
 */
#ifndef HOPE_H
#define HOPE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  HOPE_OK = 0,
  HOPE_ERR_INVALID = -1,     /* null pointer, bad enum, bad size, misaligned buffer */
  HOPE_ERR_UNSUPPORTED = -2, /* order/scheme/n combination not built */
  HOPE_ERR_HIP = -3,         /* a HIP runtime call failed */
  HOPE_ERR_NOMEM = -4,       /* device or host allocation failed in create */
  HOPE_ERR_NUMERIC = -5      /* hope_check_state found a bad cell; or the
                                ghost-map construction did not converge, or its rows
                                are not images of each other under the cube's rotations */
};

enum { HOPE_SCHEME_TPP = 0, HOPE_SCHEME_WENO = 1 };
enum { HOPE_RK_SSP3 = 0, HOPE_RK_WS3 = 1 };

typedef struct hope_grid hope_grid;

/* Problem statement (sections 2-3).  Zero fields take the defaults shown. */
typedef struct hope_grid_desc {
  int32_t struct_size;   /* sizeof(hope_grid_desc) */
  int32_t n;             /* cells per panel edge (C<n>), n >= order */
  int32_t order;         /* stencil width k = order of accuracy, odd:
                            TPP (3.7)-(3.15): 3,5,7,9,11,13; WENO (3.16)-(3.25): 3,5 */
  int32_t scheme;        /* HOPE_SCHEME_TPP or HOPE_SCHEME_WENO */
  int32_t n_gauss;       /* Gauss points per edge (3.5); 0 or (order+1)/2 */
  int32_t ghost_iters;   /* ghost map (7.12): 0 = the exact fixed point of the
                            ghost interpolation (section 3.3.1); N in 1..300 =
                            the map of N Jacobi sweeps from g = 0 (the paper
                            uses 10) */
  double radius;         /* sphere radius a in m (default 6.371e6) */
  double gravity;        /* g in m/s^2 (default 9.80616), informational */
  double omega;          /* rotation rate Omega in 1/s (default 7.292e-5) */
  double axis_tilt;      /* tilt alpha of the rotation axis towards -x (radians);
                            Coriolis f = 2 Omega (-sin(a) x + cos(a) z) at the
                            unit position (x, y, z); 0 gives f = 2 Omega sin(theta) */
  double weno_eps;       /* epsilon of (3.23) (default 1e-12) */
  double split_theta;    /* theta of the weight split (3.20) (default 3) */
  const char* cache_dir; /* NULL, or an existing directory for cached host
                            tables: hope_grid_create reads the tables of the
                            same (n, order, scheme, radius, weno_eps,
                            split_theta, ghost_iters) and library build from
                            a file there instead of building them, and
                            otherwise builds them and writes the file (about
                            40 MB at C360).  A file that does not match or
                            fails its checksum or range checks is rebuilt; a
                            directory that cannot be written only costs the
                            build. */
  /* Bottom topography (section 2, (2.13)-(2.14)): NULL for none.  Otherwise
   * a host function that hope_grid_create calls, on its own thread, to
   * evaluate the surface geopotential phi_s = g h_s (m^2/s^2) at count points:
   * xyz[3i], xyz[3i+1], xyz[3i+2] is the i-th unit vector (the panel maps
   * above), and phis[i] receives phi_s there (finite values; the create call
   * fails with HOPE_ERR_INVALID otherwise).  It is called a few times per
   * panel with up to 16 n^2 points.  The state stays the layer's own
   * (sqrtG phi, sqrtG phi u, sqrtG phi v); the grid then reconstructs
   * sqrtG phi_t = sqrtG (phi + phi_s), uses phi_t in the pressure of the
   * flux (3.38) and adds psi_B of (2.14) to the sources. */
  void (*surface_geopotential)(int64_t count, const double* xyz, double* phis, void* user);
  void* surface_user;    /* passed back to surface_geopotential */
} hope_grid_desc;

/* Sizes a caller needs to allocate buffers (all counts are elements). */
typedef struct hope_layout {
  int32_t n, r, padded, n_gauss;
  int64_t state_elems;      /* 3*6*P*P: one padded state */
  int64_t interior_elems;   /* 3*6*n*n: one unpadded field */
  int64_t rk_workspace_bytes;  /* workspace of hope_rk_step: two padded states, then
                                  tendency_workspace_bytes */
  int64_t vjp_workspace_bytes;     /* workspace of hope_tendency_vjp */
  int64_t rk_vjp_workspace_bytes;  /* workspace of hope_rk_step_vjp */
  int64_t ghost_cells;      /* ghost cells per variable, all panels */
  int64_t ghost_nnz;        /* stored entries of the ghost map */
  int64_t device_bytes;     /* device memory owned by the grid (tables, maps, scratch) */
  int32_t ghost_sweeps;     /* sweeps of the ghost-map build (ghost_iters if set) */
  int32_t tables_cached;    /* 1 if the host tables were read from cache_dir */
  int64_t tendency_workspace_bytes;  /* workspace of hope_tendency: the panel-edge
                                        traces of one stage (8 * 24 * n * n_gauss * 3
                                        bytes rounded up to 256), then the segment
                                        seams of the current launch shape (none for
                                        segments of one row or one segment per panel;
                                        otherwise 8 * 6 * n * (segments - 1) *
                                        (6 n_gauss + 11) bytes rounded up to 256) */
  int64_t fill_blocks;      /* row blocks of the LDS-staged ghost fill (0: the fill reads
                               the state directly) */
} hope_layout;

/* Build a grid: equiangular metrics, reconstruction and WENO tables, the
 * ghost-cell map G of appendix (7.12) (the exact fixed point of the iterative
 * interpolation of section 3.3.1, with owner-panel conversion (3.26)-(3.29),
 * or with ghost_iters set the map of that many sweeps), and the panel-edge
 * trace maps; with cache_dir set, the host tables may come from a file;
 * with surface_geopotential set, the topography tables (cell averages of
 * sqrtG phi_s by a 4 x 4 Gauss rule, their image under G on the ghost cells,
 * and sqrtG phi_s at every edge and cell Gauss point).  G commutes with the cube's 24 rotations;
 * each row is replaced by the rotation image of one of r*(n+r) canonical rows
 * (they agree to rounding; the build fails with HOPE_ERR_NUMERIC otherwise),
 * and the device keeps the values once per canonical row.  Host work plus
 * device uploads; synchronous.
 * On success *out owns device memory until hope_grid_destroy. */
int hope_grid_create(const hope_grid_desc* desc, hope_grid** out);
void hope_grid_destroy(hope_grid* grid);
/* A grid equal to base except for the tilt of the rotation axis (the
 * Coriolis term (2.3) with f of a tilted axis): it shares base's ghost map,
 * its transpose and the panel-edge map on the device and copies only the small
 * constant tables, so it is cheap to make one per ensemble member.  base must
 * outlive it.  Synchronous. */
int hope_grid_derive(const hope_grid* base, double axis_tilt, hope_grid** out);
int hope_grid_layout(const hope_grid* grid, hope_layout* out);

/* Ghost fill g = G q (7.12): overwrites the ghost rings of the padded state q
 * (all 3 variables, 6 panels) from its interior cells.  Mass rows are scalar,
 * momentum rows are 2x2 blocks (the conversion (3.29) at each ghost Gauss
 * point).  Interior cells are read only. */
int hope_fill_halo(const hope_grid* grid, double* q, void* stream);

/* State check for a run that may have left the shallow-water system's
 * domain: counts the interior cells of the padded state q whose layer
 * thickness sqrtG*phi (variable 0, section 2) is not a positive finite
 * number, or whose momentum (variables 1, 2) is not finite.  Ghost rings are
 * not read.  The count goes to *n_bad (host memory, may be NULL).  Waits for
 * the work queued on the stream before it, so call it between steps, not
 * inside a captured graph.  It counts in a word the grid owns; calls from
 * several threads take turns on it (a lock held until the count is read).
 * Returns HOPE_ERR_NUMERIC when the count is not zero,
 * else HOPE_OK. */
int hope_check_state(const hope_grid* grid, const double* q, int64_t* n_bad, void* stream);

/* Tendency dq/dt of (3.1): fills the ghost rings of q (they are scratch),
 * then for every interior cell reconstructs to the edge and cell Gauss
 * points (TPP or genuine 2D WENO), takes the neighbour panel's converted
 * trace at panel edges (3.26)-(3.29), evaluates the LMARS flux (3.30)-(3.38)
 * with upwind term |m|(q_R - q_L), integrates fluxes (3.5) and the metric and
 * Coriolis sources (2.2)-(2.3) (3.6), and writes dqdt [3][6][n][n].
 * ws: caller-owned device scratch of at least layout.tendency_workspace_bytes
 * (the converted neighbour traces at the panel-edge points and the segment
 * seams); its contents are overwritten and need not be kept.  Returns HOPE_ERR_INVALID for a null
 * or misaligned buffer or a workspace that is too small. */
int hope_tendency(const hope_grid* grid, double* q, double* dqdt, double* ws, size_t ws_bytes, void* stream);

/* Vector-Jacobian product of hope_tendency: given w = dL/d(dqdt) [3][6][n][n]
 * writes gq = dL/dq over the interior cells [3][6][n][n] (overwritten), the
 * ghost-cell cotangents folded back through G^T.  q's ghost rings are scratch.
 * Non-smooth points (|m|, |beta_i - beta_j|) take the subgradient sign(0)=0.
 * ws: caller-owned device workspace of at least layout.vjp_workspace_bytes
 * (8 * 2*3*(4m+m^2) bytes per cell for the point values and their
 * cotangents, plus 8 * 3 * order^2 for the stencil cotangents on grids of
 * n < 160 (from n = 160 those of as many variables at a time as fit take the
 * point values' space), plus one padded state, and 8 * 2 m^2 bytes per cell
 * more with topography); gq must not alias w.  With
 * topography the adjoint runs through sqrtG phi_t, the pressure with phi_s
 * and psi_B (2.14), phi_s being a constant of the grid. */
int hope_tendency_vjp(const hope_grid* grid, double* q, const double* w, double* gq, double* ws,
                      size_t ws_bytes, void* stream);

/* One three-stage Runge-Kutta step (section 3.5) in place on the padded
 * state q: HOPE_RK_SSP3 (Shu-Osher), or HOPE_RK_WS3 (3.39)-(3.41) with the
 * second stage from q^n.  ws: device workspace of at least
 * layout.rk_workspace_bytes (two padded stage states, then the workspace of
 * hope_tendency). */
int hope_rk_step(const hope_grid* grid, double* q, double dt, int32_t scheme, double* ws,
                 size_t ws_bytes, void* stream);

/* Vector-Jacobian product of one hope_rk_step from the state q = q^n
 * (padded; its ghost rings are scratch, its interior is read only): given
 * gout = dL/dq^{n+1} [3][6][n][n] writes gin = dL/dq^n [3][6][n][n]
 * (gin must not alias gout).  The stage states are recomputed, with their
 * panel-edge traces in the workspace too.  ws: at least
 * layout.rk_vjp_workspace_bytes. */
int hope_rk_step_vjp(const hope_grid* grid, double* q, double dt, int32_t scheme, const double* gout,
                     double* gin, double* ws, size_t ws_bytes, void* stream);

/* hope_rk_step without a workspace argument, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  The two stage states and the stage
 * scratch (panel-edge traces, segment seams) live instead in a static device array of 128 MiB (HOPE_STATIC_SCRATCH_BYTES)
 * that each GPU the library runs on holds until the process ends; a grid
 * whose layout.rk_workspace_bytes exceeds it is refused with
 * HOPE_ERR_INVALID (C360 at order 5 needs 98 MB with its default launch shape).  The call allocates
 * nothing: the first call on a device only looks up the array's device
 * address (hipGetSymbolAddress).  Every call on one GPU shares that GPU's
 * array, which keeps the last call's contents (a step reads nothing it did
 * not write first, so nothing needs clearing): calls that overlap on one GPU
 * (on different streams, or from different host threads before the earlier
 * call's kernels have finished) race and give wrong results; calls one
 * after another on one stream are fine.  The stream must belong to the
 * current device.  Results are bitwise those of hope_rk_step. */
enum { HOPE_STATIC_SCRATCH_BYTES = 128 << 20 };
int hope_rk_step_static(const hope_grid* grid, double* q, double dt, int32_t scheme, void* stream);

/* Message for the last error on this thread ("" if none). */
const char* hope_last_error(void);

/* Launch shape of the fused stage kernel: each workgroup (three wavefronts,
 * one per variable) owns a strip of strip_w <= 62 interior columns of one
 * panel and marches over seg_h rows; strips of strip_w <= 30 columns run two
 * per workgroup, one in each half of its lanes.  With seg_h >= 2 the flux
 * through each boundary between two segments is formed by a second kernel
 * from traces the segments store in the workspace (segment seams), so the
 * workspace sizes of hope_grid_layout (tendency, rk, rk_vjp) depend on
 * seg_h: read the layout again after changing it.  Any values in range give
 * bitwise identical results; they only change speed (the autotuner picks
 * them per grid).  Returns HOPE_ERR_INVALID out of range. */
int hope_grid_set_launch(hope_grid* grid, int32_t strip_w, int32_t seg_h);
int hope_grid_get_launch(const hope_grid* grid, int32_t* strip_w, int32_t* seg_h);

/* Per-kernel timing.  While enabled, the library brackets each kernel it
 * launches with HIP events on the launch stream (events are created on first
 * use and kept by the grid).  The fused stage's events are recorded by its
 * launches themselves (the start of the stage kernel, the end of the seam
 * kernel), which adds nothing between kernels; the other kernels' events are
 * markers between launches, each costing the stream a few microseconds.
 * Timing is skipped while the stream is being captured.
 * hope_grid_profile(g, 1) clears the record and starts timing every kernel;
 * (g, HOPE_PROFILE_SELECT | bits) does the same for the kernels whose bit
 * (1 << index, indices below) is set, so that the other launches carry no
 * events; (g, 0) stops.  hope_grid_profile_read waits for the
 * recorded events and returns the summed elapsed time and launch count of one
 * kernel: 0 ghost fill, 1 panel-edge traces, 2 fused stage, and the kernels
 * of the adjoint: 3 point values, 4 flux and source adjoints, 5 panel-edge
 * adjoints, 6 WENO adjoint, 7 gather to the padded cells, 8 G^T fold. */
enum { HOPE_PROFILE_SELECT = 0x40000000 };
int hope_grid_profile(hope_grid* grid, int32_t enable);
int hope_grid_profile_read(hope_grid* grid, int32_t kernel, double* total_ms, int64_t* launches);

/* Host-only inspection of the ghost map G of appendix (7.12) that
 * hope_grid_create would build for desc (no device use; for verification).
 * Call with null arrays to get *rows and *nnz; then with arrays of at least
 * rows (dst), rows+1 (ptr), nnz (col) and 5*nnz (val, struct of arrays:
 * mass, C11, C12, C21, C22) elements.  dst/col are offsets inside one
 * variable plane of the padded layout ((panel*P + jj)*P + ii).  Also returns
 * the number of fixed-point sweeps the construction took in *sweeps.  These
 * are the rows the device applies (the rotation images of the canonical
 * rows), entries in ascending column order. */
int hope_inspect_ghost_map(const hope_grid_desc* desc, int64_t* rows, int64_t* nnz, int32_t* sweeps,
                           int32_t* dst, int32_t* ptr, int32_t* col, double* val);

/* ------------------------------------------------------------------------
 * Batched ensemble.  Members of one order and scheme, on grids of any
 * resolutions (members may share a grid), advanced together: each kernel of
 * a stage (ghost fill, panel-edge traces, fused stage, and at WENO5 and TPP9
 * and up the segment seams) is one launch over all members, so a whole
 * Runge-Kutta step is 9 or 12 launches whatever the member count, and no call
 * below except create / set_launch / destroy allocates or synchronises: the
 * stage and step calls can be captured in a HIP graph.  The batch owns its
 * scratch (panel-edge traces and segment seams, the latter sized by the launch
 * shapes), so calls on one batch must not overlap on different streams.
 * Each member's result is bitwise the one hope_rk_step / hope_tendency give
 * on its own grid (with its own axis tilt).
 *
 * States of all members live in one caller-owned buffer q_all: member i's
 * padded state [3][6][P_i][P_i] starts at element state_offsets[i]; fields
 * (tendencies) likewise at field_offsets[i] of an unpadded buffer.
 * ------------------------------------------------------------------------ */
typedef struct hope_batch hope_batch;

typedef struct hope_batch_info {
  int32_t n_members, n_grids;
  int64_t state_elems;         /* length of q_all (elements) */
  int64_t field_elems;         /* length of an unpadded field buffer */
  int64_t rk_workspace_bytes;  /* workspace of the stage / step calls (two state sets) */
  int64_t items;               /* fused-stage work items per launch */
  int64_t blocks;              /* workgroups of the fused stage (0: one per item) */
  int64_t ghost_rows;          /* ghost rows of all distinct grids */
  int64_t fill_blocks;         /* row blocks of the LDS-staged ghost fill (0: the direct fill) */
} hope_batch_info;

/* grids[i]: the grid of member i (they must outlive the batch; grids with
 * topography are refused with HOPE_ERR_UNSUPPORTED).  axis_tilt:
 * per-member tilt of the rotation axis (radians), or NULL to use each grid's
 * own.  Allocates device tables; synchronous. */
int hope_batch_create(const hope_grid* const* grids, int32_t n_members, const double* axis_tilt,
                      hope_batch** out);
void hope_batch_destroy(hope_batch* batch);
/* state_offsets / field_offsets: NULL or arrays of n_members elements. */
int hope_batch_layout(const hope_batch* batch, hope_batch_info* out, int64_t* state_offsets,
                      int64_t* field_offsets);
/* Work-item shape per member (strip width 1..62, segment height 1..n; NULL
 * keeps the current values) and the fused-stage grid size (0: one workgroup
 * per item; otherwise that many workgroups stride the item list).  Waits for
 * the device, then rebuilds and uploads the item list and grows the segment
 * seam scratch to the new shapes (it never shrinks): allocates and
 * synchronises.  Any values give bitwise identical results.  Refused with
 * HOPE_ERR_INVALID once a stage of the batch has been recorded under stream
 * capture, since the graph refers to the item list. */
int hope_batch_set_launch(hope_batch* batch, const int32_t* strip_w, const int32_t* seg_h, int32_t blocks);
int hope_batch_get_launch(const hope_batch* batch, int32_t* strip_w, int32_t* seg_h, int32_t* blocks);
/* Tendencies (3.1) of all members: fills the ghost rings of q_all, writes
 * dqdt_all (unpadded, at field_offsets). */
int hope_batch_tendency(const hope_batch* batch, double* q_all, double* dqdt_all, void* stream);
/* Stage `stage` (0, 1, 2) of one Runge-Kutta step (section 3.5) of every
 * member with its own time step dt[i] (device array of n_members doubles, read
 * when the stage runs, so a captured graph can be replayed with new steps).
 * Stage 0 reads q_all and writes the first workspace state set, stage 1 reads
 * it and writes the second, stage 2 reads the second and writes q_all.
 * ws: at least layout.rk_workspace_bytes. */
int hope_batch_rk_stage(const hope_batch* batch, int32_t stage, int32_t scheme, double* q_all,
                        const double* dt, double* ws, size_t ws_bytes, void* stream);
/* The three stages in order. */
int hope_batch_rk_step(const hope_batch* batch, int32_t scheme, double* q_all, const double* dt, double* ws,
                       size_t ws_bytes, void* stream);

#ifdef __cplusplus
}
#endif
#endif /* HOPE_H */
