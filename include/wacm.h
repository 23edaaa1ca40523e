/*
 * wacm.h -- C ABI of the MI355X (gfx950) hot path of the wavelet-adaptive
 * block method for the penalized artificial-compressibility equations of
 * Engels, Schneider, Reiss & Farge (arXiv:1912.05371).
 *
 * The method advances U = (u, v, w, p) on a 2:1-balanced periodic octree of
 * cubic blocks (Sec. 4.1): each classical RK4 stage (Sec. 2.3) synchronises
 * ghost nodes (Sec. 4.2; same-level copy, fine->coarse decimation, coarse->fine
 * 4th-order Deslauriers-Dubuc prediction, Sec. 3.1) and evaluates the
 * penalized right-hand side (Sec. 2.2).  Wavelet details (Sec. 3.1, 3.3-3.4)
 * decide coarsening, and the grid is refined and coarsened around each step
 * (Sec. 3.5).
 *
 * Conventions shared by every call
 * ---------------------------------
 * - Return value: WACM_OK (0) or a negative WACM_E_* code.  No exception
 *   crosses the ABI.  Arguments are checked on the host before any launch;
 *   a failed check launches nothing and leaves every buffer untouched.
 *   wacm_last_error(grid) gives the text of the last failure of a call on
 *   that grid, wacm_last_error(NULL) the last failure of the calling thread.
 * - Asynchrony: calls that take a stream only enqueue work on it and return;
 *   errors raised by the device surface at the next synchronising call.
 *   Calls documented as "synchronous" wait for the stream.
 * - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 * - Ownership: the library never allocates device memory.  The caller owns
 *   every device buffer: the state, the work registers and the workspaces
 *   whose sizes the library states (wacm_workspace_bytes for the grid's
 *   tables, wacm_wavelet_workspace_bytes for CDF 4/4, wacm_adj_plan_bytes
 *   for the adjoint's transpose plans), each 256-byte aligned.  A grid keeps
 *   pointers into its workspaces until wacm_grid_destroy, so they must stay
 *   allocated until then.  The library owns only the opaque handle and its
 *   host metadata.
 *
 * Block pool layout ("pool"): a device array of `capacity` slots; slot s holds
 * 4 fields (u, v, w, p), each a padded cube of P^3 values, P = bs + 2 ng,
 * x fastest:  pool[((s*4 + c)*P + (k+ng))*P + (j+ng))*P + (i+ng)] for local
 * indices i, j, k in [-ng, bs+ng).  Interior points are [0, bs)^3; the others
 * are ghost nodes.  The element type is float (WACM_F32) or double (WACM_F64)
 * as chosen at grid creation.  Only slots of active blocks are read or written.
 *
 * Geometry: domain [0,L]^3, periodic in all directions.  A block at level J
 * with block index (bx,by,bz) in [0,2^J)^3 has spacing h_J = L/(2^J bs) and
 * interior point i at x = (bx bs + i) h_J (non-redundant blocks; bs even).
 * Treecode: one octal digit per level, level-1 digit most significant,
 * digit = xbit + 2 ybit + 4 zbit (Sec. 4.1).
 *
 * Two dimensions (wacm_grid_desc.dim = 2; the model of Sec. 2.1 with D = 2):
 * a periodic quadtree of square blocks on [0,L]^2 with the same spacing and
 * positions in x and y.  Leaves are given by the octal treecode of (bx, by, 0)
 * (digits 0..3).  The pool holds 3 fields (u, v, p) per slot, each a padded
 * square of P^2 values, x fastest:
 *   pool[((s*3 + c)*P + (j+ng))*P + (i+ng)].
 * Available in 2D: grid creation and queries, wacm_sync_ghosts, wacm_rhs_acm,
 * wacm_compute_dt, wacm_rk4_step(s), wacm_diagnostics (w and the force read
 * 0), wacm_threshold_blocks and wacm_adapt, all with the CDF 4/0 wavelet,
 * without mask, sponge or extra solid velocity (params.mask and
 * params.sponge 0, dus NULL; WACM_E_INVAL otherwise).  The other calls return
 * WACM_E_INVAL for a 2D grid.
 */
#ifndef WACM_H
#define WACM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif
#pragma GCC visibility push(default)

#define WACM_OK 0
#define WACM_E_INVAL (-1)      /* bad argument or size                         */
#define WACM_E_NOMEM (-2)      /* host or device allocation failed             */
#define WACM_E_CAPACITY (-3)   /* adaptation needs more pool slots             */
#define WACM_E_UNBALANCED (-4) /* leaves are not 2:1 graded (26 neighbours)     */
#define WACM_E_HIP (-5)        /* a HIP runtime call failed                    */
#define WACM_E_NONFINITE (-6)  /* NaN or Inf found in the state                */
#define WACM_E_TILING (-7)     /* leaves overlap, repeat or leave gaps          */

/* restriction wavelet (wacm_set_wavelet) */
#define WACM_CDF40 0
#define WACM_CDF44 1

#define WACM_F32 1
#define WACM_F64 2

#define WACM_DT_FIXED 0 /* rk4_step reads dt from *dt_dev                       */
#define WACM_DT_CFL 1   /* rk4_step computes dt from U and writes it to *dt_dev */

#define WACM_REFINE_ALL 1 /* split every block below jmax into 8 children      */
#define WACM_COARSEN 2    /* one merge pass over flagged sister groups          */

#define WACM_MASK_NONE 0
#define WACM_MASK_SPHERE 1 /* static sphere, chi = (1 - tanh(d/w))/2            */
#define WACM_MASK_PLATE 2  /* thin plate pitching about an axis parallel to y   */

typedef struct wacm_grid wacm_grid;

typedef struct {
  int32_t bs;       /* interior points per axis; even, >= 2 (ng + 3)            */
  int32_t ng;       /* ghost layers; >= 3                                        */
  int32_t jmin;     /* coarsest level allowed                                    */
  int32_t jmax;     /* finest level allowed, <= 18 (Sec. 3.5)                    */
  int32_t dtype;    /* WACM_F32 or WACM_F64                                      */
  int32_t dim;      /* 3 (octree; 0 is read as 3) or 2 (quadtree, see below)      */
  int64_t capacity; /* number of pool slots                                      */
  double L;         /* domain edge length                                        */
} wacm_grid_desc;

/* Launch schedule of the fused stage kernel of wacm_rk4_step (performance
 * only: results do not depend on it).  wg_per_cu: persistent workgroups per
 * compute unit (0: as many as are resident); xcd_map: 1 gives each of the 8
 * XCDs a contiguous run of the Morton-ordered blocks (shared faces meet in one
 * L2), 2 does the same through per-XCD work counters from which each
 * workgroup takes its next item, moving on to the other XCDs' runs when its
 * own is empty (calls on one grid must then not overlap in time: they share
 * the counters), 0 deals the work items round-robin; prefetch: 1 loads U^n and the accumulator before a plane's barrier, 0
 * after the rhs, -1 default; nontemporal: 1 streams U^n and the accumulator
 * with non-temporal loads/stores; tile_rows: 0 gives each workgroup a whole
 * block (bs^2 threads), 8 a tile of 8 rows of the block's columns (8 bs
 * threads, smaller workgroups, more of them per CU); pen_split: 2 runs the
 * blocks where the penalization and sponge terms vanish at every point (far
 * from the mask by 40 smoothing widths, 12 with clipping, and outside the
 * sponge) through the unpenalized variant and the others through the
 * penalized one, 1 does so when it pays (at least 2048 active blocks and,
 * for a static mask or sponge, at least 512 without penalization), 0 runs
 * every block through the penalized one when a mask, sponge or dus is
 * present.  Results are the same bit for bit.  Default {0, 1, -1, 1, 0, 1}. */
typedef struct {
  int32_t wg_per_cu;
  int32_t xcd_map;
  int32_t prefetch;
  int32_t nontemporal;
  int32_t tile_rows;
  int32_t pen_split;
} wacm_schedule;

/* Parameters of the penalized ACM model (Sec. 2.1-2.3). */
typedef struct {
  double nu;        /* kinematic viscosity                                        */
  double c0;        /* artificial speed of sound C0                               */
  double c_gamma;   /* dashpot damping C_gamma                                    */
  double c_eta;     /* penalization permeability C_eta                            */
  double c_sp;      /* sponge constant C_sp                                       */
  double l_sp;      /* sponge width at each face of [0,L]^3 (binary sponge)       */
  double u_inf[3];  /* sponge velocity                                            */
  double p_inf;     /* sponge pressure                                            */
  int32_t mask;     /* WACM_MASK_*                                                */
  int32_t sponge;   /* 0 off, 1 on                                                */
  int32_t clip;     /* 1: mask values below 1e-8 become exactly 0                 */
  int32_t reserved; /* must be 0                                                  */
  double w;         /* mask smoothing width                                       */
  double sph_c[3];  /* sphere centre                                              */
  double sph_r;     /* sphere radius                                              */
  double x_le[3];   /* plate: a point on its rotation axis (leading edge)          */
  double lo[3];     /* plate: body-frame box lower corner                         */
  double hi[3];     /* plate: body-frame box upper corner                         */
  double amp, freq, phase; /* plate pitch angle amp*sin(2 pi freq t + phase)     */
  double cfl, cfl_eta, cfl_nu; /* time-step constants (Sec. 2.3)                 */
} wacm_params;

/* Text of the last failed call on `grid` ("" if none), or with grid NULL of
 * the last failure on the calling thread. */
const char* wacm_last_error(const wacm_grid* grid);

/* Treecode helpers (Sec. 4.1). */
uint64_t wacm_treecode_encode(int32_t level, int64_t ix, int64_t iy, int64_t iz);
void wacm_treecode_decode(uint64_t code, int32_t level, int64_t* ix, int64_t* iy, int64_t* iz);

/*
 * wacm_workspace_bytes -- bytes of the device workspace a grid of this
 * descriptor needs for its tables (per block: the neighbour table of the
 * 27 regions around it, the adaptation work lists, the lists of faces and
 * ghost regions next to other levels, reduction partials; plus the work
 * counters of the stage kernel), sized for `capacity` blocks so that no
 * adaptation ever needs more.  0 if the descriptor is invalid.
 */
size_t wacm_workspace_bytes(const wacm_grid_desc* desc);

/*
 * wacm_grid_create -- build a grid from `nleaves` leaves (Sec. 4.1).
 * treecodes/levels: host arrays of nleaves entries.  Leaf i is placed in pool
 * slot i (so nleaves <= capacity); the active block list is kept in Morton
 * order.  workspace: caller-owned device buffer of ws_bytes >=
 * wacm_workspace_bytes(desc) bytes, 256-byte aligned, kept by the grid until
 * wacm_grid_destroy (the tables are built there; the grid never allocates
 * device memory).  Validation, all before the workspace is touched: sizes
 * and the workspace (WACM_E_INVAL), exact tiling of the periodic domain
 * (WACM_E_TILING), 2:1 grading over faces, edges and corners
 * (WACM_E_UNBALANCED).  On success *out receives a new handle.  Synchronous.
 */
int wacm_grid_create(const wacm_grid_desc* desc, int64_t nleaves, const uint64_t* treecodes,
                     const int8_t* levels, void* workspace, size_t ws_bytes, wacm_grid** out);

/* Release the handle (the caller's workspaces may be freed afterwards).  NULL
 * is accepted. */
int wacm_grid_destroy(wacm_grid* grid);

/* Number of active blocks. */
int64_t wacm_grid_nb(const wacm_grid* grid);

/*
 * wacm_grid_info -- active blocks in Morton order.  Each non-NULL host array
 * receives nb entries: pool slot, treecode, level.
 */
int wacm_grid_info(const wacm_grid* grid, int64_t* slots, uint64_t* treecodes, int8_t* levels);

/* Restriction wavelet of the grid (Sec. 3.2).  WACM_CDF40 (default):
 * restriction is decimation.  WACM_CDF44: the interpolating wavelet lifted to
 * 4 vanishing moments; restriction becomes the lifted low-pass (13 taps
 * (-1, 0, 18, -16, -63, 144, 348, 144, -63, -16, 18, 0, -1)/512 along each
 * axis, x then y then z) over the finer leaf's level-(J+1) lattice as held in
 * its padded array after the CDF 4/0 ghost fill.  It applies wherever the
 * method restricts: in wacm_sync_ghosts to every ghost point whose owner is
 * finer (a second phase after the CDF 4/0 fill; the first phase's values are
 * staged so no lifted value reads another), in wacm_adapt(REFINE_ALL)'s own
 * sync, and in wacm_adapt(COARSEN) to the parents (then U must be
 * ghost-synchronised, as it is after thresholding).  Details, prediction and
 * refinement are unchanged.  CDF 4/4 needs ng >= 6 (else WACM_E_INVAL) and
 * device buffers for its ghost phase, which the caller provides: ws, ws_bytes >=
 * wacm_wavelet_workspace_bytes(grid, WACM_CDF44), 256-byte aligned, kept by
 * the grid until it is destroyed or switched back to CDF 4/0 (ws may be NULL
 * for WACM_CDF40).  The size covers `capacity` blocks with every ghost point
 * lifted, so no adaptation needs more.  Not available with CDF 4/4:
 * wacm_filter_blocks and the adjoint (WACM_E_INVAL); wacm_rk4_step(s) take
 * the materialised path described at wacm_rk4_step.  wacm_get_wavelet
 * returns the current choice. */
size_t wacm_wavelet_workspace_bytes(const wacm_grid* grid, int32_t wavelet); /* 0: none */
int wacm_set_wavelet(wacm_grid* grid, int32_t wavelet, void* ws, size_t ws_bytes);
int wacm_get_wavelet(const wacm_grid* grid);

/* Set / read the stage-kernel schedule (values checked: wg_per_cu in [0, 16],
 * xcd_map in {0, 1, 2}, nontemporal in {0, 1}, prefetch in {-1, 0, 1}, tile_rows in
 * {0, 8}, pen_split in {0, 1, 2}). */
int wacm_set_schedule(wacm_grid* grid, const wacm_schedule* s);
int wacm_get_schedule(const wacm_grid* grid, wacm_schedule* s);

/* Bytes of the `work` buffer wacm_rk4_step / wacm_rk4_steps need (4 compact
 * registers of bs^3 points x 4 fields for every pool slot: accumulator, two
 * stage inputs and the state between the steps of one wacm_rk4_steps call;
 * plus the depth-3 halo of the 6 faces), 256-byte aligned by the caller. */
size_t wacm_work_bytes(const wacm_grid* grid);

/*
 * wacm_sync_ghosts -- ghost-node synchronisation (Sec. 4.2) of every active
 * block of the pool U, in place; interiors are not modified.  A ghost point
 * takes the value of the leaf that holds it: a copy if that leaf is on the
 * same level, the coincident fine point if it is finer (decimation, Sec. 3.1),
 * and the tensor-product 4th-order Deslauriers-Dubuc prediction from the
 * coarse lattice (Sec. 3.1) if it is coarser; coarse lattice values are read
 * from the interiors of their own leaves.  All `ng` layers including edges and
 * corners are filled.
 */
int wacm_sync_ghosts(wacm_grid* grid, void* U, void* stream);

/*
 * wacm_sync_ghosts_lattice -- the ghost points wacm_threshold_blocks reads,
 * with the values wacm_sync_ghosts gives them: the points of the block's
 * even lattice within 3 of its interior ((i, j, k) all even in
 * [-2, bs+2]^3, Sec. 3.1; each a copy from the leaf that holds it).  The
 * other ghost points keep their values.  So wacm_threshold_blocks after this
 * call gives what it gives after wacm_sync_ghosts, at about a tenth of the
 * memory traffic.  With CDF 4/4 or in two dimensions it is wacm_sync_ghosts.
 */
int wacm_sync_ghosts_lattice(wacm_grid* grid, void* U, void* stream);

/*
 * wacm_rhs_acm -- right-hand side of the penalized ACM equations (Sec. 2.2)
 * with Tam-Webb 4th-order first derivatives and the 4th-order centred second
 * derivative (Sec. 2.3), in advective form, at time t.
 * U: ghost-synchronised pool (read).  dU: pool-shaped output; interiors of
 * active blocks are written.  dus: optional (NULL) extra solid velocity, a
 * device array [capacity][3][bs^3] (x fastest) added to u_s.
 */
int wacm_rhs_acm(wacm_grid* grid, const wacm_params* prm, double t, const void* U, void* dU,
                 const void* dus, void* stream);

/*
 * wacm_compute_dt -- time step from the stability limits of Sec. 2.3:
 * min(cfl h_min/u_eig, cfl_eta C_eta [mask], cfl_eta C_sp [sponge],
 * cfl_nu h_min^2/nu), u_eig = |u|max + sqrt(|u|max^2 + C0^2), |u|max the
 * largest Euclidean velocity over interiors, h_min of the finest active level.
 * Writes one double to the device pointer dt_dev.  FP64 reduction.
 */
int wacm_compute_dt(wacm_grid* grid, const wacm_params* prm, const void* U, double* dt_dev,
                    void* stream);

/*
 * wacm_rk4_step -- one classical RK4 step (Sec. 2.3) in place on U on the
 * current grid.  Each stage synchronises ghosts and evaluates the rhs at the
 * stage time t + (0, 1/2, 1/2, 1) dt.  t_dev, dt_dev: device doubles; with
 * WACM_DT_CFL dt is first computed from U (as wacm_compute_dt) and stored in
 * *dt_dev, with WACM_DT_FIXED it is read from *dt_dev.  *t_dev is advanced by
 * dt.  work: device buffer of wacm_work_bytes().  dus: as in wacm_rhs_acm.
 * Only the interiors of U are defined on return: the stages read neighbour
 * values directly, not U's ghost layers, and those layers are left with
 * unspecified values (call wacm_sync_ghosts before a call that reads them).
 * With the CDF 4/0 wavelet: no host synchronisation and no allocation, so the
 * call may be captured in a HIP graph as long as the grid is not changed.
 * With CDF 4/4 (wacm_set_wavelet): every stage input is synchronised first,
 * as far as the stage and the lifted values read (U's ghost layers in place;
 * on return they are unspecified too), and the work buffer is 3 padded
 * registers (wacm_work_bytes); no host synchronisation or allocation either,
 * so this call may be captured in a HIP graph too.
 */
int wacm_rk4_step(wacm_grid* grid, const wacm_params* prm, double* t_dev, double* dt_dev,
                  void* U, void* work, const void* dus, int32_t dt_mode, void* stream);

/*
 * wacm_rk4_steps -- nsteps consecutive wacm_rk4_step calls in one call, with
 * the same results bit for bit.  With WACM_DT_CFL every step takes its dt
 * from the state it starts from, as in wacm_rk4_step; from the second step on,
 * the velocity maximum that rule needs is formed by the previous step's last
 * stage while it writes U, instead of by a separate pass over U.  *dt_dev
 * holds the last step's dt on return.  nsteps >= 0 (WACM_E_INVAL otherwise);
 * 0 does nothing.  Same buffers, synchronisation and graph-capture rules as
 * wacm_rk4_step.
 */
int wacm_rk4_steps(wacm_grid* grid, const wacm_params* prm, double* t_dev, double* dt_dev,
                   void* U, void* work, const void* dus, int32_t dt_mode, int64_t nsteps,
                   void* stream);

/*
 * wacm_diagnostics -- FP64 reductions over interiors at time t:
 * out[0] max Euclidean |u|, out[1..4] max |u|,|v|,|w|,|p|,
 * out[5..7] penalization force C_eta^-1 sum chi (u - u_s) h^3 (Sec. 2.2,
 * midpoint rule), out[8] energy 1/2 sum |u|^2 h^3, out[9] the number of
 * interior values that are NaN or Inf (the maxima skip them).  out: 10
 * device doubles.  Synchronous (the stream is waited for): returns
 * WACM_E_NONFINITE, with out filled, if out[9] > 0.
 */
int wacm_diagnostics(wacm_grid* grid, const wacm_params* prm, double t, const void* U,
                     const void* dus, double* out, void* stream);

/*
 * wacm_threshold_blocks -- wavelet details (Sec. 3.1) of a ghost-synchronised
 * pool U, normalised per component by the global max norm over interiors
 * (Sec. 3.4; a zero norm counts as 1).  For active block i (Morton order):
 * dmax[i] = largest normalised |u - P R u| over interior points with an odd
 * local index; mrange[i] = max chi - min chi over interior points at time t;
 * flags[i] = 1 (coarsen) iff level > jmin and either (dealias and level ==
 * jmax) or (dmax < eps and mrange == 0) (Sec. 3.3, 3.5).  dmax, mrange: device
 * doubles; flags: device int8; nb entries each.
 */
int wacm_threshold_blocks(wacm_grid* grid, const wacm_params* prm, double t, const void* U,
                          double eps, int32_t dealias, double* dmax, double* mrange,
                          int8_t* flags, void* stream);

/*
 * wacm_filter_blocks -- wavelet filtering (Sec. 3.1 details; the filtering at
 * the finest level of the results section's equidistant runs) of a
 * ghost-synchronised pool U, in place: in every active block of level
 * `level` (every block if level < 0) each interior point with an odd local
 * index is replaced by P R u, the tensor-product DD4 prediction from the
 * block's even-index points (ghost layers included), which removes the
 * block's details; points whose three indices are even, ghost layers and
 * other blocks are not changed.  Ghost layers are stale afterwards (sync
 * again before the next use).  Asynchronous on `stream`.
 */
int wacm_filter_blocks(wacm_grid* grid, void* U, int32_t level, void* stream);

/*
 * wacm_mr_forward / wacm_mr_inverse -- the multiresolution transform (Sec.
 * 3.1: details u - P R u iterated from the finest level down; Sec. 3.2:
 * lifted coarse values for CDF 4/4) of nfields periodic fields on the
 * equidistant lattice, in place.  No grid handle: u holds nfields arrays of
 * n^3 values of `dtype` (WACM_F32 / WACM_F64), x fastest, contiguous, on the
 * device.  Step m (m = 0 .. nlev-1, finest first; the inverse runs them in
 * reverse) works on the lattice of stride 2^m: its odd points (not all
 * coordinates multiples of 2^(m+1)) take their detail, the value minus the
 * tensor-product DD4 prediction from the even points; with WACM_CDF44 the
 * even points then take the lifted restriction of the stride-2^m values
 * (x, y, z), with WACM_CDF40 they keep their values (decimation).  Afterwards
 * the stride-2^nlev lattice holds the coarse approximation and a point whose
 * coordinates are all multiples of 2^m but not all of 2^(m+1) holds its
 * level-m detail.  wacm_mr_inverse reconstructs u up to rounding.
 * Requirements (WACM_E_INVAL otherwise): 4 <= n <= 1024, n a multiple of
 * 2^nlev with n / 2^nlev >= 4, 0 <= nlev <= 9, 1 <= nfields <= 65535, u not
 * NULL and aligned to two elements (16 bytes FP64, 8 bytes FP32); with
 * WACM_CDF44 and nlev > 0, work: a 256-byte aligned device buffer of
 * work_size >= wacm_mr_work_bytes(n, nfields, dtype) bytes (work may be NULL
 * and work_size 0 for WACM_CDF40 or nlev 0).  The caller owns u and work.
 * No allocation, no host synchronisation: asynchronous on `stream` and
 * graph-capturable.
 */
size_t wacm_mr_work_bytes(int64_t n, int32_t nfields, int32_t dtype); /* 0 if invalid */
int wacm_mr_forward(int64_t n, int32_t nfields, int32_t dtype, int32_t wavelet, int32_t nlev,
                    void* u, void* work, size_t work_size, void* stream);
int wacm_mr_inverse(int64_t n, int32_t nfields, int32_t dtype, int32_t wavelet, int32_t nlev,
                    void* u, void* work, size_t work_size, void* stream);

/*
 * wacm_mr_forward_noalloc -- wacm_mr_forward for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same kernels and results, with the
 * CDF 4/4 work buffer taken from a static device array of
 * WACM_MR_SCRATCH_BYTES bytes that the library holds on each GPU it runs on
 * until the process ends, instead of a `work` argument.  The caller still
 * passes u (on the current device).  No allocation of any kind.  Sizes whose
 * wacm_mr_work_bytes() exceeds WACM_MR_SCRATCH_BYTES are rejected with
 * WACM_E_INVAL when the wavelet is CDF 4/4 and nlev > 0 (e.g. FP64 allows
 * n = 128 with 4 fields; FP32 n = 256 with 1 field); other arguments as for
 * wacm_mr_forward.  Every call on one GPU shares that GPU's array: calls
 * that overlap in time on one GPU (different streams, or other threads)
 * race on it and must be ordered by the caller.  Each call writes every work
 * value it reads, so nothing carried over from an earlier call is used.
 * The first call on a device looks up the array's address there
 * (hipGetSymbolAddress), synchronously.
 */
#define WACM_MR_SCRATCH_BYTES (64 << 20)
int wacm_mr_forward_noalloc(int64_t n, int32_t nfields, int32_t dtype, int32_t wavelet,
                            int32_t nlev, void* u, void* stream);

/*
 * wacm_adapt -- change the grid (Sec. 3.5).  Synchronous.  The tables are
 * rebuilt inside the grid's workspaces; adjoint plans are dropped (set them
 * again before the next adjoint call).
 * WACM_REFINE_ALL: ghosts of U are synchronised, then every active block below
 *   jmax is replaced by its 8 children (even child points copy the parent,
 *   odd points take the tensor DD4 prediction, Sec. 3.1).  `flags` unused.
 * WACM_COARSEN: flags is a host int8 array of nb entries (Morton order, as
 *   from wacm_threshold_blocks).  8 sisters merge into their parent by
 *   decimation iff all are active and flagged and no active block touching the
 *   parent's box is finer than the sisters (grading).  One pass.
 * New blocks take free pool slots; the grid and the active blocks'
 * interiors are unchanged on error (WACM_E_CAPACITY if free slots run out;
 * free slots and ghost layers may have been written).  *nb_out (may be NULL) receives the
 * new number of active blocks.
 */
int wacm_adapt(wacm_grid* grid, int32_t op, const int8_t* flags, void* U, int64_t* nb_out,
               void* stream);

/*
 * ---- Discrete adjoint (frozen grid, fixed time step) --------------------
 * Exact transposes of the linearised operations above, for gradients of
 * J = sum_n dt F_x(U^n, t^n) (F_x: x-component of the penalization force,
 * Sec. 2.2) with respect to the plate pitch parameters theta = (amp, freq,
 * phase) and a static extra solid velocity dus.  Conventions: adjoint states
 * use the pool layout and element type; dtheta is a device array of 3
 * doubles and dusbar a device array [capacity][3][bs^3] of doubles (NULL:
 * not wanted); both are accumulated (+=), never cleared.  Reductions run in a
 * fixed order (bitwise reproducible).  wacm_sync_ghosts_adj needs the
 * transpose plan of the full ghost fill (face_only 0), wacm_rk4_step_adj the
 * plan of the depth-3 face star (face_only 1), each set once per grid with
 * wacm_adj_plan_set (WACM_E_INVAL otherwise).
 */

/* Bytes of the work buffer wacm_rk4_step_adj needs (8 pool-sized registers). */
size_t wacm_adj_work_bytes(const wacm_grid* grid);

/*
 * wacm_adj_plan_bytes / wacm_adj_plan_set -- the transpose of the ghost fill
 * as a gather plan: for every interior point some ghost value is copied or
 * predicted from (Sec. 3.1 weights), the ghost points that read it, sorted so
 * the accumulation order is fixed.  wacm_adj_plan_bytes builds the plan on
 * the host (kept in the handle) and returns its device size (0 on error);
 * wacm_adj_plan_set copies it into the caller's buffer ws (ws_bytes >= that
 * size, 256-byte aligned, kept until the grid changes or is destroyed).
 * Synchronous.  wacm_adapt drops both plans.
 */
size_t wacm_adj_plan_bytes(wacm_grid* grid, int32_t face_only);
int wacm_adj_plan_set(wacm_grid* grid, int32_t face_only, void* ws, size_t ws_bytes);

/*
 * wacm_sync_ghosts_adj -- transpose of wacm_sync_ghosts: the adjoint held at
 * every ghost point of Ub is added to the interior points its value was
 * copied or predicted from (with the prediction weights of Sec. 3.1), then
 * the ghost points are set to 0.  Interiors are accumulated.
 */
int wacm_sync_ghosts_adj(wacm_grid* grid, void* Ub, void* stream);

/*
 * wacm_rhs_acm_adj -- transpose of the rhs linearised at the ghost-synchronised
 * state U (Sec. 2.2-2.3): given the rhs adjoint V (interiors), Ub receives the
 * state adjoint at interior and depth-3 face ghost points (accumulated),
 * dtheta and dusbar the parameter adjoints at time t.
 */
int wacm_rhs_acm_adj(wacm_grid* grid, const wacm_params* prm, double t, const void* U,
                     const void* V, void* Ub, double* dtheta, double* dusbar, const void* dus,
                     void* stream);

/*
 * wacm_force_adj -- adds weight * dF_x/dU (interiors of Ub), weight * dF_x/dtheta
 * and weight * dF_x/ddus at time t, F_x = C_eta^-1 sum chi (u - u_s) h^3.
 */
int wacm_force_adj(wacm_grid* grid, const wacm_params* prm, double t, double weight,
                   const void* U, void* Ub, double* dtheta, double* dusbar, const void* dus,
                   void* stream);

/*
 * wacm_rk4_step_adj -- transpose of one wacm_rk4_step of size dt from time t
 * (fixed dt): Un is the checkpoint of the step's input (interiors); lam holds
 * the adjoint of the step's output on entry and of its input on return
 * (interiors).  Stage inputs are recomputed from Un.  work: device buffer of
 * wacm_adj_work_bytes(), 256-byte aligned.
 */
int wacm_rk4_step_adj(wacm_grid* grid, const wacm_params* prm, double t, double dt,
                      const void* Un, void* lam, double* dtheta, double* dusbar,
                      const void* dus, void* work, void* stream);

/*
 * Measurement support (not part of the method).  wacm_profile_enable(g, 1)
 * makes wacm_rk4_step / wacm_rk4_steps record a HIP event pair around each
 * group of kernels they launch on their stream; do not enable it while the
 * stream is being captured into a graph.  wacm_profile_read waits for the
 * recorded events and returns, per kernel class [0 time-step reduction,
 * 1 face halo of faces next to another level (the stage's ghost values that
 * are not read in place), 2 fused rhs + RK stage, 3 time update], the summed
 * milliseconds and the number of timed launches since the last read (host
 * arrays of 4), then resets them.
 */
int wacm_profile_enable(wacm_grid* grid, int32_t on);
int wacm_profile_read(wacm_grid* grid, double* ms, int64_t* launches);

/* Wall milliseconds of the last successful wacm_adapt on this grid, split
 * into ms[0] host work (leaf lists, merge decisions, table building and
 * uploads) and ms[1] device work (its ghost sync and refinement or
 * coarsening kernels, launch to completion); host array of 2.  Zero before
 * the first adaptation. */
int wacm_adapt_timing(const wacm_grid* grid, double* ms);

#pragma GCC visibility pop
#ifdef __cplusplus
}
#endif
#endif
