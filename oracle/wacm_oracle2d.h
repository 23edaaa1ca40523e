/*
 * wacm_oracle2d.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain FP64 CPU reference ("the oracle") for the two-dimensional form of
 * the block-structured wavelet-adaptive artificial-compressibility method of
 * Engels, Schneider, Reiss & Farge (arXiv:1912.05371): the model of Sec. 2.1
 * with D = 2 (velocity (u, v), pressure p), discretised as in Sec. 2.3 on a
 * 2:1-balanced periodic quadtree of square blocks (Sec. 4.1), ghost nodes as
 * in Sec. 4.2 with the prediction and decimation of Sec. 3.1, details and
 * coarsening as in Sec. 3.1-3.5.  No penalization and no sponge: the
 * three-vortex case of the results section is periodic without walls.
 *
 * Layout at this interface: one block = 3 fields (u, v, p), each a padded
 * square of P^2 doubles, P = bs + 2 ng, x fastest; local index i in
 * [-ng, bs+ng) maps to storage i + ng; interior points are [0, bs)^2.
 * Blocks are stored in the order in which the leaves were given.
 * Only the tests and the benchmark's CPU-baseline leg load this library; it
 * shares no source with the HIP library.
 */
#ifndef WACM_ORACLE2D_H
#define WACM_ORACLE2D_H
#include <stdint.h>

#include "wacm_oracle.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc2_grid orc2_grid;

/* Grid of quadtree leaves (level, ix, iy).  NULL and *err < 0 on invalid
 * input: -1 sizes, -2 overlap or not tiling, -3 not 2:1 balanced. */
orc2_grid* orc2_grid_create(int bs, int ng, double L, int jmin, int jmax, int64_t nleaves,
                            const int32_t* lev, const int64_t* ix, const int64_t* iy, int* err);
void orc2_grid_free(orc2_grid* g);
int64_t orc2_grid_nb(const orc2_grid* g);
void orc2_grid_leaves(const orc2_grid* g, int32_t* lev, int64_t* ix, int64_t* iy);

/* Ghost-node synchronisation of every block (all ng layers), in place. */
void orc2_sync(const orc2_grid* g, double* U);
/* Right-hand side (Sec. 2.2 with D = 2) at interior points; U synchronised;
 * only nu, c0 and c_gamma of p are used. */
void orc2_rhs(const orc2_grid* g, const orc_params* p, const double* U, double* dU);
/* Time step (Sec. 2.3): min(cfl h_min / u_eig, cfl_nu h_min^2 / nu). */
double orc2_dt(const orc2_grid* g, const orc_params* p, const double* U);
/* One classical RK4 step of size dt, in place (interiors advance). */
void orc2_rk4_step(const orc2_grid* g, const orc_params* p, double dt, double* U);
/* out[0] max|u|, out[1..2] max |u|, |v|, out[3] 0, out[4] max |p|,
 * out[5..7] 0, out[8] energy 1/2 sum |u|^2 h^2. */
void orc2_diagnostics(const orc2_grid* g, const double* U, double out[9]);
/* Per-block max detail (Sec. 3.1), normalised per field by its global max
 * norm (Sec. 3.4, a zero norm counts as 1); U synchronised. */
void orc2_details(const orc2_grid* g, const double* U, double* dmax);
/* Coarsening flags (Sec. 3.3, 3.5): J > jmin and ((dealias and J == jmax)
 * or dmax < eps). */
void orc2_flags(const orc2_grid* g, const double* dmax, double eps, int dealias, int8_t* flags);
/* Refine every leaf below jmax into 4 children (DD4 prediction from the
 * synchronised parent); children in Morton order. */
int64_t orc2_refine_count(const orc2_grid* g);
orc2_grid* orc2_refine_all(const orc2_grid* g, const double* U, double* Unew);
/* One merge pass by decimation: 4 flagged sister leaves merge unless a leaf
 * touching the parent's box is finer than the sisters. */
int64_t orc2_coarsen_count(const orc2_grid* g, const int8_t* flags);
orc2_grid* orc2_coarsen(const orc2_grid* g, const int8_t* flags, const double* U, double* Unew);

#ifdef __cplusplus
}
#endif
#endif
