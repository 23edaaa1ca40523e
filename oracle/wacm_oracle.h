/*
 * wacm_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU reference ("the oracle") for the block-structured
 * wavelet-adaptive artificial-compressibility method of Engels, Schneider,
 * Reiss & Farge, "A wavelet-adaptive method for multiscale simulation of
 * turbulent flows in flying insects" (arXiv:1912.05371).
 *
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no source with the HIP
 * library under paper_1912_05371_amd/csrc; both sides receive the same
 * seeded inputs and their outputs are compared.
 *
 * Array layout used at this interface (chosen so that tests can compare
 * against the GPU pool without reshuffling): one block = 4 fields
 * (u, v, w, p), each a padded cube of P^3 doubles with P = bs + 2 ng,
 * x fastest.  Local index i in [-ng, bs+ng) maps to storage i + ng.
 * Interior points are i in [0, bs).  Blocks are stored in the order in
 * which the leaves were given to orc_grid_create.
 */
#ifndef WACM_ORACLE_H
#define WACM_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_grid orc_grid;

/* Physical and numerical parameters (Sec. 2.1-2.3). */
typedef struct {
  double nu;        /* kinematic viscosity                                  */
  double c0;        /* artificial speed of sound                            */
  double c_gamma;   /* dashpot damping constant                             */
  double c_eta;     /* penalization permeability                            */
  double c_sp;      /* sponge constant                                      */
  double l_sp;      /* sponge layer width at every face of [0,L]^3          */
  double u_inf[3];  /* sponge target velocity                               */
  double p_inf;     /* sponge target pressure                               */
  int32_t mask;     /* 0 none, 1 static sphere, 2 rotating plate            */
  int32_t sponge;   /* 0 off, 1 binary sponge layer                         */
  int32_t clip;     /* 1: chi < 1e-8 is set to exactly 0                     */
  int32_t pad0;
  double w;         /* smoothing width of the mask                           */
  double sph_c[3];  /* sphere centre                                        */
  double sph_r;     /* sphere radius                                        */
  double x_le[3];   /* plate: point on the rotation (leading-edge) axis      */
  double lo[3];     /* plate: body-frame box, lower corner                   */
  double hi[3];     /* plate: body-frame box, upper corner                   */
  double amp, freq, phase; /* pitch angle alpha(t) = amp sin(2 pi freq t + phase) */
  double cfl, cfl_eta, cfl_nu;
} orc_params;

/* Tam-Webb first-derivative coefficients a1..a3 (derived, see source). */
void orc_tam_webb(double a[3]);

/* Treecode: octal digits, level-1 digit most significant, digit = xbit + 2 ybit + 4 zbit. */
uint64_t orc_treecode_encode(int level, int64_t ix, int64_t iy, int64_t iz);
void orc_treecode_decode(uint64_t code, int level, int64_t* ix, int64_t* iy, int64_t* iz);

/* Grid of leaves.  Returns NULL and writes an error code (<0) to *err on
 * invalid input: -1 bad sizes, -2 overlap/not tiling, -3 not 2:1 balanced. */
orc_grid* orc_grid_create(int bs, int ng, double L, int jmin, int jmax, int64_t nleaves,
                          const int32_t* lev, const int64_t* ix, const int64_t* iy,
                          const int64_t* iz, int* err);
void orc_grid_free(orc_grid* g);
int64_t orc_grid_nb(const orc_grid* g);
void orc_grid_leaves(const orc_grid* g, int32_t* lev, int64_t* ix, int64_t* iy, int64_t* iz);
int orc_is_balanced(const orc_grid* g);

/* Owner of the level-J lattice point (gx,gy,gz) (periodic).  Returns block id
 * and the local index in the owner block; -1 if the point is not a grid point
 * of its owner. */
int64_t orc_owner(const orc_grid* g, int J, int64_t gx, int64_t gy, int64_t gz,
                  int64_t* li, int64_t* lj, int64_t* lk);

/* Ghost-node synchronisation (Sec. 4.2, Sec. 3.1 prediction/decimation).
 * With the CDF 4/4 wavelet, ghost points whose owner is finer then take the
 * lifted restriction (Sec. 3.2) of the owner's synchronised padded array. */
void orc_sync(const orc_grid* g, double* U);

/* Wavelet of restriction: 0 CDF 4/0 (decimation, default), 1 CDF 4/4 (lifted;
 * needs ng >= 6).  Returns 0, or -1 for an invalid choice.  Grids made by
 * refinement or coarsening inherit it. */
int orc_set_wavelet(orc_grid* g, int wavelet);
/* Taps (offsets -6..6) of the lifted low-pass along one axis: order 4 (CDF
 * 4/4) or 2 (CDF 2/2), from the lifting steps applied to unit impulses. */
void orc_lift_lowpass(int order, double taps[13]);

/* Multiresolution transform (Sec. 3.1, 3.2), in place, of nf periodic fields
 * of n^3 points (x fastest): nlev forward steps, finest first, or their
 * inverse.  wavelet 0: CDF 4/0 (coarse values by decimation), 1: CDF 4/4
 * (lifted coarse values).  The stride-2^nlev lattice then holds the coarse
 * approximation; a point whose coordinates are all multiples of 2^m but not
 * all of 2^(m+1) holds its level-m detail.  Returns -1 unless n is a
 * multiple of 2^nlev with n / 2^nlev >= 4, nf >= 1, 0 <= nlev <= 20. */
int orc_mr_forward(int64_t n, int nf, int nlev, int wavelet, double* u);
int orc_mr_inverse(int64_t n, int nf, int nlev, int wavelet, double* u);

/* Mask and solid velocity at interior points, at time t. chi: [nb][bs^3], us: [nb][3][bs^3]. */
void orc_mask(const orc_grid* g, const orc_params* p, double t, double* chi, double* us);

/* Right-hand side of the penalized ACM equations at interior points.  U must
 * be ghost-synchronised.  dU has the padded layout; only interiors are written.
 * dus (may be NULL): extra static solid velocity [nb][3][bs^3] added to u_s. */
void orc_rhs(const orc_grid* g, const orc_params* p, double t, const double* U,
             const double* dus, double* dU);

/* Time step from the stability limits (Sec. 2.3). */
double orc_dt(const orc_grid* g, const orc_params* p, const double* U);

/* One classical RK4 step of size dt in place (interiors advance). */
void orc_rk4_step(const orc_grid* g, const orc_params* p, double t, double dt, double* U,
                  const double* dus);

/* out[0]=max|u|, out[1..4]=Linf of u,v,w,p, out[5..7]=force, out[8]=energy. */
void orc_diagnostics(const orc_grid* g, const orc_params* p, double t, const double* U,
                     const double* dus, double out[9]);

/* Detail coefficients (Sec. 3.1, eq. for the details; Sec. 3.4 normalisation).
 * U must be ghost-synchronised.  Writes per-block max normalised detail and the
 * mask range max(chi)-min(chi) over the interior (p may be NULL: range 0). */
void orc_details(const orc_grid* g, const orc_params* p, double t, const double* U,
                 double* dmax, double* mrange);
/* wavelet filtering (details removed) of the blocks of one level (all if < 0) */
void orc_filter(const orc_grid* g, int level, double* U);
/* Coarsening flags (Sec. 3.3, 3.5). */
void orc_flags(const orc_grid* g, const double* dmax, const double* mrange, double eps,
               int dealias, int8_t* flags);

/* Refine every leaf below jmax into 8 children (Sec. 3.5 step 1).  U must be
 * ghost-synchronised.  Returns a new grid; Unew must hold nb_new blocks
 * (query with orc_refine_count).  Children are listed in Morton order. */
int64_t orc_refine_count(const orc_grid* g);
orc_grid* orc_refine_all(const orc_grid* g, const double* U, double* Unew);
/* One merge pass (Sec. 3.5 step 3).  Returns the new grid (Morton order). */
int64_t orc_coarsen_count(const orc_grid* g, const int8_t* flags);
orc_grid* orc_coarsen(const orc_grid* g, const int8_t* flags, const double* U, double* Unew);

/* ---- discrete adjoint (frozen grid, fixed dt) ---------------------------- */
/* theta = (amp, freq, phase) of the plate pitch; dus = static extra solid
 * velocity [nb][3][bs^3].  All adjoint outputs are accumulated. */
void orc_rhs_adj(const orc_grid* g, const orc_params* p, double t, const double* U,
                 const double* V, double* Ubar, double dtheta[3], double* dusbar,
                 const double* dus);
void orc_sync_adj(const orc_grid* g, double* Ubar);
double orc_force_x(const orc_grid* g, const orc_params* p, double t, const double* U,
                   const double* dus);
void orc_force_x_adj(const orc_grid* g, const orc_params* p, double t, double weight,
                     const double* U, double* Ubar, double dtheta[3], double* dusbar,
                     const double* dus);
void orc_rk4_step_adj(const orc_grid* g, const orc_params* p, double t, double dt,
                      const double* Un, double* Lam, double dtheta[3], double* dusbar,
                      const double* dus);

#ifdef __cplusplus
}
#endif
#endif
