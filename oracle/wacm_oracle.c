/*
 * wacm_oracle.c -- TEST INFRASTRUCTURE ONLY (see wacm_oracle.h).
 *
 * A plain FP64 reference for the hot path of the wavelet-adaptive ACM block
 * method (arXiv:1912.05371).  Every routine follows the paper's definitions
 * in their stated order, with plain loops, no blocking and no fusion, so it
 * can be checked against the paper by eye.  Build with
 *   gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared
 * (no fast-math, no contraction).  OpenMP only splits independent blocks;
 * every reduction is serial and in block order, so results do not depend on
 * the thread count.
 *
 * Readings of points the paper leaves open (its appendices A-D are not part
 * of the text):
 *  - blocks are non-redundant: level J has 2^J blocks per axis, spacing
 *    h_J = L / (2^J bs), block interior index i in [0,bs) sits at
 *    x = (bx bs + i) h_J; bs is even so a coarse lattice point is an even
 *    point of the finer lattice and block origins align;
 *  - the ghost value of a point owned by a coarser block is the tensor
 *    product of the 4th-order Deslauriers-Dubuc prediction, read directly
 *    from the owners of the coarse lattice points (no ghost-to-ghost pass);
 *  - the grid is periodic in x, y and z and 2:1 graded across faces, edges
 *    and corners.
 */
#include "wacm_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define REF 20 /* reference level for integer positions (levels <= 18) */

struct orc_grid {
  int bs, ng, P, jmin, jmax;
  int wavelet; /* 0: CDF 4/0 (restriction = decimation), 1: CDF 4/4 (lifted) */
  double L;
  int64_t nb;
  int32_t* lev;
  int64_t *ix, *iy, *iz;
  int64_t hcap;
  uint64_t* hkey;
  int64_t* hval;
};

/* ------------------------------------------------------------------------ */
/* Tam-Webb coefficients (Sec. 2.3).  The first derivative is                 */
/*   D1 f_i = (1/h) sum_{m=1..3} a_m (f_{i+m} - f_{i-m}).                      */
/* Fourth order needs 2 sum m a_m = 1 and sum m^3 a_m = 0, which leaves       */
/* a1 = 2/3 + 5 t, a2 = -1/12 - 4 t, a3 = t.  Tam & Webb fix t by making the   */
/* modified wavenumber 2 sum a_m sin(m eta) closest to eta in the L2 sense on  */
/* 0 <= eta <= 1.1; the objective is quadratic in t, so                        */
/*   t = - int f0 f1 / int f1^2,                                               */
/*   f0 = 4/3 sin eta - 1/6 sin 2eta - eta,  f1 = 10 sin eta - 8 sin 2eta      */
/*        + 2 sin 3eta,                                                         */
/* with the integrals written out in closed form below.                       */
/* ------------------------------------------------------------------------ */
/* The closed forms cancel strongly; they are evaluated in long double so the
 * result rounds correctly to double. */
static long double int_sin_sin(int m, int n, long double X) { /* int_0^X sin(m e) sin(n e) de */
  if (m == n) return X / 2.0L - sinl(2.0L * m * X) / (4.0L * m);
  return sinl((long double)(m - n) * X) / (2.0L * (m - n)) -
         sinl((long double)(m + n) * X) / (2.0L * (m + n));
}
static long double int_e_sin(int m, long double X) { /* int_0^X e sin(m e) de */
  return sinl(m * X) / ((long double)m * m) - X * cosl(m * X) / m;
}

void orc_tam_webb(double a[3]) {
  const long double X = 1.1L;
  /* f0 = sum_m c0[m] sin(m e) - e ; f1 = sum_m c1[m] sin(m e), m = 1..3 */
  const long double c0[4] = {0.0L, 4.0L / 3.0L, -1.0L / 6.0L, 0.0L};
  const long double c1[4] = {0.0L, 10.0L, -8.0L, 2.0L};
  long double f0f1 = 0.0L, f1f1 = 0.0L;
  for (int m = 1; m <= 3; ++m) {
    for (int n = 1; n <= 3; ++n) {
      f0f1 += c0[m] * c1[n] * int_sin_sin(m, n, X);
      f1f1 += c1[m] * c1[n] * int_sin_sin(m, n, X);
    }
    f0f1 -= c1[m] * int_e_sin(m, X);
  }
  long double t = -f0f1 / f1f1;
  a[0] = (double)(2.0L / 3.0L + 5.0L * t);
  a[1] = (double)(-1.0L / 12.0L - 4.0L * t);
  a[2] = (double)t;
}

/* ------------------------------------------------------------------------ */
/* Treecode (Sec. 4.1): one octal digit per level, level 1 first.            */
/* ------------------------------------------------------------------------ */
uint64_t orc_treecode_encode(int level, int64_t ix, int64_t iy, int64_t iz) {
  uint64_t code = 0;
  for (int l = 1; l <= level; ++l) {
    int sh = level - l;
    uint64_t digit = (uint64_t)((ix >> sh) & 1) + 2u * (uint64_t)((iy >> sh) & 1) +
                     4u * (uint64_t)((iz >> sh) & 1);
    code = code * 8u + digit;
  }
  return code;
}

void orc_treecode_decode(uint64_t code, int level, int64_t* ix, int64_t* iy, int64_t* iz) {
  int64_t x = 0, y = 0, z = 0;
  for (int l = 1; l <= level; ++l) {
    int sh = 3 * (level - l);
    uint64_t digit = (code >> sh) & 7u;
    x = 2 * x + (int64_t)(digit & 1u);
    y = 2 * y + (int64_t)((digit >> 1) & 1u);
    z = 2 * z + (int64_t)((digit >> 2) & 1u);
  }
  *ix = x;
  *iy = y;
  *iz = z;
}

/* ------------------------------------------------------------------------ */
/* Grid: leaf list plus a hash from (level, block index) to block id.         */
/* ------------------------------------------------------------------------ */
static uint64_t hkey_of(int lev, int64_t x, int64_t y, int64_t z) {
  return ((uint64_t)lev << 57) | ((uint64_t)x << 38) | ((uint64_t)y << 19) | (uint64_t)z;
}
static uint64_t hmix(uint64_t k) {
  k ^= k >> 33;
  k *= 0xff51afd7ed558ccdULL;
  k ^= k >> 33;
  k *= 0xc4ceb9fe1a85ec53ULL;
  k ^= k >> 33;
  return k;
}
static int64_t hfind(const orc_grid* g, int lev, int64_t x, int64_t y, int64_t z) {
  uint64_t key = hkey_of(lev, x, y, z);
  int64_t pos = (int64_t)(hmix(key) & (uint64_t)(g->hcap - 1));
  for (;;) {
    if (g->hval[pos] < 0) return -1;
    if (g->hkey[pos] == key) return g->hval[pos];
    pos = (pos + 1) & (g->hcap - 1);
  }
}
static int hinsert(orc_grid* g, int lev, int64_t x, int64_t y, int64_t z, int64_t id) {
  uint64_t key = hkey_of(lev, x, y, z);
  int64_t pos = (int64_t)(hmix(key) & (uint64_t)(g->hcap - 1));
  for (;;) {
    if (g->hval[pos] < 0) {
      g->hkey[pos] = key;
      g->hval[pos] = id;
      return 0;
    }
    if (g->hkey[pos] == key) return -1; /* duplicate */
    pos = (pos + 1) & (g->hcap - 1);
  }
}

static int64_t wrap(int64_t a, int64_t n) {
  int64_t r = a % n;
  return r < 0 ? r + n : r;
}

void orc_grid_free(orc_grid* g) {
  if (!g) return;
  free(g->lev);
  free(g->ix);
  free(g->iy);
  free(g->iz);
  free(g->hkey);
  free(g->hval);
  free(g);
}

int64_t orc_grid_nb(const orc_grid* g) { return g->nb; }

void orc_grid_leaves(const orc_grid* g, int32_t* lev, int64_t* ix, int64_t* iy, int64_t* iz) {
  for (int64_t b = 0; b < g->nb; ++b) {
    lev[b] = g->lev[b];
    ix[b] = g->ix[b];
    iy[b] = g->iy[b];
    iz[b] = g->iz[b];
  }
}

/* Leaf whose half-open box contains the reference-lattice position (periodic). */
static int64_t leaf_at(const orc_grid* g, int64_t rx, int64_t ry, int64_t rz) {
  int64_t n = (int64_t)g->bs << REF;
  rx = wrap(rx, n);
  ry = wrap(ry, n);
  rz = wrap(rz, n);
  for (int K = g->jmin; K <= g->jmax; ++K) {
    int64_t span = (int64_t)g->bs << (REF - K);
    int64_t b = hfind(g, K, rx / span, ry / span, rz / span);
    if (b >= 0) return b;
  }
  return -1;
}

int64_t orc_owner(const orc_grid* g, int J, int64_t gx, int64_t gy, int64_t gz, int64_t* li,
                  int64_t* lj, int64_t* lk) {
  int64_t unitJ = (int64_t)1 << (REF - J);
  int64_t rx = gx * unitJ, ry = gy * unitJ, rz = gz * unitJ;
  int64_t n = (int64_t)g->bs << REF;
  rx = wrap(rx, n);
  ry = wrap(ry, n);
  rz = wrap(rz, n);
  int64_t b = leaf_at(g, rx, ry, rz);
  if (b < 0) return -1;
  int K = g->lev[b];
  int64_t unit = (int64_t)1 << (REF - K);
  int64_t span = (int64_t)g->bs << (REF - K);
  int64_t ox = rx - g->ix[b] * span, oy = ry - g->iy[b] * span, oz = rz - g->iz[b] * span;
  if (ox % unit || oy % unit || oz % unit) return -1;
  *li = ox / unit;
  *lj = oy / unit;
  *lk = oz / unit;
  return b;
}

/* Closed boxes of leaves a and b intersect (periodic). */
static int touches(const orc_grid* g, int64_t a, int64_t b) {
  int64_t n = (int64_t)g->bs << REF;
  int64_t sa = (int64_t)g->bs << (REF - g->lev[a]);
  int64_t sb = (int64_t)g->bs << (REF - g->lev[b]);
  const int64_t* ca[3] = {g->ix, g->iy, g->iz};
  for (int d = 0; d < 3; ++d) {
    int64_t a0 = ca[d][a] * sa, a1 = a0 + sa;
    int64_t b0 = ca[d][b] * sb, b1 = b0 + sb;
    int hit = 0;
    for (int s = -1; s <= 1; ++s) {
      int64_t c0 = b0 + s * n, c1 = b1 + s * n;
      if (c0 <= a1 && a0 <= c1) hit = 1;
    }
    if (!hit) return 0;
  }
  return 1;
}

int orc_is_balanced(const orc_grid* g) {
  int ok = 1;
#pragma omp parallel for schedule(dynamic, 64) reduction(&& : ok)
  for (int64_t a = 0; a < g->nb; ++a) {
    for (int64_t b = 0; b < g->nb; ++b) {
      int d = g->lev[a] - g->lev[b];
      if (d > 1 || d < -1) {
        if (touches(g, a, b)) ok = 0;
      }
    }
  }
  return ok;
}

static orc_grid* grid_alloc(int bs, int ng, double L, int jmin, int jmax, int64_t nb) {
  orc_grid* g = (orc_grid*)calloc(1, sizeof(orc_grid));
  g->bs = bs;
  g->ng = ng;
  g->P = bs + 2 * ng;
  g->jmin = jmin;
  g->jmax = jmax;
  g->L = L;
  g->nb = nb;
  g->lev = (int32_t*)malloc(sizeof(int32_t) * (nb ? nb : 1));
  g->ix = (int64_t*)malloc(sizeof(int64_t) * (nb ? nb : 1));
  g->iy = (int64_t*)malloc(sizeof(int64_t) * (nb ? nb : 1));
  g->iz = (int64_t*)malloc(sizeof(int64_t) * (nb ? nb : 1));
  int64_t cap = 16;
  while (cap < 2 * nb + 16) cap *= 2;
  g->hcap = cap;
  g->hkey = (uint64_t*)malloc(sizeof(uint64_t) * cap);
  g->hval = (int64_t*)malloc(sizeof(int64_t) * cap);
  for (int64_t i = 0; i < cap; ++i) g->hval[i] = -1;
  return g;
}

orc_grid* orc_grid_create(int bs, int ng, double L, int jmin, int jmax, int64_t nleaves,
                          const int32_t* lev, const int64_t* ix, const int64_t* iy,
                          const int64_t* iz, int* err) {
  *err = 0;
  if (bs < 2 * (ng + 3) || bs % 2 || ng < 3 || jmin < 0 || jmax > 18 || jmin > jmax ||
      nleaves <= 0 || !(L > 0)) {
    *err = -1;
    return NULL;
  }
  orc_grid* g = grid_alloc(bs, ng, L, jmin, jmax, nleaves);
  uint64_t vol = 0;
  for (int64_t b = 0; b < nleaves; ++b) {
    int J = lev[b];
    if (J < jmin || J > jmax || ix[b] < 0 || iy[b] < 0 || iz[b] < 0 ||
        ix[b] >= ((int64_t)1 << J) || iy[b] >= ((int64_t)1 << J) || iz[b] >= ((int64_t)1 << J)) {
      *err = -1;
      orc_grid_free(g);
      return NULL;
    }
    g->lev[b] = J;
    g->ix[b] = ix[b];
    g->iy[b] = iy[b];
    g->iz[b] = iz[b];
    if (hinsert(g, J, ix[b], iy[b], iz[b], b)) {
      *err = -2;
      orc_grid_free(g);
      return NULL;
    }
    vol += (uint64_t)1 << (3 * (jmax - J));
  }
  /* tiling: no leaf has a leaf ancestor, and the volumes add up to the domain */
  for (int64_t b = 0; b < nleaves; ++b) {
    for (int K = jmin; K < g->lev[b]; ++K) {
      int s = g->lev[b] - K;
      if (hfind(g, K, g->ix[b] >> s, g->iy[b] >> s, g->iz[b] >> s) >= 0) {
        *err = -2;
        orc_grid_free(g);
        return NULL;
      }
    }
  }
  if (vol != ((uint64_t)1 << (3 * jmax))) {
    *err = -2;
    orc_grid_free(g);
    return NULL;
  }
  if (!orc_is_balanced(g)) {
    *err = -3;
    orc_grid_free(g);
    return NULL;
  }
  return g;
}

/* ------------------------------------------------------------------------ */
/* Indexing helpers                                                            */
/* ------------------------------------------------------------------------ */
static inline int64_t pidx(const orc_grid* g, int64_t i, int64_t j, int64_t k) {
  int64_t P = g->P, n = g->ng;
  return ((k + n) * P + (j + n)) * P + (i + n);
}
static inline double* fld(const orc_grid* g, double* U, int64_t b, int c) {
  int64_t P3 = (int64_t)g->P * g->P * g->P;
  return U + (b * 4 + c) * P3;
}
static inline const double* cfld(const orc_grid* g, const double* U, int64_t b, int c) {
  int64_t P3 = (int64_t)g->P * g->P * g->P;
  return U + (b * 4 + c) * P3;
}
static double hlev(const orc_grid* g, int J) { return g->L / ((double)((int64_t)1 << J) * g->bs); }

/* ------------------------------------------------------------------------ */
/* Ghost-node synchronisation (Sec. 4.2) with prediction P_{J-1 -> J}         */
/* (Sec. 3.1, 4th-order Deslauriers-Dubuc) and restriction by decimation.      */
/* ------------------------------------------------------------------------ */
static const double DD4W[4] = {-1.0 / 16.0, 9.0 / 16.0, 9.0 / 16.0, -1.0 / 16.0};
static const int DD4O[4] = {-3, -1, 1, 3};

/* value of field c at the level-J lattice point G (unwrapped OK) as seen from a
 * block of level J: copy if the owner holds the point, else DD4 prediction from
 * the level-(J-1) lattice. */
static double lattice_value(const orc_grid* g, const double* U, int J, int c, int64_t gx,
                            int64_t gy, int64_t gz) {
  int64_t li, lj, lk;
  int64_t o = orc_owner(g, J, gx, gy, gz, &li, &lj, &lk);
  if (o >= 0) {
    int K = g->lev[o];
    if (K < J - 1 || K > J + 1) {
      fprintf(stderr, "oracle: owner level %d seen from level %d (grid not graded)\n", K, J);
      abort();
    }
    return cfld(g, U, o, c)[pidx(g, li, lj, lk)];
  }
  /* not a point of its owner: the owner is coarser (level J-1) */
  int64_t tx[4], ty[4], tz[4];
  double wx[4], wy[4], wz[4];
  int nx, ny, nz;
  int64_t Gs[3] = {gx, gy, gz};
  int64_t* T[3] = {tx, ty, tz};
  double* W[3] = {wx, wy, wz};
  int* N[3] = {&nx, &ny, &nz};
  for (int d = 0; d < 3; ++d) {
    if (wrap(Gs[d], 2) == 0) {
      T[d][0] = Gs[d] / 2;
      W[d][0] = 1.0;
      *N[d] = 1;
    } else {
      for (int m = 0; m < 4; ++m) {
        T[d][m] = (Gs[d] + DD4O[m]) / 2; /* exact: Gs odd, offset odd */
        W[d][m] = DD4W[m];
      }
      *N[d] = 4;
    }
  }
  double v = 0.0;
  for (int a = 0; a < nz; ++a)
    for (int b = 0; b < ny; ++b)
      for (int e = 0; e < nx; ++e) {
        int64_t si, sj, sk;
        int64_t o2 = orc_owner(g, J - 1, tx[e], ty[b], tz[a], &si, &sj, &sk);
        if (o2 < 0 || g->lev[o2] < J - 1) {
          fprintf(stderr, "oracle: coarse source not on its owner's lattice\n");
          abort();
        }
        double w = (wz[a] * wy[b]) * wx[e];
        v += w * cfld(g, U, o2, c)[pidx(g, si, sj, sk)];
      }
  return v;
}

/* ------------------------------------------------------------------------ */
/* Lifted restriction (Sec. 3.2, CDF 4/4).  Lifting the interpolating wavelet  */
/* of CDF 4/0 gives the primal wavelet 4 vanishing moments; the dual scaling   */
/* function changes with it, so restriction is no longer decimation.  Along   */
/* one axis, with u the fine values around an even point (offset 0):          */
/*   predict (the details of Sec. 3.1): d_m = u_m - P u at the odd offsets    */
/*            m = -3, -1, 1, 3, P the DD4 prediction from m-3, m-1, m+1, m+3;  */
/*   update:  c = u_0 + sum_m U_m d_m,  U = (-1, 9, 9, -1)/32 on m = -3..3,   */
/* the update of the interpolating family, half its predict filter, which    */
/* makes the low-pass keep the first 4 moments.  The linear analogue (predict */
/* (1/2, 1/2) at -1, 1, update 1/4 at -1, 1) is the CDF 2/2 case the paper    */
/* spells out.  A coarse value needs the fine values at offsets -6..6; in 3D  */
/* the axis restriction runs along x, then y, then z.                         */
/* ------------------------------------------------------------------------ */
static const double LIFTU[4] = {-1.0 / 32.0, 9.0 / 32.0, 9.0 / 32.0, -1.0 / 32.0};

static double lift_1d(int order, const double v[13]) {
  double c = v[6];
  if (order == 2) {
    for (int m = -1; m <= 1; m += 2) {
      double d = v[6 + m] - 0.5 * (v[6 + m - 1] + v[6 + m + 1]);
      c += 0.25 * d;
    }
    return c;
  }
  for (int k = 0; k < 4; ++k) {
    int m = 6 + DD4O[k];
    double pred = 0.0;
    for (int t = 0; t < 4; ++t) pred += DD4W[t] * v[m + DD4O[t]];
    c += LIFTU[k] * (v[m] - pred);
  }
  return c;
}

void orc_lift_lowpass(int order, double taps[13]) {
  for (int n = 0; n < 13; ++n) {
    double v[13] = {0};
    v[n] = 1.0;
    taps[n] = lift_1d(order, v);
  }
}

/* Lifted restriction at the even local point (i,j,k) of the padded field f. */
static double lift_restrict_3d(const orc_grid* g, const double* f, int64_t i, int64_t j,
                               int64_t k) {
  double ax[13][13];
  for (int z = 0; z < 13; ++z)
    for (int y = 0; y < 13; ++y) {
      double line[13];
      for (int x = 0; x < 13; ++x) line[x] = f[pidx(g, i - 6 + x, j - 6 + y, k - 6 + z)];
      ax[z][y] = lift_1d(4, line);
    }
  double ay[13];
  for (int z = 0; z < 13; ++z) ay[z] = lift_1d(4, ax[z]);
  return lift_1d(4, ay);
}

int orc_set_wavelet(orc_grid* g, int wavelet) {
  if (wavelet != 0 && wavelet != 1) return -1;
  if (wavelet == 1 && g->ng < 6) return -1; /* the lifted stencil reaches 6 fine points */
  g->wavelet = wavelet;
  return 0;
}

void orc_sync(const orc_grid* g, double* U) {
  const int bs = g->bs, ng = g->ng;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < g->nb; ++b) {
    int J = g->lev[b];
    int64_t ox = g->ix[b] * bs, oy = g->iy[b] * bs, oz = g->iz[b] * bs;
    for (int c = 0; c < 4; ++c) {
      double* f = fld(g, U, b, c);
      for (int64_t k = -ng; k < bs + ng; ++k)
        for (int64_t j = -ng; j < bs + ng; ++j)
          for (int64_t i = -ng; i < bs + ng; ++i) {
            int inside = (i >= 0 && i < bs && j >= 0 && j < bs && k >= 0 && k < bs);
            if (inside) continue;
            f[pidx(g, i, j, k)] = lattice_value(g, U, J, c, ox + i, oy + j, oz + k);
          }
    }
  }
  if (g->wavelet != 1) return;
  /* CDF 4/4: every ghost point whose owner is finer takes the lifted
   * restriction of the owner's level-(J+1) lattice around it, read from the
   * owner's padded array as synchronised above (CDF 4/0 values in its ghost
   * layers, which are 6 deep). */
  const int64_t n = g->nb * 4 * (int64_t)g->P * g->P * g->P;
  double* S = (double*)malloc(sizeof(double) * n);
  memcpy(S, U, sizeof(double) * n);
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < g->nb; ++b) {
    int J = g->lev[b];
    int64_t ox = g->ix[b] * bs, oy = g->iy[b] * bs, oz = g->iz[b] * bs;
    for (int64_t k = -ng; k < bs + ng; ++k)
      for (int64_t j = -ng; j < bs + ng; ++j)
        for (int64_t i = -ng; i < bs + ng; ++i) {
          int inside = (i >= 0 && i < bs && j >= 0 && j < bs && k >= 0 && k < bs);
          if (inside) continue;
          int64_t li, lj, lk;
          int64_t o = orc_owner(g, J, ox + i, oy + j, oz + k, &li, &lj, &lk);
          if (o < 0 || g->lev[o] != J + 1) continue;
          for (int c = 0; c < 4; ++c)
            fld(g, U, b, c)[pidx(g, i, j, k)] = lift_restrict_3d(g, cfld(g, S, o, c), li, lj, lk);
        }
  }
  free(S);
}

/* ------------------------------------------------------------------------ */
/* Mask chi and solid velocity u_s (Sec. 2.2).  The paper defers mask          */
/* generation to other work; here: a sphere with a tanh layer of width w, and  */
/* a thin plate rotating about its leading-edge (y) axis with                  */
/* alpha(t) = amp sin(2 pi freq t + phase).                                    */
/* ------------------------------------------------------------------------ */
static void mask_point(const orc_params* p, double t, double x, double y, double z, double* chi,
                       double us[3]) {
  us[0] = us[1] = us[2] = 0.0;
  *chi = 0.0;
  if (p->mask == 1) {
    double dx = x - p->sph_c[0], dy = y - p->sph_c[1], dz = z - p->sph_c[2];
    double d = sqrt(dx * dx + dy * dy + dz * dz) - p->sph_r;
    *chi = 0.5 * (1.0 - tanh(d / p->w));
  } else if (p->mask == 2) {
    const double twopi = 6.283185307179586476925286766559;
    double ph = twopi * p->freq * t + p->phase;
    double alpha = p->amp * sin(ph);
    double adot = p->amp * twopi * p->freq * cos(ph);
    double rx = x - p->x_le[0], ry = y - p->x_le[1], rz = z - p->x_le[2];
    double ca = cos(alpha), sa = sin(alpha);
    /* body frame: x' = R_y(alpha)^T r with R_y = [[c,0,s],[0,1,0],[-s,0,c]] */
    double xb[3];
    xb[0] = ca * rx - sa * rz;
    xb[1] = ry;
    xb[2] = sa * rx + ca * rz;
    double c = 1.0;
    for (int d = 0; d < 3; ++d)
      c *= 0.5 * (tanh((xb[d] - p->lo[d]) / p->w) - tanh((xb[d] - p->hi[d]) / p->w));
    *chi = c;
    /* u_s = alpha_dot e_y x r */
    us[0] = adot * rz;
    us[1] = 0.0;
    us[2] = -adot * rx;
  }
  if (p->clip && *chi < 1e-8) *chi = 0.0;
}

static double sponge_point(const orc_params* p, double L, double x, double y, double z) {
  if (!p->sponge) return 0.0;
  double q[3] = {x, y, z};
  for (int d = 0; d < 3; ++d)
    if (q[d] < p->l_sp || q[d] > L - p->l_sp) return 1.0;
  return 0.0;
}

void orc_mask(const orc_grid* g, const orc_params* p, double t, double* chi, double* us) {
  const int bs = g->bs;
  const int64_t n3 = (int64_t)bs * bs * bs;
  for (int64_t b = 0; b < g->nb; ++b) {
    double h = hlev(g, g->lev[b]);
    for (int k = 0; k < bs; ++k)
      for (int j = 0; j < bs; ++j)
        for (int i = 0; i < bs; ++i) {
          double x = (double)(g->ix[b] * bs + i) * h;
          double y = (double)(g->iy[b] * bs + j) * h;
          double z = (double)(g->iz[b] * bs + k) * h;
          double c, u[3];
          mask_point(p, t, x, y, z, &c, u);
          int64_t q = ((int64_t)k * bs + j) * bs + i;
          if (chi) chi[b * n3 + q] = c;
          if (us)
            for (int d = 0; d < 3; ++d) us[(b * 3 + d) * n3 + q] = u[d];
        }
  }
}

/* ------------------------------------------------------------------------ */
/* Right-hand side (Sec. 2.2, penalized momentum and pressure equations;      */
/* Sec. 2.3 finite differences).                                              */
/* ------------------------------------------------------------------------ */
void orc_rhs(const orc_grid* g, const orc_params* p, double t, const double* U,
             const double* dus, double* dU) {
  double a[3];
  orc_tam_webb(a);
  const int bs = g->bs;
  const int64_t n3 = (int64_t)bs * bs * bs;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < g->nb; ++b) {
    double h = hlev(g, g->lev[b]);
    const double* F[4];
    for (int c = 0; c < 4; ++c) F[c] = cfld(g, U, b, c);
    double* R[4];
    for (int c = 0; c < 4; ++c) R[c] = fld(g, dU, b, c);
    for (int64_t k = 0; k < bs; ++k)
      for (int64_t j = 0; j < bs; ++j)
        for (int64_t i = 0; i < bs; ++i) {
          int64_t s[3] = {1, g->P, (int64_t)g->P * g->P};
          int64_t q = pidx(g, i, j, k);
          double d1[4][3], d2[3][3];
          for (int c = 0; c < 4; ++c)
            for (int d = 0; d < 3; ++d) {
              const double* f = F[c];
              double acc = 0.0;
              for (int m = 1; m <= 3; ++m) acc += a[m - 1] * (f[q + m * s[d]] - f[q - m * s[d]]);
              d1[c][d] = acc / h;
            }
          for (int c = 0; c < 3; ++c)
            for (int d = 0; d < 3; ++d) {
              const double* f = F[c];
              double acc = -f[q - 2 * s[d]] / 12.0 + 4.0 * f[q - s[d]] / 3.0 - 5.0 * f[q] / 2.0 +
                           4.0 * f[q + s[d]] / 3.0 - f[q + 2 * s[d]] / 12.0;
              d2[c][d] = acc / (h * h);
            }
          double x = (double)(g->ix[b] * bs + i) * h;
          double y = (double)(g->iy[b] * bs + j) * h;
          double z = (double)(g->iz[b] * bs + k) * h;
          double chi, us[3];
          mask_point(p, t, x, y, z, &chi, us);
          int64_t qi = (k * bs + j) * bs + i;
          if (dus)
            for (int d = 0; d < 3; ++d) us[d] += dus[(b * 3 + d) * n3 + qi];
          double sp = sponge_point(p, g->L, x, y, z);
          double u[4];
          for (int c = 0; c < 4; ++c) u[c] = F[c][q];
          for (int c = 0; c < 3; ++c) {
            double conv = u[0] * d1[c][0] + u[1] * d1[c][1] + u[2] * d1[c][2];
            double lap = d2[c][0] + d2[c][1] + d2[c][2];
            double r = -conv - d1[3][c] + p->nu * lap;
            if (p->mask) r -= chi / p->c_eta * (u[c] - us[c]);
            if (p->sponge) r -= sp / p->c_sp * (u[c] - p->u_inf[c]);
            R[c][q] = r;
          }
          double div = d1[0][0] + d1[1][1] + d1[2][2];
          double rp = -p->c0 * p->c0 * div - p->c_gamma * u[3];
          if (p->sponge) rp -= sp / p->c_sp * (u[3] - p->p_inf);
          R[3][q] = rp;
        }
  }
}

/* ------------------------------------------------------------------------ */
/* Time step (Sec. 2.3 stability limits).                                     */
/* ------------------------------------------------------------------------ */
double orc_dt(const orc_grid* g, const orc_params* p, const double* U) {
  const int bs = g->bs;
  double umax = 0.0;
  int jfine = g->jmin;
  for (int64_t b = 0; b < g->nb; ++b) {
    if (g->lev[b] > jfine) jfine = g->lev[b];
    const double* u = cfld(g, U, b, 0);
    const double* v = cfld(g, U, b, 1);
    const double* w = cfld(g, U, b, 2);
    for (int64_t k = 0; k < bs; ++k)
      for (int64_t j = 0; j < bs; ++j)
        for (int64_t i = 0; i < bs; ++i) {
          int64_t q = pidx(g, i, j, k);
          double m = sqrt(u[q] * u[q] + v[q] * v[q] + w[q] * w[q]);
          if (m > umax) umax = m;
        }
  }
  double h = hlev(g, jfine);
  double ueig = umax + sqrt(umax * umax + p->c0 * p->c0);
  double dt = p->cfl * h / ueig;
  if (p->mask) {
    double d = p->cfl_eta * p->c_eta;
    if (d < dt) dt = d;
  }
  if (p->sponge) {
    double d = p->cfl_eta * p->c_sp;
    if (d < dt) dt = d;
  }
  if (p->nu > 0) {
    double d = p->cfl_nu * h * h / p->nu;
    if (d < dt) dt = d;
  }
  return dt;
}

/* ------------------------------------------------------------------------ */
/* Classical RK4 (Sec. 2.3).                                                  */
/* ------------------------------------------------------------------------ */
static void axpy_interior(const orc_grid* g, double* Y, const double* X, double a,
                          const double* K) { /* Y = X + a K on interiors */
  const int bs = g->bs;
#pragma omp parallel for schedule(static)
  for (int64_t b = 0; b < g->nb; ++b)
    for (int c = 0; c < 4; ++c) {
      double* y = fld(g, Y, b, c);
      const double* x = cfld(g, X, b, c);
      const double* kk = cfld(g, K, b, c);
      for (int64_t k = 0; k < bs; ++k)
        for (int64_t j = 0; j < bs; ++j)
          for (int64_t i = 0; i < bs; ++i) {
            int64_t q = pidx(g, i, j, k);
            y[q] = x[q] + a * kk[q];
          }
    }
}

void orc_rk4_step(const orc_grid* g, const orc_params* p, double t, double dt, double* U,
                  const double* dus) {
  const int64_t tot = g->nb * 4 * (int64_t)g->P * g->P * g->P;
  double* Us = (double*)calloc(tot, sizeof(double));
  double* k1 = (double*)calloc(tot, sizeof(double));
  double* k2 = (double*)calloc(tot, sizeof(double));
  double* k3 = (double*)calloc(tot, sizeof(double));
  double* k4 = (double*)calloc(tot, sizeof(double));
  memcpy(Us, U, sizeof(double) * tot);
  orc_sync(g, Us);
  orc_rhs(g, p, t, Us, dus, k1);
  axpy_interior(g, Us, U, 0.5 * dt, k1);
  orc_sync(g, Us);
  orc_rhs(g, p, t + 0.5 * dt, Us, dus, k2);
  axpy_interior(g, Us, U, 0.5 * dt, k2);
  orc_sync(g, Us);
  orc_rhs(g, p, t + 0.5 * dt, Us, dus, k3);
  axpy_interior(g, Us, U, dt, k3);
  orc_sync(g, Us);
  orc_rhs(g, p, t + dt, Us, dus, k4);
  const int bs = g->bs;
  for (int64_t b = 0; b < g->nb; ++b)
    for (int c = 0; c < 4; ++c) {
      double* u = fld(g, U, b, c);
      const double *a1 = cfld(g, k1, b, c), *a2 = cfld(g, k2, b, c), *a3 = cfld(g, k3, b, c),
                   *a4 = cfld(g, k4, b, c);
      for (int64_t k = 0; k < bs; ++k)
        for (int64_t j = 0; j < bs; ++j)
          for (int64_t i = 0; i < bs; ++i) {
            int64_t q = pidx(g, i, j, k);
            u[q] = u[q] + dt * (a1[q] + 2.0 * a2[q] + 2.0 * a3[q] + a4[q]) / 6.0;
          }
    }
  free(Us);
  free(k1);
  free(k2);
  free(k3);
  free(k4);
}

/* ------------------------------------------------------------------------ */
/* Diagnostics: max|u|, Linf norms, penalization force (Sec. 2.2, midpoint     */
/* rule) and kinetic energy.                                                   */
/* ------------------------------------------------------------------------ */
void orc_diagnostics(const orc_grid* g, const orc_params* p, double t, const double* U,
                     const double* dus, double out[9]) {
  const int bs = g->bs;
  const int64_t n3 = (int64_t)bs * bs * bs;
  for (int i = 0; i < 9; ++i) out[i] = 0.0;
  for (int64_t b = 0; b < g->nb; ++b) {
    double h = hlev(g, g->lev[b]);
    double vol = h * h * h;
    for (int64_t k = 0; k < bs; ++k)
      for (int64_t j = 0; j < bs; ++j)
        for (int64_t i = 0; i < bs; ++i) {
          int64_t q = pidx(g, i, j, k);
          double u[4];
          for (int c = 0; c < 4; ++c) u[c] = cfld(g, U, b, c)[q];
          double m = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
          if (m > out[0]) out[0] = m;
          for (int c = 0; c < 4; ++c)
            if (fabs(u[c]) > out[1 + c]) out[1 + c] = fabs(u[c]);
          if (p && p->mask) {
            double x = (double)(g->ix[b] * bs + i) * h;
            double y = (double)(g->iy[b] * bs + j) * h;
            double z = (double)(g->iz[b] * bs + k) * h;
            double chi, us[3];
            mask_point(p, t, x, y, z, &chi, us);
            int64_t qi = (k * bs + j) * bs + i;
            if (dus)
              for (int d = 0; d < 3; ++d) us[d] += dus[(b * 3 + d) * n3 + qi];
            for (int d = 0; d < 3; ++d) out[5 + d] += chi * (u[d] - us[d]) * vol / p->c_eta;
          }
          out[8] += 0.5 * (u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) * vol;
        }
  }
}

/* ------------------------------------------------------------------------ */
/* P R u of a block at its own level (Sec. 3.1): at a block-local point, the   */
/* tensor-product DD4 prediction from the block's even-index points (interior */
/* or ghost): weight 1 on each axis where the index is even, the 4 taps at    */
/* offsets -3, -1, +1, +3 where it is odd.  Summed z outer, then y, then x.    */
/* ------------------------------------------------------------------------ */
static double block_prediction(const orc_grid* g, const double* f, int64_t i, int64_t j,
                               int64_t k) {
  int64_t L[3] = {i, j, k};
  int64_t T[3][4];
  double W[3][4];
  int N[3];
  for (int d = 0; d < 3; ++d) {
    if (L[d] % 2 == 0) {
      T[d][0] = L[d];
      W[d][0] = 1.0;
      N[d] = 1;
    } else {
      for (int m = 0; m < 4; ++m) {
        T[d][m] = L[d] + DD4O[m];
        W[d][m] = DD4W[m];
      }
      N[d] = 4;
    }
  }
  double pred = 0.0;
  for (int a = 0; a < N[2]; ++a)
    for (int e = 0; e < N[1]; ++e)
      for (int x = 0; x < N[0]; ++x)
        pred += ((W[2][a] * W[1][e]) * W[0][x]) * f[pidx(g, T[0][x], T[1][e], T[2][a])];
  return pred;
}

/* ------------------------------------------------------------------------ */
/* Details (Sec. 3.1): d = u - P R u at points with an odd local index, where */
/* R keeps the even points and P is the tensor-product DD4 prediction.         */
/* Normalised per component by the global Linf norm (Sec. 3.4).               */
/* ------------------------------------------------------------------------ */
void orc_details(const orc_grid* g, const orc_params* p, double t, const double* U,
                 double* dmax, double* mrange) {
  const int bs = g->bs;
  double norm[4] = {0, 0, 0, 0};
  for (int64_t b = 0; b < g->nb; ++b)
    for (int c = 0; c < 4; ++c) {
      const double* f = cfld(g, U, b, c);
      for (int64_t k = 0; k < bs; ++k)
        for (int64_t j = 0; j < bs; ++j)
          for (int64_t i = 0; i < bs; ++i) {
            double v = fabs(f[pidx(g, i, j, k)]);
            if (v > norm[c]) norm[c] = v;
          }
    }
  for (int c = 0; c < 4; ++c)
    if (norm[c] == 0.0) norm[c] = 1.0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < g->nb; ++b) {
    double dm = 0.0;
    for (int c = 0; c < 4; ++c) {
      const double* f = cfld(g, U, b, c);
      for (int64_t k = 0; k < bs; ++k)
        for (int64_t j = 0; j < bs; ++j)
          for (int64_t i = 0; i < bs; ++i) {
            if (i % 2 == 0 && j % 2 == 0 && k % 2 == 0) continue;
            double d = fabs(f[pidx(g, i, j, k)] - block_prediction(g, f, i, j, k)) / norm[c];
            if (d > dm) dm = d;
          }
    }
    dmax[b] = dm;
    double cmin = 1e300, cmax = -1e300;
    if (p && p->mask) {
      double h = hlev(g, g->lev[b]);
      for (int64_t k = 0; k < bs; ++k)
        for (int64_t j = 0; j < bs; ++j)
          for (int64_t i = 0; i < bs; ++i) {
            double chi, us[3];
            mask_point(p, t, (double)(g->ix[b] * bs + i) * h, (double)(g->iy[b] * bs + j) * h,
                       (double)(g->iz[b] * bs + k) * h, &chi, us);
            if (chi < cmin) cmin = chi;
            if (chi > cmax) cmax = chi;
          }
      mrange[b] = cmax - cmin;
    } else {
      mrange[b] = 0.0;
    }
  }
}

/* ------------------------------------------------------------------------ */
/* Wavelet filtering of blocks at their own level: removing the details      */
/* (Sec. 3.1) sets every interior point with an odd local index to P R u; the */
/* even points are kept.  With level >= 0 only blocks of that level are       */
/* filtered (filtering at the finest level, as in the equidistant runs of the */
/* results section); level < 0 filters every block.  U must be ghost-synced.  */
/* ------------------------------------------------------------------------ */
void orc_filter(const orc_grid* g, int level, double* U) {
  const int bs = g->bs;
  const int64_t n3 = (int64_t)bs * bs * bs;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < g->nb; ++b) {
    if (level >= 0 && g->lev[b] != level) continue;
    double* pred = (double*)malloc(sizeof(double) * n3);
    for (int c = 0; c < 4; ++c) {
      double* f = fld(g, U, b, c);
      /* all predictions from the unfiltered block first, then the writes */
      for (int64_t k = 0; k < bs; ++k)
        for (int64_t j = 0; j < bs; ++j)
          for (int64_t i = 0; i < bs; ++i)
            pred[(k * bs + j) * bs + i] = block_prediction(g, f, i, j, k);
      for (int64_t k = 0; k < bs; ++k)
        for (int64_t j = 0; j < bs; ++j)
          for (int64_t i = 0; i < bs; ++i)
            if (i % 2 != 0 || j % 2 != 0 || k % 2 != 0)
              f[pidx(g, i, j, k)] = pred[(k * bs + j) * bs + i];
    }
    free(pred);
  }
}

void orc_flags(const orc_grid* g, const double* dmax, const double* mrange, double eps,
               int dealias, int8_t* flags) {
  for (int64_t b = 0; b < g->nb; ++b) {
    int J = g->lev[b];
    int f = 0;
    if (J > g->jmin) {
      if (dealias && J == g->jmax)
        f = 1;
      else if (dmax[b] < eps && mrange[b] == 0.0)
        f = 1;
    }
    flags[b] = (int8_t)f;
  }
}

/* ------------------------------------------------------------------------ */
/* Adaptation (Sec. 3.5): refine all, and one pass of the coarsening merge.   */
/* ------------------------------------------------------------------------ */
typedef struct {
  uint64_t key;
  int32_t lev;
  int64_t x, y, z;
  int64_t src;  /* source block (parent for refinement, first child for merge) */
  int32_t kind; /* 0 copy, 1 child of src, 2 merged parent */
} newleaf;

static int cmp_newleaf(const void* A, const void* B) {
  const newleaf* a = (const newleaf*)A;
  const newleaf* b = (const newleaf*)B;
  return a->key < b->key ? -1 : (a->key > b->key ? 1 : 0);
}
static uint64_t morton_key(int lev, int64_t x, int64_t y, int64_t z) {
  return orc_treecode_encode(lev, x, y, z) << (3 * (REF - lev));
}

int64_t orc_refine_count(const orc_grid* g) {
  int64_t n = 0;
  for (int64_t b = 0; b < g->nb; ++b) n += (g->lev[b] < g->jmax) ? 8 : 1;
  return n;
}

static orc_grid* grid_from_newleaves(const orc_grid* g, newleaf* nl, int64_t n) {
  qsort(nl, n, sizeof(newleaf), cmp_newleaf);
  orc_grid* h = grid_alloc(g->bs, g->ng, g->L, g->jmin, g->jmax, n);
  h->wavelet = g->wavelet;
  for (int64_t b = 0; b < n; ++b) {
    h->lev[b] = nl[b].lev;
    h->ix[b] = nl[b].x;
    h->iy[b] = nl[b].y;
    h->iz[b] = nl[b].z;
    hinsert(h, nl[b].lev, nl[b].x, nl[b].y, nl[b].z, b);
  }
  return h;
}

orc_grid* orc_refine_all(const orc_grid* g, const double* U, double* Unew) {
  const int bs = g->bs;
  const int64_t P3 = (int64_t)g->P * g->P * g->P;
  int64_t n = orc_refine_count(g);
  newleaf* nl = (newleaf*)malloc(sizeof(newleaf) * n);
  int64_t m = 0;
  for (int64_t b = 0; b < g->nb; ++b) {
    int J = g->lev[b];
    if (J < g->jmax) {
      for (int cz = 0; cz < 2; ++cz)
        for (int cy = 0; cy < 2; ++cy)
          for (int cx = 0; cx < 2; ++cx) {
            newleaf* q = &nl[m++];
            q->lev = J + 1;
            q->x = 2 * g->ix[b] + cx;
            q->y = 2 * g->iy[b] + cy;
            q->z = 2 * g->iz[b] + cz;
            q->key = morton_key(q->lev, q->x, q->y, q->z);
            q->src = b;
            q->kind = 1;
          }
    } else {
      newleaf* q = &nl[m++];
      q->lev = J;
      q->x = g->ix[b];
      q->y = g->iy[b];
      q->z = g->iz[b];
      q->key = morton_key(J, q->x, q->y, q->z);
      q->src = b;
      q->kind = 0;
    }
  }
  orc_grid* h = grid_from_newleaves(g, nl, n);
  memset(Unew, 0, sizeof(double) * n * 4 * P3);
  for (int64_t nb = 0; nb < n; ++nb) {
    const newleaf* q = &nl[nb];
    if (q->kind == 0) {
      memcpy(Unew + nb * 4 * P3, U + q->src * 4 * P3, sizeof(double) * 4 * P3);
      continue;
    }
    int64_t off[3] = {(q->x & 1) * bs, (q->y & 1) * bs, (q->z & 1) * bs};
    for (int c = 0; c < 4; ++c) {
      const double* f = cfld(g, U, q->src, c);
      double* o = fld(h, Unew, nb, c);
      for (int64_t k = 0; k < bs; ++k)
        for (int64_t j = 0; j < bs; ++j)
          for (int64_t i = 0; i < bs; ++i) {
            /* child point at parent half-index (off + i) */
            int64_t Q[3] = {off[0] + i, off[1] + j, off[2] + k};
            int64_t T[3][4];
            double W[3][4];
            int N[3];
            for (int d = 0; d < 3; ++d) {
              if (Q[d] % 2 == 0) {
                T[d][0] = Q[d] / 2;
                W[d][0] = 1.0;
                N[d] = 1;
              } else {
                for (int mm = 0; mm < 4; ++mm) {
                  T[d][mm] = (Q[d] + DD4O[mm]) / 2;
                  W[d][mm] = DD4W[mm];
                }
                N[d] = 4;
              }
            }
            double v = 0.0;
            for (int a = 0; a < N[2]; ++a)
              for (int e = 0; e < N[1]; ++e)
                for (int x = 0; x < N[0]; ++x)
                  v += ((W[2][a] * W[1][e]) * W[0][x]) * f[pidx(g, T[0][x], T[1][e], T[2][a])];
            o[pidx(h, i, j, k)] = v;
          }
    }
  }
  free(nl);
  return h;
}

/* A parent (level J-1, index x,y,z) may replace its 8 children if all are
 * flagged leaves and no leaf touching the parent's box is finer than J. */
static int can_merge(const orc_grid* g, const int8_t* flags, int J, int64_t px, int64_t py,
                     int64_t pz) {
  for (int c = 0; c < 8; ++c) {
    int64_t b = hfind(g, J, 2 * px + (c & 1), 2 * py + ((c >> 1) & 1), 2 * pz + ((c >> 2) & 1));
    if (b < 0 || !flags[b]) return 0;
  }
  int64_t n = (int64_t)g->bs << REF;
  int64_t sp = (int64_t)g->bs << (REF - (J - 1));
  int64_t P0[3] = {px * sp, py * sp, pz * sp};
  for (int64_t b = 0; b < g->nb; ++b) {
    if (g->lev[b] <= J) continue;
    int64_t sb = (int64_t)g->bs << (REF - g->lev[b]);
    int64_t B0[3] = {g->ix[b] * sb, g->iy[b] * sb, g->iz[b] * sb};
    int hit = 1;
    for (int d = 0; d < 3 && hit; ++d) {
      int any = 0;
      for (int s = -1; s <= 1; ++s) {
        int64_t c0 = B0[d] + s * n, c1 = c0 + sb;
        if (c0 <= P0[d] + sp && P0[d] <= c1) any = 1;
      }
      hit = any;
    }
    if (hit) return 0;
  }
  return 1;
}

static int64_t merge_plan(const orc_grid* g, const int8_t* flags, newleaf* nl) {
  /* Returns the number of new leaves; if nl != NULL fills them. */
  int64_t m = 0;
  for (int64_t b = 0; b < g->nb; ++b) {
    int J = g->lev[b];
    int64_t x = g->ix[b], y = g->iy[b], z = g->iz[b];
    int merged = 0, first = 0;
    if (J > g->jmin && flags[b] && can_merge(g, flags, J, x >> 1, y >> 1, z >> 1)) {
      merged = 1;
      first = ((x & 1) == 0 && (y & 1) == 0 && (z & 1) == 0);
    }
    if (!merged) {
      if (nl) {
        newleaf* q = &nl[m];
        q->lev = J;
        q->x = x;
        q->y = y;
        q->z = z;
        q->key = morton_key(J, x, y, z);
        q->src = b;
        q->kind = 0;
      }
      ++m;
    } else if (first) {
      if (nl) {
        newleaf* q = &nl[m];
        q->lev = J - 1;
        q->x = x >> 1;
        q->y = y >> 1;
        q->z = z >> 1;
        q->key = morton_key(J - 1, q->x, q->y, q->z);
        q->src = -1;
        q->kind = 2;
      }
      ++m;
    }
  }
  return m;
}

int64_t orc_coarsen_count(const orc_grid* g, const int8_t* flags) {
  return merge_plan(g, flags, NULL);
}

orc_grid* orc_coarsen(const orc_grid* g, const int8_t* flags, const double* U, double* Unew) {
  const int bs = g->bs;
  const int64_t P3 = (int64_t)g->P * g->P * g->P;
  int64_t n = merge_plan(g, flags, NULL);
  newleaf* nl = (newleaf*)malloc(sizeof(newleaf) * (n ? n : 1));
  merge_plan(g, flags, nl);
  orc_grid* h = grid_from_newleaves(g, nl, n);
  memset(Unew, 0, sizeof(double) * n * 4 * P3);
  for (int64_t nb = 0; nb < n; ++nb) {
    const newleaf* q = &nl[nb];
    if (q->kind == 0) {
      memcpy(Unew + nb * 4 * P3, U + q->src * 4 * P3, sizeof(double) * 4 * P3);
      continue;
    }
    int J = q->lev + 1;
    for (int c = 0; c < 4; ++c) {
      double* o = fld(h, Unew, nb, c);
      for (int64_t k = 0; k < bs; ++k)
        for (int64_t j = 0; j < bs; ++j)
          for (int64_t i = 0; i < bs; ++i) {
            /* decimation: parent point i is child point 2i (Sec. 3.1, R) */
            int64_t Q[3] = {2 * i, 2 * j, 2 * k};
            int64_t C[3], Lc[3];
            for (int d = 0; d < 3; ++d) {
              C[d] = Q[d] >= bs ? 1 : 0;
              Lc[d] = Q[d] - C[d] * bs;
            }
            int64_t child = hfind(g, J, 2 * q->x + C[0], 2 * q->y + C[1], 2 * q->z + C[2]);
            /* CDF 4/4: the lifted restriction over the child's synchronised
             * padded array (its 6-deep ghost layers hold the sisters' and
             * neighbours' values) */
            o[pidx(h, i, j, k)] =
                g->wavelet == 1 ? lift_restrict_3d(g, cfld(g, U, child, c), Lc[0], Lc[1], Lc[2])
                                : cfld(g, U, child, c)[pidx(g, Lc[0], Lc[1], Lc[2])];
          }
    }
  }
  free(nl);
  return h;
}

/* ======================================================================== */
/* Discrete adjoint on a frozen grid with a fixed time step.                  */
/*                                                                            */
/* Objective J = sum_n dt F_x(U^n, t^n), F_x the x-component of the          */
/* penalization force (Sec. 2.2).  Parameters: theta = (A, f, phi) of the      */
/* plate pitch angle alpha(t) = A sin(2 pi f t + phi), and a static extra      */
/* solid velocity dus(x) added to u_s.  Every routine below is the exact       */
/* transpose of the linearisation of the corresponding forward routine,        */
/* written in scatter form: each forward dependency y += c x becomes          */
/* xbar += c ybar.                                                             */
/* ======================================================================== */

/* alpha, alpha_dot and their derivatives with respect to (A, f, phi). */
static void pitch(const orc_params* p, double t, double* al, double* ad, double dal[3],
                  double dad[3]) {
  const double twopi = 6.283185307179586476925286766559;
  double ps = twopi * p->freq * t + p->phase;
  double s = sin(ps), c = cos(ps);
  *al = p->amp * s;
  *ad = p->amp * twopi * p->freq * c;
  dal[0] = s;
  dal[1] = p->amp * c * twopi * t;
  dal[2] = p->amp * c;
  dad[0] = twopi * p->freq * c;
  dad[1] = p->amp * twopi * c - p->amp * twopi * p->freq * s * twopi * t;
  dad[2] = -p->amp * twopi * p->freq * s;
}

/* plate mask, its derivative in alpha, and d u_s / d alpha_dot */
static void plate_point(const orc_params* p, double t, double x, double y, double z, double* chi,
                        double* dchi, double us[3], double dus_dad[3], double dal[3],
                        double dad[3]) {
  double al, ad;
  pitch(p, t, &al, &ad, dal, dad);
  double rx = x - p->x_le[0], ry = y - p->x_le[1], rz = z - p->x_le[2];
  double ca = cos(al), sa = sin(al);
  double xb[3] = {ca * rx - sa * rz, ry, sa * rx + ca * rz};
  double dxb[3] = {-xb[2], 0.0, xb[0]}; /* d x'/d alpha */
  double g[3], gp[3];
  for (int d = 0; d < 3; ++d) {
    double a = tanh((xb[d] - p->lo[d]) / p->w), b = tanh((xb[d] - p->hi[d]) / p->w);
    g[d] = 0.5 * (a - b);
    gp[d] = 0.5 * ((1.0 - a * a) - (1.0 - b * b)) / p->w;
  }
  *chi = g[0] * g[1] * g[2];
  *dchi = gp[0] * dxb[0] * g[1] * g[2] + g[0] * gp[1] * dxb[1] * g[2] +
          g[0] * g[1] * gp[2] * dxb[2];
  if (p->clip && *chi < 1e-8) {
    *chi = 0.0;
    *dchi = 0.0;
  }
  us[0] = ad * rz;
  us[1] = 0.0;
  us[2] = -ad * rx;
  dus_dad[0] = rz;
  dus_dad[1] = 0.0;
  dus_dad[2] = -rx;
}

/* Transpose of the linearised rhs at the synchronised state U: V holds the
 * rhs adjoint at interior points (padded layout); Ubar (padded) receives the
 * state adjoint at interior and ghost points (accumulated); dtheta and dusbar
 * (may be NULL) accumulate the parameter adjoints. */
void orc_rhs_adj(const orc_grid* g, const orc_params* p, double t, const double* U,
                 const double* V, double* Ubar, double dtheta[3], double* dusbar,
                 const double* dus) {
  double a[3];
  orc_tam_webb(a);
  const double w2[5] = {-1.0 / 12.0, 4.0 / 3.0, -5.0 / 2.0, 4.0 / 3.0, -1.0 / 12.0};
  const int bs = g->bs;
  const int64_t n3 = (int64_t)bs * bs * bs;
  for (int64_t b = 0; b < g->nb; ++b) {
    double h = hlev(g, g->lev[b]);
    const double* F[4];
    const double* R[4];
    double* B[4];
    for (int c = 0; c < 4; ++c) {
      F[c] = cfld(g, U, b, c);
      R[c] = cfld(g, V, b, c);
      B[c] = fld(g, Ubar, b, c);
    }
    int64_t s[3] = {1, g->P, (int64_t)g->P * g->P};
    for (int64_t k = 0; k < bs; ++k)
      for (int64_t j = 0; j < bs; ++j)
        for (int64_t i = 0; i < bs; ++i) {
          int64_t q = pidx(g, i, j, k);
          int64_t qi = (k * bs + j) * bs + i;
          double v[4], u[4];
          for (int c = 0; c < 4; ++c) {
            v[c] = R[c][q];
            u[c] = F[c][q];
          }
          double x = (double)(g->ix[b] * bs + i) * h;
          double y = (double)(g->iy[b] * bs + j) * h;
          double z = (double)(g->iz[b] * bs + k) * h;
          /* velocity equations */
          for (int c = 0; c < 3; ++c) {
            for (int d = 0; d < 3; ++d) {
              /* r_c -= u_d D1_d u_c */
              double d1 = 0.0;
              for (int m = 1; m <= 3; ++m)
                d1 += a[m - 1] * (F[c][q + m * s[d]] - F[c][q - m * s[d]]);
              d1 /= h;
              B[d][q] += -v[c] * d1;
              for (int m = 1; m <= 3; ++m) {
                B[c][q + m * s[d]] += -v[c] * u[d] * a[m - 1] / h;
                B[c][q - m * s[d]] += v[c] * u[d] * a[m - 1] / h;
              }
              /* r_c += nu D2_d u_c */
              for (int o = -2; o <= 2; ++o) B[c][q + o * s[d]] += p->nu * v[c] * w2[o + 2] / (h * h);
            }
            /* r_c -= D1_c p */
            for (int m = 1; m <= 3; ++m) {
              B[3][q + m * s[c]] += -v[c] * a[m - 1] / h;
              B[3][q - m * s[c]] += v[c] * a[m - 1] / h;
            }
          }
          /* pressure equation: r_p = -C0^2 sum_d D1_d u_d - C_gamma p */
          for (int d = 0; d < 3; ++d)
            for (int m = 1; m <= 3; ++m) {
              B[d][q + m * s[d]] += -p->c0 * p->c0 * v[3] * a[m - 1] / h;
              B[d][q - m * s[d]] += p->c0 * p->c0 * v[3] * a[m - 1] / h;
            }
          B[3][q] += -p->c_gamma * v[3];
          /* sponge */
          if (p->sponge) {
            double sp = sponge_point(p, g->L, x, y, z);
            for (int c = 0; c < 4; ++c) B[c][q] += -sp / p->c_sp * v[c];
          }
          /* penalization and its parameters */
          if (p->mask == 1) {
            double chi, us[3];
            mask_point(p, t, x, y, z, &chi, us);
            for (int c = 0; c < 3; ++c) {
              B[c][q] += -chi / p->c_eta * v[c];
              if (dusbar) dusbar[(b * 3 + c) * n3 + qi] += chi / p->c_eta * v[c];
            }
          } else if (p->mask == 2) {
            double chi, dchi, us[3], dsd[3], dal[3], dad[3];
            plate_point(p, t, x, y, z, &chi, &dchi, us, dsd, dal, dad);
            double e[3];
            for (int c = 0; c < 3; ++c) e[c] = dus ? dus[(b * 3 + c) * n3 + qi] : 0.0;
            double gal = 0.0, gad = 0.0;
            for (int c = 0; c < 3; ++c) {
              B[c][q] += -chi / p->c_eta * v[c];
              if (dusbar) dusbar[(b * 3 + c) * n3 + qi] += chi / p->c_eta * v[c];
              gal += -dchi / p->c_eta * (u[c] - us[c] - e[c]) * v[c];
              gad += chi / p->c_eta * dsd[c] * v[c];
            }
            for (int k2 = 0; k2 < 3; ++k2) dtheta[k2] += gal * dal[k2] + gad * dad[k2];
          }
        }
  }
}

/* Transpose of ghost synchronisation: the adjoint held at each ghost point
 * goes back to the interior points its value was copied or predicted from
 * (weights of Sec. 3.1), then the ghost entry is cleared. */
void orc_sync_adj(const orc_grid* g, double* Ubar) {
  const int bs = g->bs, ng = g->ng;
  for (int64_t b = 0; b < g->nb; ++b) {
    int J = g->lev[b];
    int64_t ox = g->ix[b] * bs, oy = g->iy[b] * bs, oz = g->iz[b] * bs;
    for (int c = 0; c < 4; ++c) {
      double* f = fld(g, Ubar, b, c);
      for (int64_t k = -ng; k < bs + ng; ++k)
        for (int64_t j = -ng; j < bs + ng; ++j)
          for (int64_t i = -ng; i < bs + ng; ++i) {
            int inside = (i >= 0 && i < bs && j >= 0 && j < bs && k >= 0 && k < bs);
            if (inside) continue;
            int64_t q = pidx(g, i, j, k);
            double gb = f[q];
            if (gb == 0.0) continue;
            f[q] = 0.0;
            int64_t G[3] = {ox + i, oy + j, oz + k};
            int64_t li, lj, lk;
            int64_t o = orc_owner(g, J, G[0], G[1], G[2], &li, &lj, &lk);
            if (o >= 0) {
              fld(g, Ubar, o, c)[pidx(g, li, lj, lk)] += gb;
              continue;
            }
            int64_t T[3][4];
            double W[3][4];
            int N[3];
            for (int d = 0; d < 3; ++d) {
              if (wrap(G[d], 2) == 0) {
                T[d][0] = G[d] / 2;
                W[d][0] = 1.0;
                N[d] = 1;
              } else {
                for (int m = 0; m < 4; ++m) {
                  T[d][m] = (G[d] + DD4O[m]) / 2;
                  W[d][m] = DD4W[m];
                }
                N[d] = 4;
              }
            }
            for (int az = 0; az < N[2]; ++az)
              for (int ay = 0; ay < N[1]; ++ay)
                for (int ax = 0; ax < N[0]; ++ax) {
                  int64_t si, sj, sk;
                  int64_t o2 = orc_owner(g, J - 1, T[0][ax], T[1][ay], T[2][az], &si, &sj, &sk);
                  double w = (W[2][az] * W[1][ay]) * W[0][ax];
                  fld(g, Ubar, o2, c)[pidx(g, si, sj, sk)] += w * gb;
                }
          }
    }
  }
}

/* x-force F_x at time t and its adjoint (weight * dF_x/d...). */
double orc_force_x(const orc_grid* g, const orc_params* p, double t, const double* U,
                   const double* dus) {
  double out[9];
  orc_diagnostics(g, p, t, U, dus, out);
  return out[5];
}

void orc_force_x_adj(const orc_grid* g, const orc_params* p, double t, double weight,
                     const double* U, double* Ubar, double dtheta[3], double* dusbar,
                     const double* dus) {
  const int bs = g->bs;
  const int64_t n3 = (int64_t)bs * bs * bs;
  if (!p->mask) return;
  for (int64_t b = 0; b < g->nb; ++b) {
    double h = hlev(g, g->lev[b]);
    double vol = h * h * h;
    for (int64_t k = 0; k < bs; ++k)
      for (int64_t j = 0; j < bs; ++j)
        for (int64_t i = 0; i < bs; ++i) {
          int64_t q = pidx(g, i, j, k);
          int64_t qi = (k * bs + j) * bs + i;
          double x = (double)(g->ix[b] * bs + i) * h;
          double y = (double)(g->iy[b] * bs + j) * h;
          double z = (double)(g->iz[b] * bs + k) * h;
          double e = dus ? dus[(b * 3 + 0) * n3 + qi] : 0.0;
          double u = cfld(g, U, b, 0)[q];
          if (p->mask == 1) {
            double chi, us[3];
            mask_point(p, t, x, y, z, &chi, us);
            fld(g, Ubar, b, 0)[q] += weight * chi * vol / p->c_eta;
            if (dusbar) dusbar[(b * 3 + 0) * n3 + qi] += -weight * chi * vol / p->c_eta;
          } else {
            double chi, dchi, us[3], dsd[3], dal[3], dad[3];
            plate_point(p, t, x, y, z, &chi, &dchi, us, dsd, dal, dad);
            fld(g, Ubar, b, 0)[q] += weight * chi * vol / p->c_eta;
            if (dusbar) dusbar[(b * 3 + 0) * n3 + qi] += -weight * chi * vol / p->c_eta;
            double gal = weight * dchi * (u - us[0] - e) * vol / p->c_eta;
            double gad = -weight * chi * dsd[0] * vol / p->c_eta;
            for (int k2 = 0; k2 < 3; ++k2) dtheta[k2] += gal * dal[k2] + gad * dad[k2];
          }
        }
  }
}

/* Adjoint of one RK4 step from the checkpoint Un (interiors) at time t with
 * step dt: Lam holds lambda^{n+1} on interiors on entry and lambda^n on
 * return (padded layout; ghosts are scratch). */
void orc_rk4_step_adj(const orc_grid* g, const orc_params* p, double t, double dt,
                      const double* Un, double* Lam, double dtheta[3], double* dusbar,
                      const double* dus) {
  const int64_t tot = g->nb * 4 * (int64_t)g->P * g->P * g->P;
  double* S[4];
  double* K = (double*)calloc(tot, sizeof(double));
  for (int s = 0; s < 4; ++s) S[s] = (double*)calloc(tot, sizeof(double));
  const double cs[4] = {0.0, 0.5, 0.5, 1.0};
  const double as[4] = {0.0, 0.5, 0.5, 1.0};
  /* recompute the synchronised stage inputs */
  memcpy(S[0], Un, sizeof(double) * tot);
  orc_sync(g, S[0]);
  for (int s = 1; s < 4; ++s) {
    orc_rhs(g, p, t + cs[s - 1] * dt, S[s - 1], dus, K);
    axpy_interior(g, S[s], Un, as[s] * dt, K);
    orc_sync(g, S[s]);
  }
  /* reverse sweep */
  const int bs = g->bs;
  double* lamU = (double*)calloc(tot, sizeof(double));
  double* kb[4];
  for (int s = 0; s < 4; ++s) kb[s] = (double*)calloc(tot, sizeof(double));
  const double bw[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
  for (int64_t b = 0; b < g->nb; ++b)
    for (int c = 0; c < 4; ++c)
      for (int64_t k = 0; k < bs; ++k)
        for (int64_t j = 0; j < bs; ++j)
          for (int64_t i = 0; i < bs; ++i) {
            int64_t q = (b * 4 + c) * (int64_t)g->P * g->P * g->P + pidx(g, i, j, k);
            lamU[q] = Lam[q];
            for (int s = 0; s < 4; ++s) kb[s][q] = dt * bw[s] * Lam[q];
          }
  double* Bb = (double*)calloc(tot, sizeof(double));
  for (int s = 3; s >= 0; --s) {
    memset(Bb, 0, sizeof(double) * tot);
    orc_rhs_adj(g, p, t + cs[s] * dt, S[s], kb[s], Bb, dtheta, dusbar, dus);
    orc_sync_adj(g, Bb);
    for (int64_t b = 0; b < g->nb; ++b)
      for (int c = 0; c < 4; ++c)
        for (int64_t k = 0; k < bs; ++k)
          for (int64_t j = 0; j < bs; ++j)
            for (int64_t i = 0; i < bs; ++i) {
              int64_t q = (b * 4 + c) * (int64_t)g->P * g->P * g->P + pidx(g, i, j, k);
              lamU[q] += Bb[q];
              if (s > 0) kb[s - 1][q] += as[s] * dt * Bb[q];
            }
  }
  memcpy(Lam, lamU, sizeof(double) * tot);
  free(Bb);
  free(lamU);
  for (int s = 0; s < 4; ++s) {
    free(kb[s]);
    free(S[s]);
  }
  free(K);
}

/* ------------------------------------------------------------------------ */
/* Multiresolution transform (Sec. 3.1; lifted coarse values of Sec. 3.2) of */
/* nf periodic fields of n^3 points each (x fastest), in place.  The level-m */
/* step works on the lattice of stride s = 2^m: a point of it is even when   */
/* all three of its coordinates are multiples of 2s, odd otherwise.          */
/*   forward, m = 0 .. nlev-1: every odd point takes its detail, the value   */
/*     minus the tensor DD4 prediction from the even points; with CDF 4/4    */
/*     every even point takes the lifted restriction of the stride-s values  */
/*     (the x, y, z lifting of lift_1d at stride s), with CDF 4/0 it keeps   */
/*     its value (decimation).  Both from the values before the step.        */
/*   inverse, m = nlev-1 .. 0: with CDF 4/4 the even values are recovered    */
/*     as c - L(delta), delta the stride-s lattice with the details at the   */
/*     odd points and zeros at the even ones, L the lifted restriction       */
/*     (L is linear and returns e when applied to e extended by prediction,  */
/*     so c = L(u) = e + L(delta)); then every odd point becomes its detail   */
/*     plus the prediction from the even values.                             */
/* After a forward transform the stride-2^nlev lattice holds the coarse       */
/* approximation and a point whose coordinates are all multiples of 2^m but  */
/* not all of 2^(m+1) holds its level-m detail.  n must be a multiple of     */
/* 2^nlev with n / 2^nlev >= 4.                                              */
/* ------------------------------------------------------------------------ */
static int mr_is_odd(int64_t x, int64_t y, int64_t z, int64_t s) {
  return (x / s) % 2 != 0 || (y / s) % 2 != 0 || (z / s) % 2 != 0;
}

/* tensor DD4 prediction at the stride-s lattice point G from the stride-2s
 * lattice of f */
static double mr_prediction(const double* f, int64_t n, int64_t s, int64_t gx, int64_t gy,
                            int64_t gz) {
  int64_t T[3][4];
  double W[3][4];
  int N[3];
  const int64_t G[3] = {gx, gy, gz};
  for (int d = 0; d < 3; ++d) {
    if ((G[d] / s) % 2 == 0) {
      T[d][0] = G[d];
      W[d][0] = 1.0;
      N[d] = 1;
    } else {
      for (int m = 0; m < 4; ++m) {
        T[d][m] = wrap(G[d] + DD4O[m] * s, n);
        W[d][m] = DD4W[m];
      }
      N[d] = 4;
    }
  }
  double v = 0.0;
  for (int a = 0; a < N[2]; ++a)
    for (int b = 0; b < N[1]; ++b)
      for (int e = 0; e < N[0]; ++e) {
        double w = (W[2][a] * W[1][b]) * W[0][e];
        v += w * f[(T[2][a] * n + T[1][b]) * n + T[0][e]];
      }
  return v;
}

/* lifted restriction at the stride-2s point G from the stride-s lattice of f */
static double mr_lifted(const double* f, int64_t n, int64_t s, int64_t gx, int64_t gy,
                        int64_t gz) {
  double ax[13][13];
  for (int z = 0; z < 13; ++z)
    for (int y = 0; y < 13; ++y) {
      double line[13];
      int64_t zz = wrap(gz + (z - 6) * s, n), yy = wrap(gy + (y - 6) * s, n);
      for (int x = 0; x < 13; ++x) line[x] = f[(zz * n + yy) * n + wrap(gx + (x - 6) * s, n)];
      ax[z][y] = lift_1d(4, line);
    }
  double ay[13];
  for (int z = 0; z < 13; ++z) ay[z] = lift_1d(4, ax[z]);
  return lift_1d(4, ay);
}

static int mr_valid(int64_t n, int nf, int nlev, int wavelet) {
  if (n < 4 || nf < 1 || nlev < 0 || nlev > 20 || (wavelet != 0 && wavelet != 1)) return 0;
  if (n % ((int64_t)1 << nlev) != 0 || (n >> nlev) < 4) return 0;
  return 1;
}

int orc_mr_forward(int64_t n, int nf, int nlev, int wavelet, double* u) {
  if (!mr_valid(n, nf, nlev, wavelet)) return -1;
  const int64_t n3 = n * n * n;
  double* f0 = (double*)malloc(sizeof(double) * n3);
  for (int c = 0; c < nf; ++c) {
    double* f = u + c * n3;
    for (int m = 0; m < nlev; ++m) {
      const int64_t s = (int64_t)1 << m;
      memcpy(f0, f, sizeof(double) * n3);
#pragma omp parallel for schedule(static)
      for (int64_t z = 0; z < n; z += s)
        for (int64_t y = 0; y < n; y += s)
          for (int64_t x = 0; x < n; x += s) {
            if (mr_is_odd(x, y, z, s))
              f[(z * n + y) * n + x] = f0[(z * n + y) * n + x] - mr_prediction(f0, n, s, x, y, z);
            else if (wavelet == 1)
              f[(z * n + y) * n + x] = mr_lifted(f0, n, s, x, y, z);
          }
    }
  }
  free(f0);
  return 0;
}

int orc_mr_inverse(int64_t n, int nf, int nlev, int wavelet, double* u) {
  if (!mr_valid(n, nf, nlev, wavelet)) return -1;
  const int64_t n3 = n * n * n;
  double* f0 = (double*)malloc(sizeof(double) * n3);
  for (int c = 0; c < nf; ++c) {
    double* f = u + c * n3;
    for (int m = nlev - 1; m >= 0; --m) {
      const int64_t s = (int64_t)1 << m;
      if (wavelet == 1) {
        /* delta: details at the odd points, zeros at the even ones */
        memcpy(f0, f, sizeof(double) * n3);
        for (int64_t z = 0; z < n; z += 2 * s)
          for (int64_t y = 0; y < n; y += 2 * s)
            for (int64_t x = 0; x < n; x += 2 * s) f0[(z * n + y) * n + x] = 0.0;
#pragma omp parallel for schedule(static)
        for (int64_t z = 0; z < n; z += 2 * s)
          for (int64_t y = 0; y < n; y += 2 * s)
            for (int64_t x = 0; x < n; x += 2 * s)
              f[(z * n + y) * n + x] -= mr_lifted(f0, n, s, x, y, z);
      }
      memcpy(f0, f, sizeof(double) * n3);
#pragma omp parallel for schedule(static)
      for (int64_t z = 0; z < n; z += s)
        for (int64_t y = 0; y < n; y += s)
          for (int64_t x = 0; x < n; x += s)
            if (mr_is_odd(x, y, z, s))
              f[(z * n + y) * n + x] = f0[(z * n + y) * n + x] + mr_prediction(f0, n, s, x, y, z);
    }
  }
  free(f0);
  return 0;
}
