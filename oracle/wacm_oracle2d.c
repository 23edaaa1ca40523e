/*
 * wacm_oracle2d.c -- TEST INFRASTRUCTURE ONLY (see wacm_oracle2d.h).
 *
 * The two-dimensional form of the method (model of Sec. 2.1 with D = 2),
 * written as plainly as its 3D counterpart wacm_oracle.c and with the same
 * readings: non-redundant blocks (level J has 2^J blocks per axis, spacing
 * h_J = L / (2^J bs), block interior index i at x = (bx bs + i) h_J); a ghost
 * value is the value of the leaf holding its position -- a copy from a leaf of
 * the same level, the coincident point of a finer leaf (decimation), or the
 * tensor-product 4th-order Deslauriers-Dubuc prediction from the coarse
 * lattice values held by their owners (Sec. 3.1); periodic in x and y; 2:1
 * graded across edges and corners.  Build together with wacm_oracle.c:
 *   gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared
 * OpenMP only splits independent blocks; reductions are serial.
 */
#include "wacm_oracle2d.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define REF2 20 /* reference level for integer positions */

struct orc2_grid {
  int bs, ng, P, jmin, jmax;
  double L;
  int64_t nb;
  int32_t* lev;
  int64_t *ix, *iy;
  int64_t hcap;
  uint64_t* hkey;
  int64_t* hval;
};

static uint64_t key2(int lev, int64_t x, int64_t y) {
  return ((uint64_t)lev << 50) | ((uint64_t)x << 25) | (uint64_t)y;
}
static uint64_t mix2(uint64_t k) {
  k ^= k >> 31;
  k *= 0x9e3779b97f4a7c15ULL;
  k ^= k >> 29;
  return k;
}
static int64_t find2(const orc2_grid* g, int lev, int64_t x, int64_t y) {
  uint64_t k = key2(lev, x, y);
  int64_t pos = (int64_t)(mix2(k) & (uint64_t)(g->hcap - 1));
  for (;;) {
    if (g->hval[pos] < 0) return -1;
    if (g->hkey[pos] == k) return g->hval[pos];
    pos = (pos + 1) & (g->hcap - 1);
  }
}
static int insert2(orc2_grid* g, int lev, int64_t x, int64_t y, int64_t id) {
  uint64_t k = key2(lev, x, y);
  int64_t pos = (int64_t)(mix2(k) & (uint64_t)(g->hcap - 1));
  for (;;) {
    if (g->hval[pos] < 0) {
      g->hkey[pos] = k;
      g->hval[pos] = id;
      return 0;
    }
    if (g->hkey[pos] == k) return -1;
    pos = (pos + 1) & (g->hcap - 1);
  }
}
static int64_t wrap2(int64_t a, int64_t n) {
  int64_t r = a % n;
  return r < 0 ? r + n : r;
}

static orc2_grid* alloc2(int bs, int ng, double L, int jmin, int jmax, int64_t nb) {
  orc2_grid* g = (orc2_grid*)calloc(1, sizeof(orc2_grid));
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
  int64_t cap = 16;
  while (cap < 2 * nb + 16) cap *= 2;
  g->hcap = cap;
  g->hkey = (uint64_t*)malloc(sizeof(uint64_t) * cap);
  g->hval = (int64_t*)malloc(sizeof(int64_t) * cap);
  for (int64_t i = 0; i < cap; ++i) g->hval[i] = -1;
  return g;
}

void orc2_grid_free(orc2_grid* g) {
  if (!g) return;
  free(g->lev);
  free(g->ix);
  free(g->iy);
  free(g->hkey);
  free(g->hval);
  free(g);
}

int64_t orc2_grid_nb(const orc2_grid* g) { return g->nb; }

void orc2_grid_leaves(const orc2_grid* g, int32_t* lev, int64_t* ix, int64_t* iy) {
  for (int64_t b = 0; b < g->nb; ++b) {
    lev[b] = g->lev[b];
    ix[b] = g->ix[b];
    iy[b] = g->iy[b];
  }
}

/* Closed squares of leaves a and b intersect (periodic). */
static int touch2(const orc2_grid* g, int64_t a, int64_t b) {
  int64_t n = (int64_t)g->bs << REF2;
  int64_t sa = (int64_t)g->bs << (REF2 - g->lev[a]);
  int64_t sb = (int64_t)g->bs << (REF2 - g->lev[b]);
  const int64_t* ca[2] = {g->ix, g->iy};
  for (int d = 0; d < 2; ++d) {
    int64_t a0 = ca[d][a] * sa, a1 = a0 + sa;
    int64_t b0 = ca[d][b] * sb, b1 = b0 + sb;
    int hit = 0;
    for (int s = -1; s <= 1; ++s)
      if (b0 + s * n <= a1 && a0 <= b1 + s * n) hit = 1;
    if (!hit) return 0;
  }
  return 1;
}

orc2_grid* orc2_grid_create(int bs, int ng, double L, int jmin, int jmax, int64_t nleaves,
                            const int32_t* lev, const int64_t* ix, const int64_t* iy, int* err) {
  *err = 0;
  if (bs < 2 * (ng + 3) || bs % 2 || ng < 3 || jmin < 0 || jmax > 18 || jmin > jmax ||
      nleaves <= 0 || !(L > 0)) {
    *err = -1;
    return NULL;
  }
  orc2_grid* g = alloc2(bs, ng, L, jmin, jmax, nleaves);
  uint64_t area = 0;
  for (int64_t b = 0; b < nleaves; ++b) {
    int J = lev[b];
    int64_t n = (int64_t)1 << J;
    if (J < jmin || J > jmax || ix[b] < 0 || iy[b] < 0 || ix[b] >= n || iy[b] >= n) {
      *err = -1;
      orc2_grid_free(g);
      return NULL;
    }
    g->lev[b] = J;
    g->ix[b] = ix[b];
    g->iy[b] = iy[b];
    if (insert2(g, J, ix[b], iy[b], b)) {
      *err = -2;
      orc2_grid_free(g);
      return NULL;
    }
    area += (uint64_t)1 << (2 * (jmax - J));
  }
  for (int64_t b = 0; b < nleaves; ++b)
    for (int K = jmin; K < g->lev[b]; ++K) {
      int s = g->lev[b] - K;
      if (find2(g, K, g->ix[b] >> s, g->iy[b] >> s) >= 0) {
        *err = -2;
        orc2_grid_free(g);
        return NULL;
      }
    }
  if (area != ((uint64_t)1 << (2 * jmax))) {
    *err = -2;
    orc2_grid_free(g);
    return NULL;
  }
  for (int64_t a = 0; a < nleaves; ++a)
    for (int64_t b = 0; b < nleaves; ++b) {
      int d = g->lev[a] - g->lev[b];
      if ((d > 1 || d < -1) && touch2(g, a, b)) {
        *err = -3;
        orc2_grid_free(g);
        return NULL;
      }
    }
  return g;
}

static inline int64_t pix(const orc2_grid* g, int64_t i, int64_t j) {
  return (j + g->ng) * g->P + (i + g->ng);
}
static inline double* fl2(const orc2_grid* g, double* U, int64_t b, int c) {
  return U + (b * 3 + c) * (int64_t)g->P * g->P;
}
static inline const double* cfl2(const orc2_grid* g, const double* U, int64_t b, int c) {
  return U + (b * 3 + c) * (int64_t)g->P * g->P;
}
static double h2(const orc2_grid* g, int J) { return g->L / ((double)((int64_t)1 << J) * g->bs); }

/* Leaf holding the level-J lattice point (gx, gy) (periodic) and the local
 * index of the point in it; -1 if the point is not on its owner's lattice
 * (the owner is coarser). */
static int64_t owner2(const orc2_grid* g, int J, int64_t gx, int64_t gy, int64_t* li,
                      int64_t* lj) {
  int64_t n = (int64_t)g->bs << REF2;
  int64_t u = (int64_t)1 << (REF2 - J);
  int64_t rx = wrap2(gx * u, n), ry = wrap2(gy * u, n);
  for (int K = g->jmin; K <= g->jmax; ++K) {
    int64_t span = (int64_t)g->bs << (REF2 - K);
    int64_t b = find2(g, K, rx / span, ry / span);
    if (b < 0) continue;
    int64_t unit = (int64_t)1 << (REF2 - K);
    int64_t ox = rx - g->ix[b] * span, oy = ry - g->iy[b] * span;
    if (ox % unit || oy % unit) return -1;
    *li = ox / unit;
    *lj = oy / unit;
    return b;
  }
  fprintf(stderr, "oracle2d: no leaf holds a position\n");
  abort();
}

static const double W4[4] = {-1.0 / 16.0, 9.0 / 16.0, 9.0 / 16.0, -1.0 / 16.0};
static const int O4[4] = {-3, -1, 1, 3};

/* Field c at the level-J lattice point G seen from a level-J block: the
 * owner's value if the point is on its lattice, else the DD4 prediction from
 * the level-(J-1) lattice (y outer, x inner). */
static double value2(const orc2_grid* g, const double* U, int J, int c, int64_t gx, int64_t gy) {
  int64_t li, lj;
  int64_t o = owner2(g, J, gx, gy, &li, &lj);
  if (o >= 0) {
    if (g->lev[o] < J - 1 || g->lev[o] > J + 1) {
      fprintf(stderr, "oracle2d: grid not graded\n");
      abort();
    }
    return cfl2(g, U, o, c)[pix(g, li, lj)];
  }
  int64_t G[2] = {gx, gy}, T[2][4];
  double W[2][4];
  int N[2];
  for (int d = 0; d < 2; ++d) {
    if (wrap2(G[d], 2) == 0) {
      T[d][0] = G[d] / 2;
      W[d][0] = 1.0;
      N[d] = 1;
    } else {
      for (int m = 0; m < 4; ++m) {
        T[d][m] = (G[d] + O4[m]) / 2;
        W[d][m] = W4[m];
      }
      N[d] = 4;
    }
  }
  double v = 0.0;
  for (int b = 0; b < N[1]; ++b)
    for (int a = 0; a < N[0]; ++a) {
      int64_t si, sj;
      int64_t o2 = owner2(g, J - 1, T[0][a], T[1][b], &si, &sj);
      if (o2 < 0) {
        fprintf(stderr, "oracle2d: coarse source not on its owner's lattice\n");
        abort();
      }
      v += (W[1][b] * W[0][a]) * cfl2(g, U, o2, c)[pix(g, si, sj)];
    }
  return v;
}

void orc2_sync(const orc2_grid* g, double* U) {
  const int bs = g->bs, ng = g->ng;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < g->nb; ++b) {
    int J = g->lev[b];
    for (int c = 0; c < 3; ++c)
      for (int64_t j = -ng; j < bs + ng; ++j)
        for (int64_t i = -ng; i < bs + ng; ++i) {
          if (i >= 0 && i < bs && j >= 0 && j < bs) continue;
          fl2(g, U, b, c)[pix(g, i, j)] =
              value2(g, U, J, c, g->ix[b] * bs + i, g->iy[b] * bs + j);
        }
  }
}

/* Sec. 2.2 with D = 2, advective form: for i = x, y
 *   du_i/dt = -(u D1_x + v D1_y) u_i - D1_i p + nu (D2_x + D2_y) u_i,
 *   dp/dt   = -C0^2 (D1_x u + D1_y v) - C_gamma p,
 * D1 the Tam-Webb stencil, D2 the 5-point 4th-order stencil (Sec. 2.3). */
void orc2_rhs(const orc2_grid* g, const orc_params* p, const double* U, double* dU) {
  double a[3];
  orc_tam_webb(a);
  const int bs = g->bs;
#pragma omp parallel for schedule(dynamic, 1)
  for (int64_t b = 0; b < g->nb; ++b) {
    double h = h2(g, g->lev[b]);
    const double* F[3];
    for (int c = 0; c < 3; ++c) F[c] = cfl2(g, U, b, c);
    for (int64_t j = 0; j < bs; ++j)
      for (int64_t i = 0; i < bs; ++i) {
        int64_t s[2] = {1, g->P};
        int64_t q = pix(g, i, j);
        double d1[3][2], d2[2][2];
        for (int c = 0; c < 3; ++c)
          for (int d = 0; d < 2; ++d) {
            double acc = 0.0;
            for (int m = 1; m <= 3; ++m) acc += a[m - 1] * (F[c][q + m * s[d]] - F[c][q - m * s[d]]);
            d1[c][d] = acc / h;
          }
        for (int c = 0; c < 2; ++c)
          for (int d = 0; d < 2; ++d) {
            const double* f = F[c];
            d2[c][d] = (-f[q - 2 * s[d]] / 12.0 + 4.0 * f[q - s[d]] / 3.0 - 5.0 * f[q] / 2.0 +
                        4.0 * f[q + s[d]] / 3.0 - f[q + 2 * s[d]] / 12.0) /
                       (h * h);
          }
        double u = F[0][q], v = F[1][q], pr = F[2][q];
        for (int c = 0; c < 2; ++c)
          fl2(g, dU, b, c)[q] = -(u * d1[c][0] + v * d1[c][1]) - d1[2][c] +
                                p->nu * (d2[c][0] + d2[c][1]);
        fl2(g, dU, b, 2)[q] = -p->c0 * p->c0 * (d1[0][0] + d1[1][1]) - p->c_gamma * pr;
      }
  }
}

double orc2_dt(const orc2_grid* g, const orc_params* p, const double* U) {
  const int bs = g->bs;
  double umax = 0.0;
  int jfine = g->jmin;
  for (int64_t b = 0; b < g->nb; ++b) {
    if (g->lev[b] > jfine) jfine = g->lev[b];
    for (int64_t j = 0; j < bs; ++j)
      for (int64_t i = 0; i < bs; ++i) {
        double u = cfl2(g, U, b, 0)[pix(g, i, j)], v = cfl2(g, U, b, 1)[pix(g, i, j)];
        double m = sqrt(u * u + v * v);
        if (m > umax) umax = m;
      }
  }
  double h = h2(g, jfine);
  double dt = p->cfl * h / (umax + sqrt(umax * umax + p->c0 * p->c0));
  if (p->nu > 0) {
    double d = p->cfl_nu * h * h / p->nu;
    if (d < dt) dt = d;
  }
  return dt;
}

/* Y = X + a K on interiors */
static void axpy2(const orc2_grid* g, double* Y, const double* X, double a, const double* K) {
  const int bs = g->bs;
  for (int64_t b = 0; b < g->nb; ++b)
    for (int c = 0; c < 3; ++c)
      for (int64_t j = 0; j < bs; ++j)
        for (int64_t i = 0; i < bs; ++i) {
          int64_t q = pix(g, i, j);
          fl2(g, Y, b, c)[q] = cfl2(g, X, b, c)[q] + a * cfl2(g, K, b, c)[q];
        }
}

/* Classical RK4 (Sec. 2.3): k_s = rhs(sync(U_s)), U_s = U + c_s dt k_{s-1},
 * U <- U + dt (k1 + 2 k2 + 2 k3 + k4) / 6 on interiors. */
void orc2_rk4_step(const orc2_grid* g, const orc_params* p, double dt, double* U) {
  const int64_t tot = g->nb * 3 * (int64_t)g->P * g->P;
  double* Us = (double*)calloc(tot, sizeof(double));
  double* k[4];
  for (int s = 0; s < 4; ++s) k[s] = (double*)calloc(tot, sizeof(double));
  const double cs[3] = {0.5, 0.5, 1.0};
  memcpy(Us, U, sizeof(double) * tot);
  for (int s = 0; s < 4; ++s) {
    orc2_sync(g, Us);
    orc2_rhs(g, p, Us, k[s]);
    if (s < 3) axpy2(g, Us, U, cs[s] * dt, k[s]);
  }
  const int bs = g->bs;
  for (int64_t b = 0; b < g->nb; ++b)
    for (int c = 0; c < 3; ++c)
      for (int64_t j = 0; j < bs; ++j)
        for (int64_t i = 0; i < bs; ++i) {
          int64_t q = pix(g, i, j);
          double* u = fl2(g, U, b, c);
          u[q] = u[q] + dt * (cfl2(g, k[0], b, c)[q] + 2.0 * cfl2(g, k[1], b, c)[q] +
                              2.0 * cfl2(g, k[2], b, c)[q] + cfl2(g, k[3], b, c)[q]) /
                            6.0;
        }
  free(Us);
  for (int s = 0; s < 4; ++s) free(k[s]);
}

void orc2_diagnostics(const orc2_grid* g, const double* U, double out[9]) {
  const int bs = g->bs;
  for (int i = 0; i < 9; ++i) out[i] = 0.0;
  for (int64_t b = 0; b < g->nb; ++b) {
    double h = h2(g, g->lev[b]);
    for (int64_t j = 0; j < bs; ++j)
      for (int64_t i = 0; i < bs; ++i) {
        int64_t q = pix(g, i, j);
        double u = cfl2(g, U, b, 0)[q], v = cfl2(g, U, b, 1)[q], pr = cfl2(g, U, b, 2)[q];
        double m = sqrt(u * u + v * v);
        if (m > out[0]) out[0] = m;
        if (fabs(u) > out[1]) out[1] = fabs(u);
        if (fabs(v) > out[2]) out[2] = fabs(v);
        if (fabs(pr) > out[4]) out[4] = fabs(pr);
        out[8] += 0.5 * (u * u + v * v) * h * h;
      }
  }
}

/* P R u at a block-local point from the block's own even points (Sec. 3.1). */
static double pred2(const orc2_grid* g, const double* f, int64_t i, int64_t j) {
  int64_t L[2] = {i, j}, T[2][4];
  double W[2][4];
  int N[2];
  for (int d = 0; d < 2; ++d) {
    if (L[d] % 2 == 0) {
      T[d][0] = L[d];
      W[d][0] = 1.0;
      N[d] = 1;
    } else {
      for (int m = 0; m < 4; ++m) {
        T[d][m] = L[d] + O4[m];
        W[d][m] = W4[m];
      }
      N[d] = 4;
    }
  }
  double v = 0.0;
  for (int b = 0; b < N[1]; ++b)
    for (int a = 0; a < N[0]; ++a) v += (W[1][b] * W[0][a]) * f[pix(g, T[0][a], T[1][b])];
  return v;
}

void orc2_details(const orc2_grid* g, const double* U, double* dmax) {
  const int bs = g->bs;
  double norm[3] = {0, 0, 0};
  for (int64_t b = 0; b < g->nb; ++b)
    for (int c = 0; c < 3; ++c)
      for (int64_t j = 0; j < bs; ++j)
        for (int64_t i = 0; i < bs; ++i) {
          double v = fabs(cfl2(g, U, b, c)[pix(g, i, j)]);
          if (v > norm[c]) norm[c] = v;
        }
  for (int c = 0; c < 3; ++c)
    if (norm[c] == 0.0) norm[c] = 1.0;
  for (int64_t b = 0; b < g->nb; ++b) {
    double dm = 0.0;
    for (int c = 0; c < 3; ++c) {
      const double* f = cfl2(g, U, b, c);
      for (int64_t j = 0; j < bs; ++j)
        for (int64_t i = 0; i < bs; ++i) {
          if (i % 2 == 0 && j % 2 == 0) continue;
          double d = fabs(f[pix(g, i, j)] - pred2(g, f, i, j)) / norm[c];
          if (d > dm) dm = d;
        }
    }
    dmax[b] = dm;
  }
}

void orc2_flags(const orc2_grid* g, const double* dmax, double eps, int dealias, int8_t* flags) {
  for (int64_t b = 0; b < g->nb; ++b) {
    int J = g->lev[b], f = 0;
    if (J > g->jmin) f = (dealias && J == g->jmax) || dmax[b] < eps;
    flags[b] = (int8_t)f;
  }
}

/* ---- adaptation ---------------------------------------------------------- */
typedef struct {
  uint64_t key;
  int32_t lev;
  int64_t x, y, src;
  int kind; /* 0 copy, 1 child of src, 2 merged parent */
} nleaf2;

static int cmp2(const void* A, const void* B) {
  uint64_t a = ((const nleaf2*)A)->key, b = ((const nleaf2*)B)->key;
  return a < b ? -1 : (a > b ? 1 : 0);
}
/* quadtree Morton key at the reference level: x bit below y bit */
static uint64_t morton2(int lev, int64_t x, int64_t y) {
  uint64_t k = 0;
  for (int l = 1; l <= lev; ++l) {
    int sh = lev - l;
    k = (k << 2) | (uint64_t)((x >> sh) & 1) | ((uint64_t)((y >> sh) & 1) << 1);
  }
  return k << (2 * (REF2 - lev));
}

static orc2_grid* from_leaves2(const orc2_grid* g, nleaf2* nl, int64_t n) {
  qsort(nl, n, sizeof(nleaf2), cmp2);
  orc2_grid* h = alloc2(g->bs, g->ng, g->L, g->jmin, g->jmax, n);
  for (int64_t b = 0; b < n; ++b) {
    h->lev[b] = nl[b].lev;
    h->ix[b] = nl[b].x;
    h->iy[b] = nl[b].y;
    insert2(h, nl[b].lev, nl[b].x, nl[b].y, b);
  }
  return h;
}

int64_t orc2_refine_count(const orc2_grid* g) {
  int64_t n = 0;
  for (int64_t b = 0; b < g->nb; ++b) n += g->lev[b] < g->jmax ? 4 : 1;
  return n;
}

orc2_grid* orc2_refine_all(const orc2_grid* g, const double* U, double* Unew) {
  const int bs = g->bs;
  const int64_t P2 = (int64_t)g->P * g->P;
  int64_t n = orc2_refine_count(g), m = 0;
  nleaf2* nl = (nleaf2*)malloc(sizeof(nleaf2) * n);
  for (int64_t b = 0; b < g->nb; ++b) {
    int J = g->lev[b];
    if (J < g->jmax) {
      for (int c = 0; c < 4; ++c) {
        nleaf2* q = &nl[m++];
        q->lev = J + 1;
        q->x = 2 * g->ix[b] + (c & 1);
        q->y = 2 * g->iy[b] + (c >> 1);
        q->key = morton2(q->lev, q->x, q->y);
        q->src = b;
        q->kind = 1;
      }
    } else {
      nleaf2* q = &nl[m++];
      q->lev = J;
      q->x = g->ix[b];
      q->y = g->iy[b];
      q->key = morton2(J, q->x, q->y);
      q->src = b;
      q->kind = 0;
    }
  }
  orc2_grid* h = from_leaves2(g, nl, n);
  memset(Unew, 0, sizeof(double) * n * 3 * P2);
  for (int64_t nb = 0; nb < n; ++nb) {
    const nleaf2* q = &nl[nb];
    if (q->kind == 0) {
      memcpy(Unew + nb * 3 * P2, U + q->src * 3 * P2, sizeof(double) * 3 * P2);
      continue;
    }
    int64_t off[2] = {(q->x & 1) * bs, (q->y & 1) * bs};
    for (int c = 0; c < 3; ++c) {
      const double* f = cfl2(g, U, q->src, c);
      for (int64_t j = 0; j < bs; ++j)
        for (int64_t i = 0; i < bs; ++i) {
          /* child point at parent half-index off + (i, j): even -> the parent
           * point, odd -> DD4 from the parent's padded array */
          int64_t Q[2] = {off[0] + i, off[1] + j}, T[2][4];
          double W[2][4];
          int N[2];
          for (int d = 0; d < 2; ++d) {
            if (Q[d] % 2 == 0) {
              T[d][0] = Q[d] / 2;
              W[d][0] = 1.0;
              N[d] = 1;
            } else {
              for (int mm = 0; mm < 4; ++mm) {
                T[d][mm] = (Q[d] + O4[mm]) / 2;
                W[d][mm] = W4[mm];
              }
              N[d] = 4;
            }
          }
          double v = 0.0;
          for (int e = 0; e < N[1]; ++e)
            for (int a = 0; a < N[0]; ++a) v += (W[1][e] * W[0][a]) * f[pix(g, T[0][a], T[1][e])];
          fl2(h, Unew, nb, c)[pix(h, i, j)] = v;
        }
    }
  }
  free(nl);
  return h;
}

static int can_merge2(const orc2_grid* g, const int8_t* flags, int J, int64_t px, int64_t py) {
  for (int c = 0; c < 4; ++c) {
    int64_t b = find2(g, J, 2 * px + (c & 1), 2 * py + (c >> 1));
    if (b < 0 || !flags[b]) return 0;
  }
  int64_t n = (int64_t)g->bs << REF2;
  int64_t sp = (int64_t)g->bs << (REF2 - (J - 1));
  int64_t P0[2] = {px * sp, py * sp};
  for (int64_t b = 0; b < g->nb; ++b) {
    if (g->lev[b] <= J) continue;
    int64_t sb = (int64_t)g->bs << (REF2 - g->lev[b]);
    int64_t B0[2] = {g->ix[b] * sb, g->iy[b] * sb};
    int hit = 1;
    for (int d = 0; d < 2 && hit; ++d) {
      int any = 0;
      for (int s = -1; s <= 1; ++s)
        if (B0[d] + s * n <= P0[d] + sp && P0[d] <= B0[d] + s * n + sb) any = 1;
      hit = any;
    }
    if (hit) return 0;
  }
  return 1;
}

static int64_t plan2(const orc2_grid* g, const int8_t* flags, nleaf2* nl) {
  int64_t m = 0;
  for (int64_t b = 0; b < g->nb; ++b) {
    int J = g->lev[b];
    int64_t x = g->ix[b], y = g->iy[b];
    int merged = J > g->jmin && flags[b] && can_merge2(g, flags, J, x >> 1, y >> 1);
    if (!merged) {
      if (nl) nl[m] = (nleaf2){morton2(J, x, y), J, x, y, b, 0};
      ++m;
    } else if ((x & 1) == 0 && (y & 1) == 0) {
      if (nl) nl[m] = (nleaf2){morton2(J - 1, x >> 1, y >> 1), J - 1, x >> 1, y >> 1, -1, 2};
      ++m;
    }
  }
  return m;
}

int64_t orc2_coarsen_count(const orc2_grid* g, const int8_t* flags) { return plan2(g, flags, NULL); }

orc2_grid* orc2_coarsen(const orc2_grid* g, const int8_t* flags, const double* U, double* Unew) {
  const int bs = g->bs;
  const int64_t P2 = (int64_t)g->P * g->P;
  int64_t n = plan2(g, flags, NULL);
  nleaf2* nl = (nleaf2*)malloc(sizeof(nleaf2) * (n ? n : 1));
  plan2(g, flags, nl);
  orc2_grid* h = from_leaves2(g, nl, n);
  memset(Unew, 0, sizeof(double) * n * 3 * P2);
  for (int64_t nb = 0; nb < n; ++nb) {
    const nleaf2* q = &nl[nb];
    if (q->kind == 0) {
      memcpy(Unew + nb * 3 * P2, U + q->src * 3 * P2, sizeof(double) * 3 * P2);
      continue;
    }
    int J = q->lev + 1;
    for (int c = 0; c < 3; ++c)
      for (int64_t j = 0; j < bs; ++j)
        for (int64_t i = 0; i < bs; ++i) {
          /* decimation: parent point (i, j) is the child point (2i, 2j) */
          int64_t Q[2] = {2 * i, 2 * j};
          int cx = Q[0] >= bs, cy = Q[1] >= bs;
          int64_t child = find2(g, J, 2 * q->x + cx, 2 * q->y + cy);
          fl2(h, Unew, nb, c)[pix(h, i, j)] =
              cfl2(g, U, child, c)[pix(g, Q[0] - cx * bs, Q[1] - cy * bs)];
        }
  }
  free(nl);
  return h;
}
