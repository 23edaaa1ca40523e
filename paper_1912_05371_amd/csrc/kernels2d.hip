// Two-dimensional form of the method (the model of Sec. 2.1 with D = 2) on a
// periodic quadtree of square blocks, for gfx950.
//
// Pool: U[slot][3][P][P] (u, v, p), x fastest, P = bs + 2 ng.  The grid's
// tables are the 3D ones restricted to the plane: region r = rx + 3 ry + 9 of
// a block (rz = 1), kind -1/0/+1, and the finer sub-boxes sx + 2 sy.
//
// Kernels: the ghost fill (copy, decimation, tensor DD4 prediction from the
// coarse lattice's owners, Sec. 3.1 / 4.2), the fused rhs + RK4 stage over an
// LDS tile of the synchronised block (Sec. 2.2 with D = 2, Sec. 2.3), the
// CFL maximum, diagnostics, max norms, details and flags (Sec. 3.1, 3.3-3.5),
// refinement and decimation (Sec. 3.5).  Every kernel is memory-bound; no
// MFMA.
#include <hip/hip_runtime.h>

#include "resolve.h"
#include "resolve2d.h"
#include "wacm_internal.h"

namespace wacm {

hipError_t finalize_dt(const double* part, int64_t n, const wacm_params& p, double hmin,
                       double* dt_dev, hipStream_t st);
hipError_t finalize_diag(const double* part, int64_t n, double* out, hipStream_t st);
hipError_t finalize_norm(const double* part, int64_t n, double* norm, hipStream_t st);
hipError_t add_dt_to_time(double* t_dev, const double* dt_dev, hipStream_t st);

namespace d2 {

Lay pool_layout(const wacm_grid* g) {
  Lay L;
  L.P = g->P;
  L.ng = g->d.ng;
  L.fstride = (int64_t)g->P * g->P;
  L.bstride = 3 * L.fstride;
  return L;
}

// every ghost point of every active block, all ng layers; one thread per
// (block, ghost point), the 3 fields together
template <typename T>
__global__ __launch_bounds__(NT_GEN) void sync2d_kernel(const Tab* __restrict__ tab, int64_t nb,
                                                        T* __restrict__ U, Lay L, int bs) {
  const int P = L.P, ng = L.ng;
  const int nghost = P * P - bs * bs;
  const int64_t total = nb * nghost;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t ib = q / nghost;
    int i, j;
    ghost_point((int)(q - ib * nghost), bs, ng, i, j);
    const Tab& t = tab[ib];
    T* dst = U + (int64_t)t.meta[0] * L.bstride + (int64_t)(j + ng) * P + (i + ng);
    for (int c = 0; c < 3; ++c) dst[c * L.fstride] = ghost_value(t, U, L, bs, c, i, j);
  }
}

// Fused rhs + RK4 stage on the synchronised stage input `in` (own ghost
// layers), one workgroup per block, one thread per point; the 3-deep halo
// and the block in an LDS tile.  Registers (pool layout): U^n `un`, the
// accumulator `acc`, the next stage input `out`.
//   MODE 0: out = rhs(in)
//   MODE 1: acc = U^n + dt/6 k;  out = U^n + dt/2 k
//   MODE 2: acc += dt/3 k;       out = U^n + dt/2 k
//   MODE 3: acc += dt/3 k;       out = U^n + dt k
//   MODE 4: U^n = acc + dt/6 k   (out = un)
template <typename T, int BS, int MODE>
__global__ __launch_bounds__(BS* BS) void stage2d_kernel(const Tab* __restrict__ tab, int64_t nb,
                                                         const T* __restrict__ in, T* un, T* acc,
                                                         T* out, Lay L, double Ldom,
                                                         wacm_params p,
                                                         const double* __restrict__ dt_dev) {
  constexpr int W = BS + 6;
  __shared__ T tile[3][W * W];
  const int tid = threadIdx.x, x = tid % BS, y = tid / BS;
  const double dt = MODE == 0 ? 0.0 : *dt_dev;
  const T a1 = T(TW1), a2 = T(TW2), a3 = T(TW3);
  const T c2a = T(D2A), c2b = T(D2B), c2c = T(D2C);
  const T nu = T(p.nu), c0sq = T(p.c0 * p.c0), cg = T(p.c_gamma);
  for (int64_t ib = blockIdx.x; ib < nb; ib += gridDim.x) {
    const int slot = tab[ib].meta[0], J = tab[ib].meta[1];
    const double h = Ldom / (double(int64_t(1) << J) * BS);
    const T ih = T(1.0 / h), ih2 = T(1.0 / (h * h));
    const T* src = in + (int64_t)slot * L.bstride;
    __syncthreads();  // the previous block's tile is no longer read
    for (int q = tid; q < W * W; q += BS * BS) {
      const int tx = q % W, ty = q / W;
      const int64_t o = (int64_t)(ty - 3 + L.ng) * L.P + (tx - 3 + L.ng);
      for (int c = 0; c < 3; ++c) tile[c][q] = src[c * L.fstride + o];
    }
    __syncthreads();
    const int ct = (y + 3) * W + (x + 3);
    T dx[3], dy[3], lap[2];
    for (int c = 0; c < 3; ++c) {
      const T* s = tile[c];
      dx[c] = (a1 * (s[ct + 1] - s[ct - 1]) + a2 * (s[ct + 2] - s[ct - 2]) +
               a3 * (s[ct + 3] - s[ct - 3])) *
              ih;
      dy[c] = (a1 * (s[ct + W] - s[ct - W]) + a2 * (s[ct + 2 * W] - s[ct - 2 * W]) +
               a3 * (s[ct + 3 * W] - s[ct - 3 * W])) *
              ih;
      if (c < 2)
        lap[c] = ((c2a * s[ct - 2] + c2b * s[ct - 1] + c2c * s[ct] + c2b * s[ct + 1] +
                   c2a * s[ct + 2]) +
                  (c2a * s[ct - 2 * W] + c2b * s[ct - W] + c2c * s[ct] + c2b * s[ct + W] +
                   c2a * s[ct + 2 * W])) *
                 ih2;
    }
    const T u = tile[0][ct], v = tile[1][ct], pr = tile[2][ct];
    T r[3];
    r[0] = -(u * dx[0] + v * dy[0]) - dx[2] + nu * lap[0];
    r[1] = -(u * dx[1] + v * dy[1]) - dy[2] + nu * lap[1];
    r[2] = -c0sq * (dx[0] + dy[1]) - cg * pr;
    const int64_t o = (int64_t)slot * L.bstride + (int64_t)(y + L.ng) * L.P + (x + L.ng);
    for (int c = 0; c < 3; ++c) {
      const int64_t oc = o + c * L.fstride;
      if (MODE == 0) {
        out[oc] = r[c];
      } else if (MODE == 1) {
        const T u0 = un[oc];
        acc[oc] = u0 + T(dt / 6.0) * r[c];
        out[oc] = u0 + T(0.5 * dt) * r[c];
      } else if (MODE == 2 || MODE == 3) {
        acc[oc] = acc[oc] + T(dt / 3.0) * r[c];
        out[oc] = un[oc] + T(MODE == 2 ? 0.5 * dt : dt) * r[c];
      } else {
        un[oc] = acc[oc] + T(dt / 6.0) * r[c];
      }
    }
  }
}

// per block: largest |u|^2 (CFL) -> part[ib]
template <typename T>
__global__ __launch_bounds__(NT_GEN) void maxu2d_kernel(const Tab* __restrict__ tab, int64_t nb,
                                                        const T* __restrict__ U, Lay L, int bs,
                                                        double* __restrict__ part) {
  __shared__ double red[NT_GEN / 64];
  for (int64_t ib = blockIdx.x; ib < nb; ib += gridDim.x) {
    const T* b = U + (int64_t)tab[ib].meta[0] * L.bstride;
    double m = 0.0;
    for (int q = threadIdx.x; q < bs * bs; q += blockDim.x) {
      const int64_t o = (int64_t)(q / bs + L.ng) * L.P + (q % bs + L.ng);
      const double u = b[o], v = b[o + L.fstride];
      m = fmax(m, __builtin_fma(v, v, u * u));
    }
    for (int s = 32; s > 0; s >>= 1) m = fmax(m, __shfl_xor(m, s, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      double r = red[0];
      for (int w = 1; w < NT_GEN / 64; ++w) r = fmax(r, red[w]);
      part[ib] = r;
    }
  }
}

// per block: the 10 diagnostics partials of the 3D path with w = 0 and no
// force: [max|u|^2, max|u|, max|v|, 0, max|p|, 0, 0, 0, 1/2 sum |u|^2 h^2,
// number of NaN/Inf values]; the maxima skip NaN, the count sees it
template <typename T>
__global__ __launch_bounds__(NT_GEN) void diag2d_kernel(const Tab* __restrict__ tab, int64_t nb,
                                                        const T* __restrict__ U, Lay L, int bs,
                                                        double Ldom, double* __restrict__ part) {
  constexpr int NM = 4;  // maxima |u|^2, |u|, |v|, |p|; then the two sums
  __shared__ double red[NM + 2][NT_GEN];
  for (int64_t ib = blockIdx.x; ib < nb; ib += gridDim.x) {
    const int J = tab[ib].meta[1];
    const double h = Ldom / (double(int64_t(1) << J) * bs);
    const T* b = U + (int64_t)tab[ib].meta[0] * L.bstride;
    double acc[NM + 2] = {0, 0, 0, 0, 0, 0};
    for (int q = threadIdx.x; q < bs * bs; q += blockDim.x) {
      const int64_t o = (int64_t)(q / bs + L.ng) * L.P + (q % bs + L.ng);
      const double u = b[o], v = b[o + L.fstride], pr = b[o + 2 * L.fstride];
      const double m2 = u * u + v * v;
      acc[0] = fmax(acc[0], m2);
      acc[1] = fmax(acc[1], fabs(u));
      acc[2] = fmax(acc[2], fabs(v));
      acc[3] = fmax(acc[3], fabs(pr));
      acc[4] += m2;
      acc[5] += (isfinite(u) ? 0.0 : 1.0) + (isfinite(v) ? 0.0 : 1.0) +
                (isfinite(pr) ? 0.0 : 1.0);
    }
    __syncthreads();
    for (int c = 0; c < NM + 2; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int s = NT_GEN / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
        for (int c = 0; c < NM; ++c)
          red[c][threadIdx.x] = fmax(red[c][threadIdx.x], red[c][threadIdx.x + s]);
        for (int c = NM; c < NM + 2; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      double* o = part + ib * 10;
      o[0] = red[0][0];
      o[1] = red[1][0];
      o[2] = red[2][0];
      o[3] = 0.0;
      o[4] = red[3][0];
      o[5] = o[6] = o[7] = 0.0;
      o[8] = 0.5 * red[4][0] * h * h;
      o[9] = red[5][0];
    }
  }
}

// per block: max |u|, |v|, |p| over interiors -> part[ib * 4 + (0, 1, 3)],
// part[ib * 4 + 2] = 0 (the 3D layout, w absent)
template <typename T>
__global__ __launch_bounds__(NT_GEN) void norm2d_kernel(const Tab* __restrict__ tab, int64_t nb,
                                                        const T* __restrict__ U, Lay L, int bs,
                                                        double* __restrict__ part) {
  __shared__ double red[3][NT_GEN / 64];
  for (int64_t ib = blockIdx.x; ib < nb; ib += gridDim.x) {
    const T* b = U + (int64_t)tab[ib].meta[0] * L.bstride;
    double m[3] = {0, 0, 0};
    for (int q = threadIdx.x; q < bs * bs; q += blockDim.x) {
      const int64_t o = (int64_t)(q / bs + L.ng) * L.P + (q % bs + L.ng);
      for (int c = 0; c < 3; ++c) m[c] = fmax(m[c], fabs((double)b[o + c * L.fstride]));
    }
    __syncthreads();
    for (int c = 0; c < 3; ++c) {
      double v = m[c];
      for (int s = 32; s > 0; s >>= 1) v = fmax(v, __shfl_xor(v, s, 64));
      if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
      double r = red[threadIdx.x][0];
      for (int w = 1; w < NT_GEN / 64; ++w) r = fmax(r, red[threadIdx.x][w]);
      const int slot = threadIdx.x == 2 ? 3 : threadIdx.x;
      part[ib * 4 + slot] = r;
    }
    if (threadIdx.x == 0) part[ib * 4 + 2] = 0.0;
  }
}

// Details (Sec. 3.1): at interior points with an odd index, |u - P R u| with
// P the tensor DD4 prediction from the block's own even points (ghosts
// included), normalised per field by its global max norm (Sec. 3.4); the
// block's maximum, and the coarsening flag (Sec. 3.3, 3.5; no mask in 2D).
template <typename T>
__global__ __launch_bounds__(NT_GEN) void detail2d_kernel(
    const Tab* __restrict__ tab, int64_t nb, const T* __restrict__ U, Lay L, int bs,
    const double* __restrict__ norm, double eps, int dealias, int jmin, int jmax,
    double* __restrict__ dmax, double* __restrict__ mrange, int8_t* __restrict__ flags) {
  __shared__ double red[NT_GEN / 64];
  constexpr double W[4] = {DDW0, DDW1, DDW1, DDW0};
  constexpr int O[4] = {-3, -1, 1, 3};
  const double inv[3] = {1.0 / norm[0], 1.0 / norm[1], 1.0 / norm[3]};
  for (int64_t ib = blockIdx.x; ib < nb; ib += gridDim.x) {
    const T* b = U + (int64_t)tab[ib].meta[0] * L.bstride;
    double m = 0.0;
    for (int q = threadIdx.x; q < bs * bs; q += blockDim.x) {
      const int i = q % bs, j = q / bs;
      if (!(i & 1) && !(j & 1)) continue;
      const int nx = (i & 1) ? 4 : 1, ny = (j & 1) ? 4 : 1;
      for (int c = 0; c < 3; ++c) {
        const T* f = b + c * L.fstride;
        double pv = 0.0;
        for (int e = 0; e < ny; ++e) {
          const int py = ny == 1 ? j : j + O[e];
          const double wy = ny == 1 ? 1.0 : W[e];
          for (int a = 0; a < nx; ++a) {
            const int px = nx == 1 ? i : i + O[a];
            const double wx = nx == 1 ? 1.0 : W[a];
            pv += (wy * wx) * (double)f[(int64_t)(py + L.ng) * L.P + (px + L.ng)];
          }
        }
        const double d = fabs((double)f[(int64_t)(j + L.ng) * L.P + (i + L.ng)] - pv) * inv[c];
        m = fmax(m, d);
      }
    }
    for (int s = 32; s > 0; s >>= 1) m = fmax(m, __shfl_xor(m, s, 64));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
    __syncthreads();
    if (threadIdx.x == 0) {
      double r = red[0];
      for (int w = 1; w < NT_GEN / 64; ++w) r = fmax(r, red[w]);
      const int J = tab[ib].meta[1];
      dmax[ib] = r;
      mrange[ib] = 0.0;
      flags[ib] = (int8_t)(J > jmin && ((dealias && J == jmax) || r < eps));
    }
  }
}

// refinement: list entries (parent slot, child slot, quadrant); child point
// (i, j) sits at the parent's half-index off + (i, j): even -> the parent
// point, odd -> DD4 from the parent's padded array (synchronised)
template <typename T>
__global__ __launch_bounds__(NT_GEN) void prolong2d_kernel(const int32_t* __restrict__ list,
                                                           int64_t n, T* __restrict__ U, Lay L,
                                                           int bs) {
  constexpr double W[4] = {DDW0, DDW1, DDW1, DDW0};
  constexpr int O[4] = {-3, -1, 1, 3};
  for (int64_t w = blockIdx.x; w < n; w += gridDim.x) {
    const int32_t* e = list + 3 * w;
    const T* par = U + (int64_t)e[0] * L.bstride;
    T* ch = U + (int64_t)e[1] * L.bstride;
    const int ox = (e[2] & 1) * bs, oy = ((e[2] >> 1) & 1) * bs;
    for (int q = threadIdx.x; q < bs * bs; q += blockDim.x) {
      const int i = q % bs, j = q / bs;
      const int Qx = ox + i, Qy = oy + j;
      const int nx = (Qx & 1) ? 4 : 1, ny = (Qy & 1) ? 4 : 1;
      for (int c = 0; c < 3; ++c) {
        const T* f = par + c * L.fstride;
        double v = 0.0;
        for (int b = 0; b < ny; ++b) {
          const int ty = ny == 1 ? Qy / 2 : (Qy + O[b]) / 2;
          const double wy = ny == 1 ? 1.0 : W[b];
          for (int a = 0; a < nx; ++a) {
            const int tx = nx == 1 ? Qx / 2 : (Qx + O[a]) / 2;
            const double wx = nx == 1 ? 1.0 : W[a];
            v += (wy * wx) * (double)f[(int64_t)(ty + L.ng) * L.P + (tx + L.ng)];
          }
        }
        ch[c * L.fstride + (int64_t)(j + L.ng) * L.P + (i + L.ng)] = T(v);
      }
    }
  }
}

// merge: list entries (parent slot, 4 child slots, unused...); parent point
// (i, j) is the child point (2i, 2j) (decimation)
template <typename T>
__global__ __launch_bounds__(NT_GEN) void decimate2d_kernel(const int32_t* __restrict__ list,
                                                            int64_t n, T* __restrict__ U, Lay L,
                                                            int bs) {
  for (int64_t w = blockIdx.x; w < n; w += gridDim.x) {
    const int32_t* e = list + 10 * w;
    T* par = U + (int64_t)e[0] * L.bstride;
    for (int q = threadIdx.x; q < bs * bs; q += blockDim.x) {
      const int i = q % bs, j = q / bs;
      const int cx = 2 * i >= bs, cy = 2 * j >= bs;
      const T* ch = U + (int64_t)e[1 + cx + 2 * cy] * L.bstride;
      const int64_t os = (int64_t)(2 * j - cy * bs + L.ng) * L.P + (2 * i - cx * bs + L.ng);
      const int64_t od = (int64_t)(j + L.ng) * L.P + (i + L.ng);
      for (int c = 0; c < 3; ++c) par[od + c * L.fstride] = ch[os + c * L.fstride];
    }
  }
}

// ---------------------------------------------------------------- launchers
unsigned blocks_for(int64_t n, int per_cu = 8) {
  static int cus = 0;
  if (!cus) {
    int dev = 0;
    hipDeviceProp_t prop;
    cus = (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
              ? prop.multiProcessorCount
              : 256;
  }
  const int64_t cap = (int64_t)cus * per_cu;
  return (unsigned)(n < 1 ? 1 : (n < cap ? n : cap));
}

template <typename T>
hipError_t sync_t(const wacm_grid* g, T* U, hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  const Lay L = pool_layout(g);
  const int64_t total = g->nb * (int64_t)(L.P * L.P - g->d.bs * g->d.bs);
  sync2d_kernel<T><<<blocks_for((total + NT_GEN - 1) / NT_GEN, 16), NT_GEN, 0, st>>>(
      g->d_tab, g->nb, U, L, g->d.bs);
  return hipGetLastError();
}

template <typename T, int BS, int MODE>
hipError_t stage_bs(const wacm_grid* g, const wacm_params* p, const T* in, T* un, T* acc, T* out,
                    const double* dt_dev, hipStream_t st) {
  stage2d_kernel<T, BS, MODE><<<blocks_for(g->nb, 4), BS * BS, 0, st>>>(
      g->d_tab, g->nb, in, un, acc, out, pool_layout(g), g->d.L, *p, dt_dev);
  return hipGetLastError();
}

template <typename T, int MODE>
hipError_t stage_t(const wacm_grid* g, const wacm_params* p, const T* in, T* un, T* acc, T* out,
                   const double* dt_dev, hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  switch (g->d.bs) {
    case 16:
      return stage_bs<T, 16, MODE>(g, p, in, un, acc, out, dt_dev, st);
    case 24:
      return stage_bs<T, 24, MODE>(g, p, in, un, acc, out, dt_dev, st);
    case 32:
      return stage_bs<T, 32, MODE>(g, p, in, un, acc, out, dt_dev, st);
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
hipError_t dt_t(const wacm_grid* g, const wacm_params* p, const T* U, double* dt_dev,
                hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  maxu2d_kernel<T><<<blocks_for(g->nb), NT_GEN, 0, st>>>(g->d_tab, g->nb, U, pool_layout(g),
                                                          g->d.bs, g->d_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const double hmin = g->d.L / (double(int64_t(1) << g->jfine) * g->d.bs);
  return finalize_dt(g->d_part, g->nb, *p, hmin, dt_dev, st);
}

size_t work_bytes(const wacm_grid* g) {
  const size_t es = g->d.dtype == WACM_F64 ? 8 : 4;
  const size_t reg = ((size_t)g->d.capacity * 3 * g->P * g->P * es + 255) / 256 * 256;
  return 3 * reg;
}

template <typename T>
hipError_t rk4_t(const wacm_grid* g, const wacm_params* p, double* t_dev, double* dt_dev, T* U,
                 void* work, int dt_mode, int64_t nsteps, hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  const size_t reg = work_bytes(g) / 3;
  T* Ya = (T*)work;
  T* Yb = (T*)((char*)work + reg);
  T* acc = (T*)((char*)work + 2 * reg);
  hipError_t e;
  for (int64_t k = 0; k < nsteps; ++k) {
    if (dt_mode == WACM_DT_CFL && (e = dt_t<T>(g, p, U, dt_dev, st)) != hipSuccess) return e;
    T* ins[4] = {U, Ya, Yb, Ya};
    T* outs[4] = {Ya, Yb, Ya, U};
    for (int s = 0; s < 4; ++s) {
      if ((e = sync_t<T>(g, ins[s], st)) != hipSuccess) return e;
      switch (s) {
        case 0:
          e = stage_t<T, 1>(g, p, ins[s], U, acc, outs[s], dt_dev, st);
          break;
        case 1:
          e = stage_t<T, 2>(g, p, ins[s], U, acc, outs[s], dt_dev, st);
          break;
        case 2:
          e = stage_t<T, 3>(g, p, ins[s], U, acc, outs[s], dt_dev, st);
          break;
        default:
          e = stage_t<T, 4>(g, p, ins[s], U, acc, outs[s], dt_dev, st);
          break;
      }
      if (e != hipSuccess) return e;
    }
    if ((e = add_dt_to_time(t_dev, dt_dev, st)) != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t diag_t(const wacm_grid* g, const T* U, double* out, hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  diag2d_kernel<T><<<blocks_for(g->nb), NT_GEN, 0, st>>>(g->d_tab, g->nb, U, pool_layout(g),
                                                          g->d.bs, g->d.L, g->d_part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return finalize_diag(g->d_part, g->nb, out, st);
}

template <typename T>
hipError_t thr_t(const wacm_grid* g, const T* U, double eps, int dealias, double* dmax,
                 double* mrange, int8_t* flags, hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  const Lay L = pool_layout(g);
  norm2d_kernel<T><<<blocks_for(g->nb), NT_GEN, 0, st>>>(g->d_tab, g->nb, U, L, g->d.bs,
                                                          g->d_part);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) e = finalize_norm(g->d_part, g->nb, g->d_norm, st);
  if (e != hipSuccess) return e;
  detail2d_kernel<T><<<blocks_for(g->nb), NT_GEN, 0, st>>>(
      g->d_tab, g->nb, U, L, g->d.bs, g->d_norm, eps, dealias, g->d.jmin, g->d.jmax, dmax,
      mrange, flags);
  return hipGetLastError();
}

}  // namespace d2

// ---------------------------------------------------------------- entry points used by api.cpp
size_t work_bytes_2d(const wacm_grid* g) { return d2::work_bytes(g); }

hipError_t launch_sync_2d(const wacm_grid* g, void* U, hipStream_t st) {
  return g->d.dtype == WACM_F64 ? d2::sync_t(g, (double*)U, st) : d2::sync_t(g, (float*)U, st);
}

hipError_t launch_rhs_2d(const wacm_grid* g, const wacm_params* p, const void* U, void* dU,
                         hipStream_t st) {
  if (g->d.dtype == WACM_F64)
    return d2::stage_t<double, 0>(g, p, (const double*)U, nullptr, nullptr, (double*)dU,
                                  nullptr, st);
  return d2::stage_t<float, 0>(g, p, (const float*)U, nullptr, nullptr, (float*)dU, nullptr,
                               st);
}

hipError_t launch_dt_2d(const wacm_grid* g, const wacm_params* p, const void* U, double* dt_dev,
                        hipStream_t st) {
  return g->d.dtype == WACM_F64 ? d2::dt_t(g, p, (const double*)U, dt_dev, st)
                                : d2::dt_t(g, p, (const float*)U, dt_dev, st);
}

hipError_t launch_rk4_2d(const wacm_grid* g, const wacm_params* p, double* t_dev, double* dt_dev,
                         void* U, void* work, int dt_mode, int64_t nsteps, hipStream_t st) {
  return g->d.dtype == WACM_F64
             ? d2::rk4_t(g, p, t_dev, dt_dev, (double*)U, work, dt_mode, nsteps, st)
             : d2::rk4_t(g, p, t_dev, dt_dev, (float*)U, work, dt_mode, nsteps, st);
}

hipError_t launch_diag_2d(const wacm_grid* g, const void* U, double* out, hipStream_t st) {
  return g->d.dtype == WACM_F64 ? d2::diag_t(g, (const double*)U, out, st)
                                : d2::diag_t(g, (const float*)U, out, st);
}

hipError_t launch_threshold_2d(const wacm_grid* g, const void* U, double eps, int dealias,
                               double* dmax, double* mrange, int8_t* flags, hipStream_t st) {
  return g->d.dtype == WACM_F64
             ? d2::thr_t(g, (const double*)U, eps, dealias, dmax, mrange, flags, st)
             : d2::thr_t(g, (const float*)U, eps, dealias, dmax, mrange, flags, st);
}

hipError_t launch_prolong_2d(const wacm_grid* g, void* U, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const d2::Lay L = d2::pool_layout(g);
  if (g->d.dtype == WACM_F64)
    d2::prolong2d_kernel<double><<<d2::blocks_for(n), NT_GEN, 0, st>>>(g->d_list, n, (double*)U,
                                                                       L, g->d.bs);
  else
    d2::prolong2d_kernel<float><<<d2::blocks_for(n), NT_GEN, 0, st>>>(g->d_list, n, (float*)U,
                                                                      L, g->d.bs);
  return hipGetLastError();
}

hipError_t launch_decimate_2d(const wacm_grid* g, void* U, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  const d2::Lay L = d2::pool_layout(g);
  if (g->d.dtype == WACM_F64)
    d2::decimate2d_kernel<double><<<d2::blocks_for(n), NT_GEN, 0, st>>>(g->d_list, n,
                                                                        (double*)U, L, g->d.bs);
  else
    d2::decimate2d_kernel<float><<<d2::blocks_for(n), NT_GEN, 0, st>>>(g->d_list, n, (float*)U,
                                                                       L, g->d.bs);
  return hipGetLastError();
}

}  // namespace wacm
