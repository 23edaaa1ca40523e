// HIP kernels of libwacm for gfx950 (MI355X).
//
// Data: the block pool U[slot][4][P][P][P] (x fastest, P = bs + 2 ng), RK
// registers in the same padded layout or compact (bs^3 per field), and the
// per-block neighbour tables (Tab) built on the host.  All kernels are
// memory-bound stencils: no MFMA; wave64 reductions; LDS slabs.
#include <cmath>
#include <mutex>

#include "resolve.h"
#include "wacm_internal.h"

namespace wacm {

__device__ __forceinline__ void load_tab(const Tab* __restrict__ g, Tab& s) {
  const int32_t* src = reinterpret_cast<const int32_t*>(g);
  int32_t* dst = reinterpret_cast<int32_t*>(&s);
  for (int q = threadIdx.x; q < (int)(sizeof(Tab) / 4); q += blockDim.x) dst[q] = src[q];
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// --------------------------------------------------------------------------
// ghost synchronisation
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT_GEN) void sync_kernel(const Tab* __restrict__ tab, int64_t nb,
                                                      T* __restrict__ U, Layout L, int bs,
                                                      int mode) {
  __shared__ Tab st;
  const int npts = mode == 1 ? 18 * bs * bs : L.P * L.P * L.P - bs * bs * bs;
  for (int64_t ib = blockIdx.x; ib < nb; ib += gridDim.x) {
    __syncthreads();
    load_tab(tab + ib, st);
    __syncthreads();
    T* dst = U + (int64_t)st.meta[0] * L.bstride;
    for (int p = threadIdx.x; p < npts; p += blockDim.x) {
      int i, j, k;
      shell_point(p, bs, L.ng, L.P, mode, i, j, k);
      T v[4];
      ghost_value<T>(st, bs, L, U, i, j, k, v);
      const int64_t o = ((int64_t)(k + L.ng) * L.P + (j + L.ng)) * L.P + (i + L.ng);
#pragma unroll
      for (int c = 0; c < 4; ++c) dst[o + c * L.fstride] = v[c];
    }
  }
}

// --------------------------------------------------------------------------
// fused rhs + RK4 stage (Sec. 2.2-2.3)
// --------------------------------------------------------------------------
template <typename T>
struct StageArgs {
  const Tab* tab;
  int64_t nb;
  const T* in;  // stage input, padded, face ghosts valid
  Layout Lin;
  T* un;  // U^n register (pool)
  Layout Lun;
  T* acc;  // accumulator (compact)
  Layout Lacc;
  T* out;  // next stage input, or dU for the rhs-only mode
  Layout Lout;
  const T* dus;  // extra solid velocity [slot][3][bs^3] or null
  const double* t_dev;
  const double* dt_dev;
  double t_host;
  double L;
  wacm_params p;
};

// MODE 0: dU = rhs(U).  MODE s = 1..4: classical RK4 stage s with registers
// U^n, acc, and the stage inputs:
//   s1: acc = U^n + dt/6 k1, out = U^n + dt/2 k1   (input = U^n)
//   s2: acc += dt/3 k2,      out = U^n + dt/2 k2
//   s3: acc += dt/3 k3,      out = U^n + dt k3
//   s4: U^n = acc + dt/6 k4
template <typename T, int BS, int MODE>
__global__ __launch_bounds__(BS* BS) void stage_kernel(StageArgs<T> a) {
  constexpr int H = 3, W = BS + 2 * H, NT = BS * BS;
  __shared__ T slab[4][W * W];
  const int tid = threadIdx.x;
  const int x = tid % BS, y = tid / BS;
  const T a1 = T(TW1), a2 = T(TW2), a3 = T(TW3);
  const T c2a = T(D2A), c2b = T(D2B), c2c = T(D2C);
  double tc = a.t_host, dt = 0.0;
  if (MODE != 0) {
    tc = *a.t_dev;
    dt = *a.dt_dev;
  }
  const double ts = tc + (MODE == 2 || MODE == 3 ? 0.5 * dt : (MODE == 4 ? dt : 0.0));
  const wacm_params& p = a.p;
  const T nu = T(p.nu), c0sq = T(p.c0 * p.c0), cg = T(p.c_gamma);
  const T iceta = p.mask ? T(1.0 / p.c_eta) : T(0), icsp = p.sponge ? T(1.0 / p.c_sp) : T(0);
  const T fA = T(MODE == 1 ? dt / 6.0 : (MODE == 4 ? dt / 6.0 : dt / 3.0));
  const T fB = T(MODE == 3 ? dt : 0.5 * dt);
  const int64_t fin = a.Lin.fstride;
  const int ngi = a.Lin.ng, Pi = a.Lin.P;
  const int cidx = (y + H) * W + (x + H);

  for (int64_t ib = blockIdx.x; ib < a.nb; ib += gridDim.x) {
    const int32_t* m = a.tab[ib].meta;
    const int slot = m[0], J = m[1], bx = m[2], by = m[3], bz = m[4];
    const double hd = a.L / (double(int64_t(1) << J) * BS);
    const T ih = T(1.0 / hd), ih2 = T(1.0 / (hd * hd));
    const T* __restrict__ in = a.in + (int64_t)slot * a.Lin.bstride;
    auto gi = [&](int i, int j, int k) -> int64_t {
      return ((int64_t)(k + ngi) * Pi + (j + ngi)) * Pi + (i + ngi);
    };
    T q[4][7];
#pragma unroll
    for (int c = 0; c < 4; ++c)
#pragma unroll
      for (int mm = 0; mm < 7; ++mm) q[c][mm] = in[c * fin + gi(x, y, mm - 3)];

    for (int z = 0; z < BS; ++z) {
      // prefetch the next column value
      T nq[4];
      if (z + 1 < BS) {
#pragma unroll
        for (int c = 0; c < 4; ++c) nq[c] = in[c * fin + gi(x, y, z + 4)];
      }
      __syncthreads();
#pragma unroll
      for (int c = 0; c < 4; ++c) slab[c][cidx] = q[c][3];
      for (int pp = tid; pp < 12 * BS; pp += NT) {
        const int f = pp / (3 * BS);
        const int rem = pp - f * 3 * BS;
        const int d = rem / BS, s = rem - d * BS;
        int hx, hy;
        if (f == 0) {
          hx = -1 - d;
          hy = s;
        } else if (f == 1) {
          hx = BS + d;
          hy = s;
        } else if (f == 2) {
          hx = s;
          hy = -1 - d;
        } else {
          hx = s;
          hy = BS + d;
        }
        const int li = (hy + H) * W + (hx + H);
        const int64_t g = gi(hx, hy, z);
#pragma unroll
        for (int c = 0; c < 4; ++c) slab[c][li] = in[c * fin + g];
      }
      __syncthreads();

      T d1[4][3], d2[3][3], val[4];
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const T* s = slab[c];
        val[c] = q[c][3];
        d1[c][0] = (a1 * (s[cidx + 1] - s[cidx - 1]) + a2 * (s[cidx + 2] - s[cidx - 2]) +
                    a3 * (s[cidx + 3] - s[cidx - 3])) *
                   ih;
        d1[c][1] = (a1 * (s[cidx + W] - s[cidx - W]) + a2 * (s[cidx + 2 * W] - s[cidx - 2 * W]) +
                    a3 * (s[cidx + 3 * W] - s[cidx - 3 * W])) *
                   ih;
        d1[c][2] = (a1 * (q[c][4] - q[c][2]) + a2 * (q[c][5] - q[c][1]) +
                    a3 * (q[c][6] - q[c][0])) *
                   ih;
        if (c < 3) {
          d2[c][0] = (c2a * s[cidx - 2] + c2b * s[cidx - 1] + c2c * s[cidx] + c2b * s[cidx + 1] +
                      c2a * s[cidx + 2]) *
                     ih2;
          d2[c][1] = (c2a * s[cidx - 2 * W] + c2b * s[cidx - W] + c2c * s[cidx] +
                      c2b * s[cidx + W] + c2a * s[cidx + 2 * W]) *
                     ih2;
          d2[c][2] = (c2a * q[c][1] + c2b * q[c][2] + c2c * q[c][3] + c2b * q[c][4] +
                      c2a * q[c][5]) *
                     ih2;
        }
      }
      T chi = T(0), sp = T(0), us[3] = {T(0), T(0), T(0)};
      if (p.mask || p.sponge) {
        const double xg = (double)(bx * BS + x) * hd, yg = (double)(by * BS + y) * hd,
                     zg = (double)(bz * BS + z) * hd;
        if (p.mask) {
          double cd, u3[3];
          mask_eval(p, ts, xg, yg, zg, cd, u3);
          chi = T(cd);
          us[0] = T(u3[0]);
          us[1] = T(u3[1]);
          us[2] = T(u3[2]);
        }
        if (p.sponge) sp = T(sponge_eval(p, a.L, xg, yg, zg));
      }
      if (a.dus) {
        const T* du = a.dus + (int64_t)slot * 3 * BS * BS * BS + (z * BS + y) * BS + x;
        us[0] += du[0];
        us[1] += du[BS * BS * BS];
        us[2] += du[2 * BS * BS * BS];
      }
      T r[4];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        T rc = -(val[0] * d1[c][0] + val[1] * d1[c][1] + val[2] * d1[c][2]) - d1[3][c] +
               nu * (d2[c][0] + d2[c][1] + d2[c][2]);
        if (p.mask) rc -= chi * iceta * (val[c] - us[c]);
        if (p.sponge) rc -= sp * icsp * (val[c] - T(p.u_inf[c]));
        r[c] = rc;
      }
      {
        T rp = -c0sq * (d1[0][0] + d1[1][1] + d1[2][2]) - cg * val[3];
        if (p.sponge) rp -= sp * icsp * (val[3] - T(p.p_inf));
        r[3] = rp;
      }

      if (MODE == 0) {
        T* o = a.out + (int64_t)slot * a.Lout.bstride;
        const int64_t oi = ((int64_t)(z + a.Lout.ng) * a.Lout.P + (y + a.Lout.ng)) * a.Lout.P +
                           (x + a.Lout.ng);
#pragma unroll
        for (int c = 0; c < 4; ++c) o[oi + c * a.Lout.fstride] = r[c];
      } else {
        T* accp = a.acc + (int64_t)slot * a.Lacc.bstride;
        const int64_t ai = ((int64_t)(z + a.Lacc.ng) * a.Lacc.P + (y + a.Lacc.ng)) * a.Lacc.P +
                           (x + a.Lacc.ng);
        T* unp = a.un + (int64_t)slot * a.Lun.bstride;
        const int64_t ui = ((int64_t)(z + a.Lun.ng) * a.Lun.P + (y + a.Lun.ng)) * a.Lun.P +
                           (x + a.Lun.ng);
        if (MODE == 1 || MODE == 2 || MODE == 3) {
          T* o = a.out + (int64_t)slot * a.Lout.bstride;
          const int64_t oi = ((int64_t)(z + a.Lout.ng) * a.Lout.P + (y + a.Lout.ng)) * a.Lout.P +
                             (x + a.Lout.ng);
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const T u0 = MODE == 1 ? val[c] : unp[ui + c * a.Lun.fstride];
            const T ac = MODE == 1 ? u0 : accp[ai + c * a.Lacc.fstride];
            accp[ai + c * a.Lacc.fstride] = ac + fA * r[c];
            o[oi + c * a.Lout.fstride] = u0 + fB * r[c];
          }
        } else {
#pragma unroll
          for (int c = 0; c < 4; ++c)
            unp[ui + c * a.Lun.fstride] = accp[ai + c * a.Lacc.fstride] + fA * r[c];
        }
      }
      if (z + 1 < BS) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
#pragma unroll
          for (int mm = 0; mm < 6; ++mm) q[c][mm] = q[c][mm + 1];
          q[c][6] = nq[c];
        }
      }
    }
  }
}

// --------------------------------------------------------------------------
// reductions (FP64 accumulation, fixed order -> deterministic)
// --------------------------------------------------------------------------
// per block: max over interior points of |u|^2 -> part[ib]
template <typename T>
__global__ __launch_bounds__(NT_GEN) void maxu_kernel(const Tab* __restrict__ tab, int64_t nb,
                                                      const T* __restrict__ U, Layout L, int bs,
                                                      double* __restrict__ part) {
  __shared__ double red[NT_GEN / 64];
  const int n3 = bs * bs * bs;
  for (int64_t ib = blockIdx.x; ib < nb; ib += gridDim.x) {
    const T* b = U + (int64_t)tab[ib].meta[0] * L.bstride;
    double m = 0.0;
    for (int q = threadIdx.x; q < n3; q += blockDim.x) {
      const int i = q % bs, j = (q / bs) % bs, k = q / (bs * bs);
      const int64_t o = ((int64_t)(k + L.ng) * L.P + (j + L.ng)) * L.P + (i + L.ng);
      const double u = b[o], v = b[o + L.fstride], w = b[o + 2 * L.fstride];
      m = fmax(m, u * u + v * v + w * w);
    }
    m = wave_max(m);
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

__global__ __launch_bounds__(NT_GEN) void dt_finalize(const double* __restrict__ part, int64_t nb,
                                                      wacm_params p, double hmin,
                                                      double* __restrict__ dt_out) {
  __shared__ double red[NT_GEN / 64];
  double m = 0.0;
  for (int64_t q = threadIdx.x; q < nb; q += blockDim.x) m = fmax(m, part[q]);
  m = wave_max(m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = red[0];
    for (int w = 1; w < NT_GEN / 64; ++w) r = fmax(r, red[w]);
    const double umax = sqrt(r);
    const double ueig = umax + sqrt(umax * umax + p.c0 * p.c0);
    double dt = p.cfl * hmin / ueig;
    if (p.mask) dt = fmin(dt, p.cfl_eta * p.c_eta);
    if (p.sponge) dt = fmin(dt, p.cfl_eta * p.c_sp);
    if (p.nu > 0) dt = fmin(dt, p.cfl_nu * hmin * hmin / p.nu);
    *dt_out = dt;
  }
}

__global__ void advance_time(double* t, const double* dt) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *t = *t + *dt;
}

// diagnostics partials per block: [max|u|^2, max|u|, max|v|, max|w|, max|p|,
// sum chi(u-us) x3 (times h^3/C_eta), sum |u|^2 (times h^3/2)]
template <typename T>
__global__ __launch_bounds__(NT_GEN) void diag_kernel(const Tab* __restrict__ tab, int64_t nb,
                                                      const T* __restrict__ U, Layout L, int bs,
                                                      const T* __restrict__ dus, double Ldom,
                                                      wacm_params p, double t,
                                                      double* __restrict__ part) {
  __shared__ double red[9][NT_GEN];
  const int n3 = bs * bs * bs;
  for (int64_t ib = blockIdx.x; ib < nb; ib += gridDim.x) {
    const int32_t* m = tab[ib].meta;
    const int slot = m[0], J = m[1];
    const double h = Ldom / (double(int64_t(1) << J) * bs);
    const T* b = U + (int64_t)slot * L.bstride;
    double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int q = threadIdx.x; q < n3; q += blockDim.x) {
      const int i = q % bs, j = (q / bs) % bs, k = q / (bs * bs);
      const int64_t o = ((int64_t)(k + L.ng) * L.P + (j + L.ng)) * L.P + (i + L.ng);
      double u[4];
      for (int c = 0; c < 4; ++c) u[c] = b[o + c * L.fstride];
      const double m2 = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
      acc[0] = fmax(acc[0], m2);
      for (int c = 0; c < 4; ++c) acc[1 + c] = fmax(acc[1 + c], fabs(u[c]));
      if (p.mask) {
        double chi, us[3];
        mask_eval(p, t, (double)(m[2] * bs + i) * h, (double)(m[3] * bs + j) * h,
                  (double)(m[4] * bs + k) * h, chi, us);
        if (dus)
          for (int d = 0; d < 3; ++d) us[d] += (double)dus[((int64_t)slot * 3 + d) * n3 + q];
        for (int d = 0; d < 3; ++d) acc[5 + d] += chi * (u[d] - us[d]);
      }
      acc[8] += m2;
    }
    __syncthreads();
    for (int c = 0; c < 9; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int s = NT_GEN / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
        for (int c = 0; c < 5; ++c)
          red[c][threadIdx.x] = fmax(red[c][threadIdx.x], red[c][threadIdx.x + s]);
        for (int c = 5; c < 9; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const double vol = h * h * h;
      for (int c = 0; c < 5; ++c) part[ib * 9 + c] = red[c][0];
      for (int c = 5; c < 8; ++c) part[ib * 9 + c] = p.mask ? red[c][0] * vol / p.c_eta : 0.0;
      part[ib * 9 + 8] = 0.5 * red[8][0] * vol;
    }
  }
}

__global__ __launch_bounds__(NT_GEN) void diag_finalize(const double* __restrict__ part,
                                                        int64_t nb, double* __restrict__ out) {
  __shared__ double red[9][NT_GEN];
  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t q = threadIdx.x; q < nb; q += blockDim.x) {
    for (int c = 0; c < 5; ++c) acc[c] = fmax(acc[c], part[q * 9 + c]);
    for (int c = 5; c < 9; ++c) acc[c] += part[q * 9 + c];
  }
  for (int c = 0; c < 9; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int s = NT_GEN / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      for (int c = 0; c < 5; ++c)
        red[c][threadIdx.x] = fmax(red[c][threadIdx.x], red[c][threadIdx.x + s]);
      for (int c = 5; c < 9; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sqrt(red[0][0]);
    for (int c = 1; c < 9; ++c) out[c] = red[c][0];
  }
}

// --------------------------------------------------------------------------
// wavelet details and coarsening flags (Sec. 3.1, 3.3-3.5)
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT_GEN) void norm_kernel(const Tab* __restrict__ tab, int64_t nb,
                                                      const T* __restrict__ U, Layout L, int bs,
                                                      double* __restrict__ part) {
  __shared__ double red[4][NT_GEN / 64];
  const int n3 = bs * bs * bs;
  for (int64_t ib = blockIdx.x; ib < nb; ib += gridDim.x) {
    const T* b = U + (int64_t)tab[ib].meta[0] * L.bstride;
    double m[4] = {0, 0, 0, 0};
    for (int q = threadIdx.x; q < n3; q += blockDim.x) {
      const int i = q % bs, j = (q / bs) % bs, k = q / (bs * bs);
      const int64_t o = ((int64_t)(k + L.ng) * L.P + (j + L.ng)) * L.P + (i + L.ng);
      for (int c = 0; c < 4; ++c) m[c] = fmax(m[c], fabs((double)b[o + c * L.fstride]));
    }
    __syncthreads();
    for (int c = 0; c < 4; ++c) {
      const double v = wave_max(m[c]);
      if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = v;
    }
    __syncthreads();
    if (threadIdx.x < 4) {
      double r = red[threadIdx.x][0];
      for (int w = 1; w < NT_GEN / 64; ++w) r = fmax(r, red[threadIdx.x][w]);
      part[ib * 4 + threadIdx.x] = r;
    }
  }
}

__global__ __launch_bounds__(NT_GEN) void norm_finalize(const double* __restrict__ part,
                                                        int64_t nb, double* __restrict__ norm) {
  __shared__ double red[4][NT_GEN / 64];
  double m[4] = {0, 0, 0, 0};
  for (int64_t q = threadIdx.x; q < nb; q += blockDim.x)
    for (int c = 0; c < 4; ++c) m[c] = fmax(m[c], part[q * 4 + c]);
  for (int c = 0; c < 4; ++c) {
    const double v = wave_max(m[c]);
    if ((threadIdx.x & 63) == 0) red[c][threadIdx.x >> 6] = v;
  }
  __syncthreads();
  if (threadIdx.x < 4) {
    double r = red[threadIdx.x][0];
    for (int w = 1; w < NT_GEN / 64; ++w) r = fmax(r, red[threadIdx.x][w]);
    norm[threadIdx.x] = r > 0.0 ? r : 1.0;
  }
}

template <typename T>
__global__ __launch_bounds__(NT_GEN) void detail_kernel(
    const Tab* __restrict__ tab, int64_t nb, const T* __restrict__ U, Layout L, int bs,
    const double* __restrict__ norm, double Ldom, wacm_params p, double t, double eps,
    int dealias, int jmin, int jmax, double* __restrict__ dmax, double* __restrict__ mrange,
    int8_t* __restrict__ flags) {
  __shared__ double red[3][NT_GEN / 64];
  const int n3 = bs * bs * bs;
  double inv[4];
  for (int c = 0; c < 4; ++c) inv[c] = 1.0 / norm[c];
  for (int64_t ib = blockIdx.x; ib < nb; ib += gridDim.x) {
    const int32_t* m = tab[ib].meta;
    const int slot = m[0], J = m[1];
    const double h = Ldom / (double(int64_t(1) << J) * bs);
    const T* b = U + (int64_t)slot * L.bstride;
    double dm = 0.0, cmin = 1e300, cmax = -1e300;
    for (int q = threadIdx.x; q < n3; q += blockDim.x) {
      const int i = q % bs, j = (q / bs) % bs, k = q / (bs * bs);
      if (p.mask) {
        double chi, us[3];
        mask_eval(p, t, (double)(m[2] * bs + i) * h, (double)(m[3] * bs + j) * h,
                  (double)(m[4] * bs + k) * h, chi, us);
        cmin = fmin(cmin, chi);
        cmax = fmax(cmax, chi);
      }
      if (((i | j | k) & 1) == 0) continue;
      int tx[4], ty[4], tz[4];
      T wx[4], wy[4], wz[4];
      int nx, ny, nz;
      auto taps = [](int q2, int* tq, T* wq, int& n) {
        if ((q2 & 1) == 0) {
          tq[0] = q2;
          wq[0] = T(1);
          n = 1;
        } else {
          tq[0] = q2 - 3;
          tq[1] = q2 - 1;
          tq[2] = q2 + 1;
          tq[3] = q2 + 3;
          wq[0] = T(DDW0);
          wq[1] = T(DDW1);
          wq[2] = T(DDW1);
          wq[3] = T(DDW0);
          n = 4;
        }
      };
      taps(i, tx, wx, nx);
      taps(j, ty, wy, ny);
      taps(k, tz, wz, nz);
      T pred[4] = {T(0), T(0), T(0), T(0)};
      for (int aa = 0; aa < nz; ++aa)
        for (int bb = 0; bb < ny; ++bb) {
          const T wzy = wz[aa] * wy[bb];
          for (int e = 0; e < nx; ++e) {
            const T w = wzy * wx[e];
            const int64_t o = ((int64_t)(tz[aa] + L.ng) * L.P + (ty[bb] + L.ng)) * L.P +
                              (tx[e] + L.ng);
            for (int c = 0; c < 4; ++c) pred[c] += w * b[o + c * L.fstride];
          }
        }
      const int64_t o = ((int64_t)(k + L.ng) * L.P + (j + L.ng)) * L.P + (i + L.ng);
      for (int c = 0; c < 4; ++c) {
        const T d = b[o + c * L.fstride] - pred[c];
        dm = fmax(dm, fabs((double)d) * inv[c]);
      }
    }
    dm = wave_max(dm);
    cmin = wave_min(cmin);
    cmax = wave_max(cmax);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) {
      red[0][threadIdx.x >> 6] = dm;
      red[1][threadIdx.x >> 6] = cmin;
      red[2][threadIdx.x >> 6] = cmax;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      double r0 = red[0][0], r1 = red[1][0], r2 = red[2][0];
      for (int w = 1; w < NT_GEN / 64; ++w) {
        r0 = fmax(r0, red[0][w]);
        r1 = fmin(r1, red[1][w]);
        r2 = fmax(r2, red[2][w]);
      }
      const double mr = p.mask ? r2 - r1 : 0.0;
      dmax[ib] = r0;
      mrange[ib] = mr;
      int f = 0;
      if (J > jmin) {
        if (dealias && J == jmax)
          f = 1;
        else if (r0 < eps && mr == 0.0)
          f = 1;
      }
      flags[ib] = (int8_t)f;
    }
  }
}

// --------------------------------------------------------------------------
// refinement (prediction into 8 children) and coarsening (decimation)
// --------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(NT_GEN) void prolong_kernel(const int32_t* __restrict__ list,
                                                         int64_t n, T* __restrict__ U, Layout L,
                                                         int bs) {
  const int n3 = bs * bs * bs;
  for (int64_t w = blockIdx.x; w < n; w += gridDim.x) {
    const int32_t ps = list[3 * w], cs = list[3 * w + 1], oct = list[3 * w + 2];
    const int off[3] = {(oct & 1) * bs, ((oct >> 1) & 1) * bs, ((oct >> 2) & 1) * bs};
    const T* par = U + (int64_t)ps * L.bstride;
    T* ch = U + (int64_t)cs * L.bstride;
    for (int q = threadIdx.x; q < n3; q += blockDim.x) {
      const int i = q % bs, j = (q / bs) % bs, k = q / (bs * bs);
      const int Q[3] = {off[0] + i, off[1] + j, off[2] + k};
      int tq[3][4];
      T wq[3][4];
      int nq[3];
      for (int d = 0; d < 3; ++d) {
        if ((Q[d] & 1) == 0) {
          tq[d][0] = Q[d] >> 1;
          wq[d][0] = T(1);
          nq[d] = 1;
        } else {
          tq[d][0] = (Q[d] - 3) >> 1;
          tq[d][1] = (Q[d] - 1) >> 1;
          tq[d][2] = (Q[d] + 1) >> 1;
          tq[d][3] = (Q[d] + 3) >> 1;
          wq[d][0] = T(DDW0);
          wq[d][1] = T(DDW1);
          wq[d][2] = T(DDW1);
          wq[d][3] = T(DDW0);
          nq[d] = 4;
        }
      }
      T acc[4] = {T(0), T(0), T(0), T(0)};
      for (int a = 0; a < nq[2]; ++a)
        for (int b = 0; b < nq[1]; ++b) {
          const T wzy = wq[2][a] * wq[1][b];
          for (int e = 0; e < nq[0]; ++e) {
            const T wgt = wzy * wq[0][e];
            const int64_t o = ((int64_t)(tq[2][a] + L.ng) * L.P + (tq[1][b] + L.ng)) * L.P +
                              (tq[0][e] + L.ng);
            for (int c = 0; c < 4; ++c) acc[c] += wgt * par[o + c * L.fstride];
          }
        }
      const int64_t o = ((int64_t)(k + L.ng) * L.P + (j + L.ng)) * L.P + (i + L.ng);
      for (int c = 0; c < 4; ++c) ch[o + c * L.fstride] = acc[c];
    }
  }
}

template <typename T>
__global__ __launch_bounds__(NT_GEN) void decimate_kernel(const int32_t* __restrict__ list,
                                                          int64_t n, T* __restrict__ U, Layout L,
                                                          int bs) {
  const int n3 = bs * bs * bs;
  for (int64_t w = blockIdx.x; w < n; w += gridDim.x) {
    const int32_t* e = list + 10 * w;
    T* par = U + (int64_t)e[0] * L.bstride;
    for (int q = threadIdx.x; q < n3; q += blockDim.x) {
      const int i = q % bs, j = (q / bs) % bs, k = q / (bs * bs);
      const int ci = 2 * i >= bs, cj = 2 * j >= bs, ck = 2 * k >= bs;
      const T* ch = U + (int64_t)e[1 + ci + 2 * cj + 4 * ck] * L.bstride;
      const int64_t os = ((int64_t)(2 * k - ck * bs + L.ng) * L.P + (2 * j - cj * bs + L.ng)) *
                             L.P +
                         (2 * i - ci * bs + L.ng);
      const int64_t od = ((int64_t)(k + L.ng) * L.P + (j + L.ng)) * L.P + (i + L.ng);
      for (int c = 0; c < 4; ++c) par[od + c * L.fstride] = ch[os + c * L.fstride];
    }
  }
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
static int num_cus() {
  static int cus = 0;
  static std::once_flag once;
  std::call_once(once, [] {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
      cus = prop.multiProcessorCount;
    if (cus <= 0) cus = 256;
  });
  return cus;
}

// Records an event pair around the launches in its scope when profiling is on.
class ProfScope {
 public:
  ProfScope(const wacm_grid* g, int cls, hipStream_t st) : g_(g), st_(st) {
    if (!g_->prof.on) return;
    Profiler& p = g_->prof;
    if (p.recs.size() >= 4096) (void)profile_flush(g_);
    hipEvent_t e[2];
    for (int i = 0; i < 2; ++i) {
      if (!p.spare.empty()) {
        e[i] = p.spare.back();
        p.spare.pop_back();
      } else if (hipEventCreate(&e[i]) != hipSuccess) {
        e[i] = nullptr;
      }
    }
    if (!e[0] || !e[1]) return;
    rec_ = {cls, e[0], e[1]};
    active_ = hipEventRecord(e[0], st_) == hipSuccess;
  }
  ~ProfScope() {
    if (!active_) return;
    if (hipEventRecord(rec_.b, st_) == hipSuccess) g_->prof.recs.push_back(rec_);
  }

 private:
  const wacm_grid* g_;
  hipStream_t st_;
  Profiler::Rec rec_{};
  bool active_ = false;
};

hipError_t profile_flush(const wacm_grid* g) {
  Profiler& p = g->prof;
  hipError_t err = hipSuccess;
  for (const auto& r : p.recs) {
    float ms = 0.f;
    hipError_t e = hipEventSynchronize(r.b);
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
    if (e == hipSuccess) {
      p.ms[r.cls] += ms;
      p.n[r.cls] += 1;
    } else {
      err = e;
    }
    p.spare.push_back(r.a);
    p.spare.push_back(r.b);
  }
  p.recs.clear();
  return err;
}

static Layout pool_layout(const wacm_grid* g) {
  Layout L;
  L.P = g->P;
  L.ng = g->d.ng;
  L.fstride = (int64_t)g->P * g->P * g->P;
  L.bstride = 4 * L.fstride;
  return L;
}
static Layout compact_layout(const wacm_grid* g) {
  Layout L;
  L.P = g->d.bs;
  L.ng = 0;
  L.fstride = (int64_t)g->d.bs * g->d.bs * g->d.bs;
  L.bstride = 4 * L.fstride;
  return L;
}

static unsigned grid_for(int64_t n, int per_cu) {
  int64_t cap = (int64_t)num_cus() * per_cu;
  return (unsigned)(n < cap ? (n > 0 ? n : 1) : cap);
}

size_t work_bytes(const wacm_grid* g) {
  const size_t es = g->d.dtype == WACM_F64 ? 8 : 4;
  const size_t cap = (size_t)g->d.capacity;
  const size_t P3 = (size_t)g->P * g->P * g->P, b3 = (size_t)g->d.bs * g->d.bs * g->d.bs;
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  return up(cap * 4 * b3 * es) + 2 * up(cap * 4 * P3 * es);
}

template <typename T>
static hipError_t sync_t(const wacm_grid* g, T* U, int mode, hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  sync_kernel<T><<<grid_for(g->nb, 8), NT_GEN, 0, st>>>(g->d_tab, g->nb, U, pool_layout(g),
                                                        g->d.bs, mode);
  return hipGetLastError();
}

hipError_t launch_sync(const wacm_grid* g, void* U, int face_only, hipStream_t st) {
  return g->d.dtype == WACM_F64 ? sync_t(g, (double*)U, face_only ? 1 : 0, st)
                                : sync_t(g, (float*)U, face_only ? 1 : 0, st);
}

template <typename T, int BS, int MODE>
static hipError_t stage_launch(const StageArgs<T>& a, hipStream_t st) {
  const int per_cu = BS <= 16 ? 8 : 2;
  stage_kernel<T, BS, MODE><<<grid_for(a.nb, per_cu), BS * BS, 0, st>>>(a);
  return hipGetLastError();
}

template <typename T, int MODE>
static hipError_t stage_dispatch(int bs, const StageArgs<T>& a, hipStream_t st) {
  switch (bs) {
    case 16:
      return stage_launch<T, 16, MODE>(a, st);
    case 24:
      return stage_launch<T, 24, MODE>(a, st);
    case 32:
      return stage_launch<T, 32, MODE>(a, st);
    default:
      return hipErrorInvalidValue;
  }
}

template <typename T>
static StageArgs<T> base_args(const wacm_grid* g, const wacm_params* p) {
  StageArgs<T> a{};
  a.tab = g->d_tab;
  a.nb = g->nb;
  a.L = g->d.L;
  a.p = *p;
  return a;
}

template <typename T>
static hipError_t rhs_t(const wacm_grid* g, const wacm_params* p, double t, const T* U, T* dU,
                        const T* dus, hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  StageArgs<T> a = base_args<T>(g, p);
  a.in = U;
  a.Lin = pool_layout(g);
  a.out = dU;
  a.Lout = pool_layout(g);
  a.dus = dus;
  a.t_host = t;
  return stage_dispatch<T, 0>(g->d.bs, a, st);
}

hipError_t launch_rhs(const wacm_grid* g, const wacm_params* p, double t, const void* U,
                      void* dU, const void* dus, hipStream_t st) {
  return g->d.dtype == WACM_F64
             ? rhs_t(g, p, t, (const double*)U, (double*)dU, (const double*)dus, st)
             : rhs_t(g, p, t, (const float*)U, (float*)dU, (const float*)dus, st);
}

template <typename T>
static hipError_t dt_t(const wacm_grid* g, const wacm_params* p, const T* U, double* dt_dev,
                       hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  maxu_kernel<T><<<grid_for(g->nb, 8), NT_GEN, 0, st>>>(g->d_tab, g->nb, U, pool_layout(g),
                                                        g->d.bs, g->d_part);
  const double hmin = g->d.L / (double(int64_t(1) << g->jfine) * g->d.bs);
  dt_finalize<<<1, NT_GEN, 0, st>>>(g->d_part, g->nb, *p, hmin, dt_dev);
  return hipGetLastError();
}

hipError_t launch_dt(const wacm_grid* g, const wacm_params* p, const void* U, double* dt_dev,
                     hipStream_t st) {
  return g->d.dtype == WACM_F64 ? dt_t(g, p, (const double*)U, dt_dev, st)
                                : dt_t(g, p, (const float*)U, dt_dev, st);
}

template <typename T>
static hipError_t rk4_t(const wacm_grid* g, const wacm_params* p, double* t_dev, double* dt_dev,
                        T* U, void* work, const T* dus, int dt_mode, hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  hipError_t e;
  if (dt_mode == WACM_DT_CFL) {
    ProfScope ps(g, 0, st);
    if ((e = dt_t<T>(g, p, U, dt_dev, st)) != hipSuccess) return e;
  }
  const size_t es = sizeof(T);
  const size_t cap = (size_t)g->d.capacity;
  const size_t P3 = (size_t)g->P * g->P * g->P, b3 = (size_t)g->d.bs * g->d.bs * g->d.bs;
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  char* w = (char*)work;
  T* acc = (T*)w;
  T* ping = (T*)(w + up(cap * 4 * b3 * es));
  T* pong = (T*)(w + up(cap * 4 * b3 * es) + up(cap * 4 * P3 * es));
  StageArgs<T> a = base_args<T>(g, p);
  a.un = U;
  a.Lun = pool_layout(g);
  a.acc = acc;
  a.Lacc = compact_layout(g);
  a.dus = dus;
  a.t_dev = t_dev;
  a.dt_dev = dt_dev;
  const Layout Lp = pool_layout(g);
  T* ins[4] = {U, ping, pong, ping};
  T* outs[4] = {ping, pong, ping, nullptr};
  for (int s = 0; s < 4; ++s) {
    {
      ProfScope ps(g, 1, st);
      if ((e = sync_t<T>(g, ins[s], 1, st)) != hipSuccess) return e;
    }
    ProfScope ps(g, 2, st);
    a.in = ins[s];
    a.Lin = Lp;
    a.out = outs[s];
    a.Lout = Lp;
    switch (s) {
      case 0:
        e = stage_dispatch<T, 1>(g->d.bs, a, st);
        break;
      case 1:
        e = stage_dispatch<T, 2>(g->d.bs, a, st);
        break;
      case 2:
        e = stage_dispatch<T, 3>(g->d.bs, a, st);
        break;
      default:
        e = stage_dispatch<T, 4>(g->d.bs, a, st);
        break;
    }
    if (e != hipSuccess) return e;
  }
  ProfScope ps(g, 3, st);
  advance_time<<<1, 64, 0, st>>>(t_dev, dt_dev);
  return hipGetLastError();
}

hipError_t launch_rk4(const wacm_grid* g, const wacm_params* p, double* t_dev, double* dt_dev,
                      void* U, void* work, const void* dus, int dt_mode, hipStream_t st) {
  return g->d.dtype == WACM_F64
             ? rk4_t(g, p, t_dev, dt_dev, (double*)U, work, (const double*)dus, dt_mode, st)
             : rk4_t(g, p, t_dev, dt_dev, (float*)U, work, (const float*)dus, dt_mode, st);
}

template <typename T>
static hipError_t diag_t(const wacm_grid* g, const wacm_params* p, double t, const T* U,
                         const T* dus, double* out, hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  diag_kernel<T><<<grid_for(g->nb, 8), NT_GEN, 0, st>>>(g->d_tab, g->nb, U, pool_layout(g),
                                                        g->d.bs, dus, g->d.L, *p, t, g->d_part);
  diag_finalize<<<1, NT_GEN, 0, st>>>(g->d_part, g->nb, out);
  return hipGetLastError();
}

hipError_t launch_diag(const wacm_grid* g, const wacm_params* p, double t, const void* U,
                       const void* dus, double* out, hipStream_t st) {
  return g->d.dtype == WACM_F64
             ? diag_t(g, p, t, (const double*)U, (const double*)dus, out, st)
             : diag_t(g, p, t, (const float*)U, (const float*)dus, out, st);
}

template <typename T>
static hipError_t thr_t(const wacm_grid* g, const wacm_params* p, double t, const T* U,
                        double eps, int dealias, double* dmax, double* mrange, int8_t* flags,
                        hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  norm_kernel<T><<<grid_for(g->nb, 8), NT_GEN, 0, st>>>(g->d_tab, g->nb, U, pool_layout(g),
                                                        g->d.bs, g->d_part);
  norm_finalize<<<1, NT_GEN, 0, st>>>(g->d_part, g->nb, g->d_norm);
  detail_kernel<T><<<grid_for(g->nb, 8), NT_GEN, 0, st>>>(
      g->d_tab, g->nb, U, pool_layout(g), g->d.bs, g->d_norm, g->d.L, *p, t, eps, dealias,
      g->d.jmin, g->d.jmax, dmax, mrange, flags);
  return hipGetLastError();
}

hipError_t launch_threshold(const wacm_grid* g, const wacm_params* p, double t, const void* U,
                            double eps, int dealias, double* dmax, double* mrange,
                            int8_t* flags, hipStream_t st) {
  return g->d.dtype == WACM_F64
             ? thr_t(g, p, t, (const double*)U, eps, dealias, dmax, mrange, flags, st)
             : thr_t(g, p, t, (const float*)U, eps, dealias, dmax, mrange, flags, st);
}

hipError_t launch_prolong(const wacm_grid* g, void* U, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (g->d.dtype == WACM_F64)
    prolong_kernel<double><<<grid_for(n, 8), NT_GEN, 0, st>>>(g->d_list, n, (double*)U,
                                                             pool_layout(g), g->d.bs);
  else
    prolong_kernel<float><<<grid_for(n, 8), NT_GEN, 0, st>>>(g->d_list, n, (float*)U,
                                                            pool_layout(g), g->d.bs);
  return hipGetLastError();
}

hipError_t launch_decimate(const wacm_grid* g, void* U, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (g->d.dtype == WACM_F64)
    decimate_kernel<double><<<grid_for(n, 8), NT_GEN, 0, st>>>(g->d_list, n, (double*)U,
                                                              pool_layout(g), g->d.bs);
  else
    decimate_kernel<float><<<grid_for(n, 8), NT_GEN, 0, st>>>(g->d_list, n, (float*)U,
                                                             pool_layout(g), g->d.bs);
  return hipGetLastError();
}

}  // namespace wacm
