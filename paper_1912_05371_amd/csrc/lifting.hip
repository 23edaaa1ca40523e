// CDF 4/4 lifted restriction (Sec. 3.2) on the device: the second phase of
// the ghost synchronisation (ghost points whose owner is finer) and the
// parents of merged families.
//
// Lifting the interpolating CDF 4/0 wavelet to 4 vanishing moments turns
// restriction from decimation into a low-pass filter.  Along one axis the
// coarse value at an even fine point is
//   c = u_0 + sum_m U_m (u_m - P u_m),  m = -3, -1, 1, 3,
// P the DD4 prediction from the neighbours m-3, m-1, m+1, m+3 and
// U = (-1, 9, 9, -1)/32; expanded, a 13-tap filter on the offsets -6..6
// (zero at +-5).  In 3D it is applied along x, y and z.  The fine values are
// read from the finer leaf's padded array after the CDF 4/0 ghost fill, whose
// ghost layers must be at least 6 deep.
#include <hip/hip_runtime.h>

#include "resolve.h"
#include "wacm_internal.h"

namespace wacm {

// Expanded lifted low-pass, offsets -6..6.
constexpr double LIFT_TAP[13] = {-1.0 / 512,  0.0,         18.0 / 512,  -16.0 / 512, -63.0 / 512,
                                 144.0 / 512, 348.0 / 512, 144.0 / 512, -63.0 / 512, -16.0 / 512,
                                 18.0 / 512,  0.0,         -1.0 / 512};

// One work item: a box of nx x ny x nz coarse outputs.  Source: the padded
// array of pool slot `sslot`; the output (dx, dy, dz) is centred on the
// source's fine point (fx0 + 2 dx, fy0 + 2 dy, fz0 + 2 dz).  Items of the
// ghost phase write into a staging buffer (4 fields, [c][dz][dy][dx], at 4 *
// base values), so that no item reads a ghost value another item rewrites;
// items of a merge write the parent's interior directly (parent slots are
// fresh).  Each output is a z-march over the 13 fine planes around it: for
// every fine plane an x pass on the fine rows into LDS, a y pass per output
// column into a register ring of the last 13 planes, and the z pass once the
// ring holds an output's 13 planes.  A workgroup takes NF of the 4 fields of
// an item at a time (one work unit).
//
// mode 0: `items` holds 12 int32 per item (dst slot, i0, j0, k0, nx, ny, nz,
//         src slot, fx0, fy0, fz0, base); outputs to `out` at 4 * base.
// mode 1: `items` is the merge list (10 int32 per parent: parent slot, 8
//         child slots, unused); item w is octant w % 8 of parent w / 8, a box
//         of (bs/2)^3 outputs at the octant's offset, centred on the child's
//         even points from (0, 0, 0); outputs into U at the parent.
template <typename T, int BS, int NF, bool INPLACE>
__global__ __launch_bounds__(NT_GEN) void lift_box_kernel(const int32_t* __restrict__ items,
                                                          int64_t n, const T* U, Layout L,
                                                          T* out, int mode,
                                                          const Tab* __restrict__ tab,
                                                          const int32_t* __restrict__ stab) {
  constexpr int NM = BS / 2;           // largest box edge
  constexpr int NROW = 2 * NM + 11;    // fine rows a box needs
  constexpr int NU = 4 / NF;           // work units per item
  __shared__ T xq[NF][NROW * NM];      // x pass of the current fine plane
  __shared__ Tab ft;                   // the finer leaf's table (in-place reads)
  __shared__ int64_t rowo[3][NROW];    // per fine row of the plane: offsets of x = 0
  const int tid = threadIdx.x;
  // INPLACE (mode 0): values of the finer leaf's ghost regions whose level-J
  // box is a leaf are read from that leaf's interior (the same values its
  // ghost fill would copy there); the other ghost regions from its array
  constexpr bool inplace = INPLACE;
  T h[13];
#pragma unroll
  for (int q = 0; q < 13; ++q) h[q] = T(LIFT_TAP[q]);
  for (int64_t u = blockIdx.x; u < n * NU; u += gridDim.x) {
    const int64_t w = u / NU;
    const int c0 = (int)(u - w * NU) * NF;  // first field of this unit
    int dslot, i0, j0, k0, nx, ny, nz, sslot, fx0, fy0, fz0;
    int64_t base = 0;
    if (mode == 0) {
      const int32_t* e = items + 12 * w;
      dslot = e[0], i0 = e[1], j0 = e[2], k0 = e[3], nx = e[4], ny = e[5], nz = e[6];
      sslot = e[7], fx0 = e[8], fy0 = e[9], fz0 = e[10];
      base = (int64_t)e[11] * 4;
    } else {
      const int32_t* e = items + 10 * (w >> 3);
      const int oc = (int)(w & 7);
      dslot = e[0];
      sslot = e[1 + oc];
      i0 = (oc & 1) * NM, j0 = ((oc >> 1) & 1) * NM, k0 = (oc >> 2) * NM;
      nx = ny = nz = NM;
      fx0 = fy0 = fz0 = 0;
    }
    const T* src = U + c0 * L.fstride;
    if (inplace) {
      __syncthreads();  // ft is free again
      const int32_t* ts = reinterpret_cast<const int32_t*>(tab + stab[sslot]);
      int32_t* td = reinterpret_cast<int32_t*>(&ft);
      for (int q = tid; q < (int)(sizeof(Tab) / 4); q += NT_GEN) td[q] = ts[q];
      __syncthreads();
    }
    const int nrow = 2 * ny + 11, nplane = 2 * nz + 11, nxp = nrow * nx;
    const bool own = tid < nx * ny;
    const int dx = own ? tid % nx : 0, dy = own ? tid / nx : 0;
    T ring[NF][13];
#pragma unroll
    for (int c = 0; c < NF; ++c)
#pragma unroll
      for (int q = 0; q < 13; ++q) ring[c][q] = T(0);
    for (int zf = 0; zf < nplane; ++zf) {
      const int z = fz0 - 6 + zf;
      // element offsets of each fine row's point x = 0 for x < 0, 0 <= x < bs
      // and x >= bs (the three regions along x); the last plane's x pass,
      // which read them, ended before its second barrier
      if (inplace && tid < 3 * nrow) {
        const int rx = tid / nrow, yf = tid - rx * nrow;
        const int y = fy0 - 6 + yf;
        int64_t o = (int64_t)sslot * L.bstride + ((int64_t)(z + L.ng) * L.P + (y + L.ng)) * L.P + L.ng;
        const int ry = y < 0 ? 0 : (y < BS ? 1 : 2), rz = z < 0 ? 0 : (z < BS ? 1 : 2);
        const int r = rx + 3 * ry + 9 * rz;
        if (r != 13 && ft.kind[r] == 0) {
          const int sy = ry == 0 ? BS : (ry == 2 ? -BS : 0);
          const int sz = rz == 0 ? BS : (rz == 2 ? -BS : 0);
          o = (int64_t)ft.slot[r][0] * L.bstride +
              ((int64_t)(z + sz + L.ng) * L.P + (y + sy + L.ng)) * L.P + L.ng +
              (rx == 0 ? BS : (rx == 2 ? -BS : 0));
        }
        rowo[rx][yf] = o;
      }
      __syncthreads();  // xq is free again, rowo is written
      for (int it = tid; it < NF * nxp; it += NT_GEN) {
        const int c = it / nxp, rem = it - c * nxp;
        const int yf = rem / nx, ox = rem - yf * nx;
        const T* sc = src + c * L.fstride;
        const int x0 = fx0 + 2 * ox - 6;  // the taps' window is x0..x0+12
        T v = T(0);
        if constexpr (inplace) {
          const int64_t r0 = rowo[0][yf], r1 = rowo[1][yf], r2 = rowo[2][yf];
#pragma unroll
          for (int q = 0; q < 13; ++q)
            if (q != 1 && q != 11) {
              const int x = x0 + q;
              v += h[q] * sc[(x < 0 ? r0 : (x < BS ? r1 : r2)) + x];
            }
        } else {
          const int y = fy0 - 6 + yf;
          const T* row = sc + (int64_t)sslot * L.bstride +
                         ((int64_t)(z + L.ng) * L.P + (y + L.ng)) * L.P + L.ng + x0;
#pragma unroll
          for (int q = 0; q < 13; ++q)
            if (q != 1 && q != 11) v += h[q] * row[q];
        }
        xq[c][yf * NM + ox] = v;
      }
      __syncthreads();
      if (own) {
        const bool emit = zf >= 12 && ((zf - 12) & 1) == 0;
        const int k = (zf - 12) >> 1;
#pragma unroll
        for (int c = 0; c < NF; ++c) {
          T v = T(0);
#pragma unroll
          for (int q = 0; q < 13; ++q)
            if (q != 1 && q != 11) v += h[q] * xq[c][(2 * dy + q) * NM + dx];
#pragma unroll
          for (int q = 0; q < 12; ++q) ring[c][q] = ring[c][q + 1];
          ring[c][12] = v;
          if (emit) {
            T o = T(0);
#pragma unroll
            for (int q = 0; q < 13; ++q)
              if (q != 1 && q != 11) o += h[q] * ring[c][q];
            const int cf = c0 + c;
            if (mode == 0)
              out[base + ((int64_t)(cf * nz + k) * ny + dy) * nx + dx] = o;
            else
              out[(int64_t)dslot * L.bstride + cf * L.fstride +
                  ((int64_t)(k0 + k + L.ng) * L.P + (j0 + dy + L.ng)) * L.P + (i0 + dx + L.ng)] = o;
          }
        }
      }
    }
  }
}

// Staged ghost values (mode 0 items) into the ghost layers.
template <typename T>
__global__ __launch_bounds__(NT_GEN) void lift_scatter_kernel(const int32_t* __restrict__ items,
                                                              int64_t n, const T* __restrict__ tmp,
                                                              T* __restrict__ U, Layout L) {
  for (int64_t w = blockIdx.x; w < n; w += gridDim.x) {
    const int32_t* e = items + 12 * w;
    const int dslot = e[0], i0 = e[1], j0 = e[2], k0 = e[3], nx = e[4], ny = e[5], nz = e[6];
    const int64_t base = (int64_t)e[11] * 4;
    const int np = nx * ny * nz;
    T* dst = U + (int64_t)dslot * L.bstride;
    for (int p = threadIdx.x; p < 4 * np; p += blockDim.x) {
      const int c = p / np, q = p - c * np;
      const int dx = q % nx, dy = (q / nx) % ny, dz = q / (nx * ny);
      dst[c * L.fstride + ((int64_t)(k0 + dz + L.ng) * L.P + (j0 + dy + L.ng)) * L.P +
          (i0 + dx + L.ng)] = tmp[base + p];
    }
  }
}

static Layout lift_layout(const wacm_grid* g) {
  Layout L;
  L.P = g->P;
  L.ng = g->d.ng;
  L.fstride = (int64_t)g->P * g->P * g->P;
  L.bstride = 4 * L.fstride;
  return L;
}

static unsigned lift_grid(int64_t n) {
  const int64_t cap = 2048;
  return (unsigned)(n < cap ? (n > 0 ? n : 1) : cap);
}

// two fields per work unit: measured a little faster than one or four (the
// kernel is bound by its gathers, not by its occupancy)
template <typename T, int BS>
static hipError_t lift_box_t(const wacm_grid* g, const int32_t* items, int64_t n, T* U, T* out,
                             int mode, bool inplace, hipStream_t st) {
  constexpr int NF = 2;
  if (inplace)
    lift_box_kernel<T, BS, NF, true><<<lift_grid(n * (4 / NF)), NT_GEN, 0, st>>>(
        items, n, U, lift_layout(g), out, mode, g->d_tab, lift_slot_tab(g));
  else
    lift_box_kernel<T, BS, NF, false><<<lift_grid(n * (4 / NF)), NT_GEN, 0, st>>>(
        items, n, U, lift_layout(g), out, mode, nullptr, nullptr);
  return hipGetLastError();
}

template <typename T>
static hipError_t lift_box(const wacm_grid* g, const int32_t* items, int64_t n, T* U, T* out,
                           int mode, bool inplace, hipStream_t st) {
  switch (g->d.bs) {
    case 24:
      return lift_box_t<T, 24>(g, items, n, U, out, mode, inplace, st);
    case 32:
      return lift_box_t<T, 32>(g, items, n, U, out, mode, inplace, st);
    default:
      return hipErrorInvalidValue;  // CDF 4/4 needs ng >= 6, hence bs >= 18
  }
}

// the first n items of the list (all of them, or the face star's); inplace:
// same-level values read from the neighbours' interiors
template <typename T>
static hipError_t lift_sync_t(const wacm_grid* g, T* U, int64_t n, bool inplace, hipStream_t st) {
  if (g->n_lift < 0) return hipErrorOutOfMemory;  // the last item build failed
  if (n == 0) return hipSuccess;
  if (inplace && !lift_slot_tab(g)) return hipErrorInvalidValue;
  T* tmp = (T*)g->d_lift_tmp;
  hipError_t e = lift_box<T>(g, g->d_lift, n, U, tmp, 0, inplace, st);
  if (e != hipSuccess) return e;
  lift_scatter_kernel<T><<<lift_grid(n), NT_GEN, 0, st>>>(g->d_lift, n, tmp, U, lift_layout(g));
  return hipGetLastError();
}

hipError_t launch_lift_sync(const wacm_grid* g, void* U, hipStream_t st) {
  return g->d.dtype == WACM_F64 ? lift_sync_t(g, (double*)U, g->n_lift, false, st)
                                : lift_sync_t(g, (float*)U, g->n_lift, false, st);
}

hipError_t launch_lift_sync_face(const wacm_grid* g, void* U, hipStream_t st) {
  return g->d.dtype == WACM_F64 ? lift_sync_t(g, (double*)U, g->n_lift_face, true, st)
                                : lift_sync_t(g, (float*)U, g->n_lift_face, true, st);
}

hipError_t launch_lift_coarsen(const wacm_grid* g, void* U, int64_t nparents, hipStream_t st) {
  if (nparents == 0) return hipSuccess;
  return g->d.dtype == WACM_F64
             ? lift_box<double>(g, g->d_list, 8 * nparents, (double*)U, (double*)U, 1, false, st)
             : lift_box<float>(g, g->d_list, 8 * nparents, (float*)U, (float*)U, 1, false, st);
}

// --------------------------------------------------------------------------
// Classical RK4 with CDF 4/4 ghosts.  The CDF 4/0 step reads same-level
// halos in place and fills face halos next to other levels itself; with the
// lifted restriction each stage input's ghost layers are filled first (the
// CDF 4/0 values of the regions in a coarser leaf and of the boxes the
// face-star lifted values read from finer leaves' padded arrays; then the
// lifted phase of the face star), and the fused stage kernel reads
// same-level halos in place and the others from those ghost layers: per
// stage a fill and one stage kernel, with the CDF 4/0 step's register
// arrangement (Y2/Y4, Y3 and W) in `work`, Y2/Y4 and Y3 in the padded pool
// layout, W compact.
// --------------------------------------------------------------------------
struct LiftWork {
  size_t y, k, a, total;
};
static LiftWork lift_work(const wacm_grid* g) {
  const size_t es = g->d.dtype == WACM_F64 ? 8 : 4;
  const size_t reg = (size_t)g->d.capacity * 4 * (size_t)g->P * g->P * g->P * es;
  const size_t up = (reg + 255) / 256 * 256;
  return LiftWork{0, up, 2 * up, 3 * up};
}

size_t lift_work_bytes(const wacm_grid* g) { return lift_work(g).total; }

__global__ void lift_advance_time(double* t_dev, const double* dt_dev) {
  if (threadIdx.x == 0) t_dev[0] += dt_dev[0];
}

template <typename T>
static hipError_t rk4_lifted_t(const wacm_grid* g, const wacm_params* p, double* t_dev,
                               double* dt_dev, T* U, void* work, const void* dus, int dt_mode,
                               int64_t nsteps, hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  const LiftWork wp = lift_work(g);
  T* Ya = (T*)((char*)work + wp.y);  // Y2, then Y4
  T* Yb = (T*)((char*)work + wp.k);  // Y3
  T* Wr = (T*)((char*)work + wp.a);  // W = (U^n + Y2)/3 + dt/3 k2, compact layout
  hipError_t e;
  // per stage: the CDF 4/0 fill of the input's ghosts that the stage and the
  // face-star lifted values read, the lifted values of the face star, then
  // the fused stage (same-level halos in place, the others from the ghost
  // layers); t and dt stay on the device
  auto stage = [&](int s, T* in, T* out) {
    hipError_t r = launch_sync_lifted_stage(g, in, g->d_lift_mask, st);
    if (r == hipSuccess) r = launch_lift_sync_face(g, in, st);
    if (r == hipSuccess) r = launch_stage_owng(g, p, s, t_dev, dt_dev, in, U, out, Wr, dus, st);
    return r;
  };
  for (int64_t n = 0; n < nsteps; ++n) {
    if (dt_mode == WACM_DT_CFL && (e = launch_dt(g, p, U, dt_dev, st)) != hipSuccess) return e;
    if ((e = stage(1, U, Ya)) != hipSuccess || (e = stage(2, Ya, Yb)) != hipSuccess ||
        (e = stage(3, Yb, Ya)) != hipSuccess || (e = stage(4, Ya, U)) != hipSuccess)
      return e;
    lift_advance_time<<<1, 64, 0, st>>>(t_dev, dt_dev);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_rk4_lifted(const wacm_grid* g, const wacm_params* p, double* t_dev,
                             double* dt_dev, void* U, void* work, const void* dus, int dt_mode,
                             int64_t nsteps, hipStream_t st) {
  return g->d.dtype == WACM_F64
             ? rk4_lifted_t(g, p, t_dev, dt_dev, (double*)U, work, dus, dt_mode, nsteps, st)
             : rk4_lifted_t(g, p, t_dev, dt_dev, (float*)U, work, dus, dt_mode, nsteps, st);
}

}  // namespace wacm
