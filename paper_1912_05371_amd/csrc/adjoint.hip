// Discrete adjoint of the hot path on a frozen grid with a fixed time step:
// transposes of the ghost synchronisation (Sec. 4.2 / 3.1), of the linearised
// penalized ACM right-hand side (Sec. 2.2-2.3) and of one classical RK4 step,
// plus the gradient of the x-component of the penalization force (Sec. 2.2).
// Parameters: theta = (amp, freq, phase) of the plate pitch and a static
// extra solid velocity dus.  Every reduction runs in a fixed order, so the
// results are bitwise reproducible.
#include <algorithm>
#include <tuple>

#include "resolve.h"
#include "wacm_internal.h"

namespace wacm {

// --------------------------------------------------------------------------
// transpose of the ghost fill: CSR gather plan built on the host
// --------------------------------------------------------------------------
void free_adj_plans(wacm_grid* g) {
  g->plan[0] = AdjPlan{};
  g->plan[1] = AdjPlan{};
}

// Every ghost point of the set (0: all ng layers, 1: depth-3 face star) of
// every active block, with the interior points its value was taken from:
// rows are the source interior points, entries the ghost points that read
// them with their prediction weights, sorted so the gather is deterministic.
// Host part only (kept until the grid changes); upload_adj_plan copies it
// into the caller's buffer.
int build_adj_plan(wacm_grid* g, int face_only, std::string& err) {
  AdjPlan& pl = g->plan[face_only ? 1 : 0];
  if (pl.built || !pl.h_ptr.empty()) return WACM_OK;
  (void)err;
  const int bs = g->d.bs, ng = g->d.ng, P = g->P;
  Layout L;
  L.P = P;
  L.ng = ng;
  L.fstride = (int64_t)P * P * P;
  L.bstride = 4 * L.fstride;
  const int npts = face_only ? 18 * bs * bs : P * P * P - bs * bs * bs;
  std::vector<std::tuple<int64_t, int64_t, double>> ent;
  std::vector<int64_t> ghosts;
  ghosts.reserve((size_t)g->nb * npts);
  ent.reserve((size_t)g->nb * npts * 2);
  for (int64_t ib = 0; ib < g->nb; ++ib) {
    const Tab& t = g->h_tab[ib];
    const int64_t base = (int64_t)t.meta[0] * L.bstride;
    for (int p = 0; p < npts; ++p) {
      int i, j, k;
      shell_point(p, bs, ng, P, face_only ? 1 : 0, i, j, k);
      const int64_t go = base + ((int64_t)(k + ng) * P + (j + ng)) * P + (i + ng);
      ghosts.push_back(go);
      ghost_taps<double>(t, bs, L, i, j, k,
                         [&](int64_t off, double w) { ent.emplace_back(off, go, w); });
    }
  }
  std::sort(ent.begin(), ent.end());
  AdjPlan np;
  np.h_src.reserve(ent.size());
  np.h_w.reserve(ent.size());
  for (size_t e = 0; e < ent.size(); ++e) {
    if (e == 0 || std::get<0>(ent[e]) != std::get<0>(ent[e - 1])) {
      np.h_dst.push_back(std::get<0>(ent[e]));
      np.h_ptr.push_back((int64_t)e);
    }
    np.h_src.push_back(std::get<1>(ent[e]));
    np.h_w.push_back(std::get<2>(ent[e]));
  }
  np.h_ptr.push_back((int64_t)ent.size());
  np.h_ghost.swap(ghosts);
  np.nrows = (int64_t)np.h_dst.size();
  np.nnz = (int64_t)np.h_src.size();
  np.nghost = (int64_t)np.h_ghost.size();
  pl = std::move(np);
  return WACM_OK;
}

static size_t up256(size_t v) { return (v + 255) / 256 * 256; }

// device bytes of a plan: dst, ptr, src, w, ghost, each 256-byte aligned
size_t adj_plan_bytes(const AdjPlan& p) {
  return up256(8 * p.h_dst.size()) + up256(8 * p.h_ptr.size()) + up256(8 * p.h_src.size()) +
         up256(8 * p.h_w.size()) + up256(8 * p.h_ghost.size());
}

int upload_adj_plan(wacm_grid* g, int face_only, void* ws, size_t bytes, std::string& err) {
  AdjPlan& pl = g->plan[face_only ? 1 : 0];
  if (int rc = build_adj_plan(g, face_only, err)) return rc;
  if (bytes < adj_plan_bytes(pl)) {
    err = "adjoint plan buffer smaller than wacm_adj_plan_bytes()";
    return WACM_E_INVAL;
  }
  char* w = (char*)ws;
  hipError_t e = hipSuccess;
  auto put = [&](auto** d, const auto& v) {
    using E = typename std::remove_reference<decltype(v)>::type::value_type;
    *d = reinterpret_cast<E*>(w);
    if (e == hipSuccess && !v.empty())
      e = hipMemcpy(w, v.data(), sizeof(E) * v.size(), hipMemcpyHostToDevice);
    w += up256(sizeof(E) * v.size());
  };
  put(&pl.d_dst, pl.h_dst);
  put(&pl.d_ptr, pl.h_ptr);
  put(&pl.d_src, pl.h_src);
  put(&pl.d_w, pl.h_w);
  put(&pl.d_ghost, pl.h_ghost);
  if (e != hipSuccess) {
    pl.built = 0;
    err = std::string("adjoint plan upload: ") + hipGetErrorString(e);
    return WACM_E_HIP;
  }
  pl.built = 1;
  return WACM_OK;
}

template <typename T>
__global__ __launch_bounds__(NT_GEN) void sync_adj_gather(const int64_t* __restrict__ dst,
                                                          const int64_t* __restrict__ ptr,
                                                          const int64_t* __restrict__ src,
                                                          const double* __restrict__ w,
                                                          int64_t nrows, T* __restrict__ U,
                                                          int64_t fs) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < nrows;
       r += (int64_t)gridDim.x * blockDim.x) {
    double acc[4] = {0, 0, 0, 0};
    for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) {
      const double we = w[e];
#pragma unroll
      for (int c = 0; c < 4; ++c) acc[c] += we * (double)U[src[e] + c * fs];
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) U[dst[r] + c * fs] += T(acc[c]);
  }
}

template <typename T>
__global__ __launch_bounds__(NT_GEN) void zero_points(const int64_t* __restrict__ idx, int64_t n,
                                                      T* __restrict__ U, int64_t fs) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 4; ++c) U[idx[r] + c * fs] = T(0);
  }
}

// --------------------------------------------------------------------------
// transpose of the linearised rhs, gather form within each block
// --------------------------------------------------------------------------
// For a point j of the block (interior, or face star of depth 3), with v the
// rhs adjoint (zero outside the interior) and u the synchronised state:
//   Ubar_c += sum_d D1_d[v_c u_d] + nu sum_d D2_d[v_c] + C0^2 D1_c[v_p]
//             - [j interior] (sum_c' v_c' D1_c u_c' + chi/C_eta v_c + sponge)
//   Ubar_p += sum_d D1_d[v_d] - [j interior] (C_gamma + sponge) v_p
// (D1, D2 the forward stencils applied to fields that vanish outside the
// interior: the transpose of the antisymmetric D1 moves its sign into the
// convective and gradient terms).
template <typename T>
struct AdjArgs {
  const Tab* tab;
  int64_t nb;
  const T* U;
  const T* V;
  T* Ub;
  Layout L;
  int bs;
  double Ldom;
  double t;
  wacm_params p;
  const T* dus;    // [slot][3][bs^3] or null
  double* dusbar;  // [slot][3][bs^3] or null (accumulated, FP64)
  double* part;    // per-block theta partials [nb][3]
  double weight;   // force adjoint weight
};

template <typename T>
__global__ __launch_bounds__(NT_GEN) void rhs_adj_kernel(AdjArgs<T> a) {
  __shared__ double red[3][NT_GEN];
  const int bs = a.bs, ng = a.L.ng, P = a.L.P;
  const int64_t fs = a.L.fstride;
  const int n3 = bs * bs * bs, nf = 18 * bs * bs;
  const double tw[3] = {TW1, TW2, TW3};
  const double w2[5] = {D2A, D2B, D2C, D2B, D2A};
  const wacm_params& p = a.p;
  for (int64_t ib = blockIdx.x; ib < a.nb; ib += gridDim.x) {
    const int32_t* m = a.tab[ib].meta;
    const int slot = m[0], J = m[1];
    const double h = a.Ldom / (double(int64_t(1) << J) * bs);
    const T ih = T(1.0 / h), ih2 = T(1.0 / (h * h));
    const int64_t base = (int64_t)slot * a.L.bstride;
    const T* U = a.U + base;
    const T* V = a.V + base;
    T* B = a.Ub + base;
    auto idx = [&](int i, int j, int k) -> int64_t {
      return ((int64_t)(k + ng) * P + (j + ng)) * P + (i + ng);
    };
    auto inside = [&](int i, int j, int k) {
      return i >= 0 && i < bs && j >= 0 && j < bs && k >= 0 && k < bs;
    };
    double th[3] = {0, 0, 0};
    for (int pt = threadIdx.x; pt < n3 + nf; pt += blockDim.x) {
      int q[3];
      if (pt < n3) {
        q[0] = pt % bs;
        q[1] = (pt / bs) % bs;
        q[2] = pt / (bs * bs);
      } else {
        shell_point(pt - n3, bs, ng, P, 1, q[0], q[1], q[2]);
      }
      const bool in = pt < n3;
      T acc[4] = {T(0), T(0), T(0), T(0)};
      for (int d = 0; d < 3; ++d) {
        for (int mm = 1; mm <= 3; ++mm) {
          int qp[3] = {q[0], q[1], q[2]}, qm[3] = {q[0], q[1], q[2]};
          qp[d] += mm;
          qm[d] -= mm;
          const bool ip = inside(qp[0], qp[1], qp[2]), im = inside(qm[0], qm[1], qm[2]);
          T vp[4] = {T(0), T(0), T(0), T(0)}, vm[4] = {T(0), T(0), T(0), T(0)};
          T up = T(0), um = T(0);
          if (ip) {
            const int64_t o = idx(qp[0], qp[1], qp[2]);
            for (int c = 0; c < 4; ++c) vp[c] = V[o + c * fs];
            up = U[o + d * fs];
          }
          if (im) {
            const int64_t o = idx(qm[0], qm[1], qm[2]);
            for (int c = 0; c < 4; ++c) vm[c] = V[o + c * fs];
            um = U[o + d * fs];
          }
          const T am = T(tw[mm - 1]) * ih;
          for (int c = 0; c < 3; ++c) acc[c] += am * (vp[c] * up - vm[c] * um);
          acc[d] += T(p.c0 * p.c0) * am * (vp[3] - vm[3]);
          acc[3] += am * (vp[d] - vm[d]);
        }
        for (int o = -2; o <= 2; ++o) {
          int qo[3] = {q[0], q[1], q[2]};
          qo[d] += o;
          if (!inside(qo[0], qo[1], qo[2])) continue;
          const int64_t oo = idx(qo[0], qo[1], qo[2]);
          const T wgt = T(p.nu * w2[o + 2]) * ih2;
          for (int c = 0; c < 3; ++c) acc[c] += wgt * V[oo + c * fs];
        }
      }
      const int64_t oj = idx(q[0], q[1], q[2]);
      if (in) {
        T v[4], u[4];
        for (int c = 0; c < 4; ++c) {
          v[c] = V[oj + c * fs];
          u[c] = U[oj + c * fs];
        }
        // pointwise: - sum_c' v_c' D1_c u_c'
        for (int c = 0; c < 3; ++c) {
          const int64_t st = c == 0 ? 1 : (c == 1 ? P : (int64_t)P * P);
          for (int c2 = 0; c2 < 3; ++c2) {
            const T* f = U + c2 * fs;
            const T d1 = (T(TW1) * (f[oj + st] - f[oj - st]) +
                          T(TW2) * (f[oj + 2 * st] - f[oj - 2 * st]) +
                          T(TW3) * (f[oj + 3 * st] - f[oj - 3 * st])) *
                         ih;
            acc[c] -= v[c2] * d1;
          }
        }
        acc[3] -= T(p.c_gamma) * v[3];
        const double xg = (double)(m[2] * bs + q[0]) * h, yg = (double)(m[3] * bs + q[1]) * h,
                     zg = (double)(m[4] * bs + q[2]) * h;
        if (p.sponge) {
          const T sp = T(sponge_eval(p, a.Ldom, xg, yg, zg) / p.c_sp);
          for (int c = 0; c < 4; ++c) acc[c] -= sp * v[c];
        }
        if (p.mask) {
          const int qi = (q[2] * bs + q[1]) * bs + q[0];
          double chi, dchi = 0.0, us[3], dsd[3] = {0, 0, 0}, dal[3] = {0, 0, 0},
                      dad[3] = {0, 0, 0};
          if (p.mask == WACM_MASK_PLATE)
            plate_eval_adj(p, a.t, xg, yg, zg, chi, dchi, us, dsd, dal, dad);
          else
            mask_eval(p, a.t, xg, yg, zg, chi, us);
          double gal = 0.0, gad = 0.0;
          for (int c = 0; c < 3; ++c) {
            acc[c] -= T(chi / p.c_eta) * v[c];
            if (a.dusbar)
              a.dusbar[((int64_t)slot * 3 + c) * n3 + qi] += chi / p.c_eta * (double)v[c];
            const double e = a.dus ? (double)a.dus[((int64_t)slot * 3 + c) * n3 + qi] : 0.0;
            gal += -dchi / p.c_eta * ((double)u[c] - us[c] - e) * (double)v[c];
            gad += chi / p.c_eta * dsd[c] * (double)v[c];
          }
          for (int k2 = 0; k2 < 3; ++k2) th[k2] += gal * dal[k2] + gad * dad[k2];
        }
      }
      for (int c = 0; c < 4; ++c) B[oj + c * fs] += acc[c];
    }
    __syncthreads();
    for (int k2 = 0; k2 < 3; ++k2) red[k2][threadIdx.x] = th[k2];
    __syncthreads();
    for (int s = NT_GEN / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s)
        for (int k2 = 0; k2 < 3; ++k2) red[k2][threadIdx.x] += red[k2][threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0)
      for (int k2 = 0; k2 < 3; ++k2) a.part[ib * 3 + k2] = red[k2][0];
  }
}

// Gradient of weight * F_x (the x-force, Sec. 2.2 midpoint rule) at time t.
template <typename T>
__global__ __launch_bounds__(NT_GEN) void force_adj_kernel(AdjArgs<T> a) {
  __shared__ double red[3][NT_GEN];
  const int bs = a.bs, ng = a.L.ng, P = a.L.P;
  const int n3 = bs * bs * bs;
  const wacm_params& p = a.p;
  for (int64_t ib = blockIdx.x; ib < a.nb; ib += gridDim.x) {
    const int32_t* m = a.tab[ib].meta;
    const int slot = m[0], J = m[1];
    const double h = a.Ldom / (double(int64_t(1) << J) * bs);
    const double vol = h * h * h;
    const int64_t base = (int64_t)slot * a.L.bstride;
    double th[3] = {0, 0, 0};
    for (int qi = threadIdx.x; qi < n3; qi += blockDim.x) {
      const int i = qi % bs, j = (qi / bs) % bs, k = qi / (bs * bs);
      const int64_t o = base + ((int64_t)(k + ng) * P + (j + ng)) * P + (i + ng);
      const double xg = (double)(m[2] * bs + i) * h, yg = (double)(m[3] * bs + j) * h,
                   zg = (double)(m[4] * bs + k) * h;
      double chi, dchi = 0.0, us[3], dsd[3] = {0, 0, 0}, dal[3] = {0, 0, 0}, dad[3] = {0, 0, 0};
      if (p.mask == WACM_MASK_PLATE)
        plate_eval_adj(p, a.t, xg, yg, zg, chi, dchi, us, dsd, dal, dad);
      else
        mask_eval(p, a.t, xg, yg, zg, chi, us);
      const double cw = a.weight * chi * vol / p.c_eta;
      a.Ub[o] += T(cw);
      if (a.dusbar) a.dusbar[((int64_t)slot * 3) * n3 + qi] -= cw;
      const double e = a.dus ? (double)a.dus[((int64_t)slot * 3) * n3 + qi] : 0.0;
      const double gal = a.weight * dchi * ((double)a.U[o] - us[0] - e) * vol / p.c_eta;
      const double gad = -cw * dsd[0];
      for (int k2 = 0; k2 < 3; ++k2) th[k2] += gal * dal[k2] + gad * dad[k2];
    }
    __syncthreads();
    for (int k2 = 0; k2 < 3; ++k2) red[k2][threadIdx.x] = th[k2];
    __syncthreads();
    for (int s = NT_GEN / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s)
        for (int k2 = 0; k2 < 3; ++k2) red[k2][threadIdx.x] += red[k2][threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0)
      for (int k2 = 0; k2 < 3; ++k2) a.part[ib * 3 + k2] = red[k2][0];
  }
}

// dtheta += sum over blocks of the partials (fixed order)
__global__ __launch_bounds__(NT_GEN) void theta_finalize(const double* __restrict__ part,
                                                         int64_t nb, double* __restrict__ dtheta) {
  __shared__ double red[3][NT_GEN];
  double s[3] = {0, 0, 0};
  for (int64_t q = threadIdx.x; q < nb; q += blockDim.x)
    for (int k = 0; k < 3; ++k) s[k] += part[q * 3 + k];
  for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int st = NT_GEN / 2; st > 0; st >>= 1) {
    if ((int)threadIdx.x < st)
      for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + st];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int k = 0; k < 3; ++k) dtheta[k] += red[k][0];
}

// --------------------------------------------------------------------------
// elementwise helpers on pool-layout registers
// --------------------------------------------------------------------------
// Y = a X + b Z on the interior points of every active block (X, Z may be null)
template <typename T>
__global__ __launch_bounds__(NT_GEN) void axpby_interior(const Tab* __restrict__ tab, int64_t nb,
                                                         Layout L, int bs, T* Y, double a,
                                                         const T* X, double b, const T* Z) {
  const int n3 = bs * bs * bs;
  for (int64_t ib = blockIdx.x; ib < nb; ib += gridDim.x) {
    const int64_t base = (int64_t)tab[ib].meta[0] * L.bstride;
    for (int q = threadIdx.x; q < 4 * n3; q += blockDim.x) {
      const int c = q / n3, r = q - c * n3;
      const int i = r % bs, j = (r / bs) % bs, k = r / (bs * bs);
      const int64_t o = base + c * L.fstride + ((int64_t)(k + L.ng) * L.P + (j + L.ng)) * L.P +
                        (i + L.ng);
      T v = T(0);
      if (X) v += T(a) * X[o];
      if (Z) v += T(b) * Z[o];
      Y[o] = v;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(NT_GEN) void fill_zero(T* Y, int64_t n) {
  for (int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; r < n;
       r += (int64_t)gridDim.x * blockDim.x)
    Y[r] = T(0);
}

// --------------------------------------------------------------------------
// launchers
// --------------------------------------------------------------------------
static Layout pool_L(const wacm_grid* g) {
  Layout L;
  L.P = g->P;
  L.ng = g->d.ng;
  L.fstride = (int64_t)g->P * g->P * g->P;
  L.bstride = 4 * L.fstride;
  return L;
}

static unsigned grid_n(int64_t n) {
  int64_t cap = 2048;
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>(n, cap));
}

size_t adj_work_bytes(const wacm_grid* g) {
  const size_t es = g->d.dtype == WACM_F64 ? 8 : 4;
  const size_t reg = (size_t)g->d.capacity * 4 * g->P * g->P * g->P * es;
  return 8 * ((reg + 255) / 256 * 256);
}

template <typename T>
static hipError_t sync_adj_t(const wacm_grid* g, T* Ub, int face_only, hipStream_t st) {
  const AdjPlan& pl = g->plan[face_only ? 1 : 0];
  const int64_t fs = (int64_t)g->P * g->P * g->P;
  if (pl.nrows > 0)
    sync_adj_gather<T><<<grid_n((pl.nrows + NT_GEN - 1) / NT_GEN), NT_GEN, 0, st>>>(
        pl.d_dst, pl.d_ptr, pl.d_src, pl.d_w, pl.nrows, Ub, fs);
  if (pl.nghost > 0)
    zero_points<T><<<grid_n((pl.nghost + NT_GEN - 1) / NT_GEN), NT_GEN, 0, st>>>(
        pl.d_ghost, pl.nghost, Ub, fs);
  return hipGetLastError();
}

hipError_t launch_sync_adj(const wacm_grid* g, void* Ub, int face_only, hipStream_t st) {
  return g->d.dtype == WACM_F64 ? sync_adj_t(g, (double*)Ub, face_only, st)
                                : sync_adj_t(g, (float*)Ub, face_only, st);
}

template <typename T>
static AdjArgs<T> adj_args(const wacm_grid* g, const wacm_params* p, double t, const T* U,
                           const T* V, T* Ub, double* dusbar, const T* dus) {
  AdjArgs<T> a{};
  a.tab = g->d_tab;
  a.nb = g->nb;
  a.U = U;
  a.V = V;
  a.Ub = Ub;
  a.L = pool_L(g);
  a.bs = g->d.bs;
  a.Ldom = g->d.L;
  a.t = t;
  a.p = *p;
  a.dus = dus;
  a.dusbar = dusbar;
  a.part = g->d_part;
  return a;
}

template <typename T>
static hipError_t rhs_adj_t(const wacm_grid* g, const wacm_params* p, double t, const T* U,
                            const T* V, T* Ub, double* dtheta, double* dusbar, const T* dus,
                            hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  AdjArgs<T> a = adj_args<T>(g, p, t, U, V, Ub, dusbar, dus);
  rhs_adj_kernel<T><<<grid_n(g->nb), NT_GEN, 0, st>>>(a);
  theta_finalize<<<1, NT_GEN, 0, st>>>(g->d_part, g->nb, dtheta);
  return hipGetLastError();
}

hipError_t launch_rhs_adj(const wacm_grid* g, const wacm_params* p, double t, const void* U,
                          const void* V, void* Ub, double* dtheta, double* dusbar,
                          const void* dus, hipStream_t st) {
  return g->d.dtype == WACM_F64
             ? rhs_adj_t(g, p, t, (const double*)U, (const double*)V, (double*)Ub, dtheta,
                         dusbar, (const double*)dus, st)
             : rhs_adj_t(g, p, t, (const float*)U, (const float*)V, (float*)Ub, dtheta, dusbar,
                         (const float*)dus, st);
}

template <typename T>
static hipError_t force_adj_t(const wacm_grid* g, const wacm_params* p, double t, double weight,
                              const T* U, T* Ub, double* dtheta, double* dusbar, const T* dus,
                              hipStream_t st) {
  if (g->nb == 0 || !p->mask) return hipSuccess;
  AdjArgs<T> a = adj_args<T>(g, p, t, U, nullptr, Ub, dusbar, dus);
  a.weight = weight;
  force_adj_kernel<T><<<grid_n(g->nb), NT_GEN, 0, st>>>(a);
  theta_finalize<<<1, NT_GEN, 0, st>>>(g->d_part, g->nb, dtheta);
  return hipGetLastError();
}

hipError_t launch_force_adj(const wacm_grid* g, const wacm_params* p, double t, double weight,
                            const void* U, void* Ub, double* dtheta, double* dusbar,
                            const void* dus, hipStream_t st) {
  return g->d.dtype == WACM_F64
             ? force_adj_t(g, p, t, weight, (const double*)U, (double*)Ub, dtheta, dusbar,
                           (const double*)dus, st)
             : force_adj_t(g, p, t, weight, (const float*)U, (float*)Ub, dtheta, dusbar,
                           (const float*)dus, st);
}

// One RK4 step backwards: recompute the synchronised stage inputs from the
// checkpoint Un, then sweep the stages in reverse:
//   kb_4 = dt/6 lam, kb_3 = dt/3 lam + dt B_4, kb_2 = dt/3 lam + dt/2 B_3,
//   kb_1 = dt/6 lam + dt/2 B_2, with B_s = S^T J_rhs(U_s)^T kb_s, and
//   lam_n = lam + B_4 + B_3 + B_2 + B_1.
template <typename T>
static hipError_t rk4_adj_t(const wacm_grid* g, const wacm_params* p, double t, double dt,
                            const T* Un, T* lam, double* dtheta, double* dusbar, const T* dus,
                            void* work, hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  const Layout L = pool_L(g);
  const size_t reg = ((size_t)g->d.capacity * L.bstride * sizeof(T) + 255) / 256 * 256;
  char* w = (char*)work;
  T* S[4];
  for (int s = 0; s < 4; ++s) S[s] = (T*)(w + s * reg);
  T* K = (T*)(w + 4 * reg);
  T* kb = (T*)(w + 5 * reg);
  T* B = (T*)(w + 6 * reg);
  T* lamU = (T*)(w + 7 * reg);
  const int64_t nall = (int64_t)g->d.capacity * L.bstride;
  const unsigned gb = grid_n(g->nb);
  const int bs = g->d.bs;
  hipError_t e;
  const double cs[4] = {0.0, 0.5, 0.5, 1.0};
  // forward recompute
  axpby_interior<T><<<gb, NT_GEN, 0, st>>>(g->d_tab, g->nb, L, bs, S[0], 1.0, Un, 0.0, nullptr);
  if ((e = launch_sync(g, S[0], 1, st)) != hipSuccess) return e;
  for (int s = 1; s < 4; ++s) {
    if ((e = launch_rhs(g, p, t + cs[s - 1] * dt, S[s - 1], K, dus, st)) != hipSuccess) return e;
    axpby_interior<T><<<gb, NT_GEN, 0, st>>>(g->d_tab, g->nb, L, bs, S[s], 1.0, Un, cs[s] * dt,
                                             K);
    if ((e = launch_sync(g, S[s], 1, st)) != hipSuccess) return e;
  }
  // reverse sweep
  axpby_interior<T><<<gb, NT_GEN, 0, st>>>(g->d_tab, g->nb, L, bs, lamU, 1.0, lam, 0.0, nullptr);
  axpby_interior<T><<<gb, NT_GEN, 0, st>>>(g->d_tab, g->nb, L, bs, kb, dt / 6.0, lam, 0.0,
                                           nullptr);
  const double lamw[4] = {dt / 6.0, dt / 3.0, dt / 3.0, dt / 6.0};
  for (int s = 3; s >= 0; --s) {
    fill_zero<T><<<grid_n((nall + NT_GEN - 1) / NT_GEN), NT_GEN, 0, st>>>(B, nall);
    if ((e = rhs_adj_t<T>(g, p, t + cs[s] * dt, S[s], kb, B, dtheta, dusbar, dus, st)) !=
        hipSuccess)
      return e;
    if ((e = sync_adj_t<T>(g, B, 1, st)) != hipSuccess) return e;
    axpby_interior<T><<<gb, NT_GEN, 0, st>>>(g->d_tab, g->nb, L, bs, lamU, 1.0, lamU, 1.0, B);
    if (s > 0)
      axpby_interior<T><<<gb, NT_GEN, 0, st>>>(g->d_tab, g->nb, L, bs, kb, lamw[s - 1], lam,
                                               cs[s] * dt, B);
  }
  axpby_interior<T><<<gb, NT_GEN, 0, st>>>(g->d_tab, g->nb, L, bs, lam, 1.0, lamU, 0.0, nullptr);
  return hipGetLastError();
}

hipError_t launch_rk4_adj(const wacm_grid* g, const wacm_params* p, double t, double dt,
                          const void* Un, void* lam, double* dtheta, double* dusbar,
                          const void* dus, void* work, hipStream_t st) {
  return g->d.dtype == WACM_F64
             ? rk4_adj_t(g, p, t, dt, (const double*)Un, (double*)lam, dtheta, dusbar,
                         (const double*)dus, work, st)
             : rk4_adj_t(g, p, t, dt, (const float*)Un, (float*)lam, dtheta, dusbar,
                         (const float*)dus, work, st);
}

}  // namespace wacm
