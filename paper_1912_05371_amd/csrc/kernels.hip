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
// |u|^2 in FP64 with one fixed operation order: the maximum fused into the
// last RK4 stage and the stand-alone reduction agree bit for bit.
__device__ __forceinline__ double speed2(double u, double v, double w) {
  return __builtin_fma(w, w, __builtin_fma(v, v, u * u));
}
template <typename T>
__device__ __forceinline__ T wave_min(T v) {
  for (int o = 32; o > 0; o >>= 1) v = fmin(v, __shfl_xor(v, o, 64));
  return v;
}

// --------------------------------------------------------------------------
// ghost synchronisation
// --------------------------------------------------------------------------
// Point-wise ghost fill: mode 0 every ghost point of all ng layers, mode 1 the
// depth-3 face star (the points the rhs stencils read).  With skip_coarser,
// points of regions that lie in a coarser leaf are left to
// sync_coarser_kernel.  With `box` (the lifted step's read boxes,
// LIFT_BOX_WORDS per block; mode 0): only the points inside the boxes of
// regions in a finer leaf (the lifted phase reads same-level ones from the
// neighbours' interiors), and the face star of regions in a coarser leaf
// unless those are skipped; the rest of the face star is read in place (same
// level) or overwritten by the lifted phase (finer leaf).  A block without
// such boxes visits its face star alone, or nothing.
template <typename T>
__global__ __launch_bounds__(NT_GEN) void sync_kernel(const Tab* __restrict__ tab, int64_t nb,
                                                      T* __restrict__ U, Layout L, int bs,
                                                      int mode, int skip_coarser,
                                                      const int32_t* __restrict__ box) {
  __shared__ Tab st;
  __shared__ int32_t sbox[LIFT_BOX_WORDS];
  for (int64_t ib = blockIdx.x; ib < nb; ib += gridDim.x) {
    __syncthreads();
    load_tab(tab + ib, st);
    if (box && threadIdx.x < LIFT_BOX_WORDS)
      sbox[threadIdx.x] = box[ib * LIFT_BOX_WORDS + threadIdx.x];
    __syncthreads();
    T* dst = U + (int64_t)st.meta[0] * L.bstride;
    int32_t have = 0;  // boxes of regions in a finer leaf (uniform)
    if (box)
      for (int r = 0; r < 27; ++r)
        if (r != 13 && st.kind[r] > 0) have |= sbox[13] & (int32_t(1) << r);
    if (box && have == 0 && skip_coarser) continue;
    const int md = box && have == 0 ? 1 : mode;
    const int npts = md == 1 ? 18 * bs * bs : L.P * L.P * L.P - bs * bs * bs;
    for (int p = threadIdx.x; p < npts; p += blockDim.x) {
      int i, j, k;
      shell_point(p, bs, L.ng, L.P, md, i, j, k);
      const int r = region_of(i, bs) + 3 * region_of(j, bs) + 9 * region_of(k, bs);
      if (skip_coarser && st.kind[r] < 0) continue;
      if (box) {
        bool in = false;
        if ((have >> r) & 1) {
          const int32_t b = sbox[r];
          const int q[3] = {i, j, k};
          in = true;
#pragma unroll
          for (int d = 0; d < 3; ++d) {
            const int o = q[d] - (q[d] < 0 ? -L.ng : (q[d] < bs ? 0 : bs));
            in = in && o >= ((b >> (10 * d)) & 31) && o <= ((b >> (10 * d + 5)) & 31);
          }
        }
        if (!in) {
          const int out = (i < 0 || i >= bs) + (j < 0 || j >= bs) + (k < 0 || k >= bs);
          if (st.kind[r] >= 0 || out != 1 || i < -3 || i >= bs + 3 || j < -3 || j >= bs + 3 ||
              k < -3 || k >= bs + 3)
            continue;
        }
      }
      T v[4];
      ghost_value<T>(st, bs, L, U, i, j, k, v);
      const int64_t o = ((int64_t)(k + L.ng) * L.P + (j + L.ng)) * L.P + (i + L.ng);
#pragma unroll
      for (int c = 0; c < 4; ++c) dst[o + c * L.fstride] = v[c];
    }
  }
}

// Ghost points of the even lattice within 3 of the block: (i, j, k) all even
// in [-2, bs+2]^3 outside the interior, the points the wavelet details read
// (detail_kernel).  Each is a copy: an even point is a lattice point of a
// coarser leaf and coincides with a point of a finer one (Sec. 3.1), and
// every source is an interior point of its leaf, so no write is read.
template <typename T, int BS>
__global__ __launch_bounds__(NT_GEN) void sync_lattice_kernel(const Tab* __restrict__ tab,
                                                              int64_t nb, T* __restrict__ U,
                                                              Layout L) {
  constexpr int S = BS / 2 + 3, S3 = S * S * S;  // even positions -2, 0, ..., bs+2
  __shared__ Tab st;
  for (int64_t ib = blockIdx.x; ib < nb; ib += gridDim.x) {
    __syncthreads();
    load_tab(tab + ib, st);
    __syncthreads();
    T* dst = U + (int64_t)st.meta[0] * L.bstride;
    for (int q = threadIdx.x; q < S3; q += NT_GEN) {
      const int a = q % S, b = (q / S) % S, c = q / (S * S);
      const int i = 2 * a - 2, j = 2 * b - 2, k = 2 * c - 2;
      if (i >= 0 && i < BS && j >= 0 && j < BS && k >= 0 && k < BS) continue;
      const int64_t so = point_offset(st, BS, L, i, j, k);
      const int64_t o = ((int64_t)(k + L.ng) * L.P + (j + L.ng)) * L.P + (i + L.ng);
      T v[4];
#pragma unroll
      for (int f = 0; f < 4; ++f) v[f] = U[so + f * L.fstride];
#pragma unroll
      for (int f = 0; f < 4; ++f) dst[o + f * L.fstride] = v[f];
    }
  }
}

// Ghost regions that lie in a coarser leaf (Sec. 3.1 prediction, Sec. 4.2):
// one work item per (block, region).  The region's box of ghost points is
// predicted separably: the even lattice box around it (read from whichever
// leaves hold it) is gathered for all 4 fields at once into registers, then,
// one field at a time through LDS, predicted along x, y and z and written.
// The same tensor-product DD4 values as the point-wise fill, summed in
// another order.  Requires ng <= SC_MAXG (checked by the launcher).
constexpr int SC_MAXG = 6;
template <int BS>
struct SyncCoarseDims {
  static constexpr int S = BS / 2 + 3;       // lattice points along an interior axis
  static constexpr int MG = SC_MAXG;         // lattice points along a ghost axis, ng <= 6
  static constexpr int NSRC = MG * S * S;    // largest lattice box (a face region)
  static constexpr int NA = MG * S * BS;     // largest x-pass box
  static constexpr int NB = MG * BS * BS;    // largest y-pass box
};
template <typename T, int BS>
__global__ __launch_bounds__(NT_GEN) void sync_coarser_kernel(const Tab* __restrict__ tab,
                                                              const int32_t* __restrict__ cr,
                                                              int64_t n, T* __restrict__ U,
                                                              Layout L) {
  using D = SyncCoarseDims<BS>;
  constexpr int PER = (D::NSRC + NT_GEN - 1) / NT_GEN;
  __shared__ Tab st;
  __shared__ T buf0[D::NSRC > D::NB ? D::NSRC : D::NB];  // lattice, then the y pass
  __shared__ T buf1[D::NA];                               // x pass
  const T w0 = T(DDW0), w1 = T(DDW1);
  const int tid = threadIdx.x, ng = L.ng, P = L.P;
  const int64_t fs = L.fstride;
  for (int64_t wk = blockIdx.x; wk < n; wk += gridDim.x) {
    const int32_t ib = cr[2 * wk], r = cr[2 * wk + 1];
    __syncthreads();
    load_tab(tab + ib, st);
    __syncthreads();
    T* dst = U + (int64_t)st.meta[0] * L.bstride;
    // box lo..lo+n-1 per axis, and its even lattice e0, e0+2, ... (m points)
    int lo[3], nn[3], e0[3], m[3];
    const int rd[3] = {r % 3, (r / 3) % 3, r / 9};
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      lo[d] = rd[d] == 0 ? -ng : (rd[d] == 1 ? 0 : BS);
      nn[d] = rd[d] == 1 ? BS : ng;
      const int hi = lo[d] + nn[d] - 1;
      e0[d] = (lo[d] & ~1) - 2;
      m[d] = (hi + ((hi & 1) ? 3 : 2) - e0[d]) / 2 + 1;
    }
    const int nsrc = m[0] * m[1] * m[2];
    T v[PER][4];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
      const int p = tid + q * NT_GEN;
      if (p < nsrc) {
        const int ax = p % m[0], rest = p / m[0], ay = rest % m[1], az = rest / m[1];
        const int64_t o = point_offset(st, BS, L, e0[0] + 2 * ax, e0[1] + 2 * ay, e0[2] + 2 * az);
#pragma unroll
        for (int c = 0; c < 4; ++c) v[q][c] = U[o + c * fs];
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int p = tid + q * NT_GEN;
        if (p < nsrc) buf0[p] = v[q][c];
      }
      __syncthreads();
      // x pass: buf1[az][ay][i], i over the box
      for (int p = tid; p < m[2] * m[1] * nn[0]; p += NT_GEN) {
        const int ii = p % nn[0], row = p / nn[0];
        const int i = lo[0] + ii;
        const T* s = buf0 + row * m[0];
        T val;
        if ((i & 1) == 0) {
          val = s[(i - e0[0]) / 2];
        } else {
          const int a = (i - 3 - e0[0]) / 2;
          val = w0 * s[a] + w1 * s[a + 1] + w1 * s[a + 2] + w0 * s[a + 3];
        }
        buf1[p] = val;
      }
      __syncthreads();
      // y pass: buf0[az][j][i]
      for (int p = tid; p < m[2] * nn[1] * nn[0]; p += NT_GEN) {
        const int ii = p % nn[0], rest = p / nn[0], jj = rest % nn[1], az = rest / nn[1];
        const int j = lo[1] + jj;
        const T* s = buf1 + az * m[1] * nn[0] + ii;
        T val;
        if ((j & 1) == 0) {
          val = s[((j - e0[1]) / 2) * nn[0]];
        } else {
          const int a = (j - 3 - e0[1]) / 2;
          val = w0 * s[a * nn[0]] + w1 * s[(a + 1) * nn[0]] + w1 * s[(a + 2) * nn[0]] +
                w0 * s[(a + 3) * nn[0]];
        }
        buf0[p] = val;
      }
      __syncthreads();
      // z pass into the ghost points
      const int plane = nn[1] * nn[0];
      for (int p = tid; p < nn[2] * plane; p += NT_GEN) {
        const int kk = p / plane, q2 = p - kk * plane;
        const int k = lo[2] + kk;
        const T* s = buf0 + q2;
        T val;
        if ((k & 1) == 0) {
          val = s[((k - e0[2]) / 2) * plane];
        } else {
          const int a = (k - 3 - e0[2]) / 2;
          val = w0 * s[a * plane] + w1 * s[(a + 1) * plane] + w1 * s[(a + 2) * plane] +
                w0 * s[(a + 3) * plane];
        }
        const int jj = q2 / nn[0], ii = q2 - jj * nn[0];
        const int64_t o = ((int64_t)(k + ng) * P + (lo[1] + jj + ng)) * P + (lo[0] + ii + ng);
        dst[o + c * fs] = val;
      }
      __syncthreads();
    }
  }
}

// --------------------------------------------------------------------------
// fused rhs + RK4 stage (Sec. 2.2-2.3)
// --------------------------------------------------------------------------
// Barrier that orders LDS traffic only: global loads issued before it stay in
// flight (they are the next plane's prefetch).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  // s_waitcnt lgkmcnt(0): this wave's LDS writes have completed before it
  // arrives (the fence alone need not wait for them)
  __builtin_amdgcn_s_waitcnt(0xC07F);
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <typename T>
struct StageArgs {
  const Tab* tab;
  int64_t nb;
  const T* in;  // stage input register
  Layout Lin;
  const T* hb;  // halo buffer of faces next to other levels [slot][6][4][3][bs][bs]
  T* un;        // U^n register (the pool)
  Layout Lun;
  T* acc;  // accumulator (compact)
  Layout Lacc;
  T* out;  // next stage input, or dU for the rhs-only mode
  Layout Lout;
  const T* dus;  // extra solid velocity [slot][3][bs^3] or null
  const double* t_dev;
  const double* dt_dev;
  double* umax_part;  // stage 4: per work item max |u|^2 of the new U^n, or null
  // optional block list: the blocks of this launch are blist[off + i],
  // i < bcnt[bsel], off = bsel ? bcnt[0] : 0 (the list holds the blocks
  // without penalization first, then the others; null: every block)
  const int32_t* blist;
  const int32_t* bcnt;
  int bsel;
  double t_host;
  double L;
  int xcd_map;  // 1: give each XCD a contiguous run of work items
  int* queue;   // xcd_map 2: per-XCD work counters (QSTRIDE apart), zero at launch
  int nt;       // 1: non-temporal loads/stores of the streaming operands
  wacm_params p;
};

// Persistent loop over the work items (block b, tile t) = item b nty + t of
// the Morton-ordered block list.  With xcd_map, workgroup w (dispatched to XCD
// w % 8) walks a contiguous eighth of the items, so blocks that share faces
// are processed close in time on the same L2; otherwise items go round-robin.
struct BlockIter {
  int64_t ib, end, step;
  __device__ BlockIter(int64_t n, int xcd_map) {
    const int64_t G = gridDim.x, w = blockIdx.x;
    if (xcd_map && G % 8 == 0 && n >= G) {
      const int64_t per = G / 8, xcd = w % 8, lw = w / 8;
      const int64_t chunk = (n + 7) / 8;
      const int64_t start = xcd * chunk;
      end = start + chunk < n ? start + chunk : n;
      ib = start + lw;
      step = per;
    } else {
      ib = w;
      end = n;
      step = G;
    }
  }
};

// Dynamic per-XCD work queues (xcd_map 2): the Morton-ordered items are cut
// into 8 contiguous chunks, one per XCD; workgroup w (on XCD w % 8) takes the
// next item of its own chunk from that chunk's counter, so the tiles of one
// block and neighbouring blocks run together on one L2, and when its chunk is
// empty it takes items from the following chunks, so no XCD idles while
// another still has work.  Each counter increment that finds a chunk empty
// moves on to the next chunk: at most 8 misses per workgroup, so every
// workgroup ends.  Thread 0 only.
constexpr int QSTRIDE = 32;  // ints between counters: one 128-byte line each
__device__ __forceinline__ int queue_take(int* ctr, int& q, int chunk, int n, int v) {
  for (int miss = 0;;) {
    const int lo = q * chunk;
    const int hi = lo + chunk < n ? lo + chunk : n;
    if (lo + v < hi) return lo + v;
    if (++miss == 8) return n;
    q = (q + 1) & 7;
    v = atomicAdd(ctr + q * QSTRIDE, 1);
  }
}

__global__ void queue_clear(int* ctr) {
  if (threadIdx.x < 8 * QSTRIDE) ctr[threadIdx.x] = 0;
}

// Where the depth-3 halo of one face of the current block lives: element
// (field c, depth d away from the face, tangential t0 < t1 by axis order) is
// ptr[c fs + d sd + t0 s0 + t1 s1].  Same-level neighbours are read in place
// (their interior next to the face); faces next to a coarser or finer leaf
// point into the halo buffer filled by nlface_kernel; the rhs-only mode reads
// the block's own synchronised ghost layers.  With an x-split input the
// x faces stay affine (the neighbour's side columns); for the y and z faces
// mode = 1 and ptr is the neighbour's origin: each thread addresses its own
// column with xsplit_offset.
template <typename T>
struct FaceDesc {
  const T* ptr;
  int32_t fs, sd, s0, s1, mode;
};

// Where a stage reads the depth-3 halo of a face: HALO_NB same-level faces
// from the neighbour's interior, the others from the face-halo buffer;
// HALO_OWN every face from the input's own ghost layers; HALO_MIX same-level
// faces from the neighbour's interior, the others from the own ghost layers.
enum { HALO_NB = 0, HALO_OWN = 1, HALO_MIX = 2 };

template <typename T, int BS, int HALO>
__device__ __forceinline__ FaceDesc<T> face_desc(const Tab& tb, const StageArgs<T>& a, int f,
                                                 bool xin) {
  const int axis = f >> 1, side = f & 1;
  const Layout& L = a.Lin;
  const int sx[3] = {1, L.P, L.P * L.P};
  const int sa = sx[axis], st0 = sx[axis == 0 ? 1 : 0], st1 = sx[axis == 2 ? 1 : 2];
  const int slot = tb.meta[0];
  const int64_t org = ((int64_t)L.ng * L.P + L.ng) * L.P + L.ng;  // local (0,0,0)
  const int r = (axis == 0 ? 2 * side : 1) + 3 * (axis == 1 ? 2 * side : 1) +
                9 * (axis == 2 ? 2 * side : 1);
  FaceDesc<T> fd;
  fd.mode = 0;
  if (HALO == HALO_OWN || (HALO == HALO_MIX && tb.kind[r] != 0)) {
    fd.ptr = a.in + (int64_t)slot * L.bstride + org + (int64_t)(side ? BS : -1) * sa;
    fd.fs = (int)L.fstride;
    fd.sd = side ? sa : -sa;
    fd.s0 = st0;
    fd.s1 = st1;
    return fd;
  }
  if (tb.kind[r] == 0 && xin) {
    const T* nb = a.in + (int64_t)tb.slot[r][0] * L.bstride;
    fd.fs = (int)L.fstride;
    if (axis == 0) {
      // side 0 reads the neighbour's last columns from the top, side 1 its
      // first ones
      fd.ptr = nb + (side ? BS * BS * (BS - 2 * XS_H) : BS * BS * (BS - XS_H) + XS_H - 1);
      fd.sd = side ? 1 : -1;
      fd.s0 = XS_H;
      fd.s1 = XS_H * BS;
    } else {
      fd.ptr = nb;
      fd.sd = fd.s0 = fd.s1 = 0;
      fd.mode = 1;
    }
  } else if (tb.kind[r] == 0) {
    fd.ptr = a.in + (int64_t)tb.slot[r][0] * L.bstride + org + (int64_t)(side ? 0 : BS - 1) * sa;
    fd.fs = (int)L.fstride;
    fd.sd = side ? sa : -sa;
    fd.s0 = st0;
    fd.s1 = st1;
  } else {
    fd.ptr = a.hb + ((int64_t)slot * 6 + f) * 12 * BS * BS;
    fd.fs = 3 * BS * BS;
    fd.sd = BS * BS;
    fd.s0 = 1;
    fd.s1 = BS;
  }
  return fd;
}

// Streaming operands (U^n, the accumulator) are touched once per stage: load
// and store them non-temporally so the caches keep the stage input, whose
// face layers neighbouring blocks read again.
template <typename T>
__device__ __forceinline__ T ntload(const T* p, int nt) {
  return nt ? __builtin_nontemporal_load(p) : *p;
}
template <typename T>
__device__ __forceinline__ void ntstore(T v, T* p, int nt) {
  if (nt)
    __builtin_nontemporal_store(v, p);
  else
    *p = v;
}

// MODE 0: dU = rhs(U) with U's own ghost layers.  MODE s = 1..4: classical
// RK4 stage s with registers U^n, W and the stage inputs Y_s:
//   s1: out = Y2 = U^n + dt/2 k1                    (input = U^n)
//   s2: out = Y3 = U^n + dt/2 k2,  W = (U^n + Y2)/3 + dt/3 k2
//   s3: out = Y4 = U^n + dt k3
//   s4: U^{n+1} = W + Y4/3 + dt/6 k4
// Since dt k1 = 2 (Y2 - U^n) and dt k3 = Y4 - U^n, the update
// U^n + dt/6 (k1 + 2 k2 + 2 k3 + k4) equals W + Y4/3 + dt/6 k4 with
// W = 2/3 U^n + dt/6 k1 + dt/3 k2: only stage 2 writes a second register and
// stages 3 and 4 read one besides their input (same values up to rounding of
// U^n's size).
// PEN: penalization/sponge terms present.  PREF: load the epilogue operands
// (U^n, acc) before the barrier instead of after the rhs.  Work items are
// tiles of TY rows of a block's (x,y) columns (TY = BS: the whole block), one
// persistent workgroup per item at a time, one thread per column marching in
// z: z-neighbours in a register queue, the x/y cross of the current plane in a
// double-buffered LDS slab, the next plane's loads issued before the barrier.
// Rows between tiles of one block are read from the block itself.
// Occupancy: FP64 tiles are held to 2 waves per SIMD, FP32 tiles to 3; a
// whole bs-16 block (4 waves) to 2 per SIMD, which keeps two workgroups per
// CU for the penalized FP64 variant at the cost of a few spills (measured
// faster than one workgroup per CU without spills).
// MODEX = MODE (0 rhs only, 1..4 RK stage) or 10 + MODE: the RK stage with
// every register in the padded pool layout, same-level halos read from the
// neighbours' interiors and the others from the input's own synchronised
// ghost layers (the lifted-wavelet step).
template <typename T, int BS, int TY, int MODEX, bool PEN, bool PREF>
__global__ __launch_bounds__(BS* TY) __attribute__((amdgpu_waves_per_eu(TY == BS ? (BS == 16 ? 2 : 1) : (sizeof(T) == 8 ? 2 : 3))))
void stage_kernel(StageArgs<T> a) {
  constexpr int H = 3, W = BS + 2 * H, WY = TY + 2 * H, NT = BS * TY;
  constexpr int NTY = BS / TY, NH = 6 * TY + 6 * BS;
  static_assert(NH <= NT || TY == BS, "halo points per plane exceed the threads");
  constexpr int MODE = MODEX % 10;
  constexpr bool OWNG = MODEX >= 10;
  constexpr int HALO = OWNG ? HALO_MIX : (MODE == 0 ? HALO_OWN : HALO_NB);
  // the stage registers between stages are x-split; U^n is the pool or, from
  // the second step of a multi-step call on, an x-split register too
  const bool xin = !OWNG && (MODE >= 2 || (MODE == 1 && a.Lin.xs != 0));
  const bool xun = MODE >= 2 && a.Lun.xs != 0;
  constexpr bool XOUT = !OWNG && MODE >= 1 && MODE <= 3;
  __shared__ T slab[2][4][W * WY];
  __shared__ FaceDesc<T> fds[6];
  __shared__ int32_t meta[5];
  __shared__ double red[NT / 64];
  __shared__ int qitem;
  const int tid = threadIdx.x;
  const int x = tid % BS, yl = tid / BS;
  const T a1 = T(TW1), a2 = T(TW2), a3 = T(TW3);
  const T c2a = T(D2A), c2b = T(D2B), c2c = T(D2C);
  double tc = a.t_host, dt = 0.0;
  if (MODE != 0) {
    tc = *a.t_dev;
    dt = *a.dt_dev;
  }
  const T nu = T(a.p.nu), c0sq = T(a.p.c0 * a.p.c0), cg = T(a.p.c_gamma);
  const T fA = T(MODE == 4 ? dt / 6.0 : dt / 3.0);  // k weight of W (s2) and of U^{n+1} (s4)
  // the stage time and what of the mask depends on it alone
  const double ts = tc + (MODE == 2 || MODE == 3 ? 0.5 * dt : (MODE == 4 ? dt : 0.0));
  const MaskTime mt = PEN && a.p.mask ? mask_time(a.p, ts) : MaskTime{1.0, 0.0, 0.0};
  const T fB = T(MODE == 3 ? dt : 0.5 * dt);
  const int fin = (int)a.Lin.fstride, Pi = a.Lin.P;
  const int cidx = (yl + H) * W + (x + H);
  // this thread's halo point of every plane (threads < NH): x-faces of the
  // tile's rows, then the 3 rows below and above the tile
  const bool hthr = tid < NH;
  int hkind = 0, hd = 0, hs = 0, hli = 0;  // hkind: 0..3 face x-,x+,below,above
  if (hthr) {
    if (tid < 6 * TY) {
      hkind = tid / (3 * TY);
      const int rem = tid - hkind * 3 * TY;
      hd = rem / TY;
      hs = rem - hd * TY;
      const int hx = hkind == 0 ? -1 - hd : BS + hd;
      hli = (hs + H) * W + (hx + H);
    } else {
      const int q = tid - 6 * TY;
      hkind = 2 + q / (3 * BS);
      const int rem = q - (hkind - 2) * 3 * BS;
      hd = rem / BS;
      hs = rem - hd * BS;
      const int hyl = hkind == 2 ? -1 - hd : TY + hd;
      hli = (hyl + H) * W + (hs + H);
    }
  }
  // plane steps of this thread's column
  const int zs = xin ? xsplit_zstride(BS, x) : Pi * Pi;
  const int azs = a.Lacc.P * a.Lacc.P, afs = (int)a.Lacc.fstride;
  const int uzs = xun ? xsplit_zstride(BS, x) : a.Lun.P * a.Lun.P, ufs = (int)a.Lun.fstride;
  const int ozs = XOUT ? xsplit_zstride(BS, x) : a.Lout.P * a.Lout.P;
  const int ofs = (int)a.Lout.fstride;

  // work items: static (round-robin or contiguous per XCD) or from the
  // per-XCD queues, whose next item thread 0 requests while the current one
  // is processed and publishes in qitem before the loop's first barrier
  int64_t nblk = a.nb, boff = 0;
  if (a.blist) {
    boff = a.bsel ? a.bcnt[0] : 0;
    nblk = a.bcnt[a.bsel];
  }
  const int64_t nitems = nblk * NTY;
  const bool dyn = a.queue != nullptr;
  BlockIter it(nitems, a.xcd_map);
  int qh = blockIdx.x & 7, qpend = 0;
  const int qchunk = (int)((nitems + 7) / 8);
  if (dyn && tid == 0) qitem = queue_take(a.queue, qh, qchunk, (int)nitems,
                                          atomicAdd(a.queue + qh * QSTRIDE, 1));
  for (;;) {
    lds_barrier();
    const int64_t item = dyn ? (int64_t)__builtin_amdgcn_readfirstlane(qitem) : it.ib;
    if (item >= (dyn ? nitems : it.end)) break;
    if (!dyn) it.ib += it.step;
    const int64_t il = item / NTY;
    const int64_t ibk = a.blist ? a.blist[boff + il] : il;
    const int y0 = (int)(item - il * NTY) * TY;
    const int y = y0 + yl;
    if (tid < 6) fds[tid] = face_desc<T, BS, HALO>(a.tab[ibk], a, tid, xin);
    if (tid < 5) meta[tid] = a.tab[ibk].meta[tid];
    lds_barrier();
    if (dyn && tid == 0) qpend = atomicAdd(a.queue + qh * QSTRIDE, 1);
    // offsets of this thread's column in the input, accumulator and U^n
    const int col = xin ? xsplit_offset(BS, x, y, 0)
                        : (a.Lin.ng * Pi + (y + a.Lin.ng)) * Pi + (x + a.Lin.ng);
    const int acol = (a.Lacc.ng * a.Lacc.P + (y + a.Lacc.ng)) * a.Lacc.P + (x + a.Lacc.ng);
    const int ucol = xun ? xsplit_offset(BS, x, y, 0)
                         : (a.Lun.ng * a.Lun.P + (y + a.Lun.ng)) * a.Lun.P + (x + a.Lun.ng);
    const int ocol = XOUT ? xsplit_offset(BS, x, y, 0)
                          : (a.Lout.ng * a.Lout.P + (y + a.Lout.ng)) * a.Lout.P + (x + a.Lout.ng);
    // uniform over the workgroup: scalar registers
    const int slot = __builtin_amdgcn_readfirstlane(meta[0]);
    const int J = __builtin_amdgcn_readfirstlane(meta[1]);
    const double hdd = a.L / (double(int64_t(1) << J) * BS);
    const T ih = T(1.0 / hdd), ih2 = T(1.0 / (hdd * hdd));
    const T* __restrict__ inb = a.in + (int64_t)slot * a.Lin.bstride + col;
    T* accb = a.acc + (int64_t)slot * a.Lacc.bstride + acol;
    T* unb = a.un + (int64_t)slot * a.Lun.bstride + ucol;
    T* outb = a.out + (int64_t)slot * a.Lout.bstride + ocol;
    // field c of this thread's column at depth d below (f = 4) or above
    // (f = 5) the block; the descriptor is re-read from LDS at each use
    auto zface = [&](int f, int d, int c) -> T {
      const FaceDesc<T>& fz = fds[f];
      if (xin && fz.mode == 1) return fz.ptr[c * fin + col + (f == 4 ? BS - 1 - d : d) * zs];
      return fz.ptr[c * fz.fs + d * fz.sd + x * fz.s0 + y * fz.s1];
    };
    // this thread's halo point as an affine map in z: hp[c hfs + z hzs]
    const T* hp = nullptr;
    int hfs = 0, hzs = 0;
    if (hthr) {
      if (hkind < 2) {
        const FaceDesc<T>& fh = fds[hkind];
        hp = fh.ptr + hd * fh.sd + (y0 + hs) * fh.s0;
        hfs = fh.fs;
        hzs = fh.s1;
      } else {
        const int hy = hkind == 2 ? y0 - 1 - hd : y0 + TY + hd;
        if (hy < 0 || hy >= BS) {
          const FaceDesc<T>& fh = fds[hy < 0 ? 2 : 3];
          if (xin && fh.mode == 1) {
            hp = fh.ptr + xsplit_offset(BS, hs, hy < 0 ? BS + hy : hy - BS, 0);
            hfs = fin;
            hzs = xsplit_zstride(BS, hs);
          } else {
            hp = fh.ptr + (hy < 0 ? -1 - hy : hy - BS) * fh.sd + hs * fh.s0;
            hfs = fh.fs;
            hzs = fh.s1;
          }
        } else if (xin) {
          hp = a.in + (int64_t)slot * a.Lin.bstride + xsplit_offset(BS, hs, hy, 0);
          hfs = fin;
          hzs = xsplit_zstride(BS, hs);
        } else {
          hp = a.in + (int64_t)slot * a.Lin.bstride +
               (a.Lin.ng * Pi + (hy + a.Lin.ng)) * Pi + (hs + a.Lin.ng);
          hfs = fin;
          hzs = Pi * Pi;
        }
      }
    }

    double m2 = 0.0;  // stage 4: max |u|^2 of this thread's new points
    // mask, solid velocity and sponge of this thread's point of the next
    // plane, evaluated at the end of the previous plane where fewer values
    // are live
    T pchi = T(0), psp = T(0), pus[3] = {T(0), T(0), T(0)};
    auto pen_at = [&](int zz) {
      const double xg = (double)(meta[2] * BS + x) * hdd, yg = (double)(meta[3] * BS + y) * hdd,
                   zg = (double)(meta[4] * BS + zz) * hdd;
      if (a.p.mask) {
        double cd, u3[3];
        mask_point(a.p, mt, xg, yg, zg, cd, u3);
        pchi = T(cd);
        pus[0] = T(u3[0]);
        pus[1] = T(u3[1]);
        pus[2] = T(u3[2]);
      }
      if (a.p.sponge) psp = T(sponge_eval(a.p, a.L, xg, yg, zg));
    };
    if (PEN) pen_at(0);
    T q[4][7];
#pragma unroll
    for (int mm = 0; mm < 7; ++mm) {
      const int z = mm - 3;
#pragma unroll
      for (int c = 0; c < 4; ++c)
        q[c][mm] = z < 0 ? zface(4, -1 - z, c) : inb[c * fin + z * zs];
    }
    // plane 0 into slab 0
#pragma unroll
    for (int c = 0; c < 4; ++c) slab[0][c][cidx] = q[c][3];
    if (hthr) {
#pragma unroll
      for (int c = 0; c < 4; ++c) slab[0][c][hli] = hp[c * hfs];
    }

    for (int z = 0; z < BS; ++z) {
      T(*sb)[W * WY] = slab[z & 1];
      // loads for the next plane: column value at z+4 and this thread's halo point
      T nq[4], hnx[4];
      if (z + 1 < BS) {
        const int zz = z + 4;
#pragma unroll
        for (int c = 0; c < 4; ++c)
          nq[c] = zz < BS ? inb[c * fin + zz * zs] : zface(5, zz - BS, c);
        if (hthr) {
#pragma unroll
          for (int c = 0; c < 4; ++c) hnx[c] = hp[c * hfs + (z + 1) * hzs];
        }
      }
      // epilogue operands of this point, loaded early if PREF
      T unv[4], acv[4];
      if (PREF) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (MODE == 2 || MODE == 3) unv[c] = ntload(unb + c * ufs + z * uzs, a.nt);
          if (MODE == 4) acv[c] = ntload(accb + c * afs + z * azs, a.nt);
        }
      }
      lds_barrier();

      // rhs, accumulated field by field
      const T u = q[0][3], v = q[1][3], w = q[2][3], pr = q[3][3];
      T r[4], div = T(0);
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const T* s = sb[c];
        const T dx = (a1 * (s[cidx + 1] - s[cidx - 1]) + a2 * (s[cidx + 2] - s[cidx - 2]) +
                      a3 * (s[cidx + 3] - s[cidx - 3])) *
                     ih;
        const T dy = (a1 * (s[cidx + W] - s[cidx - W]) + a2 * (s[cidx + 2 * W] - s[cidx - 2 * W]) +
                      a3 * (s[cidx + 3 * W] - s[cidx - 3 * W])) *
                     ih;
        const T dz = (a1 * (q[c][4] - q[c][2]) + a2 * (q[c][5] - q[c][1]) +
                      a3 * (q[c][6] - q[c][0])) *
                     ih;
        if (c < 3) {
          const T lap = ((c2a * s[cidx - 2] + c2b * s[cidx - 1] + c2c * s[cidx] +
                          c2b * s[cidx + 1] + c2a * s[cidx + 2]) +
                         (c2a * s[cidx - 2 * W] + c2b * s[cidx - W] + c2c * s[cidx] +
                          c2b * s[cidx + W] + c2a * s[cidx + 2 * W]) +
                         (c2a * q[c][1] + c2b * q[c][2] + c2c * q[c][3] + c2b * q[c][4] +
                          c2a * q[c][5])) *
                        ih2;
          r[c] = -(u * dx + v * dy + w * dz) + nu * lap;
          div += c == 0 ? dx : (c == 1 ? dy : dz);
        } else {
          r[0] -= dx;
          r[1] -= dy;
          r[2] -= dz;
        }
      }
      r[3] = -c0sq * div - cg * pr;
      if (PEN) {
        const wacm_params& p = a.p;
        T chi = pchi, sp = psp, us[3] = {pus[0], pus[1], pus[2]};
        if (a.dus) {
          const T* du = a.dus + (int64_t)slot * 3 * BS * BS * BS + (z * BS + y) * BS + x;
          us[0] += du[0];
          us[1] += du[BS * BS * BS];
          us[2] += du[2 * BS * BS * BS];
        }
        const T iceta = p.mask ? T(1.0 / p.c_eta) : T(0), icsp = p.sponge ? T(1.0 / p.c_sp) : T(0);
        const T val[4] = {u, v, w, pr};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          if (p.mask) r[c] -= chi * iceta * (val[c] - us[c]);
          if (p.sponge) r[c] -= sp * icsp * (val[c] - T(p.u_inf[c]));
        }
        if (p.sponge) r[3] -= sp * icsp * (pr - T(p.p_inf));
      }

      if (!PREF) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          if (MODE == 2 || MODE == 3) unv[c] = ntload(unb + c * ufs + z * uzs, a.nt);
          if (MODE == 4) acv[c] = ntload(accb + c * afs + z * azs, a.nt);
        }
      }
      if (MODE == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) outb[c * ofs + z * ozs] = r[c];
      } else if (MODE == 4) {
        const T val[4] = {u, v, w, pr};
        T nv[4];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          nv[c] = acv[c] + val[c] * T(1.0 / 3.0) + fA * r[c];
          ntstore(nv[c], unb + c * ufs + z * uzs, a.nt);
        }
        // The x-ghost columns of the row are cleared too, so that every cache
        // line of the padded row is written whole: rows of partly written lines
        // store far slower.  Ghost layers carry no state between steps.
        const int gx = a.Lun.ng;
        if (!xun && (x < gx || x >= BS - gx)) {
          const int off = x < gx ? -gx : gx;
#pragma unroll
          for (int c = 0; c < 4; ++c) ntstore(T(0), unb + c * ufs + z * uzs + off, a.nt);
        }
        if (a.umax_part) m2 = fmax(m2, speed2(double(nv[0]), double(nv[1]), double(nv[2])));
      } else {
        const T val[4] = {u, v, w, pr};
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const T u0 = MODE == 1 ? val[c] : unv[c];
          // (U^n + Y2)/3 = 2/3 U^n + dt/6 k1, from the input Y2 = U^n + dt/2 k1
          if (MODE == 2) ntstore((u0 + val[c]) * T(1.0 / 3.0) + fA * r[c], accb + c * afs + z * azs, a.nt);
          outb[c * ofs + z * ozs] = u0 + fB * r[c];
        }
        // a padded output's rows are written whole as in stage 4 (the next
        // stage's fill rewrites every ghost point that is read)
        const int gx = a.Lout.ng;
        if (OWNG && (x < gx || x >= BS - gx)) {
          const int off = x < gx ? -gx : gx;
#pragma unroll
          for (int c = 0; c < 4; ++c) outb[c * ofs + z * ozs + off] = T(0);
        }
      }
      if (z + 1 < BS) {
        // plane z+1 into the other slab: it was last read before this
        // plane's barrier, which every thread has passed
        T(*nb_)[W * WY] = slab[(z + 1) & 1];
#pragma unroll
        for (int c = 0; c < 4; ++c) nb_[c][cidx] = q[c][4];
        if (hthr) {
#pragma unroll
          for (int c = 0; c < 4; ++c) nb_[c][hli] = hnx[c];
        }
#pragma unroll
        for (int c = 0; c < 4; ++c) {
#pragma unroll
          for (int mm = 0; mm < 6; ++mm) q[c][mm] = q[c][mm + 1];
          q[c][6] = nq[c];
        }
        if (PEN) pen_at(z + 1);
      }
    }
    if (MODE == 4 && a.umax_part) {
      // the work item's maximum, reduced in the workgroup; red is free again
      // by the next item's writes (several barriers later)
      m2 = wave_max(m2);
      if ((tid & 63) == 0) red[tid >> 6] = m2;
      lds_barrier();
      if (tid == 0) {
        double mx = red[0];
#pragma unroll
        for (int w = 1; w < NT / 64; ++w) mx = fmax(mx, red[w]);
        a.umax_part[boff * NTY + item] = mx;
      }
    }
    if (dyn && tid == 0) qitem = queue_take(a.queue, qh, qchunk, (int)nitems, qpend);
  }
}

// Faces next to a coarser or finer leaf: the depth-3 face halo of the stage
// input into the halo buffer the stage kernel reads.  A finer neighbour gives
// its coincident point (decimation, Sec. 3.1).  A coarser neighbour gives the
// tensor-product DD4 prediction (Sec. 3.1), computed separably: the coarse
// lattice box around the face (even local indices, read from whichever leaves
// hold them) is gathered once, then predicted along the normal and the two
// tangential axes in turn, one field at a time through LDS.  The loads of all
// 4 fields are issued together into registers before the first field's
// passes, so one memory latency per face is exposed instead of four.  With
// `queue` (schedule xcd_map 2) the faces, listed in the blocks' Morton order,
// are taken from per-XCD work counters like the stage kernel's items, so the
// faces of sister blocks, which read the same coarse data, meet in one L2.
// FP32: held to 4 waves per SIMD (a few spilled registers; 0.64 -> 0.60 ms
// per launch on the 20k-block octree); FP64 keeps its registers (2 waves:
// held to 4 it spills ~70 and slows down).
template <typename T, int BS>
__global__ __launch_bounds__(NT_GEN) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 4 ? 4 : 1)))
void nlface_kernel(const Tab* __restrict__ tab,
                                                        const int32_t* __restrict__ cf, int64_t n,
                                                        const T* __restrict__ in, Layout Lin,
                                                        T* __restrict__ hb, int* queue) {
  constexpr int S = BS / 2 + 3;   // tangential coarse positions -2, 0, ..., bs+2
  constexpr int NSRC = 5 * S * S;  // at most 5 coarse points along the normal
  constexpr int PER = (NSRC + NT_GEN - 1) / NT_GEN;
  constexpr int B2 = BS * BS;
  constexpr int NFINE = (3 * B2 + NT_GEN - 1) / NT_GEN;
  __shared__ Tab st;
  __shared__ T src[NSRC];
  __shared__ T pa[3 * S * S];
  __shared__ T pb[3 * S * BS];
  __shared__ int qitem;
  const T w0 = T(DDW0), w1 = T(DDW1);
  const int64_t fs = Lin.fstride;
  const int tid = threadIdx.x;
  const bool dyn = queue != nullptr;
  int qh = blockIdx.x & 7, qpend = 0;
  const int qchunk = (int)((n + 7) / 8);
  if (dyn && tid == 0) qitem = queue_take(queue, qh, qchunk, (int)n, atomicAdd(queue + qh * QSTRIDE, 1));
  int64_t wnext = blockIdx.x;
  for (;;) {
    __syncthreads();
    const int64_t wk = dyn ? (int64_t)__builtin_amdgcn_readfirstlane(qitem) : wnext;
    if (wk >= n) break;
    wnext += gridDim.x;
    const int32_t ib = cf[2 * wk], f = cf[2 * wk + 1];
    load_tab(tab + ib, st);
    __syncthreads();
    if (dyn && tid == 0) qpend = atomicAdd(queue + qh * QSTRIDE, 1);
    const int slot = st.meta[0];
    const int axis = f >> 1, side = f & 1;
    const int ua = axis == 0 ? 1 : 0, ub = axis == 2 ? 1 : 2;  // tangential axes t0, t1
    const int r = (axis == 0 ? 2 * side : 1) + 3 * (axis == 1 ? 2 * side : 1) +
                  9 * (axis == 2 ? 2 * side : 1);
    T* hbf = hb + ((int64_t)slot * 6 + f) * 12 * B2;
    if (st.kind[r] > 0) {
      // finer neighbour: every halo point is a point of a finer leaf; all
      // loads of this thread's points first, then the stores
      T v[NFINE][4];
#pragma unroll
      for (int k = 0; k < NFINE; ++k) {
        const int p = tid + k * NT_GEN;
        if (p < 3 * B2) {
          const int d = p / B2, qq = p - d * B2;
          int li[3];
          li[axis] = side ? BS + d : -1 - d;
          li[ua] = qq % BS;
          li[ub] = qq / BS;
          const int64_t o = point_offset(st, BS, Lin, li[0], li[1], li[2]);
#pragma unroll
          for (int c = 0; c < 4; ++c) v[k][c] = in[o + c * fs];
        }
      }
#pragma unroll
      for (int k = 0; k < NFINE; ++k) {
        const int p = tid + k * NT_GEN;
        if (p < 3 * B2) {
#pragma unroll
          for (int c = 0; c < 4; ++c) hbf[(int64_t)(c * 3) * B2 + p] = v[k][c];
        }
      }
      if (dyn && tid == 0) qitem = queue_take(queue, qh, qchunk, (int)n, qpend);
      continue;
    }
    // coarser neighbour.  Normal ghost positions g_d = bs + d (side 1) or
    // -1 - d (side 0); the even positions their stencils use run from n0 in
    // steps of 2: side 1 [bs-2, bs+4] (4 points), side 0 [-6, 2] (5 points)
    const int n0 = side ? BS - 2 : -6;
    const int NN = side ? 4 : 5;
    const int nsrc = NN * S * S;
    T v[PER][4];
#pragma unroll
    for (int k = 0; k < PER; ++k) {
      const int p = tid + k * NT_GEN;
      if (p < nsrc) {
        const int m = p / (S * S), qq = p - m * S * S;
        int li[3];
        li[axis] = n0 + 2 * m;
        li[ua] = 2 * (qq % S) - 2;
        li[ub] = 2 * (qq / S) - 2;
        const int64_t o = point_offset(st, BS, Lin, li[0], li[1], li[2]);
#pragma unroll
        for (int c = 0; c < 4; ++c) v[k][c] = in[o + c * fs];
      }
    }
#pragma unroll
    for (int c = 0; c < 4; ++c) {
#pragma unroll
      for (int k = 0; k < PER; ++k) {
        const int p = tid + k * NT_GEN;
        if (p < nsrc) src[p] = v[k][c];
      }
      __syncthreads();
      // along the normal: pa[d][t1'][t0']
      for (int p = tid; p < 3 * S * S; p += NT_GEN) {
        const int d = p / (S * S), qq = p - d * S * S;
        const int g = side ? BS + d : -1 - d;
        T val;
        if ((g & 1) == 0) {
          val = src[((g - n0) / 2) * S * S + qq];
        } else {
          const int m = (g - 3 - n0) / 2;  // taps g-3, g-1, g+1, g+3
          val = w0 * src[m * S * S + qq] + w1 * src[(m + 1) * S * S + qq] +
                w1 * src[(m + 2) * S * S + qq] + w0 * src[(m + 3) * S * S + qq];
        }
        pa[p] = val;
      }
      __syncthreads();
      // along t0: pb[d][t1'][t0], t0 in [0, bs)
      for (int p = tid; p < 3 * S * BS; p += NT_GEN) {
        const int t0 = p % BS, rest = p / BS;  // rest = d * S + t1'
        const T* row = pa + rest * S;
        T val;
        if ((t0 & 1) == 0) {
          val = row[t0 / 2 + 1];
        } else {
          const int m = (t0 - 3) / 2 + 1;  // coarse index of t0-3
          val = w0 * row[m] + w1 * row[m + 1] + w1 * row[m + 2] + w0 * row[m + 3];
        }
        pb[p] = val;
      }
      __syncthreads();
      // along t1: out[d][t1][t0]
      for (int p = tid; p < 3 * B2; p += NT_GEN) {
        const int d = p / B2, qq = p - d * B2;
        const int t0 = qq % BS, t1 = qq / BS;
        const T* colp = pb + d * S * BS + t0;
        T val;
        if ((t1 & 1) == 0) {
          val = colp[(t1 / 2 + 1) * BS];
        } else {
          const int m = (t1 - 3) / 2 + 1;
          val = w0 * colp[m * BS] + w1 * colp[(m + 1) * BS] + w1 * colp[(m + 2) * BS] +
                w0 * colp[(m + 3) * BS];
        }
        hbf[(int64_t)(c * 3) * B2 + p] = val;
      }
      __syncthreads();
    }
    if (dyn && tid == 0) qitem = queue_take(queue, qh, qchunk, (int)n, qpend);
  }
}

// --------------------------------------------------------------------------
// reductions (FP64 accumulation, fixed order -> deterministic)
// --------------------------------------------------------------------------
// per block: max over interior points of |u|^2 -> part[ib]; the block edge
// is a template constant, so that the index arithmetic needs no division
template <typename T, int bs>
__global__ __launch_bounds__(NT_GEN) void maxu_kernel(const Tab* __restrict__ tab, int64_t nb,
                                                      const T* __restrict__ U, Layout L,
                                                      double* __restrict__ part) {
  __shared__ double red[NT_GEN / 64];
  constexpr int n3 = bs * bs * bs;
  for (int64_t ib = blockIdx.x; ib < nb; ib += gridDim.x) {
    const T* b = U + (int64_t)tab[ib].meta[0] * L.bstride;
    double m = 0.0;
#pragma unroll 4
    for (int q = threadIdx.x; q < n3; q += NT_GEN) {
      const int i = q % bs, j = (q / bs) % bs, k = q / (bs * bs);
      const int64_t o = ((int64_t)(k + L.ng) * L.P + (j + L.ng)) * L.P + (i + L.ng);
      const double u = b[o], v = b[o + L.fstride], w = b[o + 2 * L.fstride];
      m = fmax(m, speed2(u, v, w));
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
// sum chi(u-us) x3 (times h^3/C_eta), sum |u|^2 (times h^3/2), number of
// NaN or Inf values]; the maxima ignore NaN, the count sees it
constexpr int NDIAG = 10;
template <typename T, int bs>
__global__ __launch_bounds__(NT_GEN) void diag_kernel(const Tab* __restrict__ tab, int64_t nb,
                                                      const T* __restrict__ U, Layout L,
                                                      const T* __restrict__ dus, double Ldom,
                                                      wacm_params p, double t,
                                                      double* __restrict__ part) {
  __shared__ double red[NDIAG][NT_GEN];
  constexpr int n3 = bs * bs * bs;
  for (int64_t ib = blockIdx.x; ib < nb; ib += gridDim.x) {
    const int32_t* m = tab[ib].meta;
    const int slot = m[0], J = m[1];
    const double h = Ldom / (double(int64_t(1) << J) * bs);
    const T* b = U + (int64_t)slot * L.bstride;
    double acc[NDIAG] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int q = threadIdx.x; q < n3; q += NT_GEN) {
      const int i = q % bs, j = (q / bs) % bs, k = q / (bs * bs);
      const int64_t o = ((int64_t)(k + L.ng) * L.P + (j + L.ng)) * L.P + (i + L.ng);
      double u[4];
      for (int c = 0; c < 4; ++c) u[c] = b[o + c * L.fstride];
      for (int c = 0; c < 4; ++c) acc[9] += isfinite(u[c]) ? 0.0 : 1.0;
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
    for (int c = 0; c < NDIAG; ++c) red[c][threadIdx.x] = acc[c];
    __syncthreads();
    for (int s = NT_GEN / 2; s > 0; s >>= 1) {
      if ((int)threadIdx.x < s) {
        for (int c = 0; c < 5; ++c)
          red[c][threadIdx.x] = fmax(red[c][threadIdx.x], red[c][threadIdx.x + s]);
        for (int c = 5; c < NDIAG; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      const double vol = h * h * h;
      for (int c = 0; c < 5; ++c) part[ib * NDIAG + c] = red[c][0];
      for (int c = 5; c < 8; ++c)
        part[ib * NDIAG + c] = p.mask ? red[c][0] * vol / p.c_eta : 0.0;
      part[ib * NDIAG + 8] = 0.5 * red[8][0] * vol;
      part[ib * NDIAG + 9] = red[9][0];
    }
  }
}

__global__ __launch_bounds__(NT_GEN) void diag_finalize(const double* __restrict__ part,
                                                        int64_t nb, double* __restrict__ out) {
  __shared__ double red[NDIAG][NT_GEN];
  double acc[NDIAG] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int64_t q = threadIdx.x; q < nb; q += blockDim.x) {
    for (int c = 0; c < 5; ++c) acc[c] = fmax(acc[c], part[q * NDIAG + c]);
    for (int c = 5; c < NDIAG; ++c) acc[c] += part[q * NDIAG + c];
  }
  for (int c = 0; c < NDIAG; ++c) red[c][threadIdx.x] = acc[c];
  __syncthreads();
  for (int s = NT_GEN / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      for (int c = 0; c < 5; ++c)
        red[c][threadIdx.x] = fmax(red[c][threadIdx.x], red[c][threadIdx.x + s]);
      for (int c = 5; c < NDIAG; ++c) red[c][threadIdx.x] += red[c][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = sqrt(red[0][0]);
    for (int c = 1; c < NDIAG; ++c) out[c] = red[c][0];
  }
}

// --------------------------------------------------------------------------
// wavelet details and coarsening flags (Sec. 3.1, 3.3-3.5)
// --------------------------------------------------------------------------
// max over blocks of the per-block field maxima part[4 ib + c] -> norm[c]
// (1 where the field vanishes); used by the two-dimensional thresholding
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

// Wavelet details (Sec. 3.1) of one block: d = u - P R u at every interior
// point with an odd index, P R u the tensor-product DD4 prediction from the
// block's even lattice (ghost-synchronised pool), evaluated separably while
// marching in z over the coarse planes k' = -2, 0, ..., bs + 2: the x pass
// gives X(i, j', k') on the coarse rows (LDS, two buffers), the y pass
// Y(i, j, k') of the thread's own column (one thread per column, the last 4
// coarse planes in registers), the z pass the prediction of the fine plane k'
// (even) and k' - 3 (odd).  All 4 fields at once: one barrier per coarse
// plane.  One workgroup per block; per block and field the maxima of |u_c|
// and |d_c| over the interior (part[8 ib + c], part[8 ib + 4 + c]), and the
// mask range (0 without a mask, and for a block where the mask vanishes at
// time t); thr_finalize turns them into the normalised detail maximum and the
// coarsening flag (Sec. 3.3-3.5).
template <typename T, int BS>
__global__ __launch_bounds__(BS* BS) void detail_kernel(const Tab* __restrict__ tab, int64_t nb,
                                                        const T* __restrict__ U, Layout L,
                                                        double Ldom, wacm_params p, double t,
                                                        double* __restrict__ part,
                                                        double* __restrict__ mrange) {
  constexpr int S = BS / 2 + 3;  // even positions -2, 0, ..., bs+2
  constexpr int NT = BS * BS;
  __shared__ T xp[2][4][S * BS];
  __shared__ double red[10][NT / 64];
  const T w0 = T(DDW0), w1 = T(DDW1);
  const int tid = threadIdx.x;
  const int i = tid % BS, j = tid / BS;
  const int P = L.P, ng = L.ng;
  const int64_t ib = blockIdx.x;
  if (ib >= nb) return;  // whole workgroup
  const int32_t* m = tab[ib].meta;
  const T* b = U + (int64_t)m[0] * L.bstride;
  auto at = [&](int c, int ii, int jj, int kk) -> T {
    return b[c * L.fstride + ((int64_t)(kk + ng) * P + (jj + ng)) * P + (ii + ng)];
  };
  double cmin = 1e300, cmax = -1e300;
  if (p.mask) {
    wacm_params pm = p;
    pm.sponge = 0;
    if (pen_far(pm, Ldom, BS, m, pitch_window(p, t, t))) {
      cmin = cmax = 0.0;  // the mask is exactly 0 on the whole block
    } else {
      const MaskTime mt = mask_time(p, t);
      const double h = Ldom / (double(int64_t(1) << m[1]) * BS);
      for (int k = 0; k < BS; ++k) {
        double chi, us[3];
        mask_point(p, mt, (double)(m[2] * BS + i) * h, (double)(m[3] * BS + j) * h,
                   (double)(m[4] * BS + k) * h, chi, us);
        cmin = fmin(cmin, chi);
        cmax = fmax(cmax, chi);
      }
    }
  }
  double dmc[4] = {0, 0, 0, 0}, umc[4] = {0, 0, 0, 0};
  T y0[4], y1[4], y2[4], y3[4];  // Y of the coarse planes mm, mm-1, mm-2, mm-3
#pragma unroll
  for (int c = 0; c < 4; ++c) y0[c] = y1[c] = y2[c] = y3[c] = T(0);
  const bool oddij = ((i | j) & 1) != 0;
  for (int mm = 0; mm < S; ++mm) {
    const int kc = 2 * mm - 2;  // coarse plane
    const int ko = kc - 3;      // odd fine plane whose prediction this plane completes
    // this thread's points of the fine planes kc and ko, loaded before the
    // x pass so that their latency overlaps it
    T ue[4], uo[4];
    const bool he = kc >= 0 && kc < BS, ho = ko >= 0 && ko < BS;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      ue[c] = he ? at(c, i, j, kc) : T(0);
      uo[c] = ho ? at(c, i, j, ko) : T(0);
    }
    // x pass on the coarse rows j' = 2 jj - 2 of plane kc; the buffer of
    // plane mm - 2 is free: every thread has passed plane mm - 1's barrier
    T(*xb)[S * BS] = xp[mm & 1];
    for (int q = tid; q < S * BS; q += NT) {
      const int jj = q / BS, ii = q - jj * BS, jc = 2 * jj - 2;
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        T v;
        if ((ii & 1) == 0)
          v = at(c, ii, jc, kc);
        else
          v = w0 * at(c, ii - 3, jc, kc) + w1 * at(c, ii - 1, jc, kc) +
              w1 * at(c, ii + 1, jc, kc) + w0 * at(c, ii + 3, jc, kc);
        xb[c][q] = v;
      }
    }
    __syncthreads();
    // y pass: Y(i, j) of plane kc for the thread's column
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      y3[c] = y2[c];
      y2[c] = y1[c];
      y1[c] = y0[c];
      if ((j & 1) == 0) {
        y0[c] = xb[c][(j / 2 + 1) * BS + i];
      } else {
        const int jj = (j - 3) / 2 + 1;  // coarse row of j - 3
        y0[c] = w0 * xb[c][jj * BS + i] + w1 * xb[c][(jj + 1) * BS + i] +
                w1 * xb[c][(jj + 2) * BS + i] + w0 * xb[c][(jj + 3) * BS + i];
      }
    }
    // z pass: the even fine plane kc and the odd fine plane kc - 3 (taps
    // kc-6, kc-4, kc-2, kc = coarse planes mm-3 .. mm)
    if (he) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const T u = ue[c];
        umc[c] = fmax(umc[c], fabs((double)u));
        if (oddij) dmc[c] = fmax(dmc[c], fabs((double)(u - y0[c])));
      }
    }
    if (ho) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const T u = uo[c];
        const T pr = w0 * y3[c] + w1 * y2[c] + w1 * y1[c] + w0 * y0[c];
        umc[c] = fmax(umc[c], fabs((double)u));
        dmc[c] = fmax(dmc[c], fabs((double)(u - pr)));
      }
    }
  }
  double v[10];
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    v[c] = wave_max(umc[c]);
    v[4 + c] = wave_max(dmc[c]);
  }
  v[8] = wave_min(cmin);
  v[9] = wave_max(cmax);
  if ((tid & 63) == 0)
#pragma unroll
    for (int q = 0; q < 10; ++q) red[q][tid >> 6] = v[q];
  __syncthreads();
  if (tid < 10) {
    double r = red[tid][0];
    for (int w = 1; w < NT / 64; ++w) r = tid == 8 ? fmin(r, red[tid][w]) : fmax(r, red[tid][w]);
    red[tid][0] = r;
  }
  __syncthreads();
  if (tid < 8) part[ib * 8 + tid] = red[tid][0];
  if (tid == 0) mrange[ib] = p.mask ? red[9][0] - red[8][0] : 0.0;
}

// One workgroup: the field norms (max |u_c| over all blocks, 1 where a field
// vanishes) into norm, then per block the normalised detail maximum
// max_c max|d_c| / norm_c (equal to the maximum of the normalised details:
// scaling by a positive factor keeps the order) and the coarsening flag:
// 1 iff J > jmin and either dealiasing at J = jmax or the maximum is below
// eps with a constant mask.
__global__ __launch_bounds__(1024) void thr_finalize(const Tab* __restrict__ tab, int64_t nb,
                                                     const double* __restrict__ part,
                                                     const double* __restrict__ mrange,
                                                     double eps, int dealias, int jmin, int jmax,
                                                     double* __restrict__ norm,
                                                     double* __restrict__ dmax,
                                                     int8_t* __restrict__ flags) {
  __shared__ double red[4][1024 / 64];
  __shared__ double inv[4];
  const int tid = threadIdx.x;
  double mx[4] = {0, 0, 0, 0};
  for (int64_t q = tid; q < nb; q += blockDim.x)
#pragma unroll
    for (int c = 0; c < 4; ++c) mx[c] = fmax(mx[c], part[q * 8 + c]);
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    const double v = wave_max(mx[c]);
    if ((tid & 63) == 0) red[c][tid >> 6] = v;
  }
  __syncthreads();
  if (tid < 4) {
    double r = red[tid][0];
    for (int w = 1; w < (int)blockDim.x / 64; ++w) r = fmax(r, red[tid][w]);
    const double nrm = r > 0.0 ? r : 1.0;
    norm[tid] = nrm;
    inv[tid] = 1.0 / nrm;
  }
  __syncthreads();
  for (int64_t q = tid; q < nb; q += blockDim.x) {
    double dm = 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) dm = fmax(dm, part[q * 8 + 4 + c] * inv[c]);
    dmax[q] = dm;
    const int J = tab[q].meta[1];
    int f = 0;
    if (J > jmin) {
      if (dealias && J == jmax)
        f = 1;
      else if (dm < eps && mrange[q] == 0.0)
        f = 1;
    }
    flags[q] = (int8_t)f;
  }
}

// Wavelet filtering of a block at its own level: removing its details (Sec.
// 3.1) sets every interior point with an odd local index to P R u, the
// tensor-product DD4 prediction from the block's even lattice (ghost layers
// included); the even points are kept.  Only blocks of level `level` are
// filtered (every block if level < 0).  Same separable, z-marching passes as
// detail_kernel.  In place: the passes read only points whose three local
// indices are even, and the writes change only points with an odd index
// (all-even points are rewritten with their own value).
template <typename T, int BS>
__global__ __launch_bounds__(NT_GEN) void filter_kernel(const Tab* __restrict__ tab, int64_t nb,
                                                        T* U, Layout L, int level) {
  constexpr int S = BS / 2 + 3;  // even positions -2, 0, ..., bs+2
  constexpr int B2 = BS * BS;
  constexpr int NX = S * BS;                             // x-pass values per field and plane
  constexpr int KX = (4 * NX + NT_GEN - 1) / NT_GEN;     // x-pass values per thread
  constexpr int KQ = (B2 + NT_GEN - 1) / NT_GEN;         // (i, j) columns per thread
  __shared__ T xp[4 * NX];  // X(i, j', k') of the current coarse plane, 4 fields
  const T w0 = T(DDW0), w1 = T(DDW1);
  const int tid = threadIdx.x;
  const int P = L.P, ng = L.ng;
  for (int64_t ib = blockIdx.x; ib < nb; ib += gridDim.x) {
    const int32_t* m = tab[ib].meta;
    const int slot = m[0], J = m[1];
    if (level >= 0 && J != level) continue;  // uniform over the workgroup
    T* b = U + (int64_t)slot * L.bstride;
    auto ix = [&](int c, int i, int j, int k) -> int64_t {
      return c * L.fstride + ((int64_t)(k + ng) * P + (j + ng)) * P + (i + ng);
    };
    // Y(i, j, k') of this thread's columns for the last 4 coarse planes
    // (oldest first), all 4 fields, in registers
    T ring[KQ][4][4] = {};
    for (int mm = 0; mm < S; ++mm) {
      const int kc = 2 * mm - 2;  // coarse plane
      __syncthreads();            // xp is free again
      // x pass on the coarse rows j' = 2 jj - 2 of plane kc, 4 fields
#pragma unroll 2
      for (int kx = 0; kx < KX; ++kx) {
        const int it = tid + kx * NT_GEN;
        if (it < 4 * NX) {
          const int c = it / NX, q = it - c * NX;
          const int jj = q / BS, i = q - jj * BS, jc = 2 * jj - 2;
          T v;
          if ((i & 1) == 0)
            v = b[ix(c, i, jc, kc)];
          else
            v = w0 * b[ix(c, i - 3, jc, kc)] + w1 * b[ix(c, i - 1, jc, kc)] +
                w1 * b[ix(c, i + 1, jc, kc)] + w0 * b[ix(c, i + 3, jc, kc)];
          xp[it] = v;
        }
      }
      __syncthreads();
      // y pass into the ring, z pass: the even fine plane kc (the whole plane
      // is stored, so that its rows are written as whole lines: at points
      // with i and j even Y is the point itself, copied through both passes
      // without arithmetic) and the odd fine plane kc - 3
#pragma unroll
      for (int kq = 0; kq < KQ; ++kq) {
        const int q = tid + kq * NT_GEN;
        if (q < B2) {
          const int j = q / BS, i = q - j * BS;
#pragma unroll
          for (int c = 0; c < 4; ++c) {
            const T* xc = xp + c * NX;
            T y;
            if ((j & 1) == 0) {
              y = xc[(j / 2 + 1) * BS + i];
            } else {
              const int jj = (j - 3) / 2 + 1;  // coarse row of j - 3
              y = w0 * xc[jj * BS + i] + w1 * xc[(jj + 1) * BS + i] + w1 * xc[(jj + 2) * BS + i] +
                  w0 * xc[(jj + 3) * BS + i];
            }
            if (kc >= 0 && kc < BS) b[ix(c, i, j, kc)] = y;
            const int ko = kc - 3;
            if (ko >= 0 && ko < BS)
              b[ix(c, i, j, ko)] = w0 * ring[kq][c][1] + w1 * ring[kq][c][2] +
                                   w1 * ring[kq][c][3] + w0 * y;
            ring[kq][c][0] = ring[kq][c][1];
            ring[kq][c][1] = ring[kq][c][2];
            ring[kq][c][2] = ring[kq][c][3];
            ring[kq][c][3] = y;
          }
        }
      }
    }
  }
}

// --------------------------------------------------------------------------
// refinement (prediction into 8 children) and coarsening (decimation)
// --------------------------------------------------------------------------
// Refinement (Sec. 3.1 prediction, Sec. 3.5): child octant oct of a
// ghost-synchronised parent.  Child point (i, j, k) is the parent's fine-grid
// point Q = off + (i, j, k), off = octant offset (0 or bs per axis); even Q
// copy the parent point Q/2, odd Q use the DD4 taps (Q-3)/2 .. (Q+3)/2 (the
// parent's ghost layers included).  Separable and z-marching as in
// detail_kernel: for each parent plane an x pass on the parent rows and a y
// pass into a ring of 4 planes in LDS, then the z pass writes the child
// planes the ring completes.
template <typename T, int BS>
__global__ __launch_bounds__(NT_GEN) void prolong_kernel(const int32_t* __restrict__ list,
                                                         int64_t n, T* __restrict__ U, Layout L) {
  constexpr int S = BS / 2 + 4;  // parent points per axis: off/2 - 2 .. off/2 + bs/2 + 1
  constexpr int B2 = BS * BS;
  __shared__ T xp[S * BS];
  __shared__ T yr[4][B2];
  const T w0 = T(DDW0), w1 = T(DDW1);
  const int tid = threadIdx.x, P = L.P, ng = L.ng;
  for (int64_t w = blockIdx.x; w < n; w += gridDim.x) {
    const int32_t ps = list[3 * w], cs = list[3 * w + 1], oct = list[3 * w + 2];
    const int h0 = (oct & 1) * (BS / 2) - 2, h1 = ((oct >> 1) & 1) * (BS / 2) - 2,
              h2 = ((oct >> 2) & 1) * (BS / 2) - 2;  // first parent index per axis
    const T* par = U + (int64_t)ps * L.bstride;
    T* ch = U + (int64_t)cs * L.bstride;
    auto pidx = [&](int i, int j, int k) -> int64_t {
      return ((int64_t)(k + ng) * P + (j + ng)) * P + (i + ng);
    };
    for (int c = 0; c < 4; ++c) {
      const T* pc = par + c * L.fstride;
      T* cc = ch + c * L.fstride;
      for (int mm = 0; mm < S; ++mm) {
        const int kz = h2 + mm;  // parent plane
        __syncthreads();
        // x pass: xp[jj][i] for the parent rows j = h1 + jj; child i has
        // Q = 2 (h0 + 2) + i, even -> parent point Q/2, odd -> taps
        for (int q = tid; q < S * BS; q += NT_GEN) {
          const int jj = q / BS, i = q - jj * BS;
          const int64_t row = pidx(0, h1 + jj, kz);
          const int base = h0 + 2 + (i >> 1);  // parent index of Q/2 (even Q)
          T v;
          if ((i & 1) == 0)
            v = pc[row + base];
          else  // taps (Q-3)/2 .. (Q+3)/2 = base-1 .. base+2
            v = w0 * pc[row + base - 1] + w1 * pc[row + base] + w1 * pc[row + base + 1] +
                w0 * pc[row + base + 2];
          xp[q] = v;
        }
        __syncthreads();
        T* yo = yr[mm & 3];
        for (int q = tid; q < B2; q += NT_GEN) {
          const int j = q / BS, i = q - j * BS;
          const int jj = 2 + (j >> 1);  // row of Q/2 in xp
          T v;
          if ((j & 1) == 0)
            v = xp[jj * BS + i];
          else
            v = w0 * xp[(jj - 1) * BS + i] + w1 * xp[jj * BS + i] + w1 * xp[(jj + 1) * BS + i] +
                w0 * xp[(jj + 2) * BS + i];
          yo[q] = v;
        }
        __syncthreads();
        // z pass: child plane k even uses plane mm = 2 + k/2; k odd uses
        // planes 1 + (k-1)/2 .. 4 + (k-1)/2, complete when mm = 4 + (k-1)/2
        const int ke = 2 * (mm - 2), ko = 2 * (mm - 4) + 1;
        for (int q = tid; q < B2; q += NT_GEN) {
          const int j = q / BS, i = q - j * BS;
          if (ke >= 0 && ke < BS) cc[pidx(i, j, ke)] = yo[q];
          if (ko >= 0 && ko < BS)
            cc[pidx(i, j, ko)] = w0 * yr[(mm + 1) & 3][q] + w1 * yr[(mm + 2) & 3][q] +
                                 w1 * yr[(mm + 3) & 3][q] + w0 * yo[q];
        }
      }
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
// blocks without penalization
// --------------------------------------------------------------------------
// Two kernels: pen_flags marks each active block (1: far, 0: not), one
// thread per block; pen_compact, one workgroup of 1024 threads, writes
// list = the far blocks (active order), then the others, and cnt = {far
// count, other count}: each thread takes a contiguous run of flags, counts,
// and places its blocks after a workgroup prefix sum of the counts, so that
// each part keeps the active (Morton) order.  With t_dev given, the plate is
// classified for the pitch angles of the window [t, t + dt] of one step;
// else for every angle.
__global__ __launch_bounds__(NT_GEN) void pen_flags(const Tab* __restrict__ tab, int64_t nb,
                                                    wacm_params p, double L, int bs,
                                                    const double* __restrict__ t_dev,
                                                    const double* __restrict__ dt_dev,
                                                    int8_t* __restrict__ flag) {
  const int64_t b = (int64_t)blockIdx.x * NT_GEN + threadIdx.x;
  if (b >= nb) return;
  PitchWindow win{1.0, 0.0, 0.0, false};
  if (t_dev) win = pitch_window(p, *t_dev, *t_dev + *dt_dev);
  flag[b] = pen_far(p, L, bs, tab[b].meta, win) ? 1 : 0;
}

__global__ __launch_bounds__(1024) void pen_compact(const int8_t* __restrict__ flag, int64_t nb,
                                                    int32_t* __restrict__ list,
                                                    int32_t* __restrict__ cnt) {
  __shared__ int32_t wsum[2][16], woff[2][16], tot;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t per = (nb + 1023) / 1024;
  const int64_t b0 = t * per < nb ? t * per : nb, b1 = b0 + per < nb ? b0 + per : nb;
  int32_t nf = 0;
  for (int64_t b = b0; b < b1; ++b) nf += flag[b];
  const int32_t nn = (int32_t)(b1 - b0) - nf;
  // inclusive scans within the wave, then over the 16 waves' totals
  int32_t sf = nf, sn = nn;
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t xf = __shfl_up(sf, o), xn = __shfl_up(sn, o);
    if (lane >= o) {
      sf += xf;
      sn += xn;
    }
  }
  if (lane == 63) {
    wsum[0][wv] = sf;
    wsum[1][wv] = sn;
  }
  __syncthreads();
  if (t == 0) {
    int32_t af = 0, an = 0;
    for (int w = 0; w < 16; ++w) {
      woff[0][w] = af;
      woff[1][w] = an;
      af += wsum[0][w];
      an += wsum[1][w];
    }
    tot = af;
    cnt[0] = af;
    cnt[1] = an;
  }
  __syncthreads();
  int32_t of = woff[0][wv] + sf - nf, on = tot + woff[1][wv] + sn - nn;
  for (int64_t b = b0; b < b1; ++b) {
    if (flag[b])
      list[of++] = (int32_t)b;
    else
      list[on++] = (int32_t)b;
  }
}

// the two lists of blocks with and without penalization, in list/cnt
static hipError_t pen_classify(const wacm_grid* g, const wacm_params* p, const double* t_dev,
                               const double* dt_dev, int32_t* list, int32_t* cnt,
                               int8_t* flag, hipStream_t st) {
  const unsigned nwg = (unsigned)((g->nb + NT_GEN - 1) / NT_GEN);
  if (nwg > 0) {
    pen_flags<<<nwg, NT_GEN, 0, st>>>(g->d_tab, g->nb, *p, g->d.L, g->d.bs, t_dev, dt_dev, flag);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  pen_compact<<<1, 1024, 0, st>>>(flag, g->nb, list, cnt);
  return hipGetLastError();
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

// the stage inputs between stages: compact, x-split
static Layout split_layout(const wacm_grid* g) {
  Layout L = compact_layout(g);
  L.xs = 1;
  return L;
}

static unsigned grid_for(int64_t n, int per_cu) {
  int64_t cap = (int64_t)num_cus() * per_cu;
  return (unsigned)(n < cap ? (n > 0 ? n : 1) : cap);
}

// The face-halo kernel follows the stage kernel's XCD mapping: with xcd_map
// 2 it takes its faces from the second set of work counters.
template <typename T>
static hipError_t nlface_launch(const wacm_grid* g, const T* in, const Layout& Lin, T* hb,
                                hipStream_t st) {
  const unsigned grid = grid_for(g->n_cface, 8);
  int* q = g->sched.xcd_map == 2 ? g->d_queue + 8 * QSTRIDE : nullptr;
  if (q) {
    queue_clear<<<1, 8 * QSTRIDE, 0, st>>>(q);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  switch (g->d.bs) {
    case 16:
      nlface_kernel<T, 16><<<grid, NT_GEN, 0, st>>>(g->d_tab, g->d_cface, g->n_cface, in, Lin, hb, q);
      break;
    case 24:
      nlface_kernel<T, 24><<<grid, NT_GEN, 0, st>>>(g->d_tab, g->d_cface, g->n_cface, in, Lin, hb, q);
      break;
    case 32:
      nlface_kernel<T, 32><<<grid, NT_GEN, 0, st>>>(g->d_tab, g->d_cface, g->n_cface, in, Lin, hb, q);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

// work buffer: acc, ping, pong (compact, bs^3 per field) and the coarse-face
// halo buffer (6 faces x 4 fields x 3 x bs^2 per slot), 256-byte aligned parts
struct WorkParts {
  size_t acc, ping, pong, uc, hb, total;
};
static WorkParts work_parts(const wacm_grid* g) {
  const size_t es = g->d.dtype == WACM_F64 ? 8 : 4;
  const size_t cap = (size_t)g->d.capacity;
  const size_t b3 = (size_t)g->d.bs * g->d.bs * g->d.bs, b2 = (size_t)g->d.bs * g->d.bs;
  auto up = [](size_t v) { return (v + 255) / 256 * 256; };
  WorkParts w;
  w.acc = 0;
  w.ping = up(cap * 4 * b3 * es);
  w.pong = w.ping + up(cap * 4 * b3 * es);
  w.uc = w.pong + up(cap * 4 * b3 * es);
  w.hb = w.uc + up(cap * 4 * b3 * es);
  w.total = w.hb + up(cap * 6 * 4 * 3 * b2 * es);
  return w;
}

size_t work_bytes(const wacm_grid* g) { return work_parts(g).total; }

template <typename T, int BS>
static void sync_coarser_launch(const wacm_grid* g, T* U, hipStream_t st) {
  sync_coarser_kernel<T, BS><<<grid_for(g->n_cregion, 8), NT_GEN, 0, st>>>(
      g->d_tab, g->d_cregion, g->n_cregion, U, pool_layout(g));
}

// Full ghost fill (mode 0): point-wise for same-level and finer regions, and
// the separable region kernel for regions in a coarser leaf; the face star
// (mode 1) point-wise.
template <typename T>
static hipError_t sync_t(const wacm_grid* g, T* U, int mode, hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  const bool split = mode == 0 && g->d.ng <= SC_MAXG && g->n_cregion > 0;
  sync_kernel<T><<<grid_for(g->nb, 8), NT_GEN, 0, st>>>(g->d_tab, g->nb, U, pool_layout(g),
                                                        g->d.bs, mode, split ? 1 : 0, nullptr);
  if (split) {
    switch (g->d.bs) {
      case 16:
        sync_coarser_launch<T, 16>(g, U, st);
        break;
      case 24:
        sync_coarser_launch<T, 24>(g, U, st);
        break;
      case 32:
        sync_coarser_launch<T, 32>(g, U, st);
        break;
      default:
        return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

template <typename T>
static hipError_t sync_lattice_t(const wacm_grid* g, T* U, hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  const unsigned grid = grid_for(g->nb, 8);
  const Layout L = pool_layout(g);
  switch (g->d.bs) {
    case 16:
      sync_lattice_kernel<T, 16><<<grid, NT_GEN, 0, st>>>(g->d_tab, g->nb, U, L);
      break;
    case 24:
      sync_lattice_kernel<T, 24><<<grid, NT_GEN, 0, st>>>(g->d_tab, g->nb, U, L);
      break;
    case 32:
      sync_lattice_kernel<T, 32><<<grid, NT_GEN, 0, st>>>(g->d_tab, g->nb, U, L);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_sync_lattice(const wacm_grid* g, void* U, hipStream_t st) {
  return g->d.dtype == WACM_F64 ? sync_lattice_t(g, (double*)U, st)
                                : sync_lattice_t(g, (float*)U, st);
}

// The CDF 4/0 phase of a lifted stage's sync: the read boxes of regions in a
// finer leaf (what the face-star lifted values read there from a block's
// padded array) and every region in a coarser leaf (whole, by the region
// kernel); the stage and the lifted values read same-level values in place,
// and the lifted phase writes the finer face halos.
template <typename T>
static hipError_t sync_lifted_stage_t(const wacm_grid* g, T* U, const int32_t* box,
                                      hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  if (g->d.ng > SC_MAXG || !box) return sync_t(g, U, 0, st);
  const bool split = g->n_cregion > 0;
  sync_kernel<T><<<grid_for(g->nb, 8), NT_GEN, 0, st>>>(g->d_tab, g->nb, U, pool_layout(g),
                                                        g->d.bs, 0, split ? 1 : 0, box);
  if (split) {
    switch (g->d.bs) {
      case 16:
        sync_coarser_launch<T, 16>(g, U, st);
        break;
      case 24:
        sync_coarser_launch<T, 24>(g, U, st);
        break;
      case 32:
        sync_coarser_launch<T, 32>(g, U, st);
        break;
      default:
        return hipErrorInvalidValue;
    }
  }
  return hipGetLastError();
}

hipError_t launch_sync_lifted_stage(const wacm_grid* g, void* U, const int32_t* box,
                                    hipStream_t st) {
  return g->d.dtype == WACM_F64 ? sync_lifted_stage_t(g, (double*)U, box, st)
                                : sync_lifted_stage_t(g, (float*)U, box, st);
}

hipError_t launch_sync(const wacm_grid* g, void* U, int face_only, hipStream_t st) {
  return g->d.dtype == WACM_F64 ? sync_t(g, (double*)U, face_only ? 1 : 0, st)
                                : sync_t(g, (float*)U, face_only ? 1 : 0, st);
}

// resident workgroups per CU of a kernel (queried once per instantiation)
template <typename K>
static int resident_per_cu(K kernel, int threads) {
  int n = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, threads, 0) != hipSuccess || n < 1)
    n = 1;
  return n;
}

template <typename T, int BS, int TY, int MODE, bool PEN, bool PREF>
static hipError_t stage_launch_t(const StageArgs<T>& a, int wg_per_cu, hipStream_t st) {
  static const int resident =
      resident_per_cu(stage_kernel<T, BS, TY, MODE, PEN, PREF>, BS * TY);
  const int per_cu = wg_per_cu > 0 ? wg_per_cu : resident;
  const int64_t items = a.nb * (BS / TY);
  int64_t grid = (int64_t)per_cu * num_cus();
  if (grid > items) grid = items;
  if (grid < 1) grid = 1;
  if (a.queue) {
    queue_clear<<<1, 8 * QSTRIDE, 0, st>>>(a.queue);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  stage_kernel<T, BS, TY, MODE, PEN, PREF><<<(unsigned)grid, BS * TY, 0, st>>>(a);
  return hipGetLastError();
}

// tile_rows 0: whole-block work items; 8: tiles of 8 rows (bs >= 24, where the
// halo of a tile plane fits in one point per thread; smaller blocks use whole
// blocks)
template <typename T, int BS, int MODE, bool PEN, bool PREF>
static hipError_t stage_launch_pp(const StageArgs<T>& a, const wacm_schedule& s,
                                  hipStream_t st) {
  if constexpr (BS >= 24) {
    if (s.tile_rows == 8) return stage_launch_t<T, BS, 8, MODE, PEN, PREF>(a, s.wg_per_cu, st);
  }
  return stage_launch_t<T, BS, BS, MODE, PEN, PREF>(a, s.wg_per_cu, st);
}

// Schedule knobs: prefetch = 1 issues the epilogue loads before the plane's
// barrier (more bytes in flight, more registers), 0 after the rhs; -1 picks
// the default (early for FP32, late for FP64, whose 9-wave workgroup is at
// its VGPR limit).
template <typename T, int BS, int MODE>
static hipError_t stage_launch(const StageArgs<T>& a, const wacm_schedule& s, hipStream_t st) {
  const bool pen = a.p.mask || a.p.sponge || a.dus;
  const bool pref = s.prefetch < 0 ? sizeof(T) == 4 : s.prefetch != 0;
  if (pen && a.blist) {
    // the blocks where the penalization vanishes take the unpenalized
    // variant, the others the penalized one
    StageArgs<T> f = a, n = a;
    f.bsel = 0;
    n.bsel = 1;
    hipError_t e = pref ? stage_launch_pp<T, BS, MODE, false, true>(f, s, st)
                        : stage_launch_pp<T, BS, MODE, false, false>(f, s, st);
    if (e != hipSuccess) return e;
    return pref ? stage_launch_pp<T, BS, MODE, true, true>(n, s, st)
                : stage_launch_pp<T, BS, MODE, true, false>(n, s, st);
  }
  if (pen)
    return pref ? stage_launch_pp<T, BS, MODE, true, true>(a, s, st)
                : stage_launch_pp<T, BS, MODE, true, false>(a, s, st);
  return pref ? stage_launch_pp<T, BS, MODE, false, true>(a, s, st)
              : stage_launch_pp<T, BS, MODE, false, false>(a, s, st);
}

template <typename T, int MODE>
static hipError_t stage_dispatch(int bs, const StageArgs<T>& a, const wacm_schedule& s,
                                 hipStream_t st) {
  switch (bs) {
    case 16:
      return stage_launch<T, 16, MODE>(a, s, st);
    case 24:
      return stage_launch<T, 24, MODE>(a, s, st);
    case 32:
      return stage_launch<T, 32, MODE>(a, s, st);
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
  a.xcd_map = g->sched.xcd_map;
  a.queue = g->sched.xcd_map == 2 ? g->d_queue : nullptr;
  a.nt = g->sched.nontemporal;
  a.p = *p;
  return a;
}

// One RK stage s (1..4) of the fused kernel for the lifted-wavelet step:
// input, U^n and output in the padded pool layout, the accumulator compact
// (bs^3 values per field, from the start of its padded-size register); same-level
// halos from the neighbours' interiors, the halos of faces next to another
// level from the input's own ghost layers (filled before each stage), no
// face-halo buffer.  Tiles of 8 rows; early epilogue loads for FP32.
template <typename T, int BS, int S>
static hipError_t stage_owng_bs(const StageArgs<T>& a, int wg_per_cu, hipStream_t st) {
  constexpr bool PREF = sizeof(T) == 4;
  return a.p.mask || a.p.sponge || a.dus
             ? stage_launch_t<T, BS, 8, 10 + S, true, PREF>(a, wg_per_cu, st)
             : stage_launch_t<T, BS, 8, 10 + S, false, PREF>(a, wg_per_cu, st);
}

template <typename T>
static hipError_t stage_owng_t(const wacm_grid* g, const wacm_params* p, int s,
                               const double* t_dev, const double* dt_dev, const T* in, T* un,
                               T* out, T* acc, const T* dus, hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  StageArgs<T> a = base_args<T>(g, p);
  const Layout L = pool_layout(g);
  a.in = in;
  a.Lin = L;
  a.un = un;
  a.Lun = L;
  a.out = out;
  a.Lout = L;
  // the accumulator is never synchronised: compact, [c][z][y][x]
  a.acc = acc;
  a.Lacc.P = g->d.bs;
  a.Lacc.ng = 0;
  a.Lacc.fstride = (int64_t)g->d.bs * g->d.bs * g->d.bs;
  a.Lacc.bstride = 4 * a.Lacc.fstride;
  a.Lacc.xs = 0;
  a.dus = dus;
  a.t_dev = t_dev;
  a.dt_dev = dt_dev;
  const int w = g->sched.wg_per_cu;
  switch (g->d.bs * 10 + s) {
    case 241: return stage_owng_bs<T, 24, 1>(a, w, st);
    case 242: return stage_owng_bs<T, 24, 2>(a, w, st);
    case 243: return stage_owng_bs<T, 24, 3>(a, w, st);
    case 244: return stage_owng_bs<T, 24, 4>(a, w, st);
    case 321: return stage_owng_bs<T, 32, 1>(a, w, st);
    case 322: return stage_owng_bs<T, 32, 2>(a, w, st);
    case 323: return stage_owng_bs<T, 32, 3>(a, w, st);
    case 324: return stage_owng_bs<T, 32, 4>(a, w, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_stage_owng(const wacm_grid* g, const wacm_params* p, int s,
                             const double* t_dev, const double* dt_dev, const void* in, void* un,
                             void* out, void* acc, const void* dus, hipStream_t st) {
  return g->d.dtype == WACM_F64
             ? stage_owng_t(g, p, s, t_dev, dt_dev, (const double*)in, (double*)un,
                            (double*)out, (double*)acc, (const double*)dus, st)
             : stage_owng_t(g, p, s, t_dev, dt_dev, (const float*)in, (float*)un, (float*)out,
                            (float*)acc, (const float*)dus, st);
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
  a.un = dU;
  a.Lun = pool_layout(g);
  a.acc = dU;
  a.Lacc = pool_layout(g);
  a.dus = dus;
  a.t_host = t;
  return stage_dispatch<T, 0>(g->d.bs, a, g->sched, st);
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
  const unsigned grid = grid_for(g->nb, 8);
  switch (g->d.bs) {
    case 16:
      maxu_kernel<T, 16><<<grid, NT_GEN, 0, st>>>(g->d_tab, g->nb, U, pool_layout(g), g->d_part);
      break;
    case 24:
      maxu_kernel<T, 24><<<grid, NT_GEN, 0, st>>>(g->d_tab, g->nb, U, pool_layout(g), g->d_part);
      break;
    case 32:
      maxu_kernel<T, 32><<<grid, NT_GEN, 0, st>>>(g->d_tab, g->nb, U, pool_layout(g), g->d_part);
      break;
    default:
      return hipErrorInvalidValue;
  }
  const double hmin = g->d.L / (double(int64_t(1) << g->jfine) * g->d.bs);
  dt_finalize<<<1, NT_GEN, 0, st>>>(g->d_part, g->nb, *p, hmin, dt_dev);
  return hipGetLastError();
}

hipError_t launch_dt(const wacm_grid* g, const wacm_params* p, const void* U, double* dt_dev,
                     hipStream_t st) {
  return g->d.dtype == WACM_F64 ? dt_t(g, p, (const double*)U, dt_dev, st)
                                : dt_t(g, p, (const float*)U, dt_dev, st);
}

// stage work items of the current schedule (whole blocks or tiles of 8 rows)
static int64_t stage_items(const wacm_grid* g) {
  const int bs = g->d.bs;
  return g->nb * ((g->sched.tile_rows == 8 && bs >= 24) ? bs / 8 : 1);
}

// nsteps classical RK4 steps.  With the CFL rule, the first step's dt comes
// from a reduction over U; every later step's from the maximum the previous
// step's last stage formed while writing U (the same value, bit for bit).
// Between the steps of one call the state stays in the x-split register uc:
// only the first step reads the pool and only the last one writes it.
// Whether to split the blocks of a penalized stage (schedule pen_split: 0
// never, 2 always, 1 when it pays).  Two launches per stage and their tails
// cost more than the unpenalized kernel saves on small grids: the split
// needs at least 2048 active blocks, and, for a static mask or sponge, at
// least 512 blocks without penalization (counted here from the host copy of
// the tables).  A pitching plate's per-step lists leave only the blocks near
// the plate penalized, so its grids need only the size.
static bool pen_split_pays(const wacm_grid* g, const wacm_params* p) {
  if (g->sched.pen_split != 1) return g->sched.pen_split == 2;
  if (g->nb < 2048) return false;
  if (p->mask == WACM_MASK_PLATE) return true;
  const PitchWindow any{1.0, 0.0, 0.0, false};
  int64_t nfar = 0;
  for (int64_t b = 0; b < g->nb && nfar < 512; ++b)
    nfar += pen_far(*p, g->d.L, g->d.bs, g->h_tab[b].meta, any) ? 1 : 0;
  return nfar >= 512;
}

template <typename T>
static hipError_t rk4_t(const wacm_grid* g, const wacm_params* p, double* t_dev, double* dt_dev,
                        T* U, void* work, const T* dus, int dt_mode, int64_t nsteps,
                        hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  hipError_t e;
  const WorkParts wp = work_parts(g);
  char* w = (char*)work;
  T* acc = (T*)(w + wp.acc);
  T* ping = (T*)(w + wp.ping);
  T* pong = (T*)(w + wp.pong);
  T* uc = (T*)(w + wp.uc);
  T* hb = (T*)(w + wp.hb);
  StageArgs<T> a = base_args<T>(g, p);
  a.acc = acc;
  a.Lacc = compact_layout(g);
  a.hb = hb;
  a.dus = dus;
  a.t_dev = t_dev;
  a.dt_dev = dt_dev;
  const Layout Lp = pool_layout(g), Ls = split_layout(g);
  T* ins[4] = {U, ping, pong, ping};
  T* outs[4] = {ping, pong, ping, U};
  Layout lins[4] = {Lp, Ls, Ls, Ls};
  const double hmin = g->d.L / (double(int64_t(1) << g->jfine) * g->d.bs);
  const int64_t items = stage_items(g);
  // blocks without penalization first (the adaptation lists are free
  // during a step: capacity entries of the list, then the 2 counts); a
  // pitching plate is classified per step, for the angles of that step
  const bool split = (p->mask || p->sponge || dus) && pen_split_pays(g, p);
  const bool split_step = split && p->mask == WACM_MASK_PLATE;
  int32_t* const plist = g->d_list;
  int32_t* const pcnt = g->d_list + g->d.capacity;
  int8_t* const pflag = reinterpret_cast<int8_t*>(g->d_list + g->d.capacity + 2);
  if (split) {
    a.blist = plist;
    a.bcnt = pcnt;
  }
  if (split && !split_step &&
      (e = pen_classify(g, p, nullptr, nullptr, plist, pcnt, pflag, st)) != hipSuccess)
    return e;
  for (int64_t k = 0; k < nsteps; ++k) {
    if (dt_mode == WACM_DT_CFL) {
      ProfScope ps(g, 0, st);
      if (k == 0) {
        if ((e = dt_t<T>(g, p, U, dt_dev, st)) != hipSuccess) return e;
      } else {
        dt_finalize<<<1, NT_GEN, 0, st>>>(g->d_part, items, *p, hmin, dt_dev);
        if ((e = hipGetLastError()) != hipSuccess) return e;
      }
    }
    // U^n of this step and U^{n+1}: the pool at the ends of the call, uc between
    T* un = k == 0 ? U : uc;
    const Layout Lun = k == 0 ? Lp : Ls;
    T* unext = k + 1 == nsteps ? U : uc;
    const Layout Lnext = k + 1 == nsteps ? Lp : Ls;
    ins[0] = un;
    lins[0] = Lun;
    for (int s = 0; s < 4; ++s) {
      a.in = ins[s];
      a.Lin = lins[s];
      a.out = s == 3 ? unext : outs[s];
      a.Lout = s == 3 ? Lnext : Ls;
      a.un = s == 3 ? unext : un;
      a.Lun = s == 3 ? Lnext : Lun;
      a.umax_part = (s == 3 && dt_mode == WACM_DT_CFL && k + 1 < nsteps) ? g->d_part : nullptr;
      if (g->n_cface > 0) {
        ProfScope ps(g, 1, st);
        if ((e = nlface_launch<T>(g, a.in, a.Lin, hb, st)) != hipSuccess) return e;
      }
      ProfScope ps(g, 2, st);
      if (s == 0 && split_step &&
          (e = pen_classify(g, p, t_dev, dt_dev, plist, pcnt, pflag, st)) != hipSuccess)
        return e;
      switch (s) {
        case 0:
          e = stage_dispatch<T, 1>(g->d.bs, a, g->sched, st);
          break;
        case 1:
          e = stage_dispatch<T, 2>(g->d.bs, a, g->sched, st);
          break;
        case 2:
          e = stage_dispatch<T, 3>(g->d.bs, a, g->sched, st);
          break;
        default:
          e = stage_dispatch<T, 4>(g->d.bs, a, g->sched, st);
          break;
      }
      if (e != hipSuccess) return e;
    }
    ProfScope ps(g, 3, st);
    advance_time<<<1, 64, 0, st>>>(t_dev, dt_dev);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_rk4(const wacm_grid* g, const wacm_params* p, double* t_dev, double* dt_dev,
                      void* U, void* work, const void* dus, int dt_mode, int64_t nsteps,
                      hipStream_t st) {
  return g->d.dtype == WACM_F64 ? rk4_t(g, p, t_dev, dt_dev, (double*)U, work,
                                        (const double*)dus, dt_mode, nsteps, st)
                                : rk4_t(g, p, t_dev, dt_dev, (float*)U, work, (const float*)dus,
                                        dt_mode, nsteps, st);
}

template <typename T>
static hipError_t diag_t(const wacm_grid* g, const wacm_params* p, double t, const T* U,
                         const T* dus, double* out, hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  const unsigned grid = grid_for(g->nb, 8);
  const Layout L = pool_layout(g);
  switch (g->d.bs) {
    case 16:
      diag_kernel<T, 16><<<grid, NT_GEN, 0, st>>>(g->d_tab, g->nb, U, L, dus, g->d.L, *p, t,
                                                   g->d_part);
      break;
    case 24:
      diag_kernel<T, 24><<<grid, NT_GEN, 0, st>>>(g->d_tab, g->nb, U, L, dus, g->d.L, *p, t,
                                                   g->d_part);
      break;
    case 32:
      diag_kernel<T, 32><<<grid, NT_GEN, 0, st>>>(g->d_tab, g->nb, U, L, dus, g->d.L, *p, t,
                                                   g->d_part);
      break;
    default:
      return hipErrorInvalidValue;
  }
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
  const Layout L = pool_layout(g);
  switch (g->d.bs) {
#define WACM_DETAIL(BSV)                                                                    \
  case BSV:                                                                                 \
    detail_kernel<T, BSV><<<(unsigned)g->nb, BSV * BSV, 0, st>>>(g->d_tab, g->nb, U, L,    \
                                                                  g->d.L, *p, t, g->d_part, \
                                                                  mrange);                  \
    break;
    WACM_DETAIL(16)
    WACM_DETAIL(24)
    WACM_DETAIL(32)
#undef WACM_DETAIL
    default:
      return hipErrorInvalidValue;
  }
  if (hipError_t e = hipGetLastError(); e != hipSuccess) return e;
  thr_finalize<<<1, 1024, 0, st>>>(g->d_tab, g->nb, g->d_part, mrange, eps, dealias, g->d.jmin,
                                   g->d.jmax, g->d_norm, dmax, flags);
  return hipGetLastError();
}

hipError_t launch_threshold(const wacm_grid* g, const wacm_params* p, double t, const void* U,
                            double eps, int dealias, double* dmax, double* mrange,
                            int8_t* flags, hipStream_t st) {
  return g->d.dtype == WACM_F64
             ? thr_t(g, p, t, (const double*)U, eps, dealias, dmax, mrange, flags, st)
             : thr_t(g, p, t, (const float*)U, eps, dealias, dmax, mrange, flags, st);
}

template <typename T>
static hipError_t filter_t(const wacm_grid* g, T* U, int level, hipStream_t st) {
  if (g->nb == 0) return hipSuccess;
  const unsigned grid = grid_for(g->nb, 8);
  const Layout L = pool_layout(g);
  switch (g->d.bs) {
    case 16:
      filter_kernel<T, 16><<<grid, NT_GEN, 0, st>>>(g->d_tab, g->nb, U, L, level);
      break;
    case 24:
      filter_kernel<T, 24><<<grid, NT_GEN, 0, st>>>(g->d_tab, g->nb, U, L, level);
      break;
    case 32:
      filter_kernel<T, 32><<<grid, NT_GEN, 0, st>>>(g->d_tab, g->nb, U, L, level);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_filter(const wacm_grid* g, void* U, int level, hipStream_t st) {
  return g->d.dtype == WACM_F64 ? filter_t(g, (double*)U, level, st)
                                : filter_t(g, (float*)U, level, st);
}

template <typename T>
static hipError_t prolong_t(const wacm_grid* g, T* U, int64_t n, hipStream_t st) {
  const unsigned grid = grid_for(n, 8);
  switch (g->d.bs) {
    case 16:
      prolong_kernel<T, 16><<<grid, NT_GEN, 0, st>>>(g->d_list, n, U, pool_layout(g));
      break;
    case 24:
      prolong_kernel<T, 24><<<grid, NT_GEN, 0, st>>>(g->d_list, n, U, pool_layout(g));
      break;
    case 32:
      prolong_kernel<T, 32><<<grid, NT_GEN, 0, st>>>(g->d_list, n, U, pool_layout(g));
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_prolong(const wacm_grid* g, void* U, int64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  return g->d.dtype == WACM_F64 ? prolong_t(g, (double*)U, n, st)
                                : prolong_t(g, (float*)U, n, st);
}

// reductions shared with the two-dimensional path (kernels2d.hip)
hipError_t finalize_dt(const double* part, int64_t n, const wacm_params& p, double hmin,
                       double* dt_dev, hipStream_t st) {
  dt_finalize<<<1, NT_GEN, 0, st>>>(part, n, p, hmin, dt_dev);
  return hipGetLastError();
}
hipError_t finalize_diag(const double* part, int64_t n, double* out, hipStream_t st) {
  diag_finalize<<<1, NT_GEN, 0, st>>>(part, n, out);
  return hipGetLastError();
}
hipError_t finalize_norm(const double* part, int64_t n, double* norm, hipStream_t st) {
  norm_finalize<<<1, NT_GEN, 0, st>>>(part, n, norm);
  return hipGetLastError();
}
hipError_t add_dt_to_time(double* t_dev, const double* dt_dev, hipStream_t st) {
  advance_time<<<1, 64, 0, st>>>(t_dev, dt_dev);
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
