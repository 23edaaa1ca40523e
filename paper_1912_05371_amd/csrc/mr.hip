// Multiresolution transform (Sec. 3.1 details iterated from the finest level
// down; Sec. 3.2 lifted coarse values) of periodic fields on the equidistant
// lattice, in place, on the device.
//
// Fields: nf arrays of n^3 values, x fastest.  Step m works on the lattice of
// stride s = 2^m; its points with all coordinates multiples of 2s are even,
// the others odd.  Forward step: every odd point takes its detail, the value
// minus the tensor DD4 prediction from the even points; with CDF 4/4 every
// even point then takes its lifted restriction, written as c = e + L(delta):
// L the lifted low-pass with decimation (13 taps per axis, x, y, z), delta
// the stride-s lattice with the details at the odd points and zeros at the
// even ones (L returns e when applied to e extended by prediction, and it is
// linear).  The inverse undoes the steps in reverse: e = c - L(delta), then
// odd = detail + prediction.  A prediction changes only odd points from
// even ones (the even half of the pairs it stores is the unchanged value),
// the update only even points from odd ones, so both run in place without
// hazards.
//
// Kernels per step: mr_predict_kernel (the 7 odd points of each coarse cell
// from its 4^3 even neighbours, interpolated along x, y, then z, marching
// along z) and, for CDF 4/4, three separable low-pass passes through a work
// buffer (x into tx, y into ty, z added into the even points).
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "wacm_internal.h"

namespace wacm {
namespace mr {

constexpr int MR_NT = 256;

// DD4 prediction weights at the odd offsets -3, -1, 1, 3 (in fine points)
__device__ constexpr double MR_DD4[4] = {-1.0 / 16, 9.0 / 16, 9.0 / 16, -1.0 / 16};
// Expanded lifted low-pass, offsets -6..6 (zero at +-5): update (-1, 9, 9,
// -1)/32 on the DD4 details of the offsets -3, -1, 1, 3.
__device__ constexpr double MR_LIFT[13] = {-1.0 / 512,  0.0,         18.0 / 512,  -16.0 / 512,
                                          -63.0 / 512, 144.0 / 512, 348.0 / 512, 144.0 / 512,
                                          -63.0 / 512, -16.0 / 512, 18.0 / 512,  0.0,
                                          -1.0 / 512};

// Workgroups are dispatched to the 8 XCDs round-robin in linear order, each
// XCD with its own L2.  Renumber them so that every XCD runs one contiguous
// range of the logical order (neighbouring (X, Y) columns, which share even
// rows, then meet in one L2).  Returns the logical linear index.
__device__ inline uint32_t xcd_contiguous(uint32_t l, uint32_t G) {
  const uint32_t x = l % 8, q = G / 8, r = G % 8;
  return (x < r ? x * (q + 1) : r * (q + 1) + (x - r) * q) + l / 8;
}

// Odd points of the stride-s lattice: u += sign * P(even).  Cell (X, Y, Z)
// of the stride-2s lattice (nc per axis) owns the odd points (2X + a, 2Y + b,
// 2Z + c) s, (a, b, c) in {0,1}^3 minus (0,0,0).  One thread per (X, Y) and
// run of lz cells along Z (field from the workgroup): per coarse plane the
// thread loads the even points (X, Y - 1 .. Y + 2) and takes those at X - 1,
// X + 1 and X + 2 from the lanes that loaded them (consecutive lanes hold
// consecutive X of one row; a lane whose neighbour is in another wave or row
// loads it itself), interpolates along x then y (the four (a, b) types of
// the plane) and keeps the last 4 planes in registers for the z
// interpolation.  The odd points are updated as (even, odd) pairs along x,
// 16-byte accesses at stride 1; the even half is stored back unchanged.
template <typename T>
struct Pair {
  T e, o;
};

template <typename T>
__device__ inline Pair<T> load_pair(const T* p, int s) {
  if (s == 1) {
    using V = HIP_vector_type<T, 2>;
    const V v = *reinterpret_cast<const V*>(p);
    return {v.x, v.y};
  }
  return {p[0], p[s]};
}

template <typename T>
__device__ inline void store_pair(T* p, int s, Pair<T> v) {
  if (s == 1) {
    using V = HIP_vector_type<T, 2>;
    *reinterpret_cast<V*>(p) = V(v.e, v.o);
  } else {
    p[0] = v.e;
    p[s] = v.o;
  }
}

template <typename T>
__device__ inline T dd4(T a0, T a1, T a2, T a3) {
  return T(MR_DD4[0]) * a0 + T(MR_DD4[1]) * a1 + T(MR_DD4[2]) * a2 + T(MR_DD4[3]) * a3;
}

template <typename T>
__global__ __launch_bounds__(MR_NT) void mr_predict_kernel(T* __restrict__ u, int64_t n, int s,
                                                           uint32_t nc, uint32_t lz, T sign) {
  const uint32_t nrun = (nc + lz - 1) / lz, total = nc * nc * nrun;
  const uint32_t lb = xcd_contiguous(blockIdx.y * gridDim.x + blockIdx.x, gridDim.x * gridDim.y);
  const uint32_t field = lb / gridDim.x;
  const uint32_t t0 = (lb % gridDim.x) * MR_NT + threadIdx.x;
  // threads past the end repeat the last valid one's loads (they take part
  // in the shuffles) but store nothing
  const bool valid = t0 < total;
  const uint32_t t = valid ? t0 : total - 1;
  const int lane = (int)(threadIdx.x & 63);
  T* f = u + (int64_t)field * n * n * n;
  const uint32_t X = t % nc, Y = (t / nc) % nc, R = t / (nc * nc);
  const uint32_t Z0 = R * lz, Z1 = min(Z0 + lz, nc);
  // the lane holding X - 1 / X + 1 / X + 2 of the same row, if any
  const bool sh0 = lane >= 1 && X >= 1;
  const bool sh2 = lane + 1 < 64 && X + 1 < nc && t0 + 1 < total;
  const bool sh3 = lane + 2 < 64 && X + 2 < nc && t0 + 2 < total;
  const int64_t s2 = 2 * (int64_t)s, pz = s2 * n * n;
  const int64_t x0 = (int64_t)((X + nc - 1) % nc) * s2, x1 = (int64_t)X * s2,
                x2 = (int64_t)((X + 1) % nc) * s2, x3 = (int64_t)((X + 2) % nc) * s2;
  int64_t yo[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) yo[q] = (int64_t)((Y + nc - 1 + q) % nc) * s2 * n;
  // x then y interpolation of one coarse plane: v[a + 2b], (a, b) = the
  // parities along x and y
  auto plane = [&](const T* pl, T(&v)[4]) {
    T ex[4], ox[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const T* row = pl + yo[j];
      const T a1 = row[x1];
      T a0 = __shfl(a1, lane - 1 < 0 ? 0 : lane - 1, 64);
      T a2 = __shfl(a1, lane + 1 > 63 ? 63 : lane + 1, 64);
      T a3 = __shfl(a1, lane + 2 > 63 ? 63 : lane + 2, 64);
      if (!sh0) a0 = row[x0];
      if (!sh2) a2 = row[x2];
      if (!sh3) a3 = row[x3];
      ex[j] = a1;
      ox[j] = dd4(a0, a1, a2, a3);
    }
    v[0] = ex[1];
    v[1] = ox[1];
    v[2] = dd4(ex[0], ex[1], ex[2], ex[3]);
    v[3] = dd4(ox[0], ox[1], ox[2], ox[3]);
  };
  T p0[4], p1[4], p2[4], p3[4];  // planes Z-1, Z, Z+1, Z+2
  plane(f + (int64_t)((Z0 + nc - 1) % nc) * pz, p0);
  plane(f + (int64_t)Z0 * pz, p1);
  plane(f + (int64_t)((Z0 + 1) % nc) * pz, p2);
  const int64_t sy = (int64_t)s * n, sz = (int64_t)s * n * n;
  for (uint32_t Z = Z0; Z < Z1; ++Z) {
    plane(f + (int64_t)((Z + 2) % nc) * pz, p3);
    T q[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) q[k] = dd4(p0[k], p1[k], p2[k], p3[k]);
    if (valid) {
      T* base = f + (int64_t)Z * pz + (int64_t)Y * s2 * n + x1;
      Pair<T> r0 = load_pair(base, s), r1 = load_pair(base + sy, s);
      Pair<T> r2 = load_pair(base + sz, s), r3 = load_pair(base + sz + sy, s);
      r0.o += sign * p1[1];
      r1.e += sign * p1[2];
      r1.o += sign * p1[3];
      r2.e += sign * q[0];
      r2.o += sign * q[1];
      r3.e += sign * q[2];
      r3.o += sign * q[3];
      store_pair(base, s, r0);
      store_pair(base + sy, s, r1);
      store_pair(base + sz, s, r2);
      store_pair(base + sz + sy, s, r3);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      p0[k] = p1[k];
      p1[k] = p2[k];
      p2[k] = p3[k];
    }
  }
}

// Low-pass along x with decimation of delta (the stride-s lattice with its
// even points taken as 0): tx[f][z][y][X] = sum_a h_a delta((2X + a - 6) s,
// y s, z s), X < nc, y, z < m = 2 nc.  A workgroup stages k = MR_XROW / m
// whole rows in LDS, then each output reads its 11 nonzero taps there.
constexpr uint32_t MR_XROW = 2048;
template <typename T>
__global__ __launch_bounds__(MR_NT) void mr_lift_x_kernel(const T* __restrict__ u,
                                                          T* __restrict__ tx, int64_t n, int s,
                                                          uint32_t nc, uint32_t k) {
  __shared__ T row[MR_XROW];
  const uint32_t m = 2 * nc;
  const uint32_t r0 = blockIdx.x * k;  // first row (y + m z) of this workgroup
  const uint32_t nr = min(k, m * m - r0);
  const T* uf = u + (int64_t)blockIdx.y * n * n * n;
  const uint32_t wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  // one row per wave at a time, the lanes along x
  for (uint32_t rr = wave; rr < nr; rr += MR_NT / 64) {
    const uint32_t r = r0 + rr, y = r % m, z = r / m;
    const bool even_line = ((y | z) & 1) == 0;
    const T* src = uf + ((int64_t)z * n + y) * n * s;
    for (uint32_t x = lane; x < m; x += 64)
      row[rr * m + x] = even_line && (x & 1) == 0 ? T(0) : src[(int64_t)x * s];
  }
  __syncthreads();
  T* out = tx + ((int64_t)blockIdx.y * m * m + r0) * nc;
  for (uint32_t rr = wave; rr < nr; rr += MR_NT / 64) {
    const T* lr = row + rr * m;
    for (uint32_t X = lane; X < nc; X += 64) {
      T acc = 0;
#pragma unroll
      for (int a = 0; a < 13; ++a) {
        if (a == 1 || a == 11) continue;  // zero taps
        int x = (int)(2 * X) + a - 6;    // |a - 6| <= 6 < m: one wrap at most
        x = x < 0 ? x + (int)m : x >= (int)m ? x - (int)m : x;
        acc += T(MR_LIFT[a]) * lr[x];
      }
      out[(int64_t)rr * nc + X] = acc;
    }
  }
}

// Low-pass with decimation along a column of stride cs (elements) and length
// m: out[j] = sum_b h_b in[(2 j + b - 6) mod m], for the run of outputs j0 ..
// j1 - 1, with a 13-value window that moves by 2 points per output.
template <typename T, typename Store>
__device__ inline void mr_lift_column(const T* __restrict__ col, int64_t cs, uint32_t m,
                                      uint32_t j0, uint32_t j1, Store store) {
  T w[13];
#pragma unroll
  for (int b = 0; b < 13; ++b) w[b] = col[(int64_t)((2 * j0 + m - 6 + b) % m) * cs];
  for (uint32_t j = j0;;) {
    T acc = 0;
#pragma unroll
    for (int b = 0; b < 13; ++b)
      if (b != 1 && b != 11) acc += T(MR_LIFT[b]) * w[b];
    store(j, acc);
    if (++j >= j1) break;
#pragma unroll
    for (int b = 0; b < 11; ++b) w[b] = w[b + 2];
    const uint32_t a = 2 * j + 5, b = a + 1;  // < m + 7: one wrap at most
    w[11] = col[(int64_t)(a >= m ? a - m : a) * cs];
    w[12] = col[(int64_t)(b >= m ? b - m : b) * cs];
  }
}

// Low-pass along y: ty[f][z][Y][X] = sum_b h_b tx[f][z][2Y + b - 6][X]; one
// thread per (X, z) and run of ry outputs along Y.
template <typename T>
__global__ __launch_bounds__(MR_NT) void mr_lift_y_kernel(const T* __restrict__ tx,
                                                          T* __restrict__ ty, uint32_t nc,
                                                          uint32_t ry) {
  const uint32_t m = 2 * nc, nrun = (nc + ry - 1) / ry;
  const uint32_t t = blockIdx.x * MR_NT + threadIdx.x;
  if (t >= nc * m * nrun) return;
  const uint32_t X = t % nc, z = (t / nc) % m, R = t / (nc * m);
  const uint32_t Y0 = R * ry, Y1 = min(Y0 + ry, nc);
  const T* col = tx + ((int64_t)blockIdx.y * m + z) * m * nc + X;
  T* out = ty + ((int64_t)blockIdx.y * m + z) * nc * nc + X;
  mr_lift_column(col, (int64_t)nc, m, Y0, Y1,
                 [&](uint32_t Y, T v) { out[(int64_t)Y * nc] = v; });
}

// Low-pass along z, added to the even points: u((2X, 2Y, 2Z) s) += sign *
// sum_c h_c ty[f][2Z + c - 6][Y][X]; one thread per (X, Y) and run of rz
// outputs along Z.
template <typename T>
__global__ __launch_bounds__(MR_NT) void mr_lift_z_kernel(T* __restrict__ u,
                                                          const T* __restrict__ ty, int64_t n,
                                                          int s, uint32_t nc, uint32_t rz,
                                                          T sign) {
  const uint32_t m = 2 * nc, nrun = (nc + rz - 1) / rz;
  const uint32_t t = blockIdx.x * MR_NT + threadIdx.x;
  if (t >= nc * nc * nrun) return;
  const uint32_t X = t % nc, Y = (t / nc) % nc, R = t / (nc * nc);
  const uint32_t Z0 = R * rz, Z1 = min(Z0 + rz, nc);
  const T* col = ty + (int64_t)blockIdx.y * m * nc * nc + (int64_t)Y * nc + X;
  const int64_t s2 = 2 * (int64_t)s;
  T* dst = u + (int64_t)blockIdx.y * n * n * n + ((int64_t)Y * n + X) * s2;
  const int64_t pz = s2 * n * n;
  mr_lift_column(col, (int64_t)nc * nc, m, Z0, Z1, [&](uint32_t Z, T v) {
    T* d = dst + (int64_t)Z * pz;
    *d = *d + sign * v;
  });
}

unsigned blocks_for(uint64_t n) { return (unsigned)((n + MR_NT - 1) / MR_NT); }

int mr_fail(int code, const std::string& msg) {
  set_error(msg);
  return code;
}

size_t elem_size(int32_t dtype) { return dtype == WACM_F64 ? 8 : dtype == WACM_F32 ? 4 : 0; }

// tx (n^3 / 2 per field) then ty (n^3 / 4 per field), each 256-byte aligned
size_t tx_bytes(int64_t n, int32_t nf, size_t es) {
  return ((size_t)nf * (size_t)(n / 2) * n * n * es + 255) / 256 * 256;
}

size_t work_bytes_of(int64_t n, int32_t nf, size_t es) {
  const size_t ty = ((size_t)nf * (size_t)(n / 2) * (n / 2) * n * es + 255) / 256 * 256;
  return tx_bytes(n, nf, es) + ty;
}

// every argument except the work buffer
int mr_validate_sizes(int64_t n, int32_t nf, int32_t dtype, int32_t wavelet, int32_t nlev,
                      const void* u) {
  if (elem_size(dtype) == 0) return mr_fail(WACM_E_INVAL, "mr: dtype must be WACM_F32 or WACM_F64");
  if (wavelet != WACM_CDF40 && wavelet != WACM_CDF44)
    return mr_fail(WACM_E_INVAL, "mr: unknown wavelet");
  if (n < 4 || n > 1024) return mr_fail(WACM_E_INVAL, "mr: n must be in [4, 1024]");
  if (nf < 1 || nf > 65535) return mr_fail(WACM_E_INVAL, "mr: nfields must be in [1, 65535]");
  if (nlev < 0 || nlev > 9) return mr_fail(WACM_E_INVAL, "mr: nlev must be in [0, 9]");
  if (n % ((int64_t)1 << nlev) != 0 || (n >> nlev) < 4)
    return mr_fail(WACM_E_INVAL, "mr: n must be a multiple of 2^nlev with n / 2^nlev >= 4");
  if (!u) return mr_fail(WACM_E_INVAL, "mr: u is NULL");
  if ((uintptr_t)u % (2 * elem_size(dtype)) != 0)
    return mr_fail(WACM_E_INVAL, "mr: u must be aligned to two elements");
  return WACM_OK;
}

int mr_validate(int64_t n, int32_t nf, int32_t dtype, int32_t wavelet, int32_t nlev,
                const void* u, const void* work, size_t work_size) {
  if (int rc = mr_validate_sizes(n, nf, dtype, wavelet, nlev, u)) return rc;
  if (wavelet == WACM_CDF44 && nlev > 0) {
    if (!work) return mr_fail(WACM_E_INVAL, "mr: CDF 4/4 needs the work buffer");
    if ((uintptr_t)work % 256 != 0)
      return mr_fail(WACM_E_INVAL, "mr: the work buffer must be 256-byte aligned");
    if (work_size < work_bytes_of(n, nf, elem_size(dtype)))
      return mr_fail(WACM_E_INVAL, "mr: the work buffer is smaller than wacm_mr_work_bytes()");
  }
  return WACM_OK;
}

// Run length along the marching axis: long runs share the window loads, short
// ones keep enough threads (about 2^18 per launch) to fill the chip.
uint32_t run_length(uint64_t outputs, uint32_t len) {
  uint64_t r = outputs / (1u << 18);
  r = r < 1 ? 1 : r > 16 ? 16 : r;
  return (uint32_t)(r > len ? len : r);
}

template <typename T>
hipError_t mr_predict(T* u, int64_t n, int32_t nf, int s, T sign, hipStream_t st) {
  const uint32_t nc = (uint32_t)(n / (2 * s));
  const uint32_t lz = run_length((uint64_t)nc * nc * nc * nf, nc);
  const uint64_t threads = (uint64_t)nc * nc * ((nc + lz - 1) / lz);
  mr_predict_kernel<T><<<dim3(blocks_for(threads), nf), MR_NT, 0, st>>>(u, n, s, nc, lz, sign);
  return hipGetLastError();
}

template <typename T>
hipError_t mr_update(T* u, void* work, int64_t n, int32_t nf, int s, T sign, hipStream_t st) {
  const uint32_t nc = (uint32_t)(n / (2 * s)), m = 2 * nc;
  T* tx = (T*)work;
  T* ty = (T*)((char*)work + tx_bytes(n, nf, sizeof(T)));
  const uint32_t k = MR_XROW / m;  // rows per workgroup (m <= 1024)
  mr_lift_x_kernel<T><<<dim3((m * m + k - 1) / k, nf), MR_NT, 0, st>>>(u, tx, n, s, nc, k);
  const uint32_t ry = run_length((uint64_t)nc * nc * m * nf, nc);
  mr_lift_y_kernel<T><<<dim3(blocks_for((uint64_t)nc * m * ((nc + ry - 1) / ry)), nf), MR_NT, 0,
                        st>>>(tx, ty, nc, ry);
  const uint32_t rz = run_length((uint64_t)nc * nc * nc * nf, nc);
  mr_lift_z_kernel<T><<<dim3(blocks_for((uint64_t)nc * nc * ((nc + rz - 1) / rz)), nf), MR_NT, 0,
                        st>>>(u, ty, n, s, nc, rz, sign);
  return hipGetLastError();
}

template <typename T>
hipError_t mr_run(int inverse, int64_t n, int32_t nf, int32_t wavelet, int32_t nlev, T* u,
                  void* work, hipStream_t st) {
  hipError_t e = hipSuccess;
  for (int q = 0; q < nlev && e == hipSuccess; ++q) {
    const int m = inverse ? nlev - 1 - q : q;
    const int s = 1 << m;
    if (!inverse) {
      e = mr_predict<T>(u, n, nf, s, T(-1), st);
      if (e == hipSuccess && wavelet == WACM_CDF44) e = mr_update<T>(u, work, n, nf, s, T(1), st);
    } else {
      if (wavelet == WACM_CDF44) e = mr_update<T>(u, work, n, nf, s, T(-1), st);
      if (e == hipSuccess) e = mr_predict<T>(u, n, nf, s, T(1), st);
    }
  }
  return e;
}

int mr_entry(int inverse, int64_t n, int32_t nf, int32_t dtype, int32_t wavelet, int32_t nlev,
             void* u, void* work, size_t work_size, void* stream) {
  int rc = mr_validate(n, nf, dtype, wavelet, nlev, u, work, work_size);
  if (rc != WACM_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = dtype == WACM_F64
                     ? mr_run<double>(inverse, n, nf, wavelet, nlev, (double*)u, work, st)
                     : mr_run<float>(inverse, n, nf, wavelet, nlev, (float*)u, work, st);
  if (e != hipSuccess)
    return mr_fail(WACM_E_HIP, std::string("mr launch: ") + hipGetErrorString(e));
  return WACM_OK;
}

// Work buffer of wacm_mr_forward_noalloc: a file-scope device array, one
// copy per GPU, alive until the process ends.  Host code never passes the
// array's name to a kernel (on the host it is only a stand-in for the
// symbol): the device address comes from hipGetSymbolAddress, fetched once
// per device with that device current and kept here.
static __device__ __align__(256) unsigned char scratch[WACM_MR_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_ptr[MAX_DEVICES] = {};

// Device address of the current device's copy of `scratch`.
int scratch_address(void** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return mr_fail(WACM_E_HIP, std::string("mr: hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= MAX_DEVICES) return mr_fail(WACM_E_INVAL, "mr: device index out of range");
  std::lock_guard<std::mutex> lk(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return mr_fail(WACM_E_HIP, std::string("mr: hipGetSymbolAddress(scratch): ") +
                                     hipGetErrorString(e));
    scratch_ptr[dev] = p;
  }
  *out = scratch_ptr[dev];
  return WACM_OK;
}

}  // namespace mr
}  // namespace wacm

extern "C" {

int wacm_mr_forward_noalloc(int64_t n, int32_t nfields, int32_t dtype, int32_t wavelet,
                            int32_t nlev, void* u, void* stream) {
  using namespace wacm::mr;
  // the checks of wacm_mr_forward, then the scratch limit
  int rc = mr_validate_sizes(n, nfields, dtype, wavelet, nlev, u);
  if (rc != WACM_OK) return rc;
  void* work = nullptr;
  size_t wbytes = 0;
  if (wavelet == WACM_CDF44 && nlev > 0) {
    wbytes = work_bytes_of(n, nfields, elem_size(dtype));
    if (wbytes > (size_t)WACM_MR_SCRATCH_BYTES)
      return mr_fail(WACM_E_INVAL, "mr noalloc: the work of this size (" +
                                       std::to_string(wbytes) + " bytes) exceeds the " +
                                       std::to_string((size_t)WACM_MR_SCRATCH_BYTES) +
                                       "-byte scratch array");
    if ((rc = scratch_address(&work)) != WACM_OK) return rc;
  }
  return mr_entry(0, n, nfields, dtype, wavelet, nlev, u, work, wbytes, stream);
}

size_t wacm_mr_work_bytes(int64_t n, int32_t nfields, int32_t dtype) {
  const size_t es = wacm::mr::elem_size(dtype);
  if (es == 0 || n < 4 || n > 1024 || nfields < 1 || nfields > 65535) return 0;
  return wacm::mr::work_bytes_of(n, nfields, es);
}

int wacm_mr_forward(int64_t n, int32_t nfields, int32_t dtype, int32_t wavelet, int32_t nlev,
                    void* u, void* work, size_t work_size, void* stream) {
  return wacm::mr::mr_entry(0, n, nfields, dtype, wavelet, nlev, u, work, work_size, stream);
}

int wacm_mr_inverse(int64_t n, int32_t nfields, int32_t dtype, int32_t wavelet, int32_t nlev,
                    void* u, void* work, size_t work_size, void* stream) {
  return wacm::mr::mr_entry(1, n, nfields, dtype, wavelet, nlev, u, work, work_size, stream);
}

}  // extern "C"
