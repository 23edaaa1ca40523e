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
// odd = detail + prediction.  A prediction reads only even points and the
// update only odd ones, so both run in place without hazards.
//
// Kernels per step: mr_predict_kernel (one thread per coarse cell: its 4^3
// even neighbours, interpolated along x, y, z, give the 7 odd points of the
// cell) and, for CDF 4/4, three separable low-pass passes through a work
// buffer (x into tx, y into ty, z added into the even points).
#include <hip/hip_runtime.h>

#include <string>

#include "wacm_internal.h"

namespace wacm {
namespace {

constexpr int MR_NT = 256;

// DD4 prediction weights at the odd offsets -3, -1, 1, 3 (in fine points)
__device__ constexpr double MR_DD4[4] = {-1.0 / 16, 9.0 / 16, 9.0 / 16, -1.0 / 16};
// Expanded lifted low-pass, offsets -6..6 (zero at +-5): update (-1, 9, 9,
// -1)/32 on the DD4 details of the offsets -3, -1, 1, 3.
__device__ constexpr double MR_LIFT[13] = {-1.0 / 512,  0.0,         18.0 / 512,  -16.0 / 512,
                                          -63.0 / 512, 144.0 / 512, 348.0 / 512, 144.0 / 512,
                                          -63.0 / 512, -16.0 / 512, 18.0 / 512,  0.0,
                                          -1.0 / 512};

// Odd points of the stride-s lattice: u += sign * P(even).  Cell (X, Y, Z)
// of the stride-2s lattice (nc per axis) owns the odd points (2X + a, 2Y + b,
// 2Z + c) s, (a, b, c) in {0,1}^3 minus (0,0,0); field blockIdx.y.
template <typename T>
__global__ __launch_bounds__(MR_NT) void mr_predict_kernel(T* __restrict__ u, int64_t n, int s,
                                                           uint32_t nc, T sign) {
  const uint32_t cell = blockIdx.x * MR_NT + threadIdx.x;
  if (cell >= nc * nc * nc) return;
  T* f = u + (int64_t)blockIdx.y * n * n * n;
  const uint32_t X = cell % nc, Y = (cell / nc) % nc, Z = cell / (nc * nc);
  const int64_t s2 = 2 * (int64_t)s;
  int64_t xo[4], yo[4], zo[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    xo[q] = (int64_t)((X + nc - 1 + q) % nc) * s2;
    yo[q] = (int64_t)((Y + nc - 1 + q) % nc) * s2 * n;
    zo[q] = (int64_t)((Z + nc - 1 + q) % nc) * s2 * n * n;
  }
  // x: even (the cell's own x) and odd (interpolated) value on each of the
  // 4 x 4 (y, z) lines
  T ex[4][4], ox[4][4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const T* row = f + zo[k] + yo[j];
      const T a0 = row[xo[0]], a1 = row[xo[1]], a2 = row[xo[2]], a3 = row[xo[3]];
      ex[k][j] = a1;
      ox[k][j] = T(MR_DD4[0]) * a0 + T(MR_DD4[1]) * a1 + T(MR_DD4[2]) * a2 + T(MR_DD4[3]) * a3;
    }
  // y: for x type tx and each z line, even and odd in y
  T v[2][2][4];  // [tx][ty][k]
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    v[0][0][k] = ex[k][1];
    v[1][0][k] = ox[k][1];
    v[0][1][k] = T(MR_DD4[0]) * ex[k][0] + T(MR_DD4[1]) * ex[k][1] + T(MR_DD4[2]) * ex[k][2] +
                 T(MR_DD4[3]) * ex[k][3];
    v[1][1][k] = T(MR_DD4[0]) * ox[k][0] + T(MR_DD4[1]) * ox[k][1] + T(MR_DD4[2]) * ox[k][2] +
                 T(MR_DD4[3]) * ox[k][3];
  }
  const int64_t bx = (int64_t)X * s2, by = (int64_t)Y * s2 * n, bz = (int64_t)Z * s2 * n * n;
  const int64_t sy = (int64_t)s * n, sz = (int64_t)s * n * n;
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        if (a + b + c == 0) continue;
        const T* w = v[a][b];
        const T p = c == 0 ? w[1]
                           : T(MR_DD4[0]) * w[0] + T(MR_DD4[1]) * w[1] + T(MR_DD4[2]) * w[2] +
                                 T(MR_DD4[3]) * w[3];
        T* dst = f + bz + c * sz + by + b * sy + bx + a * s;
        *dst = *dst + sign * p;
      }
}

// Low-pass along x with decimation of delta (the stride-s lattice with its
// even points taken as 0): tx[f][z][y][X] = sum_a h_a delta((2X + a) s, y s,
// z s), X < nc, y, z < 2 nc.
template <typename T>
__global__ __launch_bounds__(MR_NT) void mr_lift_x_kernel(const T* __restrict__ u,
                                                          T* __restrict__ tx, int64_t n, int s,
                                                          uint32_t nc) {
  const uint32_t m = 2 * nc;
  const uint32_t o = blockIdx.x * MR_NT + threadIdx.x;
  if (o >= nc * m * m) return;
  const uint32_t X = o % nc, y = (o / nc) % m, z = o / (nc * m);
  const T* row = u + (int64_t)blockIdx.y * n * n * n + ((int64_t)z * n + y) * n * s;
  const bool even_line = ((y | z) & 1) == 0;
  T acc = 0;
#pragma unroll
  for (int a = 0; a < 13; ++a) {
    if (a == 1 || a == 11) continue;  // zero taps
    if (even_line && (a & 1) == 0) continue;  // even points of delta are 0
    const uint32_t x = (2 * X + m - 6 + a) % m;
    acc += T(MR_LIFT[a]) * row[(int64_t)x * s];
  }
  tx[((int64_t)blockIdx.y * m * m + (int64_t)z * m + y) * nc + X] = acc;
}

// Low-pass along y: ty[f][z][Y][X] = sum_b h_b tx[f][z][2Y + b][X].
template <typename T>
__global__ __launch_bounds__(MR_NT) void mr_lift_y_kernel(const T* __restrict__ tx,
                                                          T* __restrict__ ty, uint32_t nc) {
  const uint32_t m = 2 * nc;
  const uint32_t o = blockIdx.x * MR_NT + threadIdx.x;
  if (o >= nc * nc * m) return;
  const uint32_t X = o % nc, Y = (o / nc) % nc, z = o / (nc * nc);
  const T* col = tx + ((int64_t)blockIdx.y * m + z) * m * nc + X;
  T acc = 0;
#pragma unroll
  for (int b = 0; b < 13; ++b) {
    if (b == 1 || b == 11) continue;
    const uint32_t y = (2 * Y + m - 6 + b) % m;
    acc += T(MR_LIFT[b]) * col[(int64_t)y * nc];
  }
  ty[((int64_t)blockIdx.y * m + z) * nc * nc + (int64_t)Y * nc + X] = acc;
}

// Low-pass along z, added to the even points: u((2X, 2Y, 2Z) s) += sign *
// sum_c h_c ty[f][2Z + c][Y][X].
template <typename T>
__global__ __launch_bounds__(MR_NT) void mr_lift_z_kernel(T* __restrict__ u,
                                                          const T* __restrict__ ty, int64_t n,
                                                          int s, uint32_t nc, T sign) {
  const uint32_t m = 2 * nc;
  const uint32_t o = blockIdx.x * MR_NT + threadIdx.x;
  if (o >= nc * nc * nc) return;
  const uint32_t X = o % nc, Y = (o / nc) % nc, Z = o / (nc * nc);
  const T* col = ty + (int64_t)blockIdx.y * m * nc * nc + (int64_t)Y * nc + X;
  T acc = 0;
#pragma unroll
  for (int c = 0; c < 13; ++c) {
    if (c == 1 || c == 11) continue;
    const uint32_t z = (2 * Z + m - 6 + c) % m;
    acc += T(MR_LIFT[c]) * col[(int64_t)z * nc * nc];
  }
  const int64_t s2 = 2 * (int64_t)s;
  T* dst = u + (int64_t)blockIdx.y * n * n * n + (((int64_t)Z * n + Y) * n + X) * s2;
  *dst = *dst + sign * acc;
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

int mr_validate(int64_t n, int32_t nf, int32_t dtype, int32_t wavelet, int32_t nlev,
                const void* u, const void* work) {
  if (elem_size(dtype) == 0) return mr_fail(WACM_E_INVAL, "mr: dtype must be WACM_F32 or WACM_F64");
  if (wavelet != WACM_CDF40 && wavelet != WACM_CDF44)
    return mr_fail(WACM_E_INVAL, "mr: unknown wavelet");
  if (n < 4 || n > 1024) return mr_fail(WACM_E_INVAL, "mr: n must be in [4, 1024]");
  if (nf < 1 || nf > 65535) return mr_fail(WACM_E_INVAL, "mr: nfields must be in [1, 65535]");
  if (nlev < 0 || nlev > 9) return mr_fail(WACM_E_INVAL, "mr: nlev must be in [0, 9]");
  if (n % ((int64_t)1 << nlev) != 0 || (n >> nlev) < 4)
    return mr_fail(WACM_E_INVAL, "mr: n must be a multiple of 2^nlev with n / 2^nlev >= 4");
  if (!u) return mr_fail(WACM_E_INVAL, "mr: u is NULL");
  if (wavelet == WACM_CDF44 && nlev > 0 && !work)
    return mr_fail(WACM_E_INVAL, "mr: CDF 4/4 needs the work buffer");
  return WACM_OK;
}

template <typename T>
hipError_t mr_predict(T* u, int64_t n, int32_t nf, int s, T sign, hipStream_t st) {
  const uint32_t nc = (uint32_t)(n / (2 * s));
  mr_predict_kernel<T><<<dim3(blocks_for((uint64_t)nc * nc * nc), nf), MR_NT, 0, st>>>(u, n, s, nc,
                                                                                      sign);
  return hipGetLastError();
}

template <typename T>
hipError_t mr_update(T* u, void* work, int64_t n, int32_t nf, int s, T sign, hipStream_t st) {
  const uint32_t nc = (uint32_t)(n / (2 * s)), m = 2 * nc;
  T* tx = (T*)work;
  T* ty = (T*)((char*)work + tx_bytes(n, nf, sizeof(T)));
  mr_lift_x_kernel<T><<<dim3(blocks_for((uint64_t)nc * m * m), nf), MR_NT, 0, st>>>(u, tx, n, s,
                                                                                    nc);
  mr_lift_y_kernel<T><<<dim3(blocks_for((uint64_t)nc * nc * m), nf), MR_NT, 0, st>>>(tx, ty, nc);
  mr_lift_z_kernel<T><<<dim3(blocks_for((uint64_t)nc * nc * nc), nf), MR_NT, 0, st>>>(u, ty, n, s,
                                                                                      nc, sign);
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
             void* u, void* work, void* stream) {
  int rc = mr_validate(n, nf, dtype, wavelet, nlev, u, work);
  if (rc != WACM_OK) return rc;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = dtype == WACM_F64
                     ? mr_run<double>(inverse, n, nf, wavelet, nlev, (double*)u, work, st)
                     : mr_run<float>(inverse, n, nf, wavelet, nlev, (float*)u, work, st);
  if (e != hipSuccess)
    return mr_fail(WACM_E_HIP, std::string("mr launch: ") + hipGetErrorString(e));
  return WACM_OK;
}

}  // namespace
}  // namespace wacm

extern "C" {

size_t wacm_mr_work_bytes(int64_t n, int32_t nfields, int32_t dtype) {
  const size_t es = wacm::elem_size(dtype);
  if (es == 0 || n < 4 || n > 1024 || nfields < 1 || nfields > 65535) return 0;
  const size_t ty = ((size_t)nfields * (size_t)(n / 2) * (n / 2) * n * es + 255) / 256 * 256;
  return wacm::tx_bytes(n, nfields, es) + ty;
}

int wacm_mr_forward(int64_t n, int32_t nfields, int32_t dtype, int32_t wavelet, int32_t nlev,
                    void* u, void* work, void* stream) {
  return wacm::mr_entry(0, n, nfields, dtype, wavelet, nlev, u, work, stream);
}

int wacm_mr_inverse(int64_t n, int32_t nfields, int32_t dtype, int32_t wavelet, int32_t nlev,
                    void* u, void* work, void* stream) {
  return wacm::mr_entry(1, n, nfields, dtype, wavelet, nlev, u, work, stream);
}

}  // extern "C"
