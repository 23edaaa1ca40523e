// Point resolution, ghost prediction and mask evaluation shared by the HIP
// kernels and by the host-side bounds harness (__host__ __device__).
#pragma once

#include <cmath>

#include "wacm_internal.h"

#define WACM_HD __host__ __device__

namespace wacm {

#if defined(WACM_HOST_CHECK)
// host harness hook: aborts unless the source is an interior point of a slot
void wacm_host_check(int slot, int li, int lj, int lk, int bs);
#endif

// Tam-Webb optimised 7-point first derivative (Sec. 2.3): 2 sum m a_m = 1,
// sum m^3 a_m = 0, and a3 chosen so that the modified wavenumber
// 2 sum a_m sin(m eta) is closest to eta in L2 over 0 <= eta <= 1.1.
constexpr double TW1 = 0.77088238051821737976;
constexpr double TW2 = -0.16670590441457390381;
constexpr double TW3 = 0.020843142770310142619;
// classical 4th-order centred second derivative
constexpr double D2A = -1.0 / 12.0, D2B = 4.0 / 3.0, D2C = -5.0 / 2.0;
// 4th-order Deslauriers-Dubuc prediction weights at fine offsets -3,-1,+1,+3
constexpr double DDW0 = -1.0 / 16.0, DDW1 = 9.0 / 16.0;

constexpr int NT_GEN = 256;  // threads of the generic (non-stage) kernels

// --------------------------------------------------------------------------
// device helpers
// --------------------------------------------------------------------------
WACM_HD inline int region_of(int i, int bs) { return i < 0 ? 0 : (i >= bs ? 2 : 1); }

// Element offset (field 0) of the lattice point (i,j,k), given in the level-J
// local index space of the block described by t.  The point must be a grid
// point of the leaf that holds it: always true for same-level and finer
// leaves, and for even (i,j,k) when that leaf is coarser.
WACM_HD inline int64_t point_offset(const Tab& t, int bs, const Layout& L, int i,
                                                int j, int k) {
  const int rx = region_of(i, bs), ry = region_of(j, bs), rz = region_of(k, bs);
  const int r = rx + 3 * ry + 9 * rz;
  int li = i - (rx - 1) * bs, lj = j - (ry - 1) * bs, lk = k - (rz - 1) * bs;
  const int kind = t.kind[r];
  int slot;
  if (kind == 0) {
    slot = t.slot[r][0];
  } else if (kind < 0) {
    slot = t.slot[r][0];
    li = (((t.meta[2] + rx - 1) & 1) * bs + li) >> 1;
    lj = (((t.meta[3] + ry - 1) & 1) * bs + lj) >> 1;
    lk = (((t.meta[4] + rz - 1) & 1) * bs + lk) >> 1;
  } else {
    const int hb = bs >> 1;
    const int sx = li >= hb, sy = lj >= hb, sz = lk >= hb;
    slot = t.slot[r][sx + 2 * sy + 4 * sz];
    li = 2 * li - sx * bs;
    lj = 2 * lj - sy * bs;
    lk = 2 * lk - sz * bs;
  }
#if defined(WACM_HOST_CHECK) && !defined(__HIP_DEVICE_COMPILE__)
  wacm_host_check(slot, li, lj, lk, bs);
#endif
  if (L.xs) return (int64_t)slot * L.bstride + xsplit_offset(bs, li, lj, lk);
  return (int64_t)slot * L.bstride +
         ((int64_t)(lk + L.ng) * L.P + (lj + L.ng)) * L.P + (li + L.ng);
}

// Ghost value of the 4 fields at (i,j,k) (Sec. 4.2 / 3.1): copy from a leaf
// holding the point, or tensor DD4 prediction from the coarse lattice, summed
// z outer, y, x inner.
template <typename T>
WACM_HD inline void ghost_value(const Tab& t, int bs, const Layout& L,
                                            const T* __restrict__ U, int i, int j, int k,
                                            T out[4]) {
  const int r = region_of(i, bs) + 3 * region_of(j, bs) + 9 * region_of(k, bs);
  if (t.kind[r] >= 0 || ((i | j | k) & 1) == 0) {
    const int64_t o = point_offset(t, bs, L, i, j, k);
#pragma unroll
    for (int c = 0; c < 4; ++c) out[c] = U[o + c * L.fstride];
    return;
  }
  int tx[4], ty[4], tz[4];
  T wx[4], wy[4], wz[4];
  int nx, ny, nz;
  auto taps = [](int q, int* tq, T* wq, int& n) {
    if ((q & 1) == 0) {
      tq[0] = q;
      wq[0] = T(1);
      n = 1;
    } else {
      tq[0] = q - 3;
      tq[1] = q - 1;
      tq[2] = q + 1;
      tq[3] = q + 3;
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
  T acc[4] = {T(0), T(0), T(0), T(0)};
  for (int a = 0; a < nz; ++a)
    for (int b = 0; b < ny; ++b) {
      const T wzy = wz[a] * wy[b];
      for (int e = 0; e < nx; ++e) {
        const T w = wzy * wx[e];
        const int64_t o = point_offset(t, bs, L, tx[e], ty[b], tz[a]);
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[c] += w * U[o + c * L.fstride];
      }
    }
#pragma unroll
  for (int c = 0; c < 4; ++c) out[c] = acc[c];
}

// The sources of the ghost value at (i,j,k): calls f(offset, weight) once for a
// copy, or for each tap of the tensor DD4 prediction (z outer, y, x inner).
// Host code uses it to build the transpose of the ghost fill.
template <typename T, typename F>
WACM_HD inline void ghost_taps(const Tab& t, int bs, const Layout& L, int i, int j, int k, F&& f) {
  const int r = region_of(i, bs) + 3 * region_of(j, bs) + 9 * region_of(k, bs);
  if (t.kind[r] >= 0 || ((i | j | k) & 1) == 0) {
    f(point_offset(t, bs, L, i, j, k), T(1));
    return;
  }
  int tq[3][4];
  T wq[3][4];
  int nq[3];
  const int q3[3] = {i, j, k};
  for (int d = 0; d < 3; ++d) {
    const int q = q3[d];
    if ((q & 1) == 0) {
      tq[d][0] = q;
      wq[d][0] = T(1);
      nq[d] = 1;
    } else {
      tq[d][0] = q - 3;
      tq[d][1] = q - 1;
      tq[d][2] = q + 1;
      tq[d][3] = q + 3;
      wq[d][0] = T(DDW0);
      wq[d][1] = T(DDW1);
      wq[d][2] = T(DDW1);
      wq[d][3] = T(DDW0);
      nq[d] = 4;
    }
  }
  for (int a = 0; a < nq[2]; ++a)
    for (int b = 0; b < nq[1]; ++b) {
      const T wzy = wq[2][a] * wq[1][b];
      for (int e = 0; e < nq[0]; ++e)
        f(point_offset(t, bs, L, tq[0][e], tq[1][b], tq[2][a]), wzy * wq[0][e]);
    }
}

// Mask chi and solid velocity u_s at a point and time (Sec. 2.2): a sphere
// with a tanh layer, or a thin box pitching about an axis through x_le
// parallel to y with alpha(t) = amp sin(2 pi freq t + phase).  mask_time holds
// what depends on t only (the pitch angle's cosine and sine and its rate), so
// that a kernel evaluates it once; mask_eval = mask_point(mask_time(t)).
struct MaskTime {
  double ca, sa, ad;
};

WACM_HD inline MaskTime mask_time(const wacm_params& p, double t) {
  MaskTime m{1.0, 0.0, 0.0};
  if (p.mask == WACM_MASK_PLATE) {
    const double twopi = 6.283185307179586476925286766559;
    const double ph = twopi * p.freq * t + p.phase;
    const double al = p.amp * sin(ph);
    m.ad = p.amp * twopi * p.freq * cos(ph);
    m.ca = cos(al);
    m.sa = sin(al);
  }
  return m;
}

WACM_HD inline void mask_point(const wacm_params& p, const MaskTime& m, double x, double y,
                               double z, double& chi, double us[3]) {
  us[0] = us[1] = us[2] = 0.0;
  chi = 0.0;
  if (p.mask == WACM_MASK_SPHERE) {
    const double dx = x - p.sph_c[0], dy = y - p.sph_c[1], dz = z - p.sph_c[2];
    const double d = sqrt(dx * dx + dy * dy + dz * dz) - p.sph_r;
    chi = 0.5 * (1.0 - tanh(d / p.w));
  } else if (p.mask == WACM_MASK_PLATE) {
    const double rx = x - p.x_le[0], ry = y - p.x_le[1], rz = z - p.x_le[2];
    const double b0 = m.ca * rx - m.sa * rz, b1 = ry, b2 = m.sa * rx + m.ca * rz;  // R^T r
    chi = 0.5 * (tanh((b0 - p.lo[0]) / p.w) - tanh((b0 - p.hi[0]) / p.w));
    chi *= 0.5 * (tanh((b1 - p.lo[1]) / p.w) - tanh((b1 - p.hi[1]) / p.w));
    chi *= 0.5 * (tanh((b2 - p.lo[2]) / p.w) - tanh((b2 - p.hi[2]) / p.w));
    us[0] = m.ad * rz;  // alpha_dot e_y x r
    us[2] = -m.ad * rx;
  }
  if (p.clip && chi < 1e-8) chi = 0.0;
}

WACM_HD inline void mask_eval(const wacm_params& p, double t, double x, double y,
                                          double z, double& chi, double us[3]) {
  mask_point(p, mask_time(p, t), x, y, z, chi, us);
}

// Plate mask with its derivative in the pitch angle, and the solid velocity
// with its derivative in the pitch rate; dal/dad: d alpha / d(A, f, phi) and
// d alpha_dot / d(A, f, phi).  Used by the adjoint kernels.
WACM_HD inline void plate_eval_adj(const wacm_params& p, double t, double x, double y, double z,
                                   double& chi, double& dchi, double us[3], double dusd[3],
                                   double dal[3], double dad[3]) {
  const double twopi = 6.283185307179586476925286766559;
  const double ph = twopi * p.freq * t + p.phase;
  const double s = sin(ph), c = cos(ph);
  const double al = p.amp * s, ad = p.amp * twopi * p.freq * c;
  dal[0] = s;
  dal[1] = p.amp * c * twopi * t;
  dal[2] = p.amp * c;
  dad[0] = twopi * p.freq * c;
  dad[1] = p.amp * twopi * c - p.amp * twopi * p.freq * s * twopi * t;
  dad[2] = -p.amp * twopi * p.freq * s;
  const double rx = x - p.x_le[0], ry = y - p.x_le[1], rz = z - p.x_le[2];
  const double ca = cos(al), sa = sin(al);
  const double b[3] = {ca * rx - sa * rz, ry, sa * rx + ca * rz};
  const double db[3] = {-b[2], 0.0, b[0]};
  double gv[3], gp[3];
  for (int d = 0; d < 3; ++d) {
    const double ta = tanh((b[d] - p.lo[d]) / p.w), tb = tanh((b[d] - p.hi[d]) / p.w);
    gv[d] = 0.5 * (ta - tb);
    gp[d] = 0.5 * ((1.0 - ta * ta) - (1.0 - tb * tb)) / p.w;
  }
  chi = gv[0] * gv[1] * gv[2];
  dchi = gp[0] * db[0] * gv[1] * gv[2] + gv[0] * gp[1] * db[1] * gv[2] +
         gv[0] * gv[1] * gp[2] * db[2];
  if (p.clip && chi < 1e-8) {
    chi = 0.0;
    dchi = 0.0;
  }
  us[0] = ad * rz;
  us[1] = 0.0;
  us[2] = -ad * rx;
  dusd[0] = rz;
  dusd[1] = 0.0;
  dusd[2] = -rx;
}

WACM_HD inline double sponge_eval(const wacm_params& p, double L, double x, double y,
                                              double z) {
  if (!p.sponge) return 0.0;
  const bool in = x < p.l_sp || x > L - p.l_sp || y < p.l_sp || y > L - p.l_sp ||
                  z < p.l_sp || z > L - p.l_sp;
  return in ? 1.0 : 0.0;
}

// mode 0: every ghost point of all ng layers; mode 1: the face star of depth 3
// (one index outside [0,bs)), which is what the rhs stencils read.
WACM_HD inline void shell_point(int idx, int bs, int ng, int P, int mode, int& i,
                                            int& j, int& k) {
  if (mode == 1) {
    const int f2 = bs * bs;
    const int f = idx / (3 * f2);
    const int rem = idx - f * 3 * f2;
    const int d = rem / f2;
    const int q = rem - d * f2;
    const int a = q % bs, b = q / bs;
    const int nrm = (f & 1) ? bs + d : -1 - d;
    const int ax = f >> 1;
    i = ax == 0 ? nrm : a;
    j = ax == 1 ? nrm : (ax == 0 ? a : b);
    k = ax == 2 ? nrm : b;
    return;
  }
  const int slab = ng * P * P;
  if (idx < 2 * slab) {
    const int zz = idx / (P * P);
    const int rem = idx - zz * P * P;
    k = zz < ng ? zz - ng : bs + (zz - ng);
    j = rem / P - ng;
    i = rem % P - ng;
    return;
  }
  const int r = idx - 2 * slab;
  const int ring = P * P - bs * bs;
  k = r / ring;
  const int q = r - k * ring;
  if (q < 2 * ng * P) {
    const int yy = q / P;
    i = q % P - ng;
    j = yy < ng ? yy - ng : bs + (yy - ng);
  } else {
    const int q2 = q - 2 * ng * P;
    j = q2 / (2 * ng);
    const int xx = q2 % (2 * ng);
    i = xx < ng ? xx - ng : bs + (xx - ng);
  }
}

// The pitch angles the plate takes over a time window [t0, t1]: alpha lies in
// [am - da, am + da], am the angle at the window's midpoint, da from the
// bound |d alpha / dt| <= |amp| 2 pi |freq| plus 1e-9 for the rounding of the
// angle here and in the stage kernel.  on = false: no window (any angle).
struct PitchWindow {
  double ca, sa, da;  // cos and sin of am
  bool on;
};

WACM_HD inline PitchWindow pitch_window(const wacm_params& p, double t0, double t1) {
  PitchWindow w{1.0, 0.0, 0.0, false};
  if (p.mask != WACM_MASK_PLATE) return w;
  const double twopi = 6.283185307179586476925286766559;
  const double am = p.amp * sin(twopi * p.freq * (0.5 * (t0 + t1)) + p.phase);
  w.ca = cos(am);
  w.sa = sin(am);
  w.da = fabs(p.amp) * twopi * fabs(p.freq) * 0.5 * fabs(t1 - t0) + 1e-9;
  w.on = true;
  return w;
}

// A block "far" from the mask and the sponge gets chi = 0 and sponge 0 at
// every interior point (at every time, or at every time of the window), so
// the penalization terms of the rhs vanish exactly there and the
// unpenalized stage kernel gives the same values.  Conservative tests, with
// a margin of 40 w beyond the body where every tanh of the smoothed mask
// (Sec. 2.2) is exactly +-1 in FP64; with clipping (chi < 1e-8 set to 0)
// 12 w suffice: beyond it one tanh factor of the mask stays below 4e-11.
//  - sphere: the distance from the centre to the block's point box exceeds
//    R + 40 w;
//  - plate, any angle: either the block's y points miss the span widened by
//    40 w, or their distance from the pitch axis (x and z relative to x_le; a
//    rotation about the axis keeps it) exceeds the farthest corner of the
//    chord x thickness rectangle widened by 40 w;
//  - plate, angles of a window: or the body-frame chord or thickness
//    coordinate of every point of the box, at every angle of the window,
//    misses the widened rectangle's range: bounded by its value at the box
//    centre and the window's mid angle, plus the box's half-widths projected,
//    plus da times the box's largest distance from the axis;
//  - sponge: the block's extreme points lie inside [l_sp, L - l_sp] on every
//    axis, evaluated with the same expressions as the stage kernel.
WACM_HD inline bool pen_far(const wacm_params& p, double L, int bs, const int32_t* m,
                            const PitchWindow& win) {
  const double h = L / (double(int64_t(1) << m[1]) * bs);
  double lo[3], hi[3];
  for (int d = 0; d < 3; ++d) {
    lo[d] = (double)(m[2 + d] * bs) * h;
    hi[d] = (double)(m[2 + d] * bs + bs - 1) * h;
  }
  if (p.sponge)
    for (int d = 0; d < 3; ++d)
      if (!(lo[d] >= p.l_sp && hi[d] <= L - p.l_sp)) return false;
  const double mg = (p.clip ? 12.0 : 40.0) * p.w;
  if (p.mask == WACM_MASK_SPHERE) {
    double s = 0.0;
    for (int d = 0; d < 3; ++d) {
      const double q = fmax(0.0, fmax(lo[d] - p.sph_c[d], p.sph_c[d] - hi[d]));
      s += q * q;
    }
    return sqrt(s) > p.sph_r + mg;
  }
  if (p.mask == WACM_MASK_PLATE) {
    const double ylo = lo[1] - p.x_le[1], yhi = hi[1] - p.x_le[1];
    if (yhi < p.lo[1] - mg || ylo > p.hi[1] + mg) return true;
    double rmax = 0.0;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        const double cx = a ? p.hi[0] + mg : p.lo[0] - mg;
        const double cz = b ? p.hi[2] + mg : p.lo[2] - mg;
        rmax = fmax(rmax, sqrt(cx * cx + cz * cz));
      }
    double s = 0.0;
    for (int d = 0; d < 3; d += 2) {
      const double q = fmax(0.0, fmax(lo[d] - p.x_le[d], p.x_le[d] - hi[d]));
      s += q * q;
    }
    if (sqrt(s) > rmax) return true;
    if (!win.on) return false;
    const double ca = win.ca, sa = win.sa;
    const double cx = 0.5 * (lo[0] + hi[0]) - p.x_le[0], cz = 0.5 * (lo[2] + hi[2]) - p.x_le[2];
    const double hx = 0.5 * (hi[0] - lo[0]), hz = 0.5 * (hi[2] - lo[2]);
    const double fx = fmax(fabs(lo[0] - p.x_le[0]), fabs(hi[0] - p.x_le[0]));
    const double fz = fmax(fabs(lo[2] - p.x_le[2]), fabs(hi[2] - p.x_le[2]));
    const double sw = win.da * sqrt(fx * fx + fz * fz);
    const double b0 = ca * cx - sa * cz, e0 = fabs(ca) * hx + fabs(sa) * hz + sw;
    const double b2 = sa * cx + ca * cz, e2 = fabs(sa) * hx + fabs(ca) * hz + sw;
    if (b0 + e0 < p.lo[0] - mg || b0 - e0 > p.hi[0] + mg) return true;
    return b2 + e2 < p.lo[2] - mg || b2 - e2 > p.hi[2] + mg;
  }
  return true;
}

}  // namespace wacm
