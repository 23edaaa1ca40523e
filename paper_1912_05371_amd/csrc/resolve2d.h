// Point resolution of the two-dimensional path (host + device): where a ghost
// point of a quadtree block takes its value from (Sec. 4.2 with the
// prediction and decimation of Sec. 3.1).  Shared by the ghost-fill kernel
// and the host harness that checks it against the oracle.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "resolve.h"
#include "wacm_internal.h"

namespace wacm {
namespace d2 {

// 2D pool layout: U[slot][3][P][P], x fastest
struct Lay {
  int P, ng;
  int64_t fstride, bstride;
};

__host__ __device__ inline int region_of(int q, int bs) { return q < 0 ? 0 : (q >= bs ? 2 : 1); }

// Ghost point g of a block (0 <= g < P^2 - bs^2) in row order, the interior
// part of the interior rows skipped: (i, j) in [-ng, bs + ng)^2 minus [0, bs)^2.
__host__ __device__ inline void ghost_point(int g, int bs, int ng, int& i, int& j) {
  const int P = bs + 2 * ng, below = ng * P, side = bs * 2 * ng;
  if (g < below) {
    j = g / P - ng;
    i = g % P - ng;
  } else if (g < below + side) {
    const int h = g - below;
    j = h / (2 * ng);
    const int s = h % (2 * ng);
    i = s < ng ? s - ng : bs + (s - ng);
  } else {
    const int h = g - below - side;
    j = bs + h / P;
    i = h % P - ng;
  }
}

// Element offset (field 0) of the value at the block-local level-J position
// (qx, qy) of block t, a position on the lattice of the leaf holding it: the
// block itself or a same-level neighbour (copy), a coarser neighbour (its
// lattice point: qx, qy even), a finer neighbour (the coincident fine
// point).  The position lies within half a block of the block, so by 2:1
// grading its leaf is one of the 9 regions' leaves.
__host__ __device__ inline int64_t lattice_offset(const Tab& t, const Lay& L, int bs, int qx,
                                                  int qy) {
  const int rx = region_of(qx, bs), ry = region_of(qy, bs);
  const int r = rx + 3 * ry + 9;
  const int lx = qx - (rx - 1) * bs, ly = qy - (ry - 1) * bs;  // in the level-J box of r
  int slot, ix, iy;
  if (r == 13 || t.kind[r] == 0) {
    slot = r == 13 ? t.meta[0] : t.slot[r][0];
    ix = lx;
    iy = ly;
  } else if (t.kind[r] < 0) {
    // the coarse leaf holds two level-J boxes per axis; (nbx & 1) is which
    const int n = 1 << t.meta[1];
    const int nbx = (t.meta[2] + rx - 1 + n) & (n - 1), nby = (t.meta[3] + ry - 1 + n) & (n - 1);
    slot = t.slot[r][0];
    ix = (nbx & 1) * (bs / 2) + lx / 2;
    iy = (nby & 1) * (bs / 2) + ly / 2;
  } else {
    const int fx = 2 * lx, fy = 2 * ly;
    const int sx = fx >= bs, sy = fy >= bs;
    slot = t.slot[r][sx + 2 * sy];
    ix = fx - sx * bs;
    iy = fy - sy * bs;
  }
#if defined(WACM_HOST_CHECK) && !defined(__HIP_DEVICE_COMPILE__)
  wacm_host_check(slot, ix, iy, 0, bs);
#endif
  return (int64_t)slot * L.bstride + (int64_t)(iy + L.ng) * L.P + (ix + L.ng);
}

// Ghost value of field c at block-local (i, j): the owner's lattice value, or
// the DD4 prediction (weights (-1, 9, 9, -1)/16 at offsets -3, -1, 1, 3 on
// each axis where the index is odd) from the coarse lattice when the owner is
// coarser; summed y outer, x inner.
template <typename T>
__host__ __device__ T ghost_value(const Tab& t, const T* __restrict__ U, const Lay& L, int bs,
                                  int c, int i, int j) {
  const int r = region_of(i, bs) + 3 * region_of(j, bs) + 9;
  if (t.kind[r] >= 0) return U[lattice_offset(t, L, bs, i, j) + c * L.fstride];
  constexpr double W[4] = {DDW0, DDW1, DDW1, DDW0};
  constexpr int O[4] = {-3, -1, 1, 3};
  const int nx = (i & 1) ? 4 : 1, ny = (j & 1) ? 4 : 1;
  double v = 0.0;
  for (int b = 0; b < ny; ++b) {
    const int py = ny == 1 ? j : j + O[b];
    const double wy = ny == 1 ? 1.0 : W[b];
    for (int a = 0; a < nx; ++a) {
      const int px = nx == 1 ? i : i + O[a];
      const double wx = nx == 1 ? 1.0 : W[a];
      v += (wy * wx) * (double)U[lattice_offset(t, L, bs, px, py) + c * L.fstride];
    }
  }
  return T(v);
}

}  // namespace d2
}  // namespace wacm
