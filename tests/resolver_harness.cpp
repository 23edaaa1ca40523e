// Host harness for the kernels' point resolver (csrc/resolve.h), built for the
// CPU by tests/test_resolver_cpu.py.  It builds the library's neighbour tables
// from a leaf list, then runs the very functions the sync kernel runs on the
// GPU -- shell enumeration and ghost_value -- over every ghost point, with
// every source access checked to be an interior point of a valid slot.
//
//   resolver_harness leaves.txt state_in.bin state_out.bin
//   resolver_harness leaves.txt lift
//   resolver_harness leaves.txt penfar params.bin [t0 t1]
//     (prints pen_far per leaf, input order; with t0 t1, for the plate's
//     pitch angles over that window, else for every angle)
// leaves.txt: "bs ng L jmin jmax capacity n" then n lines "J x y z" (slot i = line i)
// state: n * 4 * P^3 doubles (pool layout).  Exit 0 on success.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <set>
#include <string>
#include <tuple>
#include <vector>

#include "resolve.h"
#include "wacm_internal.h"

static int g_cap = 0;

namespace wacm {
int lift_items(const wacm_grid* g, const std::vector<Tab>& tabs, std::vector<int32_t>& it,
               int64_t& pts, int64_t& n_face, std::string& err);
int lift_read_boxes(const wacm_grid* g, const std::vector<Tab>& tabs,
                    const std::vector<int32_t>& it, int64_t n_face, std::vector<int32_t>& box,
                    std::string& err);
}

// The CDF 4/4 lifted ghost-phase items: every ghost point whose owner is finer
// is the output of exactly one item, no other point is, every output is
// centred on the point the resolver gives for that ghost point (the finer
// owner's coincident fine point), every 13-point stencil stays inside the
// source's padded array, and the ghost points the face-star stencils read
// lie in the read boxes the lifted step fills.
static int check_lift(const wacm_grid& g, const std::vector<wacm::Tab>& tabs) {
  using namespace wacm;
  const int bs = g.d.bs, ng = g.d.ng, P = g.P;
  Layout L;
  L.P = P;
  L.ng = ng;
  L.fstride = (int64_t)P * P * P;
  L.bstride = 4 * L.fstride;
  std::vector<int32_t> it;
  int64_t pts = 0, n_face = 0;
  std::string err;
  if (lift_items(&g, tabs, it, pts, n_face, err)) {
    std::fprintf(stderr, "lift items: %s\n", err.c_str());
    return 10;
  }
  std::vector<int> tab_of(g_cap, -1);
  for (size_t ib = 0; ib < tabs.size(); ++ib) tab_of[tabs[ib].meta[0]] = (int)ib;
  std::set<std::tuple<int, int, int, int>> covered, covered_face;
  int64_t npts = 0;
  if (n_face < 0 || n_face > (int64_t)(it.size() / 12)) return 19;
  for (size_t w = 0; w < it.size() / 12; ++w) {
    const int32_t* e = &it[12 * w];
    if (e[0] < 0 || e[0] >= g_cap || tab_of[e[0]] < 0 || e[7] < 0 || e[7] >= g_cap) return 11;
    if (e[11] != npts) return 12;
    const Tab& t = tabs[tab_of[e[0]]];
    for (int dz = 0; dz < e[6]; ++dz)
      for (int dy = 0; dy < e[5]; ++dy)
        for (int dx = 0; dx < e[4]; ++dx) {
          const int i = e[1] + dx, j = e[2] + dy, k = e[3] + dz;
          const int r = region_of(i, bs) + 3 * region_of(j, bs) + 9 * region_of(k, bs);
          if (r == 13 || t.kind[r] <= 0 || i < -ng || i >= bs + ng || j < -ng || j >= bs + ng ||
              k < -ng || k >= bs + ng)
            return 13;
          if (!covered.insert({e[0], i, j, k}).second) return 14;
          if ((int64_t)w < n_face) covered_face.insert({e[0], i, j, k});
          const int c[3] = {e[8] + 2 * dx, e[9] + 2 * dy, e[10] + 2 * dz};
          for (int d = 0; d < 3; ++d)
            if (c[d] - 6 < -ng || c[d] + 6 > bs + ng - 1) return 15;
          const int64_t want = point_offset(t, bs, L, i, j, k);
          const int64_t got = (int64_t)e[7] * L.bstride +
                              ((int64_t)(c[2] + ng) * P + (c[1] + ng)) * P + (c[0] + ng);
          if (want != got) {
            std::fprintf(stderr, "lift item %zu: centre %lld, resolver %lld\n", w, (long long)got,
                         (long long)want);
            return 16;
          }
          ++npts;
        }
  }
  if (npts != pts) return 17;
  // every ghost point with a finer owner is covered
  for (size_t ib = 0; ib < tabs.size(); ++ib)
    for (int k = -ng; k < bs + ng; ++k)
      for (int j = -ng; j < bs + ng; ++j)
        for (int i = -ng; i < bs + ng; ++i) {
          const int r = region_of(i, bs) + 3 * region_of(j, bs) + 9 * region_of(k, bs);
          if (r == 13 || tabs[ib].kind[r] <= 0) continue;
          if (!covered.count({tabs[ib].meta[0], i, j, k})) return 18;
          // the first n_face items hold exactly the face-star points (one
          // index outside [0, bs), at depth <= 3)
          const int out = (i < 0 || i >= bs) + (j < 0 || j >= bs) + (k < 0 || k >= bs);
          const bool star = out == 1 && i >= -3 && i < bs + 3 && j >= -3 && j < bs + 3 &&
                            k >= -3 && k < bs + 3;
          if (star != (covered_face.count({tabs[ib].meta[0], i, j, k}) > 0)) return 20;
        }
  // the read boxes of the lifted step's ghost fill: each inside its region,
  // and every ghost point of a finer leaf's padded array that a face-star
  // stencil reads inside the box of its region
  std::vector<int32_t> box;
  if (lift_read_boxes(&g, tabs, it, n_face, box, err)) {
    std::fprintf(stderr, "read boxes: %s\n", err.c_str());
    return 21;
  }
  if (box.size() != tabs.size() * LIFT_BOX_WORDS) return 21;
  auto rstart = [&](int q) { return q < 0 ? -ng : (q < bs ? 0 : bs); };
  for (size_t ib = 0; ib < tabs.size(); ++ib)
    for (int r = 0; r < 27; ++r) {
      if (r == 13 || !((box[ib * LIFT_BOX_WORDS + 13] >> r) & 1)) continue;
      const int rr[3] = {r % 3, (r / 3) % 3, r / 9};
      for (int d = 0; d < 3; ++d) {
        const int lo = (box[ib * LIFT_BOX_WORDS + r] >> (10 * d)) & 31;
        const int hi = (box[ib * LIFT_BOX_WORDS + r] >> (10 * d + 5)) & 31;
        if (lo > hi || hi >= (rr[d] == 1 ? bs : ng)) return 22;
      }
    }
  int64_t nread = 0;
  for (int64_t w = 0; w < n_face; ++w) {
    const int32_t* e = &it[12 * w];
    const int fb = tab_of[e[7]];
    if (fb < 0) return 23;
    const int32_t* bx = &box[(size_t)fb * LIFT_BOX_WORDS];
    for (int k = e[10] - 6; k <= e[10] + 2 * (e[6] - 1) + 6; ++k)
      for (int j = e[9] - 6; j <= e[9] + 2 * (e[5] - 1) + 6; ++j)
        for (int i = e[8] - 6; i <= e[8] + 2 * (e[4] - 1) + 6; ++i) {
          const int r = region_of(i, bs) + 3 * region_of(j, bs) + 9 * region_of(k, bs);
          if (r == 13) continue;
          ++nread;
          if (!((bx[13] >> r) & 1)) return 24;
          const int q[3] = {i, j, k};
          for (int d = 0; d < 3; ++d) {
            const int o = q[d] - rstart(q[d]);
            if (o < ((bx[r] >> (10 * d)) & 31) || o > ((bx[r] >> (10 * d + 5)) & 31)) return 24;
          }
        }
  }
  std::printf("lift items %zu (face star %lld), points %lld, ghost reads %lld\n", it.size() / 12,
              (long long)n_face, (long long)pts, (long long)nread);
  return 0;
}

namespace wacm {
void wacm_host_check(int slot, int li, int lj, int lk, int bs) {
  if (slot < 0 || slot >= g_cap || li < 0 || li >= bs || lj < 0 || lj >= bs || lk < 0 ||
      lk >= bs) {
    std::fprintf(stderr, "out-of-bounds source: slot %d local (%d,%d,%d) bs %d\n", slot, li, lj,
                 lk, bs);
    std::exit(5);
  }
}
}  // namespace wacm

using namespace wacm;

// The x-split order of the stage registers must be a bijection of [0, bs)^3
// onto [0, bs^3), affine in z along every column with xsplit_zstride.
static bool xsplit_ok(int bs) {
  std::vector<int> hit(bs * bs * bs, 0);
  for (int k = 0; k < bs; ++k)
    for (int j = 0; j < bs; ++j)
      for (int i = 0; i < bs; ++i) {
        const int o = xsplit_offset(bs, i, j, k);
        if (o < 0 || o >= bs * bs * bs || hit[o]++) return false;
        if (o != xsplit_offset(bs, i, j, 0) + k * xsplit_zstride(bs, i)) return false;
      }
  return true;
}

int main(int argc, char** argv) {
  for (int bs : {16, 24, 32})
    if (!xsplit_ok(bs)) {
      std::fprintf(stderr, "x-split order of bs %d is not a bijection\n", bs);
      return 7;
    }
  const bool penfar = (argc == 4 || argc == 6) && std::string(argv[2]) == "penfar";
  if (argc != 4 && !penfar && !(argc == 3 && std::string(argv[2]) == "lift")) return 2;
  FILE* f = std::fopen(argv[1], "r");
  if (!f) return 2;
  wacm_grid g;
  long long cap, n;
  if (std::fscanf(f, "%d %d %lf %d %d %lld %lld", &g.d.bs, &g.d.ng, &g.d.L, &g.d.jmin, &g.d.jmax,
                  &cap, &n) != 7)
    return 2;
  g.d.capacity = cap;
  g.d.dtype = WACM_F64;
  g.P = g.d.bs + 2 * g.d.ng;
  g_cap = (int)cap;
  for (long long i = 0; i < n; ++i) {
    Leaf l;
    long long x, y, z;
    if (std::fscanf(f, "%d %lld %lld %lld", &l.J, &x, &y, &z) != 4) return 2;
    l.x = x;
    l.y = y;
    l.z = z;
    g.leaves.push_back(l);
    g.slots.push_back((int32_t)i);
  }
  std::fclose(f);
  reorder_leaves(&g);
  std::vector<Tab> tabs;
  std::string err;
  int rc = build_tables(&g, tabs, err);
  if (rc) {
    std::fprintf(stderr, "tables: %s\n", err.c_str());
    return 3;
  }
  if (argc == 3) return check_lift(g, tabs);
  if (penfar) {
    // the stage kernel's classification of blocks without penalization, per
    // leaf in input order (slot i = leaf i)
    wacm_params prm;
    FILE* fp = std::fopen(argv[3], "rb");
    if (!fp || std::fread(&prm, sizeof(prm), 1, fp) != 1) return 2;
    std::fclose(fp);
    PitchWindow win{1.0, 0.0, 0.0, false};
    if (argc == 6) win = pitch_window(prm, std::atof(argv[4]), std::atof(argv[5]));
    std::vector<int> far(g.nb, -1);
    for (const Tab& t : tabs) far[t.meta[0]] = pen_far(prm, g.d.L, g.d.bs, t.meta, win) ? 1 : 0;
    for (int64_t i = 0; i < g.nb; ++i) std::printf("%d\n", far[i]);
    return 0;
  }
  const int bs = g.d.bs, ng = g.d.ng, P = g.P;
  Layout L;
  L.P = P;
  L.ng = ng;
  L.fstride = (int64_t)P * P * P;
  L.bstride = 4 * L.fstride;
  std::vector<double> U((size_t)cap * L.bstride, 0.0);
  FILE* fi = std::fopen(argv[2], "rb");
  if (!fi) return 2;
  if (std::fread(U.data(), sizeof(double), (size_t)n * L.bstride, fi) != (size_t)n * L.bstride)
    return 2;
  std::fclose(fi);

  // enumeration: mode 0 visits every ghost point once, mode 1 the depth-3 face star
  for (int mode = 0; mode < 2; ++mode) {
    const int npts = mode == 1 ? 18 * bs * bs : P * P * P - bs * bs * bs;
    std::set<std::tuple<int, int, int>> seen;
    for (int p = 0; p < npts; ++p) {
      int i, j, k;
      shell_point(p, bs, ng, P, mode, i, j, k);
      int out = (i < 0 || i >= bs) + (j < 0 || j >= bs) + (k < 0 || k >= bs);
      bool ok = i >= -ng && i < bs + ng && j >= -ng && j < bs + ng && k >= -ng && k < bs + ng &&
                out >= 1;
      if (mode == 1) ok = ok && out == 1 && i >= -3 && i < bs + 3 && j >= -3 && j < bs + 3 &&
                          k >= -3 && k < bs + 3;
      if (!ok || !seen.insert({i, j, k}).second) {
        std::fprintf(stderr, "bad shell point mode %d p %d -> (%d,%d,%d)\n", mode, p, i, j, k);
        return 4;
      }
    }
  }
  // the sync kernel's per-point work, in place like on the GPU
  const int npts = P * P * P - bs * bs * bs;
  for (int64_t ib = 0; ib < g.nb; ++ib) {
    const Tab& t = tabs[ib];
    double* dst = U.data() + (int64_t)t.meta[0] * L.bstride;
    for (int p = 0; p < npts; ++p) {
      int i, j, k;
      shell_point(p, bs, ng, P, 0, i, j, k);
      double v[4];
      ghost_value<double>(t, bs, L, U.data(), i, j, k, v);
      const int64_t o = ((int64_t)(k + ng) * P + (j + ng)) * P + (i + ng);
      for (int c = 0; c < 4; ++c) dst[o + c * L.fstride] = v[c];
    }
  }
  // ghost_taps (used to build the adjoint's transpose plan) must give the
  // same value as ghost_value, with every tap an interior point of a slot
  for (int64_t ib = 0; ib < g.nb; ++ib) {
    const Tab& t = tabs[ib];
    for (int p = 0; p < npts; ++p) {
      int i, j, k;
      shell_point(p, bs, ng, P, 0, i, j, k);
      double v[4];
      ghost_value<double>(t, bs, L, U.data(), i, j, k, v);
      double s[4] = {0, 0, 0, 0};
      ghost_taps<double>(t, bs, L, i, j, k, [&](int64_t off, double w) {
        for (int c = 0; c < 4; ++c) s[c] += w * U[off + c * L.fstride];
      });
      for (int c = 0; c < 4; ++c)
        if (std::fabs(s[c] - v[c]) > 1e-12 * (1.0 + std::fabs(v[c]))) {
          std::fprintf(stderr, "ghost_taps mismatch block %lld point (%d,%d,%d)\n",
                       (long long)ib, i, j, k);
          return 6;
        }
    }
  }
  FILE* fo = std::fopen(argv[3], "wb");
  if (!fo) return 2;
  std::fwrite(U.data(), sizeof(double), (size_t)n * L.bstride, fo);
  std::fclose(fo);
  return 0;
}
