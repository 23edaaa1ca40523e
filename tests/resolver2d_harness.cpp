// Host harness for the two-dimensional point resolver (csrc/resolve2d.h),
// built for the CPU by tests/test_resolver_cpu.py.  It builds the library's
// quadtree tables from a leaf list, then runs the very functions the 2D
// ghost-fill kernel runs -- ghost_point and ghost_value -- over every ghost
// point, with every source access checked to be an interior point of a valid
// slot, and checks that ghost_point enumerates each ghost point once.
//
//   resolver2d_harness leaves.txt state_in.bin state_out.bin
// leaves.txt: "bs ng L jmin jmax capacity n" then n lines "J x y" (slot i =
// line i); state: n * 3 * P^2 doubles (2D pool layout).  Exit 0 on success.
#include <cstdio>
#include <cstdlib>
#include <set>
#include <string>
#include <utility>
#include <vector>

#include "resolve2d.h"

static int g_cap = 0;

namespace wacm {
void wacm_host_check(int slot, int li, int lj, int lk, int bs) {
  if (slot < 0 || slot >= g_cap || li < 0 || li >= bs || lj < 0 || lj >= bs || lk != 0) {
    std::fprintf(stderr, "out-of-bounds source: slot %d local (%d,%d,%d) bs %d\n", slot, li, lj,
                 lk, bs);
    std::exit(5);
  }
}
}  // namespace wacm

using namespace wacm;

int main(int argc, char** argv) {
  if (argc != 4) return 2;
  FILE* f = std::fopen(argv[1], "r");
  if (!f) return 2;
  wacm_grid g;
  long long cap, n;
  if (std::fscanf(f, "%d %d %lf %d %d %lld %lld", &g.d.bs, &g.d.ng, &g.d.L, &g.d.jmin, &g.d.jmax,
                  &cap, &n) != 7)
    return 2;
  g.d.capacity = cap;
  g.d.dtype = WACM_F64;
  g.d.dim = 2;
  g.dim = 2;
  g.P = g.d.bs + 2 * g.d.ng;
  g_cap = (int)cap;
  for (long long i = 0; i < n; ++i) {
    Leaf l;
    long long x, y;
    if (std::fscanf(f, "%d %lld %lld", &l.J, &x, &y) != 3) return 2;
    l.x = x;
    l.y = y;
    l.z = 0;
    g.leaves.push_back(l);
    g.slots.push_back((int32_t)i);
  }
  std::fclose(f);
  reorder_leaves(&g);
  std::vector<Tab> tabs;
  std::string err;
  if (int rc = build_tables(&g, tabs, err)) {
    std::fprintf(stderr, "tables: %s\n", err.c_str());
    return 3;
  }
  const int bs = g.d.bs, ng = g.d.ng, P = g.P;
  const int nghost = P * P - bs * bs;
  // ghost_point enumerates each ghost point exactly once
  std::set<std::pair<int, int>> seen;
  for (int q = 0; q < nghost; ++q) {
    int i, j;
    d2::ghost_point(q, bs, ng, i, j);
    if (i < -ng || i >= bs + ng || j < -ng || j >= bs + ng || (i >= 0 && i < bs && j >= 0 && j < bs))
      return 6;
    if (!seen.insert({i, j}).second) return 6;
  }
  d2::Lay L;
  L.P = P;
  L.ng = ng;
  L.fstride = (int64_t)P * P;
  L.bstride = 3 * L.fstride;
  const size_t tot = (size_t)n * 3 * P * P;
  std::vector<double> U(tot), V;
  FILE* fi = std::fopen(argv[2], "rb");
  if (!fi || std::fread(U.data(), sizeof(double), tot, fi) != tot) return 2;
  std::fclose(fi);
  V = U;
  for (const Tab& t : tabs)
    for (int q = 0; q < nghost; ++q) {
      int i, j;
      d2::ghost_point(q, bs, ng, i, j);
      for (int c = 0; c < 3; ++c)
        V[(size_t)t.meta[0] * L.bstride + c * L.fstride + (size_t)(j + ng) * P + (i + ng)] =
            d2::ghost_value<double>(t, U.data(), L, bs, c, i, j);
    }
  FILE* fo = std::fopen(argv[3], "wb");
  if (!fo || std::fwrite(V.data(), sizeof(double), tot, fo) != tot) return 2;
  std::fclose(fo);
  return 0;
}
