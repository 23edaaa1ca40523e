// Internal declarations shared by the host code and the HIP kernels of libwacm.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <unordered_map>
#include <vector>

#include "wacm.h"

namespace wacm {

// Per active block: geometry and the 27-region neighbour description used to
// resolve any lattice point within half a block of the block (Sec. 4.1-4.2).
// Region r = rx + 3 ry + 9 rz, r_d = 0 (below), 1 (inside), 2 (above) the
// block's index range along axis d.  kind[r]: 0 the level-J box of that
// region is a leaf (slot[r][0]); -1 it lies inside a level-(J-1) leaf
// (slot[r][0]); +1 it is split into level-(J+1) leaves slot[r][sx+2sy+4sz]
// (only the sub-boxes touching the block are guaranteed to be leaves).
struct alignas(16) Tab {
  int32_t meta[8];  // slot, level J, bx, by, bz, unused x3
  int32_t slot[27][8];
  int8_t kind[32];
};
static_assert(sizeof(Tab) == 928, "Tab layout");

// Region index of face f = 2 axis + side (side 0: below, 1: above).
constexpr int FACE_REGION[6] = {12, 14, 10, 16, 4, 22};

// Element layout of one RK register: block slot s, field c, local (i,j,k).
struct Layout {
  int64_t bstride;  // elements per slot
  int64_t fstride;  // elements per field
  int32_t P;        // edge of the stored cube
  int32_t ng;       // ghost layers stored
  int32_t xs = 0;   // 1: compact x-split order (xsplit_offset), ng = 0
};

// Compact x-split order of a block's field (bs^3 values): the XS_H columns
// next to each x face are stored apart from the middle columns, each part
// [z][y][x] with x fastest.  A neighbour's x-face halo (the 3 columns next to
// the face) is then read from a run of short rows instead of a few values per
// cache line.  XS_H = 4 rather than 3 keeps every part's rows of a tile of 8
// rows on whole 128-byte lines (FP64), so tiles never share a line.
constexpr int XS_H = 4;
__host__ __device__ inline int xsplit_offset(int bs, int i, int j, int k) {
  const int row = k * bs + j;
  if (i < XS_H) return bs * bs * (bs - 2 * XS_H) + row * XS_H + i;
  if (i >= bs - XS_H) return bs * bs * (bs - XS_H) + row * XS_H + (i - (bs - XS_H));
  return row * (bs - 2 * XS_H) + (i - XS_H);
}
// step of xsplit_offset from plane k to k+1 of column i
__host__ __device__ inline int xsplit_zstride(int bs, int i) {
  return (i < XS_H || i >= bs - XS_H ? XS_H : bs - 2 * XS_H) * bs;
}

struct Leaf {
  int32_t J;
  int64_t x, y, z;
};

inline uint64_t leaf_key(int J, int64_t x, int64_t y, int64_t z) {
  return (uint64_t(J) << 57) | (uint64_t(x) << 38) | (uint64_t(y) << 19) | uint64_t(z);
}

// Leaf key -> active index: open addressing with linear probing in a
// power-of-two table at most half full (the table building does ~30 lookups
// per block, so this is the host-side cost of every adaptation).
class LeafIndex {
 public:
  void build(size_t n) {
    size_t cap = 16;
    int bits = 4;
    while (cap < 2 * n) {
      cap <<= 1;
      ++bits;
    }
    keys_.assign(cap, kEmpty);
    vals_.assign(cap, -1);
    mask_ = cap - 1;
    shift_ = 64 - bits;
  }
  void insert(uint64_t k, int32_t v) {
    size_t h = slot(k);
    while (keys_[h] != kEmpty && keys_[h] != k) h = (h + 1) & mask_;
    keys_[h] = k;
    vals_[h] = v;
  }
  int32_t find(uint64_t k) const {
    if (keys_.empty()) return -1;
    for (size_t h = slot(k);; h = (h + 1) & mask_) {
      if (keys_[h] == k) return vals_[h];
      if (keys_[h] == kEmpty) return -1;
    }
  }
  void swap(LeafIndex& o) {
    keys_.swap(o.keys_);
    vals_.swap(o.vals_);
    std::swap(mask_, o.mask_);
    std::swap(shift_, o.shift_);
  }

 private:
  static constexpr uint64_t kEmpty = ~uint64_t(0);  // no leaf key has all bits set
  // Fibonacci hashing: the top bits of the product mix every key bit
  size_t slot(uint64_t k) const { return (size_t)((k * 0x9E3779B97F4A7C15ull) >> shift_); }
  std::vector<uint64_t> keys_;
  std::vector<int32_t> vals_;
  size_t mask_ = 0;
  int shift_ = 60;
};

// Event-based timing of the kernels rk4_step launches (measurement only).
struct Profiler {
  struct Rec {
    int cls;
    hipEvent_t a, b;
  };
  bool on = false;
  std::vector<hipEvent_t> spare;
  std::vector<Rec> recs;
  double ms[4] = {0, 0, 0, 0};
  int64_t n[4] = {0, 0, 0, 0};
};

// Transpose of the ghost fill as a gather: for each interior point that some
// ghost value was read from (rows, element offset of field 0), the ghosts that
// read it with their weights; plus the list of ghost points to clear.  Built
// on the host (h_*), then copied into a device buffer the caller owns (d_*
// point into it; `built` once uploaded).
struct AdjPlan {
  int built = 0;
  int64_t nrows = 0, nnz = 0, nghost = 0;
  std::vector<int64_t> h_dst, h_ptr, h_src, h_ghost;
  std::vector<double> h_w;
  int64_t* d_dst = nullptr;
  int64_t* d_ptr = nullptr;
  int64_t* d_src = nullptr;
  double* d_w = nullptr;
  int64_t* d_ghost = nullptr;
};

// Device tables of a grid inside the caller's workspace (wacm_workspace_bytes),
// byte offsets of 256-byte aligned parts sized for `capacity` blocks.
struct WsParts {
  size_t tab, part, norm, queue, list, cface, cregion, total;
};
WsParts ws_parts(int64_t capacity);
// CDF 4/4 buffers (wacm_wavelet_workspace_bytes): the lifted ghost items
// (at most 56 of 12 int32 per block) and their staging values (at most the
// whole ghost shell, 4 fields per point)
constexpr int LIFT_ITEMS_PER_BLOCK = 56;
// Read boxes of the lifted step's ghost fill, LIFT_BOX_WORDS int32 per active
// block: word r (r != 13) the box of ghost region r (region index rx + 3 ry +
// 9 rz, 0 below, 1 inside, 2 above the block on each axis) that the
// face-star lifted values read, as offsets from the region's first point
// (bits 10d..10d+4 the lowest, 10d+5..10d+9 the highest along axis d); word
// 13 the bit set of the regions that have a box.
constexpr int LIFT_BOX_WORDS = 27;
size_t lift_list_bytes(int64_t capacity);   // the items alone
size_t lift_items_bytes(int64_t capacity);  // the items, read boxes, slot map
size_t lift_ws_bytes(int64_t capacity, int bs, int ng, size_t es);

}  // namespace wacm

struct wacm_grid {
  wacm_grid_desc d{};
  int dim = 3;  // 3: octree, 2: quadtree (leaves with z index 0)
  int P = 0;
  int64_t nb = 0;
  std::vector<wacm::Leaf> leaves;      // active, Morton order
  std::vector<int32_t> slots;          // pool slot of each active block
  wacm::LeafIndex index;               // leaf key -> active index
  std::vector<int32_t> free_slots;     // unused pool slots (stack)
  mutable std::string last_err;  // text of the last failed call on this grid
  // device tables, sized for `capacity` blocks, inside the caller's workspace
  void* ws = nullptr;
  wacm::Tab* d_tab = nullptr;
  double* d_part = nullptr;      // reduction partials: capacity * 16 doubles
  int32_t* d_queue = nullptr;    // work counters (schedule xcd_map 2): stage kernel, face halo
  double* d_norm = nullptr;      // 8 doubles
  int32_t* d_list = nullptr;     // adaptation work lists: capacity * 10 int32
  int32_t* d_cface = nullptr;    // (active index, face) of faces next to another level
  int64_t n_cface = 0;
  int32_t* d_cregion = nullptr;  // (active index, region) of ghost regions in a coarser leaf
  int64_t n_cregion = 0;
  int jfine = 0;                 // finest active level
  mutable wacm::Profiler prof;   // kernel timing, off by default
  std::vector<wacm::Tab> h_tab;  // host copy of the tables
  std::vector<wacm::Tab> h_tab_next;  // the next tables' buffer (allocation reused)
  double adapt_ms[2] = {0, 0};   // last wacm_adapt: host work, device work (ms)
  hipEvent_t adapt_ev[2] = {nullptr, nullptr};  // around wacm_adapt's kernels
  wacm_schedule sched{0, 1, -1, 1, 0, 1};  // launch schedule of the stage kernel
  wacm::AdjPlan plan[2];         // ghost-fill transposes: all layers / face star
  // restriction wavelet: 0 CDF 4/0 (decimation), 1 CDF 4/4 (lifted); with
  // CDF 4/4, the work items of the lifted ghost phase (12 int32 each) and
  // their staging buffer (4 fields per output point), both in the caller's
  // wavelet workspace
  int wavelet = 0;
  int32_t* d_lift = nullptr;
  int64_t n_lift = 0;
  int64_t n_lift_face = 0;  // the first items: the lifted points of the face star
  // per active block, the read boxes of its ghost regions (LIFT_BOX_WORDS),
  // then per pool slot its table index (lift_slot_tab)
  int32_t* d_lift_mask = nullptr;
  size_t lift_items_cap = 0;
  void* d_lift_tmp = nullptr;
  size_t lift_tmp_cap = 0;
};

namespace wacm {
// the table index of every pool slot (-1: inactive), kept after the read boxes
inline int32_t* lift_slot_tab(const wacm_grid* g) {
  return g->d_lift_mask ? g->d_lift_mask + (size_t)LIFT_BOX_WORDS * g->d.capacity : nullptr;
}
}  // namespace wacm

namespace wacm {

// host-side helpers (grid.cpp)
void reorder_leaves(wacm_grid* g);  // Morton order, key index, finest level
int build_tables(wacm_grid* g, std::vector<Tab>& tabs, std::string& err);
int upload_tables(wacm_grid* g, std::vector<Tab>& tabs, std::string& err);
std::vector<int32_t> coarse_faces(const std::vector<Tab>& tabs);  // non-same-level faces
std::vector<int32_t> coarser_regions(const std::vector<Tab>& tabs);  // regions in coarser leaves
// CDF 4/4: builds the lifted ghost-phase items of the current tables and
// (re)allocates their device buffers; a no-op for CDF 4/0
int build_lift(wacm_grid* g, const std::vector<Tab>& tabs, std::string& err);
uint64_t morton_key(const Leaf& l);
void set_error(const std::string& s);

// kernel launchers (kernels.hip); all enqueue on `st`
struct Regs {  // pointers and layouts of the RK registers
  void* U;
  Layout Lu;
  void* acc;
  Layout La;
  void* ping;
  void* pong;
  Layout Ls;
};

// ghost points of the even lattice within 3 of each block (CDF 4/0, 3D)
hipError_t launch_sync_lattice(const wacm_grid* g, void* U, hipStream_t st);
hipError_t launch_sync(const wacm_grid* g, void* U, int face_only, hipStream_t st);
// one RK stage (1..4) of the fused kernel reading the input's own ghost
// layers; every register in the padded pool layout
hipError_t launch_stage_owng(const wacm_grid* g, const wacm_params* p, int s,
                             const double* t_dev, const double* dt_dev, const void* in, void* un,
                             void* out, void* acc, const void* dus, hipStream_t st);
hipError_t launch_rhs(const wacm_grid* g, const wacm_params* p, double t, const void* U,
                      void* dU, const void* dus, hipStream_t st);
hipError_t launch_dt(const wacm_grid* g, const wacm_params* p, const void* U, double* dt_dev,
                     hipStream_t st);
hipError_t launch_rk4(const wacm_grid* g, const wacm_params* p, double* t_dev, double* dt_dev,
                      void* U, void* work, const void* dus, int dt_mode, int64_t nsteps,
                      hipStream_t st);
hipError_t launch_diag(const wacm_grid* g, const wacm_params* p, double t, const void* U,
                       const void* dus, double* out, hipStream_t st);
hipError_t launch_threshold(const wacm_grid* g, const wacm_params* p, double t, const void* U,
                            double eps, int dealias, double* dmax, double* mrange,
                            int8_t* flags, hipStream_t st);
hipError_t launch_filter(const wacm_grid* g, void* U, int level, hipStream_t st);
// CDF 4/4 (lifting.hip): the lifted ghost phase after the CDF 4/0 fill, and
// the parents of a merge list of n families (already in d_list)
hipError_t launch_lift_sync(const wacm_grid* g, void* U, hipStream_t st);
// the CDF 4/0 fill a lifted stage needs: the regions in a coarser leaf and
// the read boxes `box` (LIFT_BOX_WORDS per block: what the face-star lifted
// values read)
hipError_t launch_sync_lifted_stage(const wacm_grid* g, void* U, const int32_t* box,
                                    hipStream_t st);
// the lifted phase of the face star only (the points a stage reads)
hipError_t launch_lift_sync_face(const wacm_grid* g, void* U, hipStream_t st);
hipError_t launch_lift_coarsen(const wacm_grid* g, void* U, int64_t nparents, hipStream_t st);
// RK4 with CDF 4/4 ghosts: before each stage the ghosts it and the lifted
// values read are filled, then the fused stage reads same-level halos in
// place and the others from the input's ghost layers; work = 3 padded
// registers (lift_work_bytes)
hipError_t launch_rk4_lifted(const wacm_grid* g, const wacm_params* p, double* t_dev,
                             double* dt_dev, void* U, void* work, const void* dus, int dt_mode,
                             int64_t nsteps, hipStream_t st);
size_t lift_work_bytes(const wacm_grid* g);
// refine: n entries of (parent slot, child slot, octant); decimate: n entries
// of (parent slot, 8 child slots); lists already on the device in d_list.
hipError_t launch_prolong(const wacm_grid* g, void* U, int64_t n, hipStream_t st);
hipError_t launch_decimate(const wacm_grid* g, void* U, int64_t n, hipStream_t st);

size_t work_bytes(const wacm_grid* g);
// adjoint (adjoint.hip)
size_t adj_work_bytes(const wacm_grid* g);
int build_adj_plan(wacm_grid* g, int face_only, std::string& err);  // host part
size_t adj_plan_bytes(const AdjPlan& p);
int upload_adj_plan(wacm_grid* g, int face_only, void* ws, size_t bytes, std::string& err);
void free_adj_plans(wacm_grid* g);
hipError_t launch_sync_adj(const wacm_grid* g, void* Ub, int face_only, hipStream_t st);
hipError_t launch_rhs_adj(const wacm_grid* g, const wacm_params* p, double t, const void* U,
                          const void* V, void* Ub, double* dtheta, double* dusbar,
                          const void* dus, hipStream_t st);
hipError_t launch_force_adj(const wacm_grid* g, const wacm_params* p, double t, double weight,
                            const void* U, void* Ub, double* dtheta, double* dusbar,
                            const void* dus, hipStream_t st);
hipError_t launch_rk4_adj(const wacm_grid* g, const wacm_params* p, double t, double dt,
                          const void* Un, void* lam, double* dtheta, double* dusbar,
                          const void* dus, void* work, hipStream_t st);
hipError_t profile_flush(const wacm_grid* g);  // accumulate recorded events

// two dimensions (kernels2d.hip): pool [slot][3][P][P]; the RK4 work buffer
// holds 3 pool-shaped registers
size_t work_bytes_2d(const wacm_grid* g);
hipError_t launch_sync_2d(const wacm_grid* g, void* U, hipStream_t st);
hipError_t launch_rhs_2d(const wacm_grid* g, const wacm_params* p, const void* U, void* dU,
                         hipStream_t st);
hipError_t launch_dt_2d(const wacm_grid* g, const wacm_params* p, const void* U, double* dt_dev,
                        hipStream_t st);
hipError_t launch_rk4_2d(const wacm_grid* g, const wacm_params* p, double* t_dev, double* dt_dev,
                         void* U, void* work, int dt_mode, int64_t nsteps, hipStream_t st);
hipError_t launch_diag_2d(const wacm_grid* g, const void* U, double* out, hipStream_t st);
hipError_t launch_threshold_2d(const wacm_grid* g, const void* U, double eps, int dealias,
                               double* dmax, double* mrange, int8_t* flags, hipStream_t st);
hipError_t launch_prolong_2d(const wacm_grid* g, void* U, int64_t n, hipStream_t st);
hipError_t launch_decimate_2d(const wacm_grid* g, void* U, int64_t n, hipStream_t st);

}  // namespace wacm
