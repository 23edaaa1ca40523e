// Host-side block tree of libwacm: leaf index, 2:1 checks and the per-block
// neighbour tables the kernels use to resolve ghost points (Sec. 4.1-4.2).
#include <unistd.h>

#include <algorithm>
#include <condition_variable>
#include <cstring>
#include <functional>
#include <mutex>
#include <numeric>
#include <thread>

#include "wacm_internal.h"

namespace wacm {

uint64_t morton_key(const Leaf& l) {
  // treecode scaled to level 20: 3 bits per level, x in the lowest bit
  uint64_t k = 0;
  for (int b = 19; b >= 0; --b) {
    int sh = b - (20 - l.J);  // bit of the level-J index that lands on bit b
    uint64_t xb = sh >= 0 ? ((uint64_t)l.x >> sh) & 1u : 0;
    uint64_t yb = sh >= 0 ? ((uint64_t)l.y >> sh) & 1u : 0;
    uint64_t zb = sh >= 0 ? ((uint64_t)l.z >> sh) & 1u : 0;
    k = (k << 3) | (xb | (yb << 1) | (zb << 2));
  }
  return k;
}

static inline int64_t wrapi(int64_t a, int64_t n) {
  int64_t r = a % n;
  return r < 0 ? r + n : r;
}

// Slot of the active leaf (J, x, y, z), or -1.
static int32_t find_slot(const wacm_grid* g, int J, int64_t x, int64_t y, int64_t z) {
  if (J < 0) return -1;
  const int32_t i = g->index.find(leaf_key(J, x, y, z));
  return i < 0 ? -1 : g->slots[i];
}

// Sort active blocks into Morton order and rebuild the key index.
void reorder_leaves(wacm_grid* g) {
  std::vector<int64_t> ord(g->leaves.size());
  std::iota(ord.begin(), ord.end(), 0);
  std::vector<uint64_t> keys(g->leaves.size());
  for (size_t i = 0; i < keys.size(); ++i) keys[i] = morton_key(g->leaves[i]);
  std::sort(ord.begin(), ord.end(), [&](int64_t a, int64_t b) { return keys[a] < keys[b]; });
  std::vector<Leaf> L(ord.size());
  std::vector<int32_t> S(ord.size());
  for (size_t i = 0; i < ord.size(); ++i) {
    L[i] = g->leaves[ord[i]];
    S[i] = g->slots[ord[i]];
  }
  g->leaves.swap(L);
  g->slots.swap(S);
  g->nb = (int64_t)g->leaves.size();
  g->index.build(g->leaves.size());
  g->jfine = g->d.jmin;
  for (int64_t i = 0; i < g->nb; ++i) {
    const Leaf& l = g->leaves[i];
    g->index.insert(leaf_key(l.J, l.x, l.y, l.z), (int32_t)i);
    g->jfine = std::max(g->jfine, l.J);
  }
}


// In two dimensions only the 9 regions of the plane (rz = 1) and the 4
// sub-boxes with sz = 0 are filled; the others stay unused.
static int build_range(const wacm_grid* g, Tab* tabs, int64_t i0, int64_t i1, int64_t& bad,
                       std::string& err) {
  const int rz0 = g->dim == 2 ? 1 : 0, rz1 = g->dim == 2 ? 1 : 2, nsub = g->dim == 2 ? 4 : 8;
  for (int64_t i = i0; i < i1; ++i) {
    const Leaf& b = g->leaves[i];
    Tab& t = tabs[i];
    t = Tab{};
    t.meta[0] = g->slots[i];
    t.meta[1] = b.J;
    t.meta[2] = (int32_t)b.x;
    t.meta[3] = (int32_t)b.y;
    t.meta[4] = (int32_t)b.z;
    const int64_t n = int64_t(1) << b.J;
    for (int rz = rz0; rz <= rz1; ++rz)
      for (int ry = 0; ry < 3; ++ry)
        for (int rx = 0; rx < 3; ++rx) {
          int r = rx + 3 * ry + 9 * rz;
          for (int s = 0; s < 8; ++s) t.slot[r][s] = -1;
          int64_t nx = wrapi(b.x + rx - 1, n), ny = wrapi(b.y + ry - 1, n),
                  nz = wrapi(b.z + rz - 1, n);
          int32_t s0 = find_slot(g, b.J, nx, ny, nz);
          if (s0 >= 0) {
            t.kind[r] = 0;
            for (int s = 0; s < 8; ++s) t.slot[r][s] = s0;
            continue;
          }
          int32_t sc = b.J > 0 ? find_slot(g, b.J - 1, nx >> 1, ny >> 1, nz >> 1) : -1;
          if (sc >= 0) {
            t.kind[r] = -1;
            for (int s = 0; s < 8; ++s) t.slot[r][s] = sc;
            continue;
          }
          // the neighbour box must be split into level-(J+1) leaves; every
          // sub-box touching this block has to be a leaf (2:1 grading)
          bool anyfine = false;
          for (int s = 0; s < nsub; ++s) {
            int sx = s & 1, sy = (s >> 1) & 1, sz = (s >> 2) & 1;
            bool touch = (rx == 1 || sx == (rx == 0 ? 1 : 0)) &&
                         (ry == 1 || sy == (ry == 0 ? 1 : 0)) &&
                         (rz == 1 || sz == (rz == 0 ? 1 : 0));
            int32_t sf = find_slot(g, b.J + 1, 2 * nx + sx, 2 * ny + sy, 2 * nz + sz);
            if (touch && sf < 0) {
              bad = i;
              err = "grid is not 2:1 balanced around block (level " + std::to_string(b.J) +
                    ", " + std::to_string(b.x) + "," + std::to_string(b.y) + "," +
                    std::to_string(b.z) + ")";
              return WACM_E_UNBALANCED;
            }
            t.slot[r][s] = sf;
            anyfine = anyfine || sf >= 0;
          }
          if (!anyfine) {
            bad = i;
            err = "no neighbour found";
            return WACM_E_UNBALANCED;
          }
          t.kind[r] = 1;
        }
  }
  return WACM_OK;
}

// A fixed team of 7 worker threads for the table builds: spawning threads
// on every adaptation pass costs about as much as building a small grid's
// tables.  run(n, f) calls f(k) for k in [0, n), on the workers and the
// calling thread, and returns when all have finished; calls are serialised.
// In a process forked after the team started (its workers are not there)
// the calls run on the calling thread alone.
class BuildTeam {
 public:
  static BuildTeam& get() {
    static BuildTeam team;
    return team;
  }
  void run(int n, const std::function<void(int)>& f) {
    std::lock_guard<std::mutex> call(call_mu_);
    if (getpid() != pid_ || th_.empty() || n <= 1) {
      for (int k = 0; k < n; ++k) f(k);
      return;
    }
    {
      std::lock_guard<std::mutex> lk(mu_);
      job_ = &f;
      njob_ = n;
      next_ = 0;
      left_ = n;
      ++gen_;
    }
    cv_.notify_all();
    work();
    std::unique_lock<std::mutex> lk(mu_);
    done_cv_.wait(lk, [&] { return left_ == 0; });
    job_ = nullptr;
  }
  ~BuildTeam() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      stop_ = true;
    }
    cv_.notify_all();
    for (auto& t : th_) t.join();
  }

 private:
  BuildTeam() : pid_(getpid()) {
    const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    const unsigned nw = std::min(7u, hw - 1);
    for (unsigned w = 0; w < nw; ++w) th_.emplace_back([this] { loop(); });
  }
  // take indices of the current job until none is left
  void work() {
    for (;;) {
      int k;
      const std::function<void(int)>* f;
      {
        std::lock_guard<std::mutex> lk(mu_);
        if (!job_ || next_ >= njob_) return;
        k = next_++;
        f = job_;
      }
      (*f)(k);
      std::lock_guard<std::mutex> lk(mu_);
      if (--left_ == 0) done_cv_.notify_all();
    }
  }
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return stop_ || gen_ != seen; });
        if (stop_) return;
        seen = gen_;
      }
      work();
    }
  }
  const pid_t pid_;
  std::mutex call_mu_, mu_;
  std::condition_variable cv_, done_cv_;
  std::vector<std::thread> th_;
  const std::function<void(int)>* job_ = nullptr;
  int njob_ = 0, next_ = 0, left_ = 0;
  uint64_t gen_ = 0;
  bool stop_ = false;
};

// The blocks are split into contiguous runs (at most 8, of at least 256
// blocks) built by the team (each block's table depends only on the
// read-only leaf index); the error reported is that of the first failing
// block in active order, whatever the split.  `tabs` keeps its allocation
// from call to call.
int build_tables(wacm_grid* g, std::vector<Tab>& tabs, std::string& err) {
  const int64_t nb = g->nb;
  tabs.resize(nb);
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(8, (nb + 255) / 256));
  std::vector<int> rc(nt, WACM_OK);
  std::vector<int64_t> bad(nt, -1);
  std::vector<std::string> msg(nt);
  BuildTeam::get().run(nt, [&](int k) {
    const int64_t i0 = nb * k / nt, i1 = nb * (k + 1) / nt;
    rc[k] = build_range(g, tabs.data(), i0, i1, bad[k], msg[k]);
  });
  for (int k = 0; k < nt; ++k)  // runs are in active order
    if (rc[k] != WACM_OK) {
      err = msg[k];
      return rc[k];
    }
  return WACM_OK;
}

std::vector<int32_t> coarse_faces(const std::vector<Tab>& tabs) {
  size_t n = 0;
  for (const Tab& t : tabs)
    for (int f = 0; f < 6; ++f) n += t.kind[FACE_REGION[f]] != 0;
  std::vector<int32_t> cf(2 * n);
  size_t k = 0;
  for (size_t i = 0; i < tabs.size(); ++i)
    for (int f = 0; f < 6; ++f)
      if (tabs[i].kind[FACE_REGION[f]] != 0) {
        cf[k++] = (int32_t)i;
        cf[k++] = f;
      }
  return cf;
}

std::vector<int32_t> coarser_regions(const std::vector<Tab>& tabs) {
  size_t n = 0;
  for (const Tab& t : tabs)
    for (int r = 0; r < 27; ++r) n += r != 13 && t.kind[r] < 0;
  std::vector<int32_t> cr(2 * n);
  size_t k = 0;
  for (size_t i = 0; i < tabs.size(); ++i)
    for (int r = 0; r < 27; ++r)
      if (r != 13 && tabs[i].kind[r] < 0) {
        cr[k++] = (int32_t)i;
        cr[k++] = r;
      }
  return cr;
}

// Lifted ghost phase (CDF 4/4): one item per (block, ghost region in a finer
// leaf, child of that region next to the block).  Along an axis the region
// is [-ng, 0) (children of the upper half), [bs, bs+ng) (lower half) or the
// block's own range split into its two halves; an output at block-local
// coarse index i is centred on the child's fine point 2 (i - (r-1) bs) - h bs,
// whose 13-point stencil must lie in the child's padded array.  Face regions
// are cut along their normal into the 3 layers next to the block and the
// rest: the items of the first n_face of the list are exactly the lifted
// points of the depth-3 face star (what a stage reads), the others the
// remaining lifted ghost points.
// The items of the tables (12 int32 each, pts = output points); also used
// by the host harness that checks them against the point resolver.
int lift_items(const wacm_grid* g, const std::vector<Tab>& tabs, std::vector<int32_t>& it,
               int64_t& pts, int64_t& n_face, std::string& err) {
  const int bs = g->d.bs, ng = g->d.ng, hb = bs / 2;
  it.clear();
  pts = 0;
  n_face = 0;
  for (int pass = 0; pass < 2; ++pass) {
    for (size_t ib = 0; ib < tabs.size(); ++ib) {
      const Tab& t = tabs[ib];
      for (int r = 0; r < 27; ++r) {
        if (r == 13 || t.kind[r] <= 0) continue;
        const int rr[3] = {r % 3, (r / 3) % 3, r / 9};
        const bool face = (rr[0] == 1) + (rr[1] == 1) + (rr[2] == 1) == 2;
        if (pass == 0 && !face) continue;
        int st[3][2], cnt[3][2], half[3][2], nseg[3];
        for (int d = 0; d < 3; ++d) {
          if (rr[d] == 1) {
            nseg[d] = 2;
            st[d][0] = 0, cnt[d][0] = hb, half[d][0] = 0;
            st[d][1] = hb, cnt[d][1] = hb, half[d][1] = 1;
            continue;
          }
          nseg[d] = 1;
          half[d][0] = rr[d] == 0 ? 1 : 0;
          // a face region's normal range: the 3 layers next to the block
          // (pass 0) or the others (pass 1); otherwise all ng layers
          const int lo = face && pass == 1 ? 3 : 0, hi = face && pass == 0 ? 3 : ng;
          cnt[d][0] = hi - lo;
          st[d][0] = rr[d] == 0 ? -hi : bs + lo;
        }
        if (cnt[0][0] <= 0 || cnt[1][0] <= 0 || cnt[2][0] <= 0) continue;
        for (int c = 0; c < nseg[2]; ++c)
          for (int b = 0; b < nseg[1]; ++b)
            for (int a = 0; a < nseg[0]; ++a) {
              const int sg[3] = {a, b, c};
              int f0[3], n3[3], o0[3], oct = 0;
              for (int d = 0; d < 3; ++d) {
                o0[d] = st[d][sg[d]];
                n3[d] = cnt[d][sg[d]];
                f0[d] = 2 * (o0[d] - (rr[d] - 1) * bs) - half[d][sg[d]] * bs;
                oct += half[d][sg[d]] << d;
                if (f0[d] - 6 < -ng || f0[d] + 2 * (n3[d] - 1) + 6 > bs + ng - 1) {
                  err = "lifted restriction stencil leaves the child's ghost layers";
                  return WACM_E_INVAL;
                }
              }
              const int32_t item[12] = {t.meta[0], o0[0], o0[1], o0[2], n3[0], n3[1], n3[2],
                                        t.slot[r][oct], f0[0], f0[1], f0[2], (int32_t)pts};
              it.insert(it.end(), item, item + 12);
              pts += (int64_t)n3[0] * n3[1] * n3[2];
            }
      }
    }
    if (pass == 0) n_face = (int64_t)it.size() / 12;
  }
  return WACM_OK;
}

static size_t up256(size_t v) { return (v + 255) / 256 * 256; }

WsParts ws_parts(int64_t cap) {
  const size_t c = (size_t)cap;
  WsParts w;
  size_t o = 0;
  w.tab = o, o += up256(sizeof(Tab) * c);
  // reduction partials: 10 per block (diagnostics) or one per stage work item
  // (at most 4 per block), 16 reserved per block plus a margin
  w.part = o, o += up256(sizeof(double) * 16 * (c + 1024));
  w.norm = o, o += up256(sizeof(double) * 16);
  w.queue = o, o += up256(sizeof(int32_t) * 512);
  w.list = o, o += up256(sizeof(int32_t) * 10 * c);
  w.cface = o, o += up256(sizeof(int32_t) * 12 * c);
  w.cregion = o, o += up256(sizeof(int32_t) * 52 * c);
  w.total = o;
  return w;
}

size_t lift_list_bytes(int64_t cap) {
  return up256(sizeof(int32_t) * 12 * LIFT_ITEMS_PER_BLOCK * (size_t)cap);
}

// the items, then the read boxes of every block (lift_read_boxes) and the
// table index of every pool slot
size_t lift_items_bytes(int64_t cap) {
  return lift_list_bytes(cap) + up256(sizeof(int32_t) * (LIFT_BOX_WORDS + 1) * (size_t)cap);
}

// Per active block (table order), the part of each ghost region of its
// padded array that the face-star lifted values read: an item's outputs are
// centred on the finer leaf's points f0, f0 + 2, ..., whose 13-point stencils
// cover [f0 - 6, f0 + 2 (n - 1) + 6] on each axis; per region the bounding
// box of those boxes' intersections with it, packed as in LIFT_BOX_WORDS.
int lift_read_boxes(const wacm_grid* g, const std::vector<Tab>& tabs,
                    const std::vector<int32_t>& it, int64_t n_face, std::vector<int32_t>& box,
                    std::string& err) {
  const int bs = g->d.bs, ng = g->d.ng;
  if (bs > 32 || ng > 32) {
    err = "read boxes need bs and ng of at most 32";
    return WACM_E_INVAL;
  }
  std::vector<int32_t> slot_ib((size_t)g->d.capacity, -1);
  for (size_t ib = 0; ib < tabs.size(); ++ib) slot_ib[tabs[ib].meta[0]] = (int32_t)ib;
  // per (block, region): lowest and highest block-local index on each axis
  std::vector<int16_t> lh(tabs.size() * 27 * 6, 0);
  box.assign(tabs.size() * LIFT_BOX_WORDS, 0);
  for (int64_t w = 0; w < n_face; ++w) {
    const int32_t* e = &it[12 * w];
    const int32_t fb = e[7] >= 0 && e[7] < g->d.capacity ? slot_ib[e[7]] : -1;
    if (fb < 0) {
      err = "lifted item reads an inactive slot";
      return WACM_E_INVAL;
    }
    int a0[3], a1[3];
    for (int d = 0; d < 3; ++d) {
      a0[d] = e[8 + d] - 6;
      a1[d] = e[8 + d] + 2 * (e[4 + d] - 1) + 6;
    }
    for (int r = 0; r < 27; ++r) {
      if (r == 13) continue;
      const int rr[3] = {r % 3, (r / 3) % 3, r / 9};
      int lo[3], hi[3];
      bool hit = true;
      for (int d = 0; d < 3; ++d) {
        const int r0 = rr[d] == 0 ? -ng : (rr[d] == 1 ? 0 : bs);
        const int r1 = rr[d] == 0 ? -1 : (rr[d] == 1 ? bs - 1 : bs + ng - 1);
        lo[d] = std::max(r0, a0[d]);
        hi[d] = std::min(r1, a1[d]);
        hit = hit && lo[d] <= hi[d];
      }
      if (!hit) continue;
      int32_t& have = box[(size_t)fb * LIFT_BOX_WORDS + 13];
      int16_t* b = &lh[((size_t)fb * 27 + r) * 6];
      for (int d = 0; d < 3; ++d) {
        const bool first = !((have >> r) & 1);
        b[2 * d] = (int16_t)(first ? lo[d] : std::min<int>(b[2 * d], lo[d]));
        b[2 * d + 1] = (int16_t)(first ? hi[d] : std::max<int>(b[2 * d + 1], hi[d]));
      }
      have |= int32_t(1) << r;
    }
  }
  for (size_t ib = 0; ib < tabs.size(); ++ib)
    for (int r = 0; r < 27; ++r) {
      if (r == 13 || !((box[ib * LIFT_BOX_WORDS + 13] >> r) & 1)) continue;
      const int rr[3] = {r % 3, (r / 3) % 3, r / 9};
      const int16_t* b = &lh[(ib * 27 + r) * 6];
      int32_t v = 0;
      for (int d = 0; d < 3; ++d) {
        const int r0 = rr[d] == 0 ? -ng : (rr[d] == 1 ? 0 : bs);
        v |= (int32_t)(b[2 * d] - r0) << (10 * d);
        v |= (int32_t)(b[2 * d + 1] - r0) << (10 * d + 5);
      }
      box[ib * LIFT_BOX_WORDS + r] = v;
    }
  return WACM_OK;
}

size_t lift_ws_bytes(int64_t cap, int bs, int ng, size_t es) {
  const size_t P = (size_t)bs + 2 * ng;
  const size_t shell = P * P * P - (size_t)bs * bs * bs;
  return lift_items_bytes(cap) + up256((size_t)cap * shell * 4 * es);
}

// Lifted ghost items of the tables into the caller's wavelet workspace
// (d_lift, d_lift_tmp, set by wacm_set_wavelet).  Never allocates: the
// workspace is sized for `capacity` blocks with every ghost point lifted.
int build_lift(wacm_grid* g, const std::vector<Tab>& tabs, std::string& err) {
  g->n_lift = 0;
  if (g->wavelet != 1 || tabs.empty()) return WACM_OK;
  std::vector<int32_t> it;
  int64_t pts = 0, n_face = 0;
  if (int rc = lift_items(g, tabs, it, pts, n_face, err)) {
    g->n_lift = -1;
    return rc;
  }
  if (pts > (int64_t(1) << 30)) {  // staging offsets are int32
    g->n_lift = -1;
    err = "too many lifted ghost points";
    return WACM_E_CAPACITY;
  }
  const size_t es = g->d.dtype == WACM_F64 ? 8 : 4;
  const size_t ibytes = it.size() * sizeof(int32_t), tbytes = (size_t)pts * 4 * es;
  if (!g->d_lift || !g->d_lift_tmp || ibytes > g->lift_items_cap || tbytes > g->lift_tmp_cap) {
    g->n_lift = -1;
    err = "lifted ghost items exceed the wavelet workspace";
    return WACM_E_CAPACITY;
  }
  std::vector<int32_t> mask;
  if (int rc = lift_read_boxes(g, tabs, it, n_face, mask, err)) {
    g->n_lift = -1;
    return rc;
  }
  // table index of every pool slot (-1: inactive), after the boxes
  std::vector<int32_t> slot_ib((size_t)g->d.capacity, -1);
  for (size_t ib = 0; ib < tabs.size(); ++ib) slot_ib[tabs[ib].meta[0]] = (int32_t)ib;
  hipError_t e = hipSuccess;
  if (ibytes > 0) e = hipMemcpy(g->d_lift, it.data(), ibytes, hipMemcpyHostToDevice);
  if (e == hipSuccess && g->d_lift_mask && !mask.empty())
    e = hipMemcpy(g->d_lift_mask, mask.data(), sizeof(int32_t) * mask.size(),
                  hipMemcpyHostToDevice);
  if (e == hipSuccess && g->d_lift_mask)
    e = hipMemcpy(lift_slot_tab(g), slot_ib.data(), sizeof(int32_t) * slot_ib.size(),
                  hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    // no usable items: the lifted phase refuses to run until a rebuild works
    g->n_lift = -1;
    err = std::string("lifted ghost items: ") + hipGetErrorString(e);
    return WACM_E_HIP;
  }
  g->n_lift = (int64_t)it.size() / 12;
  g->n_lift_face = n_face;
  return WACM_OK;
}

// The tables become the grid's host copy by exchange: `tabs` receives the
// previous host copy, whose allocation the next build reuses.
int upload_tables(wacm_grid* g, std::vector<Tab>& tabs, std::string& err) {
  if (tabs.empty()) return WACM_OK;
  hipError_t e = hipMemcpy(g->d_tab, tabs.data(), sizeof(Tab) * tabs.size(),
                           hipMemcpyHostToDevice);
  std::vector<int32_t> cf = coarse_faces(tabs);
  if (e == hipSuccess && !cf.empty())
    e = hipMemcpy(g->d_cface, cf.data(), sizeof(int32_t) * cf.size(), hipMemcpyHostToDevice);
  std::vector<int32_t> cr = coarser_regions(tabs);
  if (e == hipSuccess && !cr.empty())
    e = hipMemcpy(g->d_cregion, cr.data(), sizeof(int32_t) * cr.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    err = std::string("hipMemcpy tables: ") + hipGetErrorString(e);
    return WACM_E_HIP;
  }
  g->n_cface = (int64_t)cf.size() / 2;
  g->n_cregion = (int64_t)cr.size() / 2;
  g->h_tab.swap(tabs);
  return build_lift(g, g->h_tab, err);
}

}  // namespace wacm
