// extern "C" entry points of libwacm (declared in include/wacm.h).
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>

#include "wacm_internal.h"

using namespace wacm;

namespace {
thread_local std::string g_err;
thread_local const wacm_grid* g_cur = nullptr;  // grid of the current entry point

// Every entry point that takes a grid opens a GridScope: a failure is then
// recorded for the calling thread and on the grid (wacm_last_error(grid)).
struct GridScope {
  const wacm_grid* prev;
  explicit GridScope(const wacm_grid* g) : prev(g_cur) { g_cur = g; }
  ~GridScope() { g_cur = prev; }
};

void record(const std::string& msg) {
  g_err = msg;
  if (g_cur) g_cur->last_err = msg;
}

int fail(int code, const std::string& msg) {
  record(msg);
  return code;
}

int hipfail(hipError_t e, const char* what) {
  record(std::string(what) + ": " + hipGetErrorString(e));
  return WACM_E_HIP;
}

bool elem_ok(const wacm_grid* g) { return g && (g->d.dtype == WACM_F32 || g->d.dtype == WACM_F64); }

// the two-dimensional path has no mask, sponge or extra solid velocity
int check_2d(const wacm_grid* g, const wacm_params* p, const void* dus) {
  if (g->dim != 2) return WACM_OK;
  if (p && (p->mask || p->sponge))
    return fail(WACM_E_INVAL, "two dimensions: no mask or sponge (params.mask, params.sponge 0)");
  if (dus) return fail(WACM_E_INVAL, "two dimensions: no extra solid velocity (dus NULL)");
  return WACM_OK;
}

int not_2d(const wacm_grid* g, const char* what) {
  return g->dim == 2 ? fail(WACM_E_INVAL, std::string(what) + " is not available in two dimensions")
                     : WACM_OK;
}

int check_params(const wacm_params* p) {
  if (!p) return fail(WACM_E_INVAL, "params is NULL");
  if (p->mask < 0 || p->mask > 2) return fail(WACM_E_INVAL, "unknown mask kind");
  if (p->mask && !(p->c_eta > 0)) return fail(WACM_E_INVAL, "c_eta must be > 0 with a mask");
  if (p->mask && !(p->w > 0)) return fail(WACM_E_INVAL, "mask width w must be > 0");
  if (p->sponge && !(p->c_sp > 0)) return fail(WACM_E_INVAL, "c_sp must be > 0 with a sponge");
  if (p->nu < 0) return fail(WACM_E_INVAL, "nu must be >= 0");
  return WACM_OK;
}

// Drops the references into the caller's buffers (the library never
// allocates device memory, so there is nothing to free) and the events of
// the profiler.
void free_dev(wacm_grid* g) {
  free_adj_plans(g);
  (void)profile_flush(g);
  for (hipEvent_t e : g->prof.spare) (void)hipEventDestroy(e);
  g->prof.spare.clear();
  for (hipEvent_t& e : g->adapt_ev) {
    if (e) (void)hipEventDestroy(e);
    e = nullptr;
  }
  g->ws = nullptr;
  g->d_lift = nullptr;
  g->d_lift_mask = nullptr;
  g->d_lift_tmp = nullptr;
  g->lift_items_cap = g->lift_tmp_cap = 0;
  g->n_lift = 0;
  g->d_cface = nullptr;
  g->d_cregion = nullptr;
  g->d_tab = nullptr;
  g->d_part = nullptr;
  g->d_norm = nullptr;
  g->d_queue = nullptr;
  g->d_list = nullptr;
}

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

// descriptor checks shared by wacm_workspace_bytes and wacm_grid_create
int check_desc(const wacm_grid_desc* d) {
  if (d->bs % 2 || d->bs < 2 * (d->ng + 3) || d->ng < 3 || d->bs > 64)
    return fail(WACM_E_INVAL, "bs must be even with 2(ng+3) <= bs <= 64 and ng >= 3");
  if (d->jmin < 0 || d->jmax > 18 || d->jmin > d->jmax)
    return fail(WACM_E_INVAL, "need 0 <= jmin <= jmax <= 18");
  if (d->dtype != WACM_F32 && d->dtype != WACM_F64) return fail(WACM_E_INVAL, "bad dtype");
  if (d->dim != 0 && d->dim != 2 && d->dim != 3) return fail(WACM_E_INVAL, "dim must be 2 or 3");
  if (!(d->L > 0)) return fail(WACM_E_INVAL, "L must be > 0");
  if (d->capacity <= 0 || d->capacity > (int64_t)1 << 30)
    return fail(WACM_E_INVAL, "need 0 < capacity <= 2^30");
  if (d->bs != 16 && d->bs != 24 && d->bs != 32)
    return fail(WACM_E_INVAL, "kernels are built for bs in {16, 24, 32}");
  return WACM_OK;
}

}  // namespace

namespace wacm {
void set_error(const std::string& s) { record(s); }
}  // namespace wacm

extern "C" {

const char* wacm_last_error(const wacm_grid* g) {
  return g ? g->last_err.c_str() : g_err.c_str();
}

size_t wacm_workspace_bytes(const wacm_grid_desc* d) {
  if (!d || check_desc(d) != WACM_OK) return 0;
  return ws_parts(d->capacity).total;
}

uint64_t wacm_treecode_encode(int32_t level, int64_t ix, int64_t iy, int64_t iz) {
  uint64_t code = 0;
  for (int l = 1; l <= level; ++l) {
    int sh = level - l;
    uint64_t d = ((uint64_t)(ix >> sh) & 1u) | (((uint64_t)(iy >> sh) & 1u) << 1) |
                 (((uint64_t)(iz >> sh) & 1u) << 2);
    code = (code << 3) | d;
  }
  return code;
}

void wacm_treecode_decode(uint64_t code, int32_t level, int64_t* ix, int64_t* iy, int64_t* iz) {
  int64_t x = 0, y = 0, z = 0;
  for (int l = 1; l <= level; ++l) {
    uint64_t d = (code >> (3 * (level - l))) & 7u;
    x = (x << 1) | (int64_t)(d & 1u);
    y = (y << 1) | (int64_t)((d >> 1) & 1u);
    z = (z << 1) | (int64_t)((d >> 2) & 1u);
  }
  if (ix) *ix = x;
  if (iy) *iy = y;
  if (iz) *iz = z;
}

int wacm_grid_create(const wacm_grid_desc* d, int64_t nleaves, const uint64_t* treecodes,
                     const int8_t* levels, void* workspace, size_t ws_bytes, wacm_grid** out) {
  if (!d || !out || !treecodes || !levels) return fail(WACM_E_INVAL, "NULL argument");
  *out = nullptr;
  if (int rc = check_desc(d)) return rc;
  if (nleaves <= 0 || nleaves > d->capacity)
    return fail(WACM_E_INVAL, "need 0 < nleaves <= capacity");
  const WsParts wp = ws_parts(d->capacity);
  if (!workspace) return fail(WACM_E_INVAL, "workspace is NULL");
  if (reinterpret_cast<uintptr_t>(workspace) % 256)
    return fail(WACM_E_INVAL, "workspace not 256-byte aligned");
  if (ws_bytes < wp.total) return fail(WACM_E_INVAL, "workspace smaller than wacm_workspace_bytes()");

  wacm_grid* g = new (std::nothrow) wacm_grid();
  if (!g) return fail(WACM_E_NOMEM, "host allocation");
  g->d = *d;
  g->dim = d->dim == 2 ? 2 : 3;
  g->P = d->bs + 2 * d->ng;
  const int vsh = g->dim;  // a level-J leaf covers 2^(dim (jmax - J)) finest boxes
  g->leaves.resize(nleaves);
  g->slots.resize(nleaves);
  // tiling: unique, in range, no leaf inside another, volumes add up
  std::unordered_map<uint64_t, int32_t> seen;
  seen.reserve(nleaves * 2);
  unsigned __int128 vol = 0;
  for (int64_t i = 0; i < nleaves; ++i) {
    int J = levels[i];
    if (J < d->jmin || J > d->jmax) {
      delete g;
      return fail(WACM_E_INVAL, "leaf level outside [jmin, jmax]");
    }
    if (J < 21 && (treecodes[i] >> (3 * J)) != 0) {
      delete g;
      return fail(WACM_E_INVAL, "treecode has digits beyond its level");
    }
    Leaf l;
    l.J = J;
    wacm_treecode_decode(treecodes[i], J, &l.x, &l.y, &l.z);
    if (g->dim == 2 && l.z != 0) {
      delete g;
      return fail(WACM_E_INVAL, "two dimensions: treecodes of (bx, by, 0) only");
    }
    if (!seen.emplace(leaf_key(J, l.x, l.y, l.z), (int32_t)i).second) {
      delete g;
      return fail(WACM_E_TILING, "repeated leaf");
    }
    g->leaves[i] = l;
    g->slots[i] = (int32_t)i;
    vol += (unsigned __int128)1 << (vsh * (d->jmax - J));
  }
  for (int64_t i = 0; i < nleaves; ++i) {
    const Leaf& l = g->leaves[i];
    for (int K = d->jmin; K < l.J; ++K) {
      int s = l.J - K;
      if (seen.count(leaf_key(K, l.x >> s, l.y >> s, l.z >> s))) {
        delete g;
        return fail(WACM_E_TILING, "a leaf lies inside another leaf");
      }
    }
  }
  if (vol != ((unsigned __int128)1 << (vsh * d->jmax))) {
    delete g;
    return fail(WACM_E_TILING, "leaves do not cover the domain");
  }
  for (int64_t s = d->capacity - 1; s >= nleaves; --s) g->free_slots.push_back((int32_t)s);
  reorder_leaves(g);

  std::vector<Tab> tabs;
  std::string err;
  int rc = build_tables(g, tabs, err);
  if (rc) {
    delete g;
    return fail(rc, err);
  }
  // every check passed: the tables go into the caller's workspace
  char* w = static_cast<char*>(workspace);
  g->ws = workspace;
  g->d_tab = reinterpret_cast<Tab*>(w + wp.tab);
  g->d_part = reinterpret_cast<double*>(w + wp.part);
  g->d_norm = reinterpret_cast<double*>(w + wp.norm);
  g->d_queue = reinterpret_cast<int32_t*>(w + wp.queue);
  g->d_list = reinterpret_cast<int32_t*>(w + wp.list);
  g->d_cface = reinterpret_cast<int32_t*>(w + wp.cface);
  g->d_cregion = reinterpret_cast<int32_t*>(w + wp.cregion);
  rc = upload_tables(g, tabs, err);
  if (rc) {
    free_dev(g);
    delete g;
    return fail(rc, err);
  }
  *out = g;
  return WACM_OK;
}

int wacm_grid_destroy(wacm_grid* g) {
  GridScope gs(g);
  if (!g) return WACM_OK;
  free_dev(g);
  delete g;
  return WACM_OK;
}

int64_t wacm_grid_nb(const wacm_grid* g) { return g ? g->nb : -1; }

int wacm_grid_info(const wacm_grid* g, int64_t* slots, uint64_t* treecodes, int8_t* levels) {
  GridScope gs(g);
  if (!g) return fail(WACM_E_INVAL, "NULL grid");
  for (int64_t i = 0; i < g->nb; ++i) {
    const Leaf& l = g->leaves[i];
    if (slots) slots[i] = g->slots[i];
    if (treecodes) treecodes[i] = wacm_treecode_encode(l.J, l.x, l.y, l.z);
    if (levels) levels[i] = (int8_t)l.J;
  }
  return WACM_OK;
}

size_t wacm_work_bytes(const wacm_grid* g) {
  GridScope gs(g);
  if (!g) return 0;
  if (g->dim == 2) return work_bytes_2d(g);
  return g->wavelet == WACM_CDF44 ? lift_work_bytes(g) : work_bytes(g);
}

int wacm_set_schedule(wacm_grid* g, const wacm_schedule* s) {
  GridScope gs(g);
  if (!g || !s) return fail(WACM_E_INVAL, "NULL argument");
  if (s->wg_per_cu < 0 || s->wg_per_cu > 16 || s->xcd_map < 0 || s->xcd_map > 2 ||
      s->prefetch < -1 || s->prefetch > 1 || (s->nontemporal != 0 && s->nontemporal != 1) ||
      (s->tile_rows != 0 && s->tile_rows != 8) || (s->pen_split < 0 || s->pen_split > 2))
    return fail(WACM_E_INVAL, "schedule value out of range");
  g->sched = *s;
  return WACM_OK;
}

int wacm_get_schedule(const wacm_grid* g, wacm_schedule* s) {
  GridScope gs(g);
  if (!g || !s) return fail(WACM_E_INVAL, "NULL argument");
  *s = g->sched;
  return WACM_OK;
}

// Full ghost fill with the grid's wavelet: the CDF 4/0 fill, then with CDF
// 4/4 the lifted values of ghost points whose owner is finer.
static hipError_t full_sync(const wacm_grid* g, void* U, hipStream_t st) {
  if (g->dim == 2) return launch_sync_2d(g, U, st);
  hipError_t e = launch_sync(g, U, 0, st);
  if (e == hipSuccess && g->wavelet == WACM_CDF44) e = launch_lift_sync(g, U, st);
  return e;
}

int wacm_sync_ghosts(wacm_grid* g, void* U, void* stream) {
  GridScope gs(g);
  if (!elem_ok(g) || !U) return fail(WACM_E_INVAL, "NULL argument");
  hipError_t e = full_sync(g, U, S(stream));
  return e == hipSuccess ? WACM_OK : hipfail(e, "sync_ghosts launch");
}

int wacm_sync_ghosts_lattice(wacm_grid* g, void* U, void* stream) {
  GridScope gs(g);
  if (!elem_ok(g) || !U) return fail(WACM_E_INVAL, "NULL argument");
  hipError_t e = g->dim == 3 && g->wavelet == WACM_CDF40 ? launch_sync_lattice(g, U, S(stream))
                                                         : full_sync(g, U, S(stream));
  return e == hipSuccess ? WACM_OK : hipfail(e, "sync_ghosts_lattice launch");
}

size_t wacm_wavelet_workspace_bytes(const wacm_grid* g, int32_t wavelet) {
  GridScope gs(g);
  if (!elem_ok(g) || wavelet != WACM_CDF44) return 0;
  return lift_ws_bytes(g->d.capacity, g->d.bs, g->d.ng, g->d.dtype == WACM_F64 ? 8 : 4);
}

int wacm_set_wavelet(wacm_grid* g, int32_t wavelet, void* ws, size_t ws_bytes) {
  GridScope gs(g);
  if (!elem_ok(g)) return fail(WACM_E_INVAL, "NULL argument");
  if (wavelet != WACM_CDF40 && wavelet != WACM_CDF44) return fail(WACM_E_INVAL, "wavelet");
  if (wavelet == WACM_CDF44) {
    if (int rc = not_2d(g, "CDF 4/4")) return rc;
    if (g->d.ng < 6)
      return fail(WACM_E_INVAL, "CDF 4/4 needs ng >= 6 (the lifted stencil reaches 6 fine points)");
    if (!ws || reinterpret_cast<uintptr_t>(ws) % 256)
      return fail(WACM_E_INVAL, "CDF 4/4 needs a 256-byte aligned wavelet workspace");
    if (ws_bytes < wacm_wavelet_workspace_bytes(g, WACM_CDF44))
      return fail(WACM_E_INVAL, "wavelet workspace smaller than wacm_wavelet_workspace_bytes()");
  }
  const int old = g->wavelet;
  int32_t* old_items = g->d_lift;
  int32_t* old_mask = g->d_lift_mask;
  void* old_tmp = g->d_lift_tmp;
  const size_t old_icap = g->lift_items_cap, old_tcap = g->lift_tmp_cap;
  g->wavelet = wavelet;
  if (wavelet == WACM_CDF44) {
    const size_t ib = lift_items_bytes(g->d.capacity);
    g->d_lift = static_cast<int32_t*>(ws);
    g->lift_items_cap = lift_list_bytes(g->d.capacity);
    g->d_lift_mask = reinterpret_cast<int32_t*>(static_cast<char*>(ws) + g->lift_items_cap);
    g->d_lift_tmp = static_cast<char*>(ws) + ib;
    g->lift_tmp_cap = ws_bytes - ib;
  } else {
    g->d_lift = nullptr;
    g->d_lift_mask = nullptr;
    g->d_lift_tmp = nullptr;
    g->lift_items_cap = g->lift_tmp_cap = 0;
  }
  std::string err;
  if (int rc = build_lift(g, g->h_tab, err)) {
    g->wavelet = old;
    g->d_lift = old_items;
    g->d_lift_mask = old_mask;
    g->d_lift_tmp = old_tmp;
    g->lift_items_cap = old_icap;
    g->lift_tmp_cap = old_tcap;
    build_lift(g, g->h_tab, err);
    return fail(rc, err);
  }
  return WACM_OK;
}

int wacm_get_wavelet(const wacm_grid* g) { return g ? g->wavelet : WACM_E_INVAL; }

int wacm_rhs_acm(wacm_grid* g, const wacm_params* p, double t, const void* U, void* dU,
                 const void* dus, void* stream) {
  GridScope gs(g);
  if (!elem_ok(g) || !U || !dU) return fail(WACM_E_INVAL, "NULL argument");
  if (int rc = check_params(p)) return rc;
  if (int rc = check_2d(g, p, dus)) return rc;
  hipError_t e = g->dim == 2 ? launch_rhs_2d(g, p, U, dU, S(stream))
                             : launch_rhs(g, p, t, U, dU, dus, S(stream));
  return e == hipSuccess ? WACM_OK : hipfail(e, "rhs_acm launch");
}

int wacm_compute_dt(wacm_grid* g, const wacm_params* p, const void* U, double* dt_dev,
                    void* stream) {
  GridScope gs(g);
  if (!elem_ok(g) || !U || !dt_dev) return fail(WACM_E_INVAL, "NULL argument");
  if (int rc = check_params(p)) return rc;
  if (int rc = check_2d(g, p, nullptr)) return rc;
  hipError_t e = g->dim == 2 ? launch_dt_2d(g, p, U, dt_dev, S(stream))
                             : launch_dt(g, p, U, dt_dev, S(stream));
  return e == hipSuccess ? WACM_OK : hipfail(e, "compute_dt launch");
}

static int rk4_common(wacm_grid* g, const wacm_params* p, double* t_dev, double* dt_dev, void* U,
                      void* work, const void* dus, int32_t dt_mode, int64_t nsteps,
                      void* stream, const char* what) {
  if (!elem_ok(g) || !U || !work || !t_dev || !dt_dev)
    return fail(WACM_E_INVAL, "NULL argument");
  if (dt_mode != WACM_DT_FIXED && dt_mode != WACM_DT_CFL) return fail(WACM_E_INVAL, "dt_mode");
  if (nsteps < 0) return fail(WACM_E_INVAL, "nsteps must be >= 0");
  if (reinterpret_cast<uintptr_t>(work) % 256) return fail(WACM_E_INVAL, "work not 256-aligned");
  if (int rc = check_params(p)) return rc;
  if (int rc = check_2d(g, p, dus)) return rc;
  if (g->dim == 2) {
    hipError_t e = launch_rk4_2d(g, p, t_dev, dt_dev, U, work, dt_mode, nsteps, S(stream));
    return e == hipSuccess ? WACM_OK : hipfail(e, what);
  }
  hipError_t e = g->wavelet == WACM_CDF44
                     ? launch_rk4_lifted(g, p, t_dev, dt_dev, U, work, dus, dt_mode, nsteps,
                                         S(stream))
                     : launch_rk4(g, p, t_dev, dt_dev, U, work, dus, dt_mode, nsteps, S(stream));
  return e == hipSuccess ? WACM_OK : hipfail(e, what);
}

int wacm_rk4_step(wacm_grid* g, const wacm_params* p, double* t_dev, double* dt_dev, void* U,
                  void* work, const void* dus, int32_t dt_mode, void* stream) {
  GridScope gs(g);
  return rk4_common(g, p, t_dev, dt_dev, U, work, dus, dt_mode, 1, stream, "rk4_step launch");
}

int wacm_rk4_steps(wacm_grid* g, const wacm_params* p, double* t_dev, double* dt_dev, void* U,
                   void* work, const void* dus, int32_t dt_mode, int64_t nsteps, void* stream) {
  GridScope gs(g);
  return rk4_common(g, p, t_dev, dt_dev, U, work, dus, dt_mode, nsteps, stream,
                    "rk4_steps launch");
}

int wacm_diagnostics(wacm_grid* g, const wacm_params* p, double t, const void* U,
                     const void* dus, double* out, void* stream) {
  GridScope gs(g);
  if (!elem_ok(g) || !U || !out) return fail(WACM_E_INVAL, "NULL argument");
  if (int rc = check_params(p)) return rc;
  if (int rc = check_2d(g, p, dus)) return rc;
  hipError_t e = g->dim == 2 ? launch_diag_2d(g, U, out, S(stream))
                             : launch_diag(g, p, t, U, dus, out, S(stream));
  if (e != hipSuccess) return hipfail(e, "diagnostics launch");
  double h[10];
  e = hipMemcpyAsync(h, out, sizeof(h), hipMemcpyDeviceToHost, S(stream));
  if (e == hipSuccess) e = hipStreamSynchronize(S(stream));
  if (e != hipSuccess) return hipfail(e, "diagnostics read-back");
  if (h[9] > 0)
    return fail(WACM_E_NONFINITE, std::to_string((int64_t)h[9]) +
                                      " interior values of the state are NaN or Inf");
  return WACM_OK;
}

int wacm_threshold_blocks(wacm_grid* g, const wacm_params* p, double t, const void* U,
                          double eps, int32_t dealias, double* dmax, double* mrange,
                          int8_t* flags, void* stream) {
  GridScope gs(g);
  if (!elem_ok(g) || !U || !dmax || !mrange || !flags) return fail(WACM_E_INVAL, "NULL argument");
  if (int rc = check_params(p)) return rc;
  if (!(eps >= 0)) return fail(WACM_E_INVAL, "eps must be >= 0");
  if (int rc = check_2d(g, p, nullptr)) return rc;
  hipError_t e = g->dim == 2
                     ? launch_threshold_2d(g, U, eps, dealias, dmax, mrange, flags, S(stream))
                     : launch_threshold(g, p, t, U, eps, dealias, dmax, mrange, flags, S(stream));
  return e == hipSuccess ? WACM_OK : hipfail(e, "threshold_blocks launch");
}

int wacm_filter_blocks(wacm_grid* g, void* U, int32_t level, void* stream) {
  GridScope gs(g);
  if (!elem_ok(g) || !U) return fail(WACM_E_INVAL, "NULL argument");
  if (int rc = not_2d(g, "wavelet filtering")) return rc;
  if (g->wavelet != WACM_CDF40) return fail(WACM_E_INVAL, "filtering is CDF 4/0 only");
  hipError_t e = launch_filter(g, U, level, S(stream));
  return e == hipSuccess ? WACM_OK : hipfail(e, "filter_blocks launch");
}

int wacm_adapt(wacm_grid* g, int32_t op, const int8_t* flags, void* U, int64_t* nb_out,
               void* stream) {
  const auto t_call = std::chrono::steady_clock::now();
  GridScope gs(g);
  if (!elem_ok(g) || !U) return fail(WACM_E_INVAL, "NULL argument");
  hipStream_t st = S(stream);
  const int bs = g->d.bs;
  (void)bs;
  std::vector<int32_t> list;
  std::vector<Leaf> newleaves;
  std::vector<int32_t> newslots;
  std::vector<int32_t> freed;
  std::vector<int32_t> freelist = g->free_slots;
  auto take = [&](int32_t& s) -> bool {
    if (freelist.empty()) return false;
    s = freelist.back();
    freelist.pop_back();
    return true;
  };
  int64_t nwork = 0;
  const int nchild = g->dim == 2 ? 4 : 8;  // children of a block
  if (op == WACM_REFINE_ALL) {
    for (int64_t i = 0; i < g->nb; ++i) {
      const Leaf& l = g->leaves[i];
      if (l.J >= g->d.jmax) {
        newleaves.push_back(l);
        newslots.push_back(g->slots[i]);
        continue;
      }
      for (int c = 0; c < nchild; ++c) {
        Leaf ch{l.J + 1, 2 * l.x + (c & 1), 2 * l.y + ((c >> 1) & 1), 2 * l.z + ((c >> 2) & 1)};
        int32_t s;
        if (!take(s)) return fail(WACM_E_CAPACITY, "refinement needs more pool slots");
        newleaves.push_back(ch);
        newslots.push_back(s);
        list.push_back(g->slots[i]);
        list.push_back(s);
        list.push_back(c);
        ++nwork;
      }
      freed.push_back(g->slots[i]);
    }
  } else if (op == WACM_COARSEN) {
    if (!flags) return fail(WACM_E_INVAL, "flags is NULL");
    // a family merges iff its 8 sisters are active and flagged and no active
    // block touching the parent box is finer than the sisters
    std::vector<char> done(g->nb, 0);
    for (int64_t i = 0; i < g->nb; ++i) {
      if (done[i]) continue;
      const Leaf& l = g->leaves[i];
      bool merge = flags[i] && l.J > g->d.jmin;
      int32_t sis[8];
      int64_t sidx[8];
      int64_t px = l.x >> 1, py = l.y >> 1, pz = l.z >> 1;
      if (merge) {
        for (int c = 0; c < nchild && merge; ++c) {
          const int32_t si = g->index.find(
              leaf_key(l.J, 2 * px + (c & 1), 2 * py + ((c >> 1) & 1), 2 * pz + ((c >> 2) & 1)));
          if (si < 0 || !flags[si]) {
            merge = false;
          } else {
            sidx[c] = si;
            sis[c] = g->slots[si];
          }
        }
      }
      if (merge) {
        // grading: the parent (level J-1) must not touch a leaf of level
        // J+1.  Such a leaf lies in a neighbour region of some sister outside
        // the family, which the sister's table then marks finer; conversely
        // every finer region of a sister holds leaves of level J+1 touching
        // the sister, hence the parent box.
        for (int c = 0; c < nchild && merge; ++c) {
          const int8_t* kd = g->h_tab[sidx[c]].kind;
          for (int r = 0; r < 27; ++r)
            if (kd[r] > 0) {
              merge = false;
              break;
            }
        }
      }
      if (!merge) {
        done[i] = 1;
        newleaves.push_back(l);
        newslots.push_back(g->slots[i]);
        continue;
      }
      int32_t s;
      if (!take(s)) return fail(WACM_E_CAPACITY, "coarsening needs a free pool slot");
      Leaf p{l.J - 1, px, py, pz};
      newleaves.push_back(p);
      newslots.push_back(s);
      list.push_back(s);
      for (int c = 0; c < 8; ++c) {
        if (c >= nchild) {
          list.push_back(-1);
          continue;
        }
        list.push_back(sis[c]);
        done[sidx[c]] = 1;
        freed.push_back(sis[c]);
      }
      list.push_back(0);
      ++nwork;
    }
  } else {
    return fail(WACM_E_INVAL, "unknown adapt op");
  }
  if (nwork == 0) {
    // nothing to refine or merge: the leaves, slots and tables stay; the
    // adjoint plans are dropped all the same, as after any adaptation
    free_adj_plans(g);
    if (nb_out) *nb_out = g->nb;
    g->adapt_ms[0] =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_call).count();
    g->adapt_ms[1] = 0.0;
    return WACM_OK;
  }
  // the new leaf set in Morton order; the kernels below need only the work
  // list, so they are launched first and the new tables are built on the host
  // while they run.  Before the tables are known to be valid only free pool
  // slots and ghost layers are written: on error the grid and the active
  // blocks' interiors are unchanged.
  wacm_grid tmp;
  tmp.d = g->d;
  tmp.dim = g->dim;
  tmp.P = g->P;
  tmp.leaves.swap(newleaves);
  tmp.slots.swap(newslots);
  reorder_leaves(&tmp);
  hipError_t e;
  for (hipEvent_t& ev : g->adapt_ev)
    if (!ev && (e = hipEventCreate(&ev)) != hipSuccess) return hipfail(e, "adapt event");
  if ((e = hipEventRecord(g->adapt_ev[0], st)) != hipSuccess) return hipfail(e, "adapt event");
  if (op == WACM_REFINE_ALL) {
    e = full_sync(g, U, st);
    if (e != hipSuccess) return hipfail(e, "adapt sync");
  }
  e = hipMemcpyAsync(g->d_list, list.data(), sizeof(int32_t) * list.size(),
                     hipMemcpyHostToDevice, st);
  if (e != hipSuccess) return hipfail(e, "adapt list upload");
  if (g->dim == 2)
    e = op == WACM_REFINE_ALL ? launch_prolong_2d(g, U, nwork, st)
                              : launch_decimate_2d(g, U, nwork, st);
  else if (op == WACM_REFINE_ALL)
    e = launch_prolong(g, U, nwork, st);
  else
    e = g->wavelet == WACM_CDF44 ? launch_lift_coarsen(g, U, nwork, st)
                                 : launch_decimate(g, U, nwork, st);
  if (e != hipSuccess) return hipfail(e, "adapt kernel");
  if ((e = hipEventRecord(g->adapt_ev[1], st)) != hipSuccess) return hipfail(e, "adapt event");
  std::vector<Tab>& tabs = g->h_tab_next;
  std::string err;
  int rc = build_tables(&tmp, tabs, err);
  e = hipStreamSynchronize(st);
  if (rc) return fail(rc, err);
  if (e != hipSuccess) return hipfail(e, "adapt synchronize");
  float dev_ms = 0.0f;
  if ((e = hipEventElapsedTime(&dev_ms, g->adapt_ev[0], g->adapt_ev[1])) != hipSuccess)
    return hipfail(e, "adapt event");
  for (int32_t s : freed) freelist.push_back(s);
  g->leaves.swap(tmp.leaves);
  g->slots.swap(tmp.slots);
  g->index.swap(tmp.index);
  g->nb = tmp.nb;
  g->jfine = tmp.jfine;
  g->free_slots.swap(freelist);
  free_adj_plans(g);
  rc = upload_tables(g, tabs, err);
  if (rc) return fail(rc, err);
  if (nb_out) *nb_out = g->nb;
  const double all_ms =
      std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_call).count();
  g->adapt_ms[0] = all_ms - dev_ms;
  g->adapt_ms[1] = dev_ms;
  return WACM_OK;
}

int wacm_adapt_timing(const wacm_grid* g, double* ms) {
  GridScope gs(g);
  if (!g || !ms) return fail(WACM_E_INVAL, "NULL argument");
  ms[0] = g->adapt_ms[0];
  ms[1] = g->adapt_ms[1];
  return WACM_OK;
}

size_t wacm_adj_work_bytes(const wacm_grid* g) { return g ? adj_work_bytes(g) : 0; }

size_t wacm_adj_plan_bytes(wacm_grid* g, int32_t face_only) {
  GridScope gs(g);
  if (!elem_ok(g) || (face_only != 0 && face_only != 1)) return 0;
  std::string err;
  if (build_adj_plan(g, face_only, err)) return 0;
  return adj_plan_bytes(g->plan[face_only]);
}

int wacm_adj_plan_set(wacm_grid* g, int32_t face_only, void* ws, size_t ws_bytes) {
  GridScope gs(g);
  if (!elem_ok(g) || !ws) return fail(WACM_E_INVAL, "NULL argument");
  if (int rc = not_2d(g, "the adjoint")) return rc;
  if (face_only != 0 && face_only != 1) return fail(WACM_E_INVAL, "face_only must be 0 or 1");
  if (g->wavelet != WACM_CDF40) return fail(WACM_E_INVAL, "the adjoint is CDF 4/0 only");
  if (reinterpret_cast<uintptr_t>(ws) % 256)
    return fail(WACM_E_INVAL, "plan buffer not 256-byte aligned");
  std::string err;
  if (int rc = upload_adj_plan(g, face_only, ws, ws_bytes, err)) return fail(rc, err);
  return WACM_OK;
}

int wacm_sync_ghosts_adj(wacm_grid* g, void* Ub, void* stream) {
  GridScope gs(g);
  if (!elem_ok(g) || !Ub) return fail(WACM_E_INVAL, "NULL argument");
  if (int rc = not_2d(g, "the adjoint")) return rc;
  if (g->wavelet != WACM_CDF40) return fail(WACM_E_INVAL, "the adjoint is CDF 4/0 only");
  if (!g->plan[0].built)
    return fail(WACM_E_INVAL, "no plan of the ghost-fill transpose: wacm_adj_plan_set(grid, 0, ...)");
  hipError_t e = launch_sync_adj(g, Ub, 0, S(stream));
  return e == hipSuccess ? WACM_OK : hipfail(e, "sync_ghosts_adj launch");
}

int wacm_rhs_acm_adj(wacm_grid* g, const wacm_params* p, double t, const void* U, const void* V,
                     void* Ub, double* dtheta, double* dusbar, const void* dus, void* stream) {
  GridScope gs(g);
  if (!elem_ok(g) || !U || !V || !Ub || !dtheta) return fail(WACM_E_INVAL, "NULL argument");
  if (int rc = not_2d(g, "the adjoint")) return rc;
  if (g->wavelet != WACM_CDF40) return fail(WACM_E_INVAL, "the adjoint is CDF 4/0 only");
  if (int rc = check_params(p)) return rc;
  hipError_t e = launch_rhs_adj(g, p, t, U, V, Ub, dtheta, dusbar, dus, S(stream));
  return e == hipSuccess ? WACM_OK : hipfail(e, "rhs_acm_adj launch");
}

int wacm_force_adj(wacm_grid* g, const wacm_params* p, double t, double weight, const void* U,
                   void* Ub, double* dtheta, double* dusbar, const void* dus, void* stream) {
  GridScope gs(g);
  if (!elem_ok(g) || !U || !Ub || !dtheta) return fail(WACM_E_INVAL, "NULL argument");
  if (int rc = not_2d(g, "the adjoint")) return rc;
  if (g->wavelet != WACM_CDF40) return fail(WACM_E_INVAL, "the adjoint is CDF 4/0 only");
  if (int rc = check_params(p)) return rc;
  hipError_t e = launch_force_adj(g, p, t, weight, U, Ub, dtheta, dusbar, dus, S(stream));
  return e == hipSuccess ? WACM_OK : hipfail(e, "force_adj launch");
}

int wacm_rk4_step_adj(wacm_grid* g, const wacm_params* p, double t, double dt, const void* Un,
                      void* lam, double* dtheta, double* dusbar, const void* dus, void* work,
                      void* stream) {
  GridScope gs(g);
  if (!elem_ok(g) || !Un || !lam || !dtheta || !work) return fail(WACM_E_INVAL, "NULL argument");
  if (int rc = not_2d(g, "the adjoint")) return rc;
  if (g->wavelet != WACM_CDF40) return fail(WACM_E_INVAL, "the adjoint is CDF 4/0 only");
  if (reinterpret_cast<uintptr_t>(work) % 256) return fail(WACM_E_INVAL, "work not 256-aligned");
  if (int rc = check_params(p)) return rc;
  if (!g->plan[1].built)
    return fail(WACM_E_INVAL, "no plan of the face-star transpose: wacm_adj_plan_set(grid, 1, ...)");
  hipError_t e = launch_rk4_adj(g, p, t, dt, Un, lam, dtheta, dusbar, dus, work, S(stream));
  return e == hipSuccess ? WACM_OK : hipfail(e, "rk4_step_adj launch");
}

int wacm_profile_enable(wacm_grid* g, int32_t on) {
  GridScope gs(g);
  if (!g) return fail(WACM_E_INVAL, "NULL grid");
  g->prof.on = on != 0;
  return WACM_OK;
}

int wacm_profile_read(wacm_grid* g, double* ms, int64_t* launches) {
  GridScope gs(g);
  if (!g || !ms || !launches) return fail(WACM_E_INVAL, "NULL argument");
  hipError_t e = profile_flush(g);
  for (int c = 0; c < 4; ++c) {
    ms[c] = g->prof.ms[c];
    launches[c] = g->prof.n[c];
    g->prof.ms[c] = 0.0;
    g->prof.n[c] = 0;
  }
  return e == hipSuccess ? WACM_OK : hipfail(e, "profile events");
}

}  // extern "C"
