// C ABI of libpamd: argument validation, launch planning, workspace layout,
// dispatch, batches, path sampling, autotuning and graph capture.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "internal.hpp"
#include "pamd.h"

using namespace pamd;

namespace {

thread_local std::string g_err;
thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

// Records the one-shot measurement events around the main kernel of a call.
struct EventScope {
  hipStream_t st;
  hipEvent_t a, b;
  explicit EventScope(hipStream_t s) : st(s), a(g_ev_start), b(g_ev_stop) {
    g_ev_start = g_ev_stop = nullptr;
    if (a) hipEventRecord(a, st);
  }
  ~EventScope() {
    if (b) hipEventRecord(b, st);
  }
};

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define PAMD_HIP(expr)                                                                 \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess) return fail(PAMD_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

constexpr size_t kLdsMax = 163840;  // LDS per workgroup on gfx950
constexpr int kMaxGrid = 2048;      // persistent-grid cap: bounds per-block scratch
constexpr size_t kAlign = 256;
constexpr double kDefaultSkin = 0.5;  // in units of sigma

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

// ---------------------------------------------------------------------------
// Validation
// ---------------------------------------------------------------------------
int check_path(const pamd_path* p) {
  if (!p) return fail(PAMD_EINVAL, "path is NULL");
  if (p->n_steps < 1) return fail(PAMD_EINVAL, "n_steps must be >= 1 (got %lld)", (long long)p->n_steps);
  if (p->n_atoms < 1) return fail(PAMD_EINVAL, "n_atoms must be >= 1 (got %d)", p->n_atoms);
  if (p->n_dim != 1 && p->n_dim != 3)
    return fail(PAMD_EUNSUPPORTED, "n_dim must be 1 or 3 (got %d)", p->n_dim);
  if (!finite_pos(p->dt)) return fail(PAMD_EINVAL, "dt must be finite and > 0");
  if (!finite_pos(p->D)) return fail(PAMD_EINVAL, "D must be finite and > 0");
  if (!finite_pos(p->gamma)) return fail(PAMD_EINVAL, "gamma must be finite and > 0");
  if (p->precision != PAMD_FP64 && p->precision != PAMD_FP32_FORCE)
    return fail(PAMD_EINVAL, "precision must be PAMD_FP64 or PAMD_FP32_FORCE (got %d)", p->precision);
  const double elems = (double)(p->n_steps + 1) * p->n_dim * p->n_atoms;
  if (elems > 9.0e15) return fail(PAMD_EINVAL, "path too large");
  return PAMD_OK;
}

int check_pot(const pamd_path* p, const pamd_potential* v) {
  if (!v) return fail(PAMD_EINVAL, "potential is NULL");
  if (v->kind == PAMD_HARMONIC) {
    if (!std::isfinite(v->k)) return fail(PAMD_EINVAL, "harmonic k must be finite");
    if (v->box != 0.0) return fail(PAMD_EUNSUPPORTED, "harmonic potential takes no periodic box (box must be 0)");
    return PAMD_OK;
  }
  if (v->kind != PAMD_LJ) return fail(PAMD_EINVAL, "unknown potential kind %d", v->kind);
  if (p->n_dim != 3) return fail(PAMD_EUNSUPPORTED, "Lennard-Jones paths need n_dim = 3 (got %d)", p->n_dim);
  if (!finite_pos(v->eps)) return fail(PAMD_EINVAL, "eps must be finite and > 0");
  if (!finite_pos(v->sigma)) return fail(PAMD_EINVAL, "sigma must be finite and > 0");
  if (!finite_pos(v->rc)) return fail(PAMD_EINVAL, "rc must be finite and > 0");
  if (!finite_pos(v->box)) return fail(PAMD_EINVAL, "box must be finite and > 0");
  if (v->rc > 0.5 * v->box)
    return fail(PAMD_EUNSUPPORTED, "rc = %g exceeds half the box (%g): minimum image would miss pairs", v->rc, 0.5 * v->box);
  if (p->n_atoms > 65535) return fail(PAMD_EUNSUPPORTED, "Lennard-Jones paths support at most 65535 atoms");
  return PAMD_OK;
}

int check_tuning(const pamd_tuning* t) {
  if (!t) return PAMD_OK;
  if (t->algo < PAMD_ALGO_AUTO || t->algo > PAMD_ALGO_PLAIN) return fail(PAMD_EINVAL, "unknown algo %d", t->algo);
  if (t->block != 0 && (t->block < 64 || t->block > 1024 || t->block % 64))
    return fail(PAMD_EINVAL, "block must be 0 or a multiple of 64 in [64, 1024] (got %d)", t->block);
  if (t->tile < 0) return fail(PAMD_EINVAL, "tile must be >= 0");
  if (t->max_neighbours < 0) return fail(PAMD_EINVAL, "max_neighbours must be >= 0");
  if (!std::isfinite(t->skin)) return fail(PAMD_EINVAL, "skin must be finite");
  if (t->neighbour_list < PAMD_LIST_AUTO || t->neighbour_list > PAMD_LIST_HALF)
    return fail(PAMD_EINVAL, "unknown neighbour_list %d", t->neighbour_list);
  if (t->slot_arrays < 0 || t->slot_arrays > 2)
    return fail(PAMD_EINVAL, "slot_arrays must be 0, 1 or 2 (got %d)", t->slot_arrays);
  return PAMD_OK;
}

// ---------------------------------------------------------------------------
// Autotune cache
// ---------------------------------------------------------------------------
std::mutex g_tune_mu;
std::map<std::string, pamd_tuning> g_tune;

std::string tune_key(const pamd_path* p, const pamd_potential* v) {
  char buf[160];
  int lg = 0;
  while (((int64_t)1 << (lg + 1)) <= p->n_steps) ++lg;
  snprintf(buf, sizeof(buf), "%d/%d/%d/%d/%.6g/%.6g", v->kind, p->n_atoms, p->precision, lg,
           v->kind == PAMD_LJ ? v->box : 0.0, v->kind == PAMD_LJ ? v->rc : 0.0);
  return buf;
}

bool cached_tuning(const pamd_path* p, const pamd_potential* v, pamd_tuning* out) {
  std::lock_guard<std::mutex> lk(g_tune_mu);
  auto it = g_tune.find(tune_key(p, v));
  if (it == g_tune.end()) return false;
  *out = it->second;
  return true;
}

// ---------------------------------------------------------------------------
// Planning
// ---------------------------------------------------------------------------
int default_kmax(double box, double radius, int n_atoms) {
  const double rho = n_atoms / (box * box * box);
  const double expect = 4.0 / 3.0 * M_PI * radius * radius * radius * rho;
  int k = (int)align_up((size_t)std::ceil(1.3 * expect + 24.0), 8);
  return std::max(1, std::min(k, n_atoms - 1 > 0 ? n_atoms - 1 : 1));
}

// Half lists: one atom per thread up to 1024 atoms, else the fewest atoms
// per thread.  Full lists: two threads per atom, up to 1024 threads.
int default_block(int n_atoms, bool half) {
  if (!half) return std::max(64, std::min(1024, (int)align_up((size_t)2 * n_atoms, 64)));
  int per = (n_atoms + 1023) / 1024;
  int b = (int)align_up((size_t)((n_atoms + per - 1) / per), 64);
  return std::max(64, std::min(1024, b));
}

struct Plan {
  int kind = 0;
  bool f32 = false;
  int algo = PAMD_ALGO_FUSED;
  int64_t steps = 0;
  int N = 0, dim = 0;
  int64_t dof = 0;
  // fused LJ
  int block = 0, tile = 0, n_tiles = 0, grid = 0, kmax = 0;
  CellGrid cells;
  double skin = 0;
  bool r_in_lds = true;
  bool lds2 = true;  // with r_in_lds: two slot arrays
  bool exl = false;  // exact lists in LDS (one slot array)
  bool half = false;
  size_t lds = 0;
  // plain LJ
  CellGrid pcells;
  int pkmax = 0;
  size_t plds = 0;
  // harmonic
  int seg = 1;
  // workspace (byte offsets)
  size_t off_step = 0, off_bnd = 0, off_nbr = 0, off_cnt = 0, off_xref = 0, off_rglob = 0;
  size_t nbr_stride = 0, cnt_stride = 0, xref_stride = 0, rglob_stride = 0;  // elements
  size_t off_pnbr = 0, off_pcnt = 0, off_F = 0, off_R = 0, off_Q = 0;
  size_t off_mh_ex = 0, off_mh_state = 0, off_mh_acc = 0;
  size_t total = 0;
};

size_t bump(size_t& cur, size_t bytes) {
  const size_t at = align_up(cur, kAlign);
  cur = at + bytes;
  return at;
}

// use_cache = false: fields left at 0 take the planner's own choices even
// when the autotuner has cached others for this problem.
int make_plan(const pamd_path* p, const pamd_potential* v, const pamd_tuning* t_in, bool mh,
              Plan& P, int grid_cap = kMaxGrid, bool use_cache = true) {
  int rc;
  if ((rc = check_path(p)) || (rc = check_pot(p, v)) || (rc = check_tuning(t_in))) return rc;
  pamd_tuning t{};
  if (t_in) t = *t_in;
  pamd_tuning cached{};
  const bool have_cache = use_cache && cached_tuning(p, v, &cached);
  P.kind = v->kind;
  P.steps = p->n_steps;
  P.N = p->n_atoms;
  P.dim = p->n_dim;
  P.dof = (int64_t)p->n_dim * p->n_atoms;
  P.f32 = v->kind == PAMD_LJ && p->precision == PAMD_FP32_FORCE;
  P.algo = t.algo == PAMD_ALGO_PLAIN ? PAMD_ALGO_PLAIN : PAMD_ALGO_FUSED;
  size_t cur = 0;
  P.off_step = bump(cur, sizeof(double) * P.steps);
  if (v->kind == PAMD_HARMONIC) {
    int seg = 1;
    while (seg < 64 && seg < P.dof) seg <<= 1;
    P.seg = seg;
  } else if (P.algo == PAMD_ALGO_FUSED) {
    const int N = P.N;
    const double L = v->box;
    P.skin = t.skin > 0 ? t.skin : (have_cache && cached.skin > 0 ? cached.skin : kDefaultSkin * v->sigma);
    const double radius = v->rc + P.skin;
    P.kmax = t.max_neighbours > 0 ? std::min(t.max_neighbours, std::max(1, N - 1))
                                  : default_kmax(L, radius, N);
    P.kmax = (int)align_up((size_t)P.kmax, 8);  // lists are read in chunks of 8
    int list = t.neighbour_list ? t.neighbour_list
                                : (have_cache && cached.neighbour_list ? cached.neighbour_list : PAMD_LIST_AUTO);
    P.block = t.block ? t.block
                      : (have_cache && cached.block ? cached.block
                                                    : default_block(N, list == PAMD_LIST_HALF));
    P.half = list == PAMD_LIST_HALF;  // automatic choice: full lists (repeatable, as fast)
    if (P.half && N > fused_half_slots() * P.block)
      return fail(PAMD_EUNSUPPORTED, "half lists need n_atoms <= %d * block", fused_half_slots());
    // residuals in LDS with two slot arrays when they fit (unless one is
    // asked for), else with one, else in global scratch
    const int slots = t.slot_arrays ? t.slot_arrays
                                    : (have_cache && cached.slot_arrays ? cached.slot_arrays : 0);
    // full lists with one slot per thread: the exact lists can live in LDS
    // (one slot array) when they fit; that is the default
    if (!P.half && slots != 2 && N <= P.block) {
      const CellGrid g = choose_cells(L, radius, N, 1 << 30);
      const size_t b = exl_lds_bytes(N, g.nc, P.block);
      if (b <= kLdsMax) {
        P.exl = true;
        P.cells = g;
        P.lds = b;
        P.r_in_lds = true;
        P.lds2 = false;
      }
    }
    if (P.exl) {
    } else if (slots != 1 && fused_cells_fit(L, radius, N, P.block, true, P.half, &P.cells, &P.lds, true)) {
      P.r_in_lds = true;
      P.lds2 = true;
    } else if (fused_cells_fit(L, radius, N, P.block, true, P.half, &P.cells, &P.lds, false)) {
      P.r_in_lds = true;
      P.lds2 = false;
    } else if (fused_cells_fit(L, radius, N, P.block, false, P.half, &P.cells, &P.lds)) {
      P.r_in_lds = false;
      P.lds2 = false;
    } else {
      return fail(PAMD_EUNSUPPORTED, "n_atoms = %d needs %zu bytes of LDS per workgroup (max %zu)", N,
                  fused_lds_bytes(N, 0, false, P.half, P.block), kLdsMax);
    }
    int tile = t.tile ? t.tile : (have_cache && cached.tile ? cached.tile : 0);
    if (tile <= 0) {
      // Enough tiles for every CU to hold as many workgroups as its wave slots
      // (16 at this kernel's register use) and LDS allow: small systems get
      // short tiles, since a workgroup walks its tile's steps in sequence.
      const int waves = (P.block + 63) / 64;
      const int by_lds = (int)std::max<size_t>(1, kLdsMax / std::max<size_t>(P.lds, 1));
      const int per_cu = std::max(1, std::min(16 / waves, by_lds));
      const int64_t slots = 256LL * per_cu;
      tile = (int)std::max<int64_t>(1, std::min<int64_t>(32, (P.steps + slots - 1) / slots));
    }
    P.tile = (int)std::min<int64_t>(tile, P.steps);
    P.n_tiles = (int)((P.steps + P.tile - 1) / P.tile);
    // No cell grid, a list sphere holding most of the box and tiles of one or
    // two steps: the list build would cost more than scanning all atoms in
    // both passes (without lists a slice costs ~1.5x, the build ~1.4 slices,
    // at 108 atoms), so the plan keeps no lists (reach -1) unless a list
    // capacity or a skin is asked for.
    if (P.exl && P.cells.nc == 0 && P.tile <= 2 && t.max_neighbours == 0 && t.skin == 0 &&
        4.0 / 3.0 * M_PI * radius * radius * radius >= 0.6 * L * L * L)
      P.cells.reach = -1;
    P.grid = std::min(P.n_tiles, std::max(1, std::min(grid_cap, kMaxGrid)));
    P.off_bnd = bump(cur, sizeof(double) * 3 * N * (size_t)std::max(0, P.n_tiles - 1));
    // neighbour lists (two rows per atom, each with a spare chunk: kmax + 32
    // per atom), then, unless the exact lists stay in LDS, room for exact
    // lists of the same size
    P.nbr_stride = (P.exl ? 1 : 2) * align_up((size_t)(P.kmax + 32) * N, 128);
    P.cnt_stride = align_up((size_t)2 * N, 64);  // list lengths: up to two rows per atom
    P.xref_stride = align_up((size_t)6 * N, 32);
    // global scratch: residuals, or with one LDS slot array the list reaches
    // (and the sequential integrator's sort scratch)
    P.rglob_stride = P.r_in_lds && P.lds2 ? 0 : align_up((size_t)3 * N, 32);
    P.off_nbr = bump(cur, sizeof(uint16_t) * P.nbr_stride * P.grid);
    P.off_cnt = bump(cur, sizeof(int32_t) * P.cnt_stride * P.grid);
    P.off_xref = bump(cur, sizeof(double) * P.xref_stride * P.grid);
    P.off_rglob = bump(cur, sizeof(double) * P.rglob_stride * P.grid);
  } else {
    const int N = P.N;
    P.pcells = choose_cells(v->box, v->rc, N, 1 << 30, 0.5);
    P.pkmax = t.max_neighbours > 0 ? std::min(t.max_neighbours, std::max(1, N - 1))
                                   : default_kmax(v->box, v->rc, N);
    // one thread per atom where a workgroup holds them all
    P.block = t.block ? t.block : (int)std::min<size_t>(1024, align_up((size_t)N, 64));
    P.plds = plain_lds_bytes(N, P.pcells.nc);
    if (P.plds > kLdsMax)
      return fail(PAMD_EUNSUPPORTED, "plain form: n_atoms = %d needs %zu bytes of LDS (max %zu)", N, P.plds, kLdsMax);
    const size_t S = (size_t)P.steps;
    P.off_pnbr = bump(cur, sizeof(uint16_t) * S * P.pkmax * N);
    P.off_pcnt = bump(cur, sizeof(int32_t) * S * N);
    P.off_F = bump(cur, sizeof(double) * S * 3 * N);
    P.off_R = bump(cur, sizeof(double) * S * 3 * N);
    P.off_Q = bump(cur, sizeof(double) * S * 3 * N);
  }
  if (mh) {
    P.off_mh_ex = bump(cur, sizeof(double) * P.steps);
    P.off_mh_state = bump(cur, sizeof(int32_t) * 4);
    P.off_mh_acc = bump(cur, sizeof(int32_t) * (P.steps + 2));
  }
  P.total = align_up(cur, kAlign);
  return PAMD_OK;
}

int check_ws(const Plan& P, void* ws, size_t ws_bytes) {
  if (ws_bytes < P.total)
    return fail(PAMD_EWORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, P.total);
  if (P.total && !ws) return fail(PAMD_EINVAL, "workspace is NULL");
  if (((uintptr_t)ws) % kAlign) return fail(PAMD_EWORKSPACE, "workspace must be 256-byte aligned");
  return PAMD_OK;
}

template <typename T>
T* at(void* ws, size_t off) {
  return reinterpret_cast<T*>(reinterpret_cast<char*>(ws) + off);
}

void fill_lj(const pamd_path* p, const pamd_potential* v, const Plan& P, PathArgs& a) {
  std::memset(&a, 0, sizeof(a));
  a.n_steps = p->n_steps;
  a.n_atoms = p->n_atoms;
  a.tile = P.tile;
  a.n_tiles = P.n_tiles;
  a.mu_dt = p->dt / p->gamma;
  a.inv4Ddt = 1.0 / (4.0 * p->D * p->dt);
  a.c = 1.0 / (2.0 * p->D * p->dt);
  a.lj.box = v->box;
  a.lj.inv_box = 1.0 / v->box;
  a.lj.rc2 = v->rc * v->rc;
  a.lj.a24 = 24.0 * v->eps;
  a.lj.sig2 = v->sigma * v->sigma;
  const double sr = v->sigma / v->rc;
  const double sr6 = sr * sr * sr * sr * sr * sr;
  a.lj.duc = -(24.0 * v->eps / v->rc) * (2.0 * sr6 * sr6 - sr6);  // u'(r_c)
  const double radius = v->rc + P.skin;
  a.rlist2 = radius * radius;
  a.half_skin2 = 0.25 * P.skin * P.skin;
  a.nc = P.cells.nc;
  a.reach = P.cells.reach;
  a.kmax = P.kmax;
  a.lds2 = P.r_in_lds && P.lds2 ? 1 : 0;
  set_box_units(a);
}

BlockScratch scratch_of(const Plan& P, void* ws) {
  BlockScratch s;
  s.nbr = at<uint16_t>(ws, P.off_nbr);
  s.cnt = at<int32_t>(ws, P.off_cnt);
  s.xref = at<double>(ws, P.off_xref);
  s.rglob = P.rglob_stride ? at<double>(ws, P.off_rglob) : nullptr;
  s.nbr_stride = (int64_t)P.nbr_stride;
  s.cnt_stride = (int64_t)P.cnt_stride;
  s.xref_stride = (int64_t)P.xref_stride;
  s.rglob_stride = (int64_t)P.rglob_stride;
  s.ex_off = P.exl ? 0 : (int64_t)P.nbr_stride / 2;
  return s;
}

FusedLaunch launch_of(const Plan& P) {
  FusedLaunch L;
  L.block = P.block;
  L.grid = P.grid;
  L.r_in_lds = P.r_in_lds;
  L.lds2 = P.lds2;
  L.f32 = P.f32;
  L.half = P.half;
  L.exl = P.exl;
  L.lds_bytes = P.lds;
  return L;
}

// Core evaluation shared by the entry points.
int evaluate(const pamd_path* p, const pamd_potential* v, const Plan& P, const double* x,
             const double* w, double* action, double* per_step, double* grad, double* excess,
             int mode, void* ws, hipStream_t st) {
  double* steps = per_step ? per_step : at<double>(ws, P.off_step);
  if (P.kind == PAMD_HARMONIC) {
    HOArgs h;
    h.x = x;
    h.weights = w;
    h.grad = grad;
    h.per_step = steps;
    h.excess = excess;
    h.n_steps = P.steps;
    h.n_dof = P.dof;
    h.k = v->k;
    h.mu_dt = p->dt / p->gamma;
    h.inv4Ddt = 1.0 / (4.0 * p->D * p->dt);
    h.c = 1.0 / (2.0 * p->D * p->dt);
    h.mode = mode;
    h.seg = P.seg;
    {
      EventScope ev(st);
      PAMD_HIP(launch_ho(h, action, st));
    }
    return PAMD_OK;
  }
  PathArgs a;
  fill_lj(p, v, P, a);
  a.x = x;
  a.weights = w;
  a.grad = grad;
  a.per_step = steps;
  a.excess = excess;
  a.mode = mode;
  if (P.algo == PAMD_ALGO_PLAIN) {
    PlainArgs pa;
    pa.p = a;
    pa.p.nc = P.pcells.nc;
    pa.p.reach = P.pcells.reach;
    pa.p.kmax = P.pkmax;
    pa.nbr = at<uint16_t>(ws, P.off_pnbr);
    pa.cnt = at<int32_t>(ws, P.off_pcnt);
    pa.F = at<double>(ws, P.off_F);
    pa.R = at<double>(ws, P.off_R);
    pa.Q = at<double>(ws, P.off_Q);
    {
      EventScope ev(st);
      PAMD_HIP(launch_lj_plain(pa, P.block, P.f32, action, st));
    }
    return PAMD_OK;
  }
  a.bnd = at<double>(ws, P.off_bnd);
  {
    EventScope ev(st);
    PAMD_HIP(launch_lj_fused(a, scratch_of(P, ws), launch_of(P), st));
  }
  if (action || (mode & MODE_GRAD)) PAMD_HIP(launch_lj_finalize(a, action, st));
  return PAMD_OK;
}

}  // namespace

namespace pamd {

// cell_cost: the cost of visiting one stencil cell, in candidate tests (0
// for the fused build, whose scan walks contiguous cell ranges; per-atom
// stencil walks pay it per cell)
CellGrid choose_cells(double box, double radius, int n_atoms, int max_cells, double cell_cost) {
  CellGrid g;
  const double rho = n_atoms / (box * box * box);
  double best = (double)n_atoms;  // all pairs
  const int cap = std::min(max_cells, std::max(64, 4 * n_atoms));
  for (int reach = 1; reach <= 3; ++reach) {
    int nc = (int)std::floor(reach * box / radius);
    while (nc >= 2 * reach + 1 && (int64_t)nc * nc * nc > cap) --nc;
    if (nc < 2 * reach + 1) continue;
    const double h = box / nc;
    const double cells = std::pow(2 * reach + 1, 3);
    const double cand = cells * h * h * h * rho + cell_cost * cells;
    if (cand < best) {
      best = cand;
      g.nc = nc;
      g.reach = reach;
    }
  }
  return g;
}

bool fused_cells_fit(double box, double radius, int n_atoms, int block, bool r_in_lds, bool half,
                     CellGrid* grid, size_t* lds, bool two, size_t cap_bytes) {
  int cap = 1 << 30;
  for (;;) {
    const CellGrid g = choose_cells(box, radius, n_atoms, cap);
    const size_t b = fused_lds_bytes(n_atoms, g.nc, r_in_lds, half, block, two);
    if (b <= cap_bytes) {
      *grid = g;
      *lds = b;
      return true;
    }
    if (g.nc == 0) return false;
    cap = g.nc * g.nc * g.nc / 2;  // fewer, larger cells
  }
}

int batch_fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}
}  // namespace pamd

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* pamd_last_error(void) { return g_err.c_str(); }

const char* pamd_version(void) { return "pamd 0.1 (gfx950)"; }

int pamd_profile_events(void* start, void* stop) {
  g_ev_start = (hipEvent_t)start;
  g_ev_stop = (hipEvent_t)stop;
  return PAMD_OK;
}

double pamd_log_norm(const pamd_path* p) {
  if (check_path(p)) return NAN;
  return (double)p->n_steps * (p->n_dim * (double)p->n_atoms / 2.0) *
         std::log(4.0 * M_PI * p->D * p->dt);
}

int pamd_workspace_size(const pamd_path* p, const pamd_potential* v, const pamd_tuning* t,
                        size_t* bytes) {
  if (!bytes) return fail(PAMD_EINVAL, "bytes is NULL");
  Plan P;
  int rc = make_plan(p, v, t, false, P);
  if (rc) return rc;
  *bytes = P.total;
  return PAMD_OK;
}

int pamd_launch_info(const pamd_path* p, const pamd_potential* v, const pamd_tuning* t,
                     pamd_launch* out) {
  if (!out) return fail(PAMD_EINVAL, "out is NULL");
  Plan P;
  int rc = make_plan(p, v, t, false, P);
  if (rc) return rc;
  std::memset(out, 0, sizeof(*out));
  if (P.kind == PAMD_HARMONIC) return PAMD_OK;
  out->algo = P.algo;
  out->skin = P.skin;
  if (P.algo == PAMD_ALGO_PLAIN) {
    out->block = P.block;
    out->cells = P.pcells.nc;
    out->reach = P.pcells.reach;
    out->max_neighbours = P.pkmax;
    out->lds_bytes = (int32_t)P.plds;
    out->tile = 1;
    out->n_tiles = (int32_t)std::min<int64_t>(P.steps, INT32_MAX);
    return PAMD_OK;
  }
  out->block = P.block;
  out->tile = P.tile;
  out->n_tiles = P.n_tiles;
  out->grid = P.grid;
  out->cells = P.cells.nc;
  out->reach = P.cells.reach;
  out->max_neighbours = P.kmax;
  out->neighbour_list = P.half ? PAMD_LIST_HALF : PAMD_LIST_FULL;
  out->lds_bytes = (int32_t)P.lds;
  out->slot_arrays = P.r_in_lds ? (P.lds2 ? 2 : 1) : 0;
  out->exact_lists = P.exl ? 1 : 0;
  return PAMD_OK;
}

int pamd_action(const pamd_path* p, const pamd_potential* v, const pamd_tuning* t,
                const double* x, double* action, double* per_step, void* ws, size_t ws_bytes,
                void* stream) {
  Plan P;
  int rc = make_plan(p, v, t, false, P);
  if (rc) return rc;
  if (!x) return fail(PAMD_EINVAL, "x is NULL");
  if (!action) return fail(PAMD_EINVAL, "action is NULL");
  if ((rc = check_ws(P, ws, ws_bytes))) return rc;
  return evaluate(p, v, P, x, nullptr, action, per_step, nullptr, nullptr, 0, ws,
                  (hipStream_t)stream);
}

int pamd_action_grad(const pamd_path* p, const pamd_potential* v, const pamd_tuning* t,
                     const double* x, const double* w, double* action, double* per_step,
                     double* grad, void* ws, size_t ws_bytes, void* stream) {
  Plan P;
  int rc = make_plan(p, v, t, false, P);
  if (rc) return rc;
  if (!x) return fail(PAMD_EINVAL, "x is NULL");
  if (!grad) return fail(PAMD_EINVAL, "grad is NULL");
  if ((rc = check_ws(P, ws, ws_bytes))) return rc;
  return evaluate(p, v, P, x, w, action, per_step, grad, nullptr, MODE_GRAD, ws,
                  (hipStream_t)stream);
}

int pamd_excess_action(const pamd_path* p, const pamd_potential* v, const pamd_tuning* t,
                       const double* x, double* excess, double* per_step, void* ws,
                       size_t ws_bytes, void* stream) {
  Plan P;
  int rc = make_plan(p, v, t, false, P);
  if (rc) return rc;
  if (!x) return fail(PAMD_EINVAL, "x is NULL");
  if (!excess) return fail(PAMD_EINVAL, "excess is NULL");
  if ((rc = check_ws(P, ws, ws_bytes))) return rc;
  return evaluate(p, v, P, x, nullptr, nullptr, per_step, nullptr, excess, MODE_EXCESS, ws,
                  (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Action and gradient without a caller workspace (see pamd.h)
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {
// Scratch of pamd_action_grad_noalloc: one array per device, loaded with the
// code object and held until the process ends.  Host code never uses the
// array's name as an address: hipGetSymbolAddress gives each device's copy.
static __device__ __align__(256) unsigned char scratch[PAMD_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch (looked up once per device).
int scratch_address(void** out) {
  int dev = 0;
  PAMD_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(PAMD_EUNSUPPORTED, "device index %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    PAMD_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(PAMD_EHIP, "hipGetSymbolAddress returned NULL for the scratch array");
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return PAMD_OK;
}

// The largest plan whose workspace fits the static scratch: the persistent
// grid shrinks (tiles are taken in a grid-stride loop, so results are the
// same) until it fits; PAMD_EWORKSPACE when even one workgroup's does not.
int noalloc_plan(const pamd_path* p, const pamd_potential* v, const pamd_tuning* t, Plan& P) {
  int rc = make_plan(p, v, t, false, P);
  if (rc) return rc;
  if (P.total <= PAMD_NOALLOC_SCRATCH_BYTES) return PAMD_OK;
  if (P.kind == PAMD_LJ && P.algo == PAMD_ALGO_FUSED && P.grid > 1) {
    int lo = 1, hi = P.grid - 1, best = 0;
    while (lo <= hi) {
      const int mid = (lo + hi) / 2;
      Plan Q;
      if ((rc = make_plan(p, v, t, false, Q, mid))) return rc;
      if (Q.total <= PAMD_NOALLOC_SCRATCH_BYTES) {
        best = mid;
        lo = mid + 1;
      } else {
        hi = mid - 1;
      }
    }
    if (best > 0) return make_plan(p, v, t, false, P, best);
  }
  return fail(PAMD_EWORKSPACE,
              "problem needs %zu bytes of scratch, more than the %llu-byte static array of "
              "pamd_action_grad_noalloc; use pamd_action_grad with a workspace",
              P.total, (unsigned long long)PAMD_NOALLOC_SCRATCH_BYTES);
}
}  // namespace

extern "C" {

int pamd_action_grad_noalloc(const pamd_path* p, const pamd_potential* v, const pamd_tuning* t,
                             const double* x, const double* w, double* action, double* per_step,
                             double* grad, void* stream) {
  Plan P;
  int rc = noalloc_plan(p, v, t, P);
  if (rc) return rc;
  if (!x) return fail(PAMD_EINVAL, "x is NULL");
  if (!grad) return fail(PAMD_EINVAL, "grad is NULL");
  void* ws = nullptr;
  if ((rc = scratch_address(&ws))) return rc;
  return evaluate(p, v, P, x, w, action, per_step, grad, nullptr, MODE_GRAD, ws,
                  (hipStream_t)stream);
}

// ---------------------------------------------------------------------------
// Path sampling
// ---------------------------------------------------------------------------
int pamd_mh_workspace_size(const pamd_path* p, const pamd_potential* v, const pamd_tuning* t,
                           size_t* bytes) {
  if (!bytes) return fail(PAMD_EINVAL, "bytes is NULL");
  Plan P;
  int rc = make_plan(p, v, t, true, P);
  if (rc) return rc;
  *bytes = P.total;
  return PAMD_OK;
}

}  // extern "C"

namespace {
int mh_step_impl(const pamd_path* p, const pamd_potential* v, const pamd_tuning* t,
                 uint64_t seed, int32_t l_min, int32_t l_max, int64_t* sweep_counter,
                 double* x, double* excess, double* trial, double* frag_delta,
                 int32_t* frag_accept, int32_t* step_info, uint64_t* level_stats, void* ws,
                 size_t ws_bytes, void* stream) {
  Plan P;
  int rc = make_plan(p, v, t, true, P);
  if (rc) return rc;
  if (!x || !excess || !trial || !sweep_counter)
    return fail(PAMD_EINVAL, "x, excess, trial and sweep_counter must be non-NULL");
  if (l_min < 1 || l_max < l_min || l_max > 30)
    return fail(PAMD_EINVAL, "levels must satisfy 1 <= l_min <= l_max <= 30 (got %d, %d)", l_min, l_max);
  if (((int64_t)1 << l_max) > p->n_steps)
    return fail(PAMD_EINVAL, "2^l_max = %lld exceeds n_steps = %lld", (long long)1 << l_max, (long long)p->n_steps);
  if ((rc = check_ws(P, ws, ws_bytes))) return rc;
  hipStream_t st = (hipStream_t)stream;
  MHArgs m;
  m.x = x;
  m.trial = trial;
  m.excess = excess;
  m.excess_trial = at<double>(ws, P.off_mh_ex);
  m.frag_delta = frag_delta;
  m.frag_accept = frag_accept;
  m.step_info = step_info;
  m.state = at<int32_t>(ws, P.off_mh_state);
  m.acc_ws = at<int32_t>(ws, P.off_mh_acc);
  m.sweep_counter = sweep_counter;
  m.level_stats = reinterpret_cast<unsigned long long*>(level_stats);
  m.n_steps = p->n_steps;
  m.n_dof = P.dof;
  m.key0 = (uint32_t)(seed & 0xffffffffu);
  m.key1 = (uint32_t)(seed >> 32);
  m.l_min = l_min;
  m.l_max = l_max;
  m.sig = std::sqrt(2.0 * p->D * p->dt);
  PAMD_HIP(launch_mh_prepare(m, st));
  PAMD_HIP(launch_mh_trial(m, st));
  rc = evaluate(p, v, P, trial, nullptr, nullptr, nullptr, nullptr, m.excess_trial, MODE_EXCESS,
                ws, st);
  if (rc) return rc;
  PAMD_HIP(launch_mh_accept(m, st));
  return PAMD_OK;
}
}  // namespace

extern "C" {

int pamd_mh_step(const pamd_path* p, const pamd_potential* v, const pamd_tuning* t,
                 uint64_t seed, int32_t l_min, int32_t l_max, int64_t* sweep_counter,
                 double* x, double* excess, double* trial, double* frag_delta,
                 int32_t* frag_accept, int32_t* step_info, void* ws, size_t ws_bytes,
                 void* stream) {
  return mh_step_impl(p, v, t, seed, l_min, l_max, sweep_counter, x, excess, trial, frag_delta,
                      frag_accept, step_info, nullptr, ws, ws_bytes, stream);
}

// ---------------------------------------------------------------------------
// Sequential Euler-Maruyama integration
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {
// The integrator runs one workgroup: its plan is that of a one-step path (one
// tile, scratch for one block).
int em_plan(const pamd_path* p, const pamd_potential* v, const pamd_tuning* t, Plan& P) {
  int rc;
  if ((rc = check_path(p))) return rc;
  pamd_path q = *p;
  q.n_steps = 1;
  if ((rc = make_plan(&q, v, t, false, P))) return rc;
  if (P.exl) {  // the integrator keeps two slot arrays (its own kernel has no exact lists)
    pamd_tuning t2 = t ? *t : pamd_tuning{};
    t2.slot_arrays = 2;
    if ((rc = make_plan(&q, v, &t2, false, P))) return rc;
  }
  if (v->kind == PAMD_LJ) {
    if (P.algo != PAMD_ALGO_FUSED)
      return fail(PAMD_EUNSUPPORTED, "the integrator uses the fused force pass (algo PLAIN given)");
    if (P.f32) return fail(PAMD_EUNSUPPORTED, "the integrator computes forces in float64 only");
    if (P.half) return fail(PAMD_EUNSUPPORTED, "the integrator uses full neighbour lists");
  }
  return PAMD_OK;
}
}  // namespace

extern "C" {

int pamd_em_workspace_size(const pamd_path* p, const pamd_potential* v, const pamd_tuning* t,
                           size_t* bytes) {
  if (!bytes) return fail(PAMD_EINVAL, "bytes is NULL");
  Plan P;
  int rc = em_plan(p, v, t, P);
  if (rc) return rc;
  *bytes = P.total;
  return PAMD_OK;
}

int pamd_em_integrate(const pamd_path* p, const pamd_potential* v, const pamd_tuning* t,
                      const double* x0, const double* noise, double* x_out, void* ws,
                      size_t ws_bytes, void* stream) {
  Plan P;
  int rc = em_plan(p, v, t, P);
  if (rc) return rc;
  if (!x0 || !noise || !x_out) return fail(PAMD_EINVAL, "x0, noise and x_out must be non-NULL");
  const size_t dof = (size_t)P.dof;
  const size_t nb = sizeof(double) * dof * (size_t)p->n_steps;
  const char *nlo = (const char*)noise, *olo = (const char*)x_out;
  if (nlo < olo + nb + sizeof(double) * dof && olo < nlo + nb)
    return fail(PAMD_EINVAL, "x_out overlaps noise");
  if ((rc = check_ws(P, ws, ws_bytes))) return rc;
  hipStream_t st = (hipStream_t)stream;
  const double amp = std::sqrt(2.0 * p->D * p->dt);
  EventScope ev(st);
  if (v->kind == PAMD_HARMONIC) {
    PAMD_HIP(launch_ho_em(x0, noise, x_out, p->n_steps, P.dof, v->k * p->dt / p->gamma, amp, st));
    return PAMD_OK;
  }
  PathArgs a;
  fill_lj(p, v, P, a);
  a.n_steps = p->n_steps;
  a.x = x0;
  a.per_step = at<double>(ws, P.off_step);
  PAMD_HIP(launch_lj_em(a, noise, amp, x_out, scratch_of(P, ws), launch_of(P), st));
  return PAMD_OK;
}

// ---------------------------------------------------------------------------
// Path-based integration: shifting events and the sample-shift-regrow loop
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {
bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  const char *pa = (const char*)a, *pb = (const char*)b;
  return pa < pb + nb && pb < pa + na;
}

// The path of steps N - n_shift .. N: the part that a shifting event regrows.
pamd_path tail_path(const pamd_path* p, int32_t n_shift) {
  pamd_path q = *p;
  q.n_steps = n_shift;
  return q;
}
}  // namespace

extern "C" {

int pamd_shift(const pamd_path* p, uint64_t seed, int32_t n_shift, int64_t* event_counter,
               const double* x_in, double* x_out, const double* excess_in, double* excess_out,
               double* traj_out, void* stream) {
  int rc;
  if ((rc = check_path(p))) return rc;
  if (n_shift < 1 || n_shift > p->n_steps)
    return fail(PAMD_EINVAL, "n_shift must be in [1, n_steps] (got %d)", n_shift);
  if (!event_counter || !x_in || !x_out)
    return fail(PAMD_EINVAL, "event_counter, x_in and x_out must be non-NULL");
  if (!excess_in != !excess_out)
    return fail(PAMD_EINVAL, "excess_in and excess_out must both be given or both be NULL");
  const int64_t dof = (int64_t)p->n_dim * p->n_atoms;
  const size_t xb = sizeof(double) * (size_t)(p->n_steps + 1) * dof;
  const size_t eb = sizeof(double) * (size_t)p->n_steps;
  if (overlap(x_in, xb, x_out, xb)) return fail(PAMD_EINVAL, "x_in and x_out overlap");
  if (excess_in && overlap(excess_in, eb, excess_out, eb))
    return fail(PAMD_EINVAL, "excess_in and excess_out overlap");
  if (traj_out && (overlap(traj_out, sizeof(double) * (size_t)n_shift * dof, x_out, xb) ||
                   overlap(traj_out, sizeof(double) * (size_t)n_shift * dof, x_in, xb)))
    return fail(PAMD_EINVAL, "traj_out overlaps x_in or x_out");
  ShiftArgs a;
  a.x_in = x_in;
  a.x_out = x_out;
  a.ex_in = excess_in;
  a.ex_out = excess_out;
  a.traj = traj_out;
  a.event_counter = event_counter;
  a.n_steps = p->n_steps;
  a.n_dof = dof;
  a.n_shift = n_shift;
  a.key0 = (uint32_t)(seed & 0xffffffffu);
  a.key1 = (uint32_t)(seed >> 32);
  a.sig = std::sqrt(2.0 * p->D * p->dt);
  PAMD_HIP(launch_shift(a, (hipStream_t)stream));
  return PAMD_OK;
}

int pamd_run_workspace_size(const pamd_path* p, const pamd_potential* v, const pamd_tuning* t,
                            int32_t n_shift, size_t* bytes) {
  if (!bytes) return fail(PAMD_EINVAL, "bytes is NULL");
  int rc;
  if ((rc = check_path(p))) return rc;
  if (n_shift < 1 || n_shift > p->n_steps)
    return fail(PAMD_EINVAL, "n_shift must be in [1, n_steps] (got %d)", n_shift);
  Plan P, Q;
  if ((rc = make_plan(p, v, t, true, P))) return rc;
  const pamd_path q = tail_path(p, n_shift);
  if ((rc = make_plan(&q, v, t, false, Q))) return rc;
  *bytes = std::max(P.total, Q.total);
  return PAMD_OK;
}

int pamd_run(const pamd_path* p, const pamd_potential* v, const pamd_tuning* t, uint64_t seed,
             int32_t l_min, int32_t l_max, int32_t n_sample, int32_t n_shift, int32_t n_events,
             int64_t* counters, double* x, double* x_alt, double* trial, double* excess,
             double* excess_alt, double* traj_out, uint64_t* level_stats, void* ws,
             size_t ws_bytes, void* stream) {
  size_t need = 0;
  int rc = pamd_run_workspace_size(p, v, t, n_shift, &need);
  if (rc) return rc;
  if (n_sample < 0 || n_events < 0)
    return fail(PAMD_EINVAL, "n_sample and n_events must be >= 0 (got %d, %d)", n_sample, n_events);
  if (l_min < 1 || l_max < l_min || l_max > 30)
    return fail(PAMD_EINVAL, "levels must satisfy 1 <= l_min <= l_max <= 30 (got %d, %d)", l_min, l_max);
  if (((int64_t)1 << l_max) > p->n_steps)
    return fail(PAMD_EINVAL, "2^l_max = %lld exceeds n_steps = %lld", (long long)1 << l_max, (long long)p->n_steps);
  if (!counters || !x || !x_alt || !trial || !excess || !excess_alt)
    return fail(PAMD_EINVAL, "counters, x, x_alt, trial, excess and excess_alt must be non-NULL");
  const int64_t dof = (int64_t)p->n_dim * p->n_atoms;
  const size_t xb = sizeof(double) * (size_t)(p->n_steps + 1) * dof;
  const size_t eb = sizeof(double) * (size_t)p->n_steps;
  if (overlap(x, xb, x_alt, xb) || overlap(x, xb, trial, xb) || overlap(x_alt, xb, trial, xb))
    return fail(PAMD_EINVAL, "x, x_alt and trial must not overlap");
  if (overlap(excess, eb, excess_alt, eb)) return fail(PAMD_EINVAL, "excess and excess_alt overlap");
  Plan W;
  W.total = need;
  if ((rc = check_ws(W, ws, ws_bytes))) return rc;
  hipStream_t st = (hipStream_t)stream;
  const pamd_path q = tail_path(p, n_shift);
  const int64_t keep = p->n_steps - n_shift;
  double *xc = x, *xo = x_alt, *ec = excess, *eo = excess_alt;
  for (int32_t e = 0; e < n_events; ++e) {
    for (int32_t k = 0; k < n_sample; ++k) {
      rc = mh_step_impl(p, v, t, seed, l_min, l_max, counters, xc, ec, trial, nullptr, nullptr,
                        nullptr, level_stats, ws, ws_bytes, stream);
      if (rc) return rc;
    }
    rc = pamd_shift(p, seed, n_shift, counters + 1, xc, xo, ec, eo,
                    traj_out ? traj_out + (size_t)e * n_shift * dof : nullptr, stream);
    if (rc) return rc;
    // excess of the regrown steps
    rc = pamd_excess_action(&q, v, t, xo + (size_t)keep * dof, eo + keep, nullptr, ws, ws_bytes,
                            stream);
    if (rc) return rc;
    std::swap(xc, xo);
    std::swap(ec, eo);
  }
  if (xc != x) {
    PAMD_HIP(launch_copy(xc, x, (int64_t)(p->n_steps + 1) * dof, st));
    PAMD_HIP(launch_copy(ec, excess, p->n_steps, st));
  }
  return PAMD_OK;
}

// ---------------------------------------------------------------------------
// Gradient-informed (Langevin) path move
// ---------------------------------------------------------------------------
}  // extern "C"

namespace {
// The move's workspace: the action+gradient plan's, then the partial sums,
// the proposal's action and the decision flag.
struct LangevinPlan {
  Plan P;
  int blocks = 1;
  size_t off_partial = 0, off_action = 0, off_flag = 0, total = 0;
};

int langevin_plan(const pamd_path* p, const pamd_potential* v, const pamd_tuning* t,
                  LangevinPlan& L) {
  int rc = make_plan(p, v, t, false, L.P);
  if (rc) return rc;
  const int64_t elems = p->n_steps * (int64_t)p->n_dim * p->n_atoms;
  L.blocks = (int)std::max<int64_t>(1, std::min<int64_t>(kLangevinBlocks, (elems + 255) / 256));
  size_t cur = L.P.total;
  L.off_partial = bump(cur, sizeof(double) * 2 * L.blocks);
  L.off_action = bump(cur, sizeof(double));
  L.off_flag = bump(cur, sizeof(int32_t));
  L.total = align_up(cur, kAlign);
  return PAMD_OK;
}
}  // namespace

extern "C" {

int pamd_langevin_workspace_size(const pamd_path* p, const pamd_potential* v,
                                 const pamd_tuning* t, size_t* bytes) {
  if (!bytes) return fail(PAMD_EINVAL, "bytes is NULL");
  LangevinPlan L;
  int rc = langevin_plan(p, v, t, L);
  if (rc) return rc;
  *bytes = L.total;
  return PAMD_OK;
}

int pamd_langevin_step(const pamd_path* p, const pamd_potential* v, const pamd_tuning* t,
                       uint64_t seed, double tau, int64_t* move_counter, double* x,
                       double* grad, double* action, double* y, double* grad_y,
                       int32_t* accepted, double* log_alpha, void* ws, size_t ws_bytes,
                       void* stream) {
  LangevinPlan L;
  int rc = langevin_plan(p, v, t, L);
  if (rc) return rc;
  if (!std::isfinite(tau) || tau <= 0.0) return fail(PAMD_EINVAL, "tau must be finite and > 0");
  if (!move_counter || !x || !grad || !action || !y || !grad_y)
    return fail(PAMD_EINVAL, "move_counter, x, grad, action, y and grad_y must be non-NULL");
  const size_t xb = sizeof(double) * (size_t)(p->n_steps + 1) * p->n_dim * p->n_atoms;
  const double* bufs[4] = {x, grad, y, grad_y};
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (overlap(bufs[i], xb, bufs[j], xb))
        return fail(PAMD_EINVAL, "x, grad, y and grad_y must not overlap");
  Plan W;
  W.total = L.total;
  if ((rc = check_ws(W, ws, ws_bytes))) return rc;
  hipStream_t st = (hipStream_t)stream;
  LangevinArgs a;
  a.x = x;
  a.grad = grad;
  a.action = action;
  a.y = y;
  a.grad_y = grad_y;
  a.action_y = at<double>(ws, L.off_action);
  a.partial = at<double>(ws, L.off_partial);
  a.flag = at<int32_t>(ws, L.off_flag);
  a.accepted = accepted;
  a.log_alpha = log_alpha;
  a.counter = move_counter;
  a.n_steps = p->n_steps;
  a.n_dof = L.P.dof;
  a.key0 = (uint32_t)(seed & 0xffffffffu);
  a.key1 = (uint32_t)(seed >> 32);
  a.tau = tau;
  a.blocks = L.blocks;
  PAMD_HIP(launch_langevin_propose(a, st));
  rc = evaluate(p, v, L.P, y, nullptr, at<double>(ws, L.off_action), nullptr, grad_y, nullptr,
                MODE_GRAD, ws, st);
  if (rc) return rc;
  PAMD_HIP(launch_langevin_accept(a, st));
  return PAMD_OK;
}

// ---------------------------------------------------------------------------
// Autotuning
// ---------------------------------------------------------------------------
int pamd_autotune(const pamd_path* p, const pamd_potential* v, const double* x,
                  double* grad_scratch, void* ws, size_t ws_bytes, void* stream,
                  pamd_tuning* best) {
  int rc;
  if ((rc = check_path(p)) || (rc = check_pot(p, v))) return rc;
  if (!x || !grad_scratch) return fail(PAMD_EINVAL, "x and grad_scratch must be non-NULL");
  hipStream_t st = (hipStream_t)stream;
  std::vector<pamd_tuning> cands;
  if (v->kind == PAMD_LJ) {
    const int N = p->n_atoms;
    for (int list : {PAMD_LIST_HALF, PAMD_LIST_FULL}) {
      std::vector<int> blocks;
      for (int b : {default_block(N, list == PAMD_LIST_HALF), (int)align_up((size_t)(N + 1) / 2, 64),
                    256, 512, 1024})
        if (b >= 64 && b <= 1024 && std::find(blocks.begin(), blocks.end(), b) == blocks.end())
          blocks.push_back(b);
      // tile 0 and skin 0 are the planner's own choices for the block, so the
      // default launch is among the candidates
      for (int b : blocks)
        for (int slots : {2, 1}) {
          for (int tile : {0, 2, 4, 8, 16, 32})
            for (double skin : {0.0, 0.2, 0.3, 0.45}) {
              pamd_tuning c{};
              c.algo = PAMD_ALGO_FUSED;
              c.block = b;
              c.tile = tile;
              c.skin = skin * v->sigma;
              c.neighbour_list = list;
              c.slot_arrays = slots;
              cands.push_back(c);
            }
        }
    }
  } else {
    cands.push_back(pamd_tuning{});
  }
  hipEvent_t e0, e1;
  PAMD_HIP(hipEventCreate(&e0));
  PAMD_HIP(hipEventCreate(&e1));
  float best_ms = 1e30f;
  pamd_tuning best_t{};
  bool found = false;
  for (const auto& c : cands) {
    Plan P;
    if (make_plan(p, v, &c, false, P, kMaxGrid, false) != PAMD_OK) continue;
    if (P.total > ws_bytes || !ws) continue;
    if (evaluate(p, v, P, x, nullptr, nullptr, nullptr, grad_scratch, nullptr, MODE_GRAD, ws, st))
      continue;
    float ms_min = 1e30f;
    for (int rep = 0; rep < 3; ++rep) {
      hipEventRecord(e0, st);
      evaluate(p, v, P, x, nullptr, nullptr, nullptr, grad_scratch, nullptr, MODE_GRAD, ws, st);
      hipEventRecord(e1, st);
      if (hipEventSynchronize(e1) != hipSuccess) break;
      float ms = 0;
      hipEventElapsedTime(&ms, e0, e1);
      ms_min = std::min(ms_min, ms);
    }
    if (ms_min < best_ms) {
      best_ms = ms_min;
      best_t = c;
      found = true;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (!found) return fail(PAMD_EWORKSPACE, "no candidate fits the %zu-byte workspace", ws_bytes);
  best_t.algo = PAMD_ALGO_AUTO;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune[tune_key(p, v)] = best_t;
  }
  if (best) *best = best_t;
  return PAMD_OK;
}

// ---------------------------------------------------------------------------
// Graphs
// ---------------------------------------------------------------------------
struct pamd_graph {
  hipGraph_t graph;
  hipGraphExec_t exec;
};

int pamd_graph_begin(void* stream) {
  if (!stream) return fail(PAMD_EINVAL, "graph capture needs a non-null stream");
  PAMD_HIP(hipStreamBeginCapture((hipStream_t)stream, hipStreamCaptureModeThreadLocal));
  return PAMD_OK;
}

int pamd_graph_end(void* stream, pamd_graph** out) {
  if (!stream || !out) return fail(PAMD_EINVAL, "stream and out must be non-NULL");
  hipGraph_t g = nullptr;
  PAMD_HIP(hipStreamEndCapture((hipStream_t)stream, &g));
  hipGraphExec_t ex = nullptr;
  hipError_t e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
  if (e != hipSuccess) {
    hipGraphDestroy(g);
    return fail(PAMD_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
  }
  *out = new pamd_graph{g, ex};
  return PAMD_OK;
}

int pamd_graph_launch(const pamd_graph* g, void* stream) {
  if (!g) return fail(PAMD_EINVAL, "graph is NULL");
  PAMD_HIP(hipGraphLaunch(g->exec, (hipStream_t)stream));
  return PAMD_OK;
}

void pamd_graph_destroy(pamd_graph* g) {
  if (!g) return;
  hipGraphExecDestroy(g->exec);
  hipGraphDestroy(g->graph);
  delete g;
}

}  // extern "C"
