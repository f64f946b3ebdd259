// Batches of independent paths: packed layout, a cost-ordered (path, tile) work
// list executed by one persistent launch for the Lennard-Jones members, and one
// streaming launch per harmonic member.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "internal.hpp"
#include "pamd.h"

using namespace pamd;

extern "C" int pamd_workspace_size(const pamd_path*, const pamd_potential*, const pamd_tuning*,
                                   size_t*);

namespace pamd {
int batch_fail(int code, const char* fmt, ...);
}

namespace {

constexpr size_t kAlign = 256;
constexpr int kMaxGrid = 2048;

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
size_t bump(size_t& cur, size_t bytes) {
  const size_t at = align_up(cur, kAlign);
  cur = at + bytes;
  return at;
}

}  // namespace

struct pamd_batch {
  std::vector<pamd_path> paths;
  std::vector<pamd_potential> pots;
  std::vector<int64_t> x_off, step_off;  // n + 1 entries
  std::vector<int> lj_ids, ho_ids;
  // device tables (host copies)
  std::vector<BatchMember> members;
  std::vector<int32_t> slots;
  std::vector<BatchItem> items;
  int max_tiles = 1;
  FusedLaunch launch{};
  BlockScratch scratch_proto{};
  bool f32 = false;
  // planning inputs: the caller's tuning (if any) and the member-tile policy
  // (tile = tile_budget / n_atoms steps, clamped to [4, 128]; skin =
  // skin_frac sigma unless the tuning fixes them)
  bool has_tuning = false;
  pamd_tuning tuning{};
  double tile_budget = 16384.0;
  double skin_frac = 0.5;
  // workspace offsets
  size_t off_actions = 0;  // n_paths doubles: the autotuner's trial actions
  size_t off_members = 0, off_slots = 0, off_items = 0, off_counter = 0, off_steps = 0,
         off_bnd = 0, off_nbr = 0, off_cnt = 0, off_xref = 0, off_rglob = 0, total = 0;
  size_t nbr_stride = 0, cnt_stride = 0, xref_stride = 0, rglob_stride = 0;
};

namespace {
// Plans the members' tiles and lists, the work list, the launch shape and the
// workspace layout from b's paths, tuning and tile policy (replaces any
// earlier plan).
int plan_batch(pamd_batch* b) {
  const pamd_tuning* tuning = b->has_tuning ? &b->tuning : nullptr;
  b->members.clear();
  b->slots.clear();
  b->items.clear();
  b->max_tiles = 1;
  b->launch = FusedLaunch{};
  // Lennard-Jones members: per-member tiles and lists, batch-wide launch shape.
  int max_n = 1;
  size_t max_nbr = 0;
  std::vector<double> radii;  // list radius per member (LJ members, in order)
  int64_t bnd_elems = 0;
  const double skin_in = tuning && tuning->skin > 0 ? tuning->skin : -1.0;
  for (int p : b->lj_ids) {
    const pamd_path& P = b->paths[p];
    const pamd_potential& V = b->pots[p];
    const int N = P.n_atoms;
    const double skin = skin_in > 0 ? skin_in : b->skin_frac * V.sigma;
    const double radius = V.rc + skin;
    radii.push_back(radius);
    const double rho = N / (V.box * V.box * V.box);
    int kmax = (int)align_up((size_t)std::ceil(1.3 * 4.0 / 3.0 * M_PI * radius * radius * radius * rho + 24.0), 8);
    if (tuning && tuning->max_neighbours > 0) kmax = tuning->max_neighbours;
    kmax = std::max(1, std::min(kmax, std::max(1, N - 1)));
    kmax = (int)align_up((size_t)kmax, 8);  // lists are read in chunks of 8
    int tile = tuning && tuning->tile > 0
                   ? tuning->tile
                   : (int)std::max(4.0, std::min(128.0, std::ceil(b->tile_budget / N)));
    tile = (int)std::min<int64_t>(tile, P.n_steps);
    BatchMember m;
    std::memset(&m, 0, sizeof(m));
    PathArgs& a = m.a;
    a.n_steps = P.n_steps;
    a.n_atoms = N;
    a.tile = tile;
    a.n_tiles = (int)((P.n_steps + tile - 1) / tile);
    a.mode = MODE_GRAD;
    a.mu_dt = P.dt / P.gamma;
    a.inv4Ddt = 1.0 / (4.0 * P.D * P.dt);
    a.c = 1.0 / (2.0 * P.D * P.dt);
    a.lj.box = V.box;
    a.lj.inv_box = 1.0 / V.box;
    a.lj.rc2 = V.rc * V.rc;
    a.lj.a24 = 24.0 * V.eps;
    a.lj.sig2 = V.sigma * V.sigma;
    const double sr = V.sigma / V.rc, sr6 = std::pow(sr, 6);
    a.lj.duc = -(24.0 * V.eps / V.rc) * (2.0 * sr6 * sr6 - sr6);
    a.rlist2 = radius * radius;
    a.half_skin2 = 0.25 * skin * skin;
    a.kmax = kmax;
    set_box_units(a);
    m.x_off = b->x_off[p];
    m.step_off = b->step_off[p];
    m.bnd_off = bnd_elems;
    bnd_elems += (int64_t)align_up((size_t)std::max(0, a.n_tiles - 1) * 3 * N, 32);
    b->members.push_back(m);
    b->slots.push_back(p);
    b->max_tiles = std::max(b->max_tiles, a.n_tiles);
    max_n = std::max(max_n, N);
    max_nbr = std::max(max_nbr, (size_t)(kmax + 32) * N);  // exact lists: 2 rows, spare chunks
  }
  // Work list: every tile of every member, largest (atoms x steps) first.
  for (int mi = 0; mi < (int)b->members.size(); ++mi) {
    const PathArgs& a = b->members[mi].a;
    for (int t = 0; t < a.n_tiles; ++t) b->items.push_back(BatchItem{mi, t});
  }
  std::stable_sort(b->items.begin(), b->items.end(), [&](const BatchItem& u, const BatchItem& v) {
    auto cost = [&](const BatchItem& it) {
      const PathArgs& a = b->members[it.path].a;
      const int64_t n0 = (int64_t)it.tile * a.tile;
      const int64_t len = std::min<int64_t>(a.tile, a.n_steps - n0);
      return (double)len * a.n_atoms;
    };
    return cost(u) > cost(v);
  });
  FusedLaunch& L = b->launch;
  L.f32 = b->f32;
  if (!b->lj_ids.empty()) {
    const int list = tuning ? tuning->neighbour_list : PAMD_LIST_AUTO;
    // full lists: two threads per atom; half lists: one atom per thread
    int block = 0;
    if (tuning && tuning->block) {
      block = tuning->block;
    } else if (list == PAMD_LIST_HALF) {
      int per = (max_n + 1023) / 1024;
      block = (int)align_up((size_t)((max_n + per - 1) / per), 64);
    } else {
      block = (int)align_up((size_t)2 * max_n, 64);
    }
    L.block = std::max(64, std::min(1024, block));
    L.half = list == PAMD_LIST_HALF;  // automatic choice: full lists
    if (L.half && max_n > fused_half_slots() * L.block) {
      return batch_fail(PAMD_EUNSUPPORTED, "half lists do not fit this batch");
    }
    // one residual placement for the whole batch: in LDS with two slot
    // arrays if every member fits so, else with one, else in global scratch;
    // each member gets the finest cell grid that fits
    auto fit_all = [&](bool r_in_lds, bool two) {
      size_t lds_max = 0;
      for (size_t mi = 0; mi < b->members.size(); ++mi) {
        PathArgs& a = b->members[mi].a;
        CellGrid g;
        size_t lds = 0;
        if (!fused_cells_fit(a.lj.box, radii[mi], a.n_atoms, L.block, r_in_lds, L.half, &g, &lds,
                             two, kBatchLdsMax))
          return false;
        a.nc = g.nc;
        a.reach = g.reach;
        a.lds2 = r_in_lds && two ? 1 : 0;
        lds_max = std::max(lds_max, lds);
      }
      L.r_in_lds = r_in_lds;
      L.lds2 = r_in_lds && two;
      L.lds_bytes = lds_max;
      return true;
    };
    if (!fit_all(true, true) && !fit_all(true, false) && !fit_all(false, false)) {
      return batch_fail(PAMD_EUNSUPPORTED, "batch member with %d atoms exceeds LDS", max_n);
    }
    L.grid = std::max(1, std::min<int>((int)b->items.size(), kMaxGrid));
  }
  b->nbr_stride = 2 * align_up(max_nbr, 128);  // neighbour list + exact list
  b->cnt_stride = align_up((size_t)2 * max_n, 64);  // list lengths: up to two rows per atom
  b->xref_stride = align_up((size_t)6 * max_n, 32);
  b->rglob_stride = L.r_in_lds && L.lds2 ? 0 : align_up((size_t)3 * max_n, 32);
  size_t cur = 0;
  b->off_members = bump(cur, sizeof(BatchMember) * std::max<size_t>(1, b->members.size()));
  b->off_slots = bump(cur, sizeof(int32_t) * std::max<size_t>(1, b->slots.size()));
  b->off_items = bump(cur, sizeof(BatchItem) * std::max<size_t>(1, b->items.size()));
  b->off_counter = bump(cur, sizeof(int32_t));
  b->off_steps = bump(cur, sizeof(double) * (size_t)b->step_off.back());
  b->off_actions = bump(cur, sizeof(double) * b->paths.size());
  b->off_bnd = bump(cur, sizeof(double) * (size_t)bnd_elems);
  const size_t G = b->lj_ids.empty() ? 0 : (size_t)L.grid;
  b->off_nbr = bump(cur, sizeof(uint16_t) * b->nbr_stride * G);
  b->off_cnt = bump(cur, sizeof(int32_t) * b->cnt_stride * G);
  b->off_xref = bump(cur, sizeof(double) * b->xref_stride * G);
  b->off_rglob = bump(cur, sizeof(double) * b->rglob_stride * G);
  b->total = align_up(cur, kAlign);
  return PAMD_OK;
}
}  // namespace

extern "C" {

int pamd_batch_create(int32_t n_paths, const pamd_path* paths, const pamd_potential* pots,
                      const pamd_tuning* tuning, pamd_batch** out) {
  if (!out) return batch_fail(PAMD_EINVAL, "out is NULL");
  *out = nullptr;
  if (n_paths < 1) return batch_fail(PAMD_EINVAL, "n_paths must be >= 1");
  if (!paths || !pots) return batch_fail(PAMD_EINVAL, "paths and pots must be non-NULL");
  if (tuning && tuning->algo == PAMD_ALGO_PLAIN)
    return batch_fail(PAMD_EUNSUPPORTED, "batches run the fused form only");
  for (int p = 0; p < n_paths; ++p) {
    size_t dummy;
    int rc = pamd_workspace_size(&paths[p], &pots[p], tuning, &dummy);
    if (rc) return rc;
    if (paths[p].precision != paths[0].precision)
      return batch_fail(PAMD_EUNSUPPORTED, "all batch members must share one precision");
    if (paths[p].n_steps > (int64_t)INT32_MAX * 16)
      return batch_fail(PAMD_EUNSUPPORTED, "member %d has too many steps for a batch", p);
  }
  pamd_batch* b = new pamd_batch;
  b->paths.assign(paths, paths + n_paths);
  b->pots.assign(pots, pots + n_paths);
  b->f32 = paths[0].precision == PAMD_FP32_FORCE;
  b->x_off.resize(n_paths + 1);
  b->step_off.resize(n_paths + 1);
  int64_t xo = 0, so = 0;
  for (int p = 0; p < n_paths; ++p) {
    b->x_off[p] = xo;
    b->step_off[p] = so;
    xo += (int64_t)align_up((size_t)((paths[p].n_steps + 1) * paths[p].n_dim * paths[p].n_atoms), 32);
    so += (int64_t)align_up((size_t)paths[p].n_steps, 32);
    (pots[p].kind == PAMD_LJ ? b->lj_ids : b->ho_ids).push_back(p);
  }
  b->x_off[n_paths] = xo;
  b->step_off[n_paths] = so;

  if (tuning) {
    b->has_tuning = true;
    b->tuning = *tuning;
  }
  int rc = plan_batch(b);
  if (rc) {
    delete b;
    return rc;
  }
  *out = b;
  return PAMD_OK;
}

void pamd_batch_destroy(pamd_batch* b) { delete b; }

int pamd_batch_layout(const pamd_batch* b, int64_t* x_offsets, int64_t* step_offsets,
                      size_t* ws_bytes) {
  if (!b) return batch_fail(PAMD_EINVAL, "batch is NULL");
  const size_t n = b->paths.size();
  if (x_offsets) std::copy(b->x_off.begin(), b->x_off.end(), x_offsets);
  if (step_offsets) std::copy(b->step_off.begin(), b->step_off.end(), step_offsets);
  if (ws_bytes) *ws_bytes = b->total;
  (void)n;
  return PAMD_OK;
}

int pamd_batch_prepare(const pamd_batch* b, void* ws, size_t ws_bytes, void* stream) {
  if (!b) return batch_fail(PAMD_EINVAL, "batch is NULL");
  if (ws_bytes < b->total) return batch_fail(PAMD_EWORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, b->total);
  if (!ws || ((uintptr_t)ws) % kAlign) return batch_fail(PAMD_EWORKSPACE, "workspace must be non-NULL and 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  char* base = (char*)ws;
  hipError_t e = hipSuccess;
  if (!b->members.empty()) {
    e = hipMemcpyAsync(base + b->off_members, b->members.data(), sizeof(BatchMember) * b->members.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(base + b->off_slots, b->slots.data(), sizeof(int32_t) * b->slots.size(), hipMemcpyHostToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(base + b->off_items, b->items.data(), sizeof(BatchItem) * b->items.size(), hipMemcpyHostToDevice, st);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) return batch_fail(PAMD_EHIP, "batch upload: %s", hipGetErrorString(e));
  return PAMD_OK;
}

}  // extern "C"

namespace {
// The batch's launches.  Packed form: member p at x_all + x_off[p] (gradient
// likewise in grad_all).  Pointer form (xs != null): member p at xs[p], its
// gradient at gs[p] (gs or gs[p] null: no gradient), per-step terms in the
// workspace.
int run_batch(const pamd_batch* b, const double* x_all, const double* w_all, double* actions,
              double* per_step_all, double* grad_all, const double* const* xs,
              double* const* gs, void* ws, hipStream_t st) {
  char* base = (char*)ws;
  double* steps = per_step_all ? per_step_all : (double*)(base + b->off_steps);
  hipError_t e = hipSuccess;
  if (!b->lj_ids.empty()) {
    BatchBase bb;
    bb.x = x_all;
    bb.weights = w_all;
    bb.grad = grad_all;
    bb.per_step = steps;
    bb.bnd = (double*)(base + b->off_bnd);
    bb.mode = 0;
    bb.pad0 = 0;
    BlockScratch s;
    s.nbr = (uint16_t*)(base + b->off_nbr);
    s.cnt = (int32_t*)(base + b->off_cnt);
    s.xref = (double*)(base + b->off_xref);
    s.rglob = b->rglob_stride ? (double*)(base + b->off_rglob) : nullptr;
    s.nbr_stride = (int64_t)b->nbr_stride;
    s.ex_off = (int64_t)b->nbr_stride / 2;
    s.cnt_stride = (int64_t)b->cnt_stride;
    s.xref_stride = (int64_t)b->xref_stride;
    s.rglob_stride = (int64_t)b->rglob_stride;
    const BatchMember* mem = (const BatchMember*)(base + b->off_members);
    int* counter = (int*)(base + b->off_counter);
    e = launch_reset_counter(counter, st);
    if (e == hipSuccess)
      e = launch_lj_batch(mem, bb, (const BatchItem*)(base + b->off_items), (int)b->items.size(),
                          counter, s, b->launch, st);
    if (e == hipSuccess)
      e = launch_batch_finalize(mem, bb, (const int32_t*)(base + b->off_slots),
                                (int)b->members.size(), actions, b->max_tiles, st);
    if (e != hipSuccess) return batch_fail(PAMD_EHIP, "batch launch: %s", hipGetErrorString(e));
  }
  for (int p : b->ho_ids) {
    const pamd_path& P = b->paths[p];
    HOArgs h;
    h.x = xs ? xs[p] : x_all + b->x_off[p];
    h.weights = w_all ? w_all + b->step_off[p] : nullptr;
    h.grad = xs ? (gs ? gs[p] : nullptr) : (grad_all ? grad_all + b->x_off[p] : nullptr);
    h.per_step = steps + b->step_off[p];
    h.excess = nullptr;
    h.n_steps = P.n_steps;
    h.n_dof = (int64_t)P.n_dim * P.n_atoms;
    h.k = b->pots[p].k;
    h.mu_dt = P.dt / P.gamma;
    h.inv4Ddt = 1.0 / (4.0 * P.D * P.dt);
    h.c = 1.0 / (2.0 * P.D * P.dt);
    h.mode = h.grad ? MODE_GRAD : 0;
    int seg = 1;
    while (seg < 64 && seg < h.n_dof) seg <<= 1;
    h.seg = seg;
    e = launch_ho(h, actions + p, st);
    if (e != hipSuccess) return batch_fail(PAMD_EHIP, "batch harmonic launch: %s", hipGetErrorString(e));
  }
  return PAMD_OK;
}

int check_batch_ws(size_t need, void* ws, size_t ws_bytes) {
  if (ws_bytes < need) return batch_fail(PAMD_EWORKSPACE, "workspace has %zu bytes, %zu needed", ws_bytes, need);
  if (!ws || ((uintptr_t)ws) % kAlign) return batch_fail(PAMD_EWORKSPACE, "workspace must be non-NULL and 256-byte aligned");
  return PAMD_OK;
}
}  // namespace

extern "C" {

int pamd_batch_run(const pamd_batch* b, const double* x_all, const double* w_all,
                   double* actions, double* per_step_all, double* grad_all, void* ws,
                   size_t ws_bytes, void* stream) {
  if (!b) return batch_fail(PAMD_EINVAL, "batch is NULL");
  if (!x_all || !actions) return batch_fail(PAMD_EINVAL, "x_all and actions must be non-NULL");
  int rc = check_batch_ws(b->total, ws, ws_bytes);
  if (rc) return rc;
  return run_batch(b, x_all, w_all, actions, per_step_all, grad_all, nullptr, nullptr, ws,
                   (hipStream_t)stream);
}

}  // extern "C"

namespace {
struct TilePolicy {
  double budget, skin_frac;
};
// Member-tile policies the batch autotuner times: tile = budget / n_atoms
// steps (so the tiles of all members hold similar work), and the list skin.
std::vector<TilePolicy> batch_policies(const pamd_batch* b) {
  const bool fixed_tile = b->has_tuning && b->tuning.tile > 0;
  const bool fixed_skin = b->has_tuning && b->tuning.skin > 0;
  std::vector<TilePolicy> out;
  for (double budget : {8192.0, 16384.0, 32768.0, 65536.0, 131072.0, 262144.0}) {
    if (fixed_tile && budget != 16384.0) continue;
    for (double skin : {0.3, 0.5}) {
      if (fixed_skin && skin != 0.5) continue;
      out.push_back({budget, skin});
    }
  }
  return out;
}
}  // namespace

extern "C" {

int pamd_batch_autotune_workspace_size(pamd_batch* b, size_t* bytes) {
  if (!b || !bytes) return batch_fail(PAMD_EINVAL, "batch and bytes must be non-NULL");
  const TilePolicy keep{b->tile_budget, b->skin_frac};
  size_t need = b->total;
  for (const TilePolicy& c : batch_policies(b)) {
    b->tile_budget = c.budget;
    b->skin_frac = c.skin_frac;
    if (plan_batch(b) == PAMD_OK) need = std::max(need, b->total);
  }
  b->tile_budget = keep.budget;
  b->skin_frac = keep.skin_frac;
  int rc = plan_batch(b);
  if (rc) return rc;
  *bytes = need;
  return PAMD_OK;
}

int pamd_batch_autotune(pamd_batch* b, const double* x_all, double* grad_all, void* ws,
                        size_t ws_bytes, void* stream, double* tile_budget, double* skin_frac) {
  if (!b) return batch_fail(PAMD_EINVAL, "batch is NULL");
  if (!x_all) return batch_fail(PAMD_EINVAL, "x_all is NULL");
  if (!ws || ((uintptr_t)ws) % kAlign) return batch_fail(PAMD_EWORKSPACE, "workspace must be non-NULL and 256-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  double* actions = nullptr;  // the trial runs' actions (workspace)
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return batch_fail(PAMD_EHIP, "hipEventCreate failed");
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return batch_fail(PAMD_EHIP, "hipEventCreate failed");
  }
  TilePolicy best{b->tile_budget, b->skin_frac};
  float best_ms = 1e30f;
  int rc = PAMD_OK;
  for (const TilePolicy& c : batch_policies(b)) {
    b->tile_budget = c.budget;
    b->skin_frac = c.skin_frac;
    if (plan_batch(b) != PAMD_OK || b->total > ws_bytes) continue;
    if ((rc = pamd_batch_prepare(b, ws, ws_bytes, stream))) break;
    actions = (double*)((char*)ws + b->off_actions);
    if ((rc = run_batch(b, x_all, nullptr, actions, nullptr, grad_all, nullptr, nullptr, ws, st)))
      break;
    float ms_min = 1e30f;
    for (int rep = 0; rep < 2; ++rep) {
      hipEventRecord(e0, st);
      rc = run_batch(b, x_all, nullptr, actions, nullptr, grad_all, nullptr, nullptr, ws, st);
      hipEventRecord(e1, st);
      if (rc) break;
      if (hipEventSynchronize(e1) != hipSuccess) {
        rc = batch_fail(PAMD_EHIP, "hipEventSynchronize failed");
        break;
      }
      float ms = 0.0f;
      hipEventElapsedTime(&ms, e0, e1);
      ms_min = std::min(ms_min, ms);
    }
    if (rc) break;
    if (ms_min < best_ms) {
      best_ms = ms_min;
      best = c;
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  b->tile_budget = best.budget;
  b->skin_frac = best.skin_frac;
  int rc2 = plan_batch(b);
  if (rc) return rc;
  if (rc2) return rc2;
  if (best_ms >= 1e30f) return batch_fail(PAMD_EWORKSPACE, "no tile policy fits the %zu-byte workspace", ws_bytes);
  if (tile_budget) *tile_budget = best.budget;
  if (skin_frac) *skin_frac = best.skin_frac;
  if (b->total > ws_bytes) return PAMD_OK;  // the caller prepares a larger workspace
  return pamd_batch_prepare(b, ws, ws_bytes, stream);
}

int pamd_batch_workspace_size(int32_t n_paths, const pamd_path* paths, const pamd_potential* pots,
                              size_t* bytes) {
  if (!bytes) return batch_fail(PAMD_EINVAL, "bytes is NULL");
  pamd_batch* b = nullptr;
  int rc = pamd_batch_create(n_paths, paths, pots, nullptr, &b);
  if (rc) return rc;
  *bytes = b->total;
  pamd_batch_destroy(b);
  return PAMD_OK;
}

int pamd_batch_action_grad(int32_t n_paths, const pamd_path* paths, const pamd_potential* pots,
                           const double* const* x, double* actions, double* const* grads,
                           void* ws, size_t ws_bytes, void* stream) {
  if (n_paths >= 1 && !x) return batch_fail(PAMD_EINVAL, "x (array of path pointers) is NULL");
  if (n_paths >= 1 && !actions) return batch_fail(PAMD_EINVAL, "actions is NULL");
  for (int32_t p = 0; p < n_paths && x; ++p)
    if (!x[p]) return batch_fail(PAMD_EINVAL, "x[%d] is NULL", p);
  pamd_batch* b = nullptr;
  int rc = pamd_batch_create(n_paths, paths, pots, nullptr, &b);
  if (rc) return rc;
  if ((rc = check_batch_ws(b->total, ws, ws_bytes))) {
    pamd_batch_destroy(b);
    return rc;
  }
  for (size_t mi = 0; mi < b->members.size(); ++mi) {
    const int p = b->slots[mi];
    b->members[mi].x_abs = x[p];
    b->members[mi].grad_abs = grads ? grads[p] : nullptr;
  }
  hipStream_t st = (hipStream_t)stream;
  rc = pamd_batch_prepare(b, ws, ws_bytes, stream);
  if (!rc) rc = run_batch(b, nullptr, nullptr, actions, nullptr, nullptr, x, grads, ws, st);
  pamd_batch_destroy(b);
  return rc;
}

}  // extern "C"
