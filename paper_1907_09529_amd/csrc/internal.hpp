// Internal interfaces between the C-ABI layer (api.cpp) and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pamd.h"

namespace pamd {

// Mode bits of a path evaluation.
enum : int {
  MODE_GRAD = 1,     // Hessian-vector pass and gradient
  MODE_EXCESS = 2,   // per-step excess action e_n = s_n - s0_n
  MODE_STEP = 4,     // per-step action s_n written to per_step
};

// Lennard-Jones pair constants (Eq. 16) prepared on the host.
struct LJConst {
  double box, inv_box;
  double rc2;        // cutoff^2: pair included when r^2 <= rc2
  double a24;        // 24 eps
  double sig2;       // sigma^2
  double duc;        // u'(r_c)
};

// The same constants in box units (positions u = x / L, displacements du,
// r^2 = |du|^2), as used by the fused kernel:
//   force      F += [a24_L p (2 sr6 - 1) + duc iru] du,
//   Hessian    K w = -fs w + [(a96_L2 p (7 sr6 - 2) + duc_L iru) ir2] (du.w) du,
// with iru = 1/|du|, ir2 = iru^2, sr6 = (sig2 ir2)^3, p = ir2 sr6 and
// fs = a24_L2 p (2 sr6 - 1) + duc_L iru (the physical -U'(r)/r).
// With ir6 = ir2^3 and ir8 = ir2 ir6 the same terms are polynomials in ir6:
//   force coefficient  ir8 (f12 ir6 - f6) + duc iru,
//   fs                 ir8 (s12 ir6 - s6) + duc_L iru,
//   bv                 [ir8 (b12 ir6 - b6) + duc_L iru] ir2.
struct BoxUnits {
  double rc2, sig2, rlist2, half_skin2;
  double a24_L, a24_L2, a96_L2, duc, duc_L, seven;
  double f12, f6, s12, s6, b12, b6;
};

// One path as seen by the LJ kernels.
struct PathArgs {
  const double* x;        // (N+1) * 3 * n_atoms
  const double* weights;  // N or null
  double* grad;           // (N+1) * 3 * n_atoms or null
  double* per_step;       // N (always provided: workspace when the caller passed null)
  double* excess;         // N or null
  double* bnd;            // (n_tiles - 1) * 3 * n_atoms boundary terms, or null
  int64_t n_steps;
  int32_t n_atoms;
  int32_t tile;           // steps per tile
  int32_t n_tiles;
  int32_t mode;
  double mu_dt;           // dt / gamma
  double inv4Ddt;         // 1 / (4 D dt)
  double c;               // 1 / (2 D dt)
  LJConst lj;
  // neighbour list geometry
  double rlist2;          // (rc + skin)^2
  double half_skin2;      // (skin / 2)^2: rebuild when an atom moved further
  int32_t nc;             // cells per axis (0: all pairs)
  int32_t reach;          // stencil half-width in cells; -1 (with nc = 0, exact-list
                          // kernel only): no lists, every pass scans all atoms
  int32_t kmax;           // list capacity per atom
  int32_t lds2;           // rho in LDS with two slot arrays (1) or one (0)
  BoxUnits bu;            // set by set_box_units() from lj, rlist2 and half_skin2
};

// Fills a.bu from the physical constants.  The list radius is widened by a
// relative 1e-12 so that rounding in box units can never drop a pair that
// the physical-unit bound keeps.
inline void set_box_units(PathArgs& a) {
  const double ib = a.lj.inv_box, ib2 = ib * ib;
  a.bu.rc2 = a.lj.rc2 * ib2;
  a.bu.sig2 = a.lj.sig2 * ib2;
  a.bu.rlist2 = a.rlist2 * ib2 * (1.0 + 1e-12);
  a.bu.half_skin2 = a.half_skin2 * ib2;
  a.bu.a24_L = a.lj.a24 * ib;
  a.bu.a24_L2 = a.lj.a24 * ib2;
  a.bu.a96_L2 = 4.0 * a.lj.a24 * ib2;
  a.bu.duc = a.lj.duc;
  a.bu.duc_L = a.lj.duc * ib;
  a.bu.seven = 7.0;
  const double sg6 = a.bu.sig2 * a.bu.sig2 * a.bu.sig2, sg12 = sg6 * sg6;
  a.bu.f12 = 2.0 * a.bu.a24_L * sg12;
  a.bu.f6 = a.bu.a24_L * sg6;
  a.bu.s12 = 2.0 * a.bu.a24_L2 * sg12;
  a.bu.s6 = a.bu.a24_L2 * sg6;
  a.bu.b12 = 7.0 * a.bu.a96_L2 * sg12;
  a.bu.b6 = 2.0 * a.bu.a96_L2 * sg6;
}

// Per-block scratch in global memory for the fused LJ kernel.
struct BlockScratch {
  uint16_t* nbr;   // per block: neighbour lists, then (unless ex_off is 0) exact lists, (kmax + 32) * n_atoms each
  int32_t* cnt;    // n_atoms per block
  double* xref;    // 6 * n_atoms per block: list-build positions, then rho_{n-1}
  double* rglob;   // 3 * n_atoms per block (residuals when they do not fit in LDS), or null
  int64_t nbr_stride, cnt_stride, xref_stride, rglob_stride;  // elements per block
  int64_t ex_off;  // elements from a block's neighbour lists to its exact lists; 0: none
};

struct FusedLaunch {
  int block;        // threads per block
  int grid;         // blocks
  bool r_in_lds;
  bool lds2;        // with r_in_lds: two slot arrays (else one)
  bool f32;
  bool half;        // half neighbour lists with LDS atomics (else full lists)
  bool exl;         // exact lists in LDS, one slot array (lj_fused_exl_kernel)
  size_t lds_bytes;
};

// Batch work item: one tile of one member path.
struct BatchItem {
  int32_t path;
  int32_t tile;
};

// Batch member descriptor (uploaded once): PathArgs with null pointers plus
// element offsets into the packed buffers passed at call time.
struct BatchMember {
  PathArgs a;
  int64_t x_off;      // into x_all / grad_all
  int64_t step_off;   // into weights_all / per_step_all
  int64_t bnd_off;    // into the workspace boundary buffer
  const double* x_abs;  // the member's own path and gradient buffers (pointer-array
  double* grad_abs;     // form); null: the packed buffers at x_off
};

// Packed buffers of one batch call.
struct BatchBase {
  const double* x;
  const double* weights;
  double* grad;
  double* per_step;
  double* bnd;
  int32_t mode;
  int32_t pad0;
};

// Shared memory of the fused kernel's workgroup (bytes).
// With rho in LDS (r_in_lds) there are two slot arrays (two) or one.
size_t fused_lds_bytes(int n_atoms, int nc, bool r_in_lds, bool half, int block, bool two = true);
int fused_half_slots();
// Shared memory of the exact-lists-in-LDS kernel (n_atoms <= block).
size_t exl_lds_bytes(int n_atoms, int nc, int block);
constexpr size_t kFusedLdsMax = 163840;  // LDS per workgroup on gfx950
// Dynamic LDS a batch launch may use: the batch kernel's own work-queue slot
// takes 16 bytes of static LDS.
constexpr size_t kBatchLdsMax = kFusedLdsMax - 16;

// Cell grid of a list build: nc cells per axis (0: all pairs), stencil
// half-width `reach` cells.
struct CellGrid {
  int nc = 0, reach = 0;
};
// Cells of edge >= radius / reach for reach in 1..3, at most max_cells of
// them (and at most 4 per atom); the variant visiting the fewest candidate
// atoms wins.
CellGrid choose_cells(double box, double radius, int n_atoms, int max_cells, double cell_cost = 0.0);
// The finest cell grid with which the fused kernel's LDS (given block size,
// residual placement and list kind) fits `cap` bytes; false if none does.
bool fused_cells_fit(double box, double radius, int n_atoms, int block, bool r_in_lds, bool half,
                     CellGrid* grid, size_t* lds, bool two = true, size_t cap = kFusedLdsMax);
size_t plain_lds_bytes(int n_atoms, int nc);

hipError_t launch_lj_fused(const PathArgs& a, const BlockScratch& s, const FusedLaunch& L,
                           hipStream_t st);
hipError_t launch_lj_finalize(const PathArgs& a, double* action, hipStream_t st);
hipError_t launch_lj_batch(const BatchMember* members, const BatchBase& base,
                           const BatchItem* items, int n_items, int* counter,
                           const BlockScratch& s, const FusedLaunch& L, hipStream_t st);
hipError_t launch_batch_finalize(const BatchMember* members, const BatchBase& base,
                                 const int32_t* member_slot, int n_members, double* actions,
                                 int max_tiles, hipStream_t st);
hipError_t launch_reset_counter(int* counter, hipStream_t st);

// Plain (unfused) LJ pipeline.
struct PlainArgs {
  PathArgs p;
  uint16_t* nbr;   // N * kmax * n_atoms
  int32_t* cnt;    // N * n_atoms
  double* F;       // N * 3 * n_atoms
  double* R;       // N * 3 * n_atoms (weighted residuals)
  double* Q;       // N * 3 * n_atoms
};
hipError_t launch_lj_plain(const PlainArgs& a, int block, bool f32, double* action,
                           hipStream_t st);

// Harmonic path.
struct HOArgs {
  const double* x;
  const double* weights;
  double* grad;
  double* per_step;
  double* excess;
  int64_t n_steps;
  int64_t n_dof;
  double k;
  double mu_dt, inv4Ddt, c;
  int32_t mode;
  int32_t seg;     // lanes per slice in the reduction (power of two <= 64)
};
hipError_t launch_ho(const HOArgs& a, double* action, hipStream_t st);

// Sequential Euler-Maruyama integrators (Eq. 2).
hipError_t launch_lj_em(const PathArgs& a, const double* xi, double amp, double* xout,
                        const BlockScratch& s, const FusedLaunch& L, hipStream_t st);
hipError_t launch_ho_em(const double* x0, const double* xi, double* xout, int64_t n_steps,
                        int64_t n_dof, double kmu, double amp, hipStream_t st);
hipError_t launch_sum(const double* v, int64_t n, double* out, hipStream_t st);

// Path sampling.
struct MHArgs {
  double* x;
  double* trial;
  double* excess;        // e_n of x
  double* excess_trial;  // e'_n (workspace)
  double* frag_delta;    // may be null
  int32_t* frag_accept;  // may be null
  int32_t* step_info;    // may be null
  int32_t* state;        // workspace: {l, u, n_frag, n_acc}
  int32_t* acc_ws;       // workspace: accept flag per fragment
  int64_t* sweep_counter;
  unsigned long long* level_stats;  // may be null: {proposed, accepted} fragments per level, summed
  int64_t n_steps;
  int64_t n_dof;
  uint32_t key0, key1;
  int32_t l_min, l_max;
  double sig;            // sqrt(2 D dt)
};
hipError_t launch_mh_prepare(const MHArgs& m, hipStream_t st);
hipError_t launch_mh_trial(const MHArgs& m, hipStream_t st);
hipError_t launch_mh_accept(const MHArgs& m, hipStream_t st);

// Shifting event of the path-based integrator.
struct ShiftArgs {
  const double* x_in;
  double* x_out;
  const double* ex_in;   // may be null (then ex_out is too)
  double* ex_out;
  double* traj;          // may be null
  int64_t* event_counter;
  int64_t n_steps;
  int64_t n_dof;
  int64_t n_shift;
  uint32_t key0, key1;
  double sig;            // sqrt(2 D dt)
};
hipError_t launch_shift(const ShiftArgs& a, hipStream_t st);

// Gradient-informed (Metropolis-adjusted Langevin) path move.
struct LangevinArgs {
  double* x;             // current path, its gradient and action (device scalar)
  double* grad;
  double* action;
  double* y;             // proposal, its gradient and action (workspace scalar)
  double* grad_y;
  const double* action_y;
  double* partial;       // workspace: 2 per partial-sum block
  int32_t* flag;         // workspace: the decision
  int32_t* accepted;     // may be null
  double* log_alpha;     // may be null
  int64_t* counter;
  int64_t n_steps;
  int64_t n_dof;
  uint32_t key0, key1;
  double tau;
  int32_t blocks;        // partial-sum blocks
};
constexpr int kLangevinBlocks = 512;
hipError_t launch_langevin_propose(const LangevinArgs& a, hipStream_t st);
hipError_t launch_langevin_accept(const LangevinArgs& a, hipStream_t st);
hipError_t launch_copy(const double* src, double* dst, int64_t n, hipStream_t st);

}  // namespace pamd
