// Fused Lennard-Jones path action + adjoint gradient (gfx950).
//
// One workgroup owns a tile of consecutive time steps [n0, n1).  For each step
// n it holds slice x_n in LDS, evaluates F(x_n) from a neighbour list,
// forms r_n = Delta_n - (dt/gamma) F(x_n) and the per-step action
// s_n = |r_n|^2/(4 D dt) (Eq. 3), stores rho_n = w_n r_n for the whole slice,
// then applies the Hessian K-sum to rho_n and writes
//     g_n = c [rho_{n-1} - rho_n + (dt/gamma) H(x_n) rho_n],  c = 1/(2 D dt).
// rho_{n-1} is carried in registers of the thread that owns the atom; at the
// tile's first step it belongs to the previous tile, which writes c rho_{n0-1}
// to a boundary buffer that the finalize kernel adds (fixed order, no atomics).
//
// Neighbour lists (radius r_c + skin) are built at the tile start from a cell
// list in LDS and reused while no atom has moved more than skin/2 from where
// the list was built (then every pair with r <= r_c at the current slice is
// in the list); otherwise the list is rebuilt on the spot.  The cutoff test
// itself is exact at every slice.
#include "lj_pair.hpp"

namespace pamd {

struct TileLDS {
  double* X;     // 3 * n_atoms, slice x_n (AoS)
  double* R;     // 3 * n_atoms, rho_n (AoS), when kept in LDS
  double* red;   // 32 doubles
  CellLDS cells;
};

__device__ inline TileLDS carve_lds(char* base, int n_atoms, int ncell, bool r_in_lds) {
  TileLDS t;
  size_t off = 0;
  t.X = reinterpret_cast<double*>(base + off);
  off += sizeof(double) * 3 * (size_t)n_atoms;
  if (r_in_lds) {
    t.R = reinterpret_cast<double*>(base + off);
    off += sizeof(double) * 3 * (size_t)n_atoms;
  } else {
    t.R = nullptr;
  }
  t.red = reinterpret_cast<double*>(base + off);
  off += sizeof(double) * 32;
  t.cells.tmp = reinterpret_cast<int*>(base + off);
  off += sizeof(int) * 16;
  t.cells.start = reinterpret_cast<int*>(base + off);
  off += sizeof(int) * (size_t)(ncell + 1);
  t.cells.fill = reinterpret_cast<int*>(base + off);
  off += sizeof(int) * (size_t)ncell;
  t.cells.atoms = reinterpret_cast<int*>(base + off);
  return t;
}

size_t fused_lds_bytes(int n_atoms, int nc, bool r_in_lds) {
  const size_t ncell = (size_t)nc * nc * nc;
  size_t b = sizeof(double) * 3 * (size_t)n_atoms * (r_in_lds ? 2 : 1);
  b += sizeof(double) * 32 + sizeof(int) * 16;
  b += sizeof(int) * (2 * ncell + 1);
  b += sizeof(int) * (size_t)n_atoms;
  return b;
}

// Per-block global scratch for one tile: lists and per-atom state that only
// the owning thread touches (atom i is owned by thread i mod blockDim).
struct TileScratch {
  uint16_t* nbr;   // kmax * n_atoms
  int* cnt;        // n_atoms
  double* xref;    // 3 * n_atoms: positions at the last list build
  double* rprev;   // 3 * n_atoms: rho_{n-1}
  double* rglob;   // 3 * n_atoms: rho_n of every atom when not in LDS
};

template <bool F32, bool RLDS>
__device__ void tile_body(const PathArgs& a, int tile, const TileScratch& ts, char* lds_base) {
  const int N = a.n_atoms;
  const int ncell = a.nc * a.nc * a.nc;
  TileLDS L = carve_lds(lds_base, N, ncell, RLDS);
  double* R = RLDS ? L.R : ts.rglob;
  const int64_t n0 = (int64_t)tile * a.tile;
  const int64_t n1 = min(n0 + (int64_t)a.tile, a.n_steps);
  const size_t slice = (size_t)3 * N;
  const bool grad = (a.mode & MODE_GRAD) != 0;
  const int B = blockDim.x;
  const double box = a.lj.box, ib = a.lj.inv_box;

  for (int i = threadIdx.x; i < N; i += B) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      L.X[3 * i + c] = a.x[(size_t)n0 * slice + (size_t)c * N + i];
      ts.rprev[3 * i + c] = 0.0;
    }
  }
  bool need_build = true;

  for (int64_t n = n0; n < n1; ++n) {
    const double w = a.weights ? a.weights[n] : 1.0;
    const double* xnext = a.x + (size_t)(n + 1) * slice;
    __syncthreads();  // X holds x_n

    if (!need_build) {
      double m = 0.0;
      for (int i = threadIdx.x; i < N; i += B) {
        const double ux = min_image(L.X[3 * i + 0] - ts.xref[3 * i + 0], box, ib);
        const double uy = min_image(L.X[3 * i + 1] - ts.xref[3 * i + 1], box, ib);
        const double uz = min_image(L.X[3 * i + 2] - ts.xref[3 * i + 2], box, ib);
        m = fmax(m, fma(ux, ux, fma(uy, uy, uz * uz)));
      }
      m = block_max_all(m, L.red);
      need_build = !(m <= a.half_skin2);
    }
    if (need_build) {
      if (a.nc > 0) build_cells(a.lj, L.X, N, a.nc, L.cells);
      for (int i = threadIdx.x; i < N; i += B) {
        ts.cnt[i] = build_list(a.lj, L.X, N, a.nc, a.reach, L.cells, a.rlist2, a.kmax,
                               ts.nbr + i, i);
#pragma unroll
        for (int c = 0; c < 3; ++c) ts.xref[3 * i + c] = L.X[3 * i + c];
      }
      need_build = false;
    }

    // ---- pass 1: force, residual, per-step action ----
    double s_loc = 0.0, e_loc = 0.0;
    for (int i = threadIdx.x; i < N; i += B) {
      const double xi = L.X[3 * i + 0], yi = L.X[3 * i + 1], zi = L.X[3 * i + 2];
      double f[3];
      force_on<F32>(a.lj, L.X, N, ts.nbr + i, ts.cnt[i], i, xi, yi, zi, f[0], f[1], f[2]);
      const double xo[3] = {xi, yi, zi};
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double d = min_image(xnext[(size_t)c * N + i] - xo[c], box, ib);
        const double r = fma(-a.mu_dt, f[c], d);
        s_loc = fma(r, r, s_loc);
        e_loc = fma(r - d, r + d, e_loc);
        if (grad) R[3 * i + c] = w * r;
      }
    }
    const double s_sum = block_sum(s_loc, L.red);
    if (threadIdx.x == 0) a.per_step[n] = s_sum * a.inv4Ddt;
    if (a.mode & MODE_EXCESS) {
      const double e_sum = block_sum(e_loc, L.red);
      if (threadIdx.x == 0) a.excess[n] = e_sum * a.inv4Ddt;
    }

    // ---- pass 2: Hessian-vector product and gradient ----
    if (grad) {
      __syncthreads();  // R holds rho_n of every atom
      for (int i = threadIdx.x; i < N; i += B) {
        const double xi = L.X[3 * i + 0], yi = L.X[3 * i + 1], zi = L.X[3 * i + 2];
        const double rx = R[3 * i + 0], ry = R[3 * i + 1], rz = R[3 * i + 2];
        double q[3];
        hv_on<F32>(a.lj, L.X, R, N, ts.nbr + i, ts.cnt[i], i, xi, yi, zi, rx, ry, rz, q[0],
                   q[1], q[2]);
        const double rho[3] = {rx, ry, rz};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const double g = a.c * (ts.rprev[3 * i + c] - rho[c] + a.mu_dt * q[c]);
          a.grad[(size_t)n * slice + (size_t)c * N + i] = g;
          ts.rprev[3 * i + c] = rho[c];
        }
      }
    }
    __syncthreads();  // every read of X (and R) for slice n is done
    for (int i = threadIdx.x; i < N; i += B) {
#pragma unroll
      for (int c = 0; c < 3; ++c) L.X[3 * i + c] = xnext[(size_t)c * N + i];
    }
  }

  if (grad) {
    for (int i = threadIdx.x; i < N; i += B) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double v = a.c * ts.rprev[3 * i + c];
        if (n1 == a.n_steps)
          a.grad[(size_t)a.n_steps * slice + (size_t)c * N + i] = v;
        else
          a.bnd[(size_t)tile * slice + (size_t)c * N + i] = v;
      }
    }
  }
  __syncthreads();  // LDS is reused by the next tile of this block
}

__device__ __forceinline__ TileScratch block_scratch(const BlockScratch& s) {
  TileScratch t;
  t.nbr = s.nbr + (size_t)blockIdx.x * s.nbr_stride;
  t.cnt = s.cnt + (size_t)blockIdx.x * s.cnt_stride;
  t.xref = s.xref + (size_t)blockIdx.x * s.xref_stride;
  t.rprev = t.xref + s.xref_stride / 2;
  t.rglob = s.rglob ? s.rglob + (size_t)blockIdx.x * s.rglob_stride : nullptr;
  return t;
}

template <bool F32, bool RLDS>
__global__ void __launch_bounds__(1024) lj_fused_kernel(PathArgs a, BlockScratch s) {
  extern __shared__ __align__(16) char lds[];
  const TileScratch ts = block_scratch(s);
  for (int t = blockIdx.x; t < a.n_tiles; t += gridDim.x) tile_body<F32, RLDS>(a, t, ts, lds);
}

__device__ __forceinline__ PathArgs member_args(const BatchMember& m, const BatchBase& b) {
  PathArgs a = m.a;
  a.x = b.x + m.x_off;
  a.weights = b.weights ? b.weights + m.step_off : nullptr;
  a.grad = b.grad ? b.grad + m.x_off : nullptr;
  a.per_step = b.per_step + m.step_off;
  a.bnd = b.bnd + m.bnd_off;
  a.excess = nullptr;
  a.mode = b.mode & ~MODE_EXCESS;
  if (!b.grad) a.mode &= ~MODE_GRAD;
  return a;
}

// Persistent batch kernel: workgroups pull (path, tile) items, largest first.
template <bool F32, bool RLDS>
__global__ void __launch_bounds__(1024) lj_batch_kernel(const BatchMember* members,
                                                        BatchBase base, const BatchItem* items,
                                                        int n_items, int* counter,
                                                        BlockScratch s) {
  extern __shared__ __align__(16) char lds[];
  __shared__ int next;
  const TileScratch ts = block_scratch(s);
  for (;;) {
    if (threadIdx.x == 0) next = atomicAdd(counter, 1);
    __syncthreads();
    const int it = __builtin_amdgcn_readfirstlane(next);
    __syncthreads();
    if (it >= n_items) break;
    const BatchItem item = items[it];
    const PathArgs a = member_args(members[item.path], base);
    tile_body<F32, RLDS>(a, item.tile, ts, lds);
  }
}

__global__ void reset_counter_kernel(int* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0;
}

// Boundary fixups (grad[(t+1) T] += bnd[t]) and the fixed-order action sum.
__global__ void lj_finalize_kernel(PathArgs a, double* action) {
  __shared__ double red[32];
  const int t = blockIdx.x;
  if (t < a.n_tiles - 1) {
    const size_t slice = (size_t)3 * a.n_atoms;
    const int64_t m = (int64_t)(t + 1) * a.tile;
    for (size_t e = threadIdx.x; e < slice; e += blockDim.x)
      a.grad[(size_t)m * slice + e] += a.bnd[(size_t)t * slice + e];
    return;
  }
  double v = 0.0;
  for (int64_t n = threadIdx.x; n < a.n_steps; n += blockDim.x) v += a.per_step[n];
  v = block_sum(v, red);
  if (threadIdx.x == 0 && action) *action = v;
}

// grid (tile, member): boundary fixups per member, last tile block sums the action.
__global__ void batch_finalize_kernel(const BatchMember* members, BatchBase base,
                                      const int32_t* slot, double* actions) {
  __shared__ double red[32];
  const PathArgs a = member_args(members[blockIdx.y], base);
  const int t = blockIdx.x;
  if (t >= a.n_tiles) return;
  if (t < a.n_tiles - 1) {
    if (!(a.mode & MODE_GRAD)) return;
    const size_t slice = (size_t)3 * a.n_atoms;
    const int64_t m = (int64_t)(t + 1) * a.tile;
    for (size_t e = threadIdx.x; e < slice; e += blockDim.x)
      a.grad[(size_t)m * slice + e] += a.bnd[(size_t)t * slice + e];
    return;
  }
  double v = 0.0;
  for (int64_t n = threadIdx.x; n < a.n_steps; n += blockDim.x) v += a.per_step[n];
  v = block_sum(v, red);
  if (threadIdx.x == 0) actions[slot[blockIdx.y]] = v;
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <bool F32, bool RLDS>
static hipError_t launch_fused_t(const PathArgs& a, const BlockScratch& s, const FusedLaunch& L,
                                 hipStream_t st) {
  auto kern = lj_fused_kernel<F32, RLDS>;
  hipError_t e = hipFuncSetAttribute((const void*)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)L.lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(L.grid), dim3(L.block), L.lds_bytes, st, a, s);
  return hipGetLastError();
}

template <bool F32, bool RLDS>
static hipError_t launch_batch_t(const BatchMember* m, const BatchBase& b, const BatchItem* it,
                                 int n, int* ctr, const BlockScratch& s, const FusedLaunch& L,
                                 hipStream_t st) {
  auto kern = lj_batch_kernel<F32, RLDS>;
  hipError_t e = hipFuncSetAttribute((const void*)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)L.lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(L.grid), dim3(L.block), L.lds_bytes, st, m, b, it, n, ctr, s);
  return hipGetLastError();
}

#define PAMD_DISPATCH(FN, ...)                                                  \
  return L.f32 ? (L.r_in_lds ? FN<true, true>(__VA_ARGS__) : FN<true, false>(__VA_ARGS__)) \
               : (L.r_in_lds ? FN<false, true>(__VA_ARGS__) : FN<false, false>(__VA_ARGS__));

hipError_t launch_lj_fused(const PathArgs& a, const BlockScratch& s, const FusedLaunch& L,
                           hipStream_t st) {
  PAMD_DISPATCH(launch_fused_t, a, s, L, st)
}

hipError_t launch_lj_batch(const BatchMember* m, const BatchBase& b, const BatchItem* it,
                           int n, int* ctr, const BlockScratch& s, const FusedLaunch& L,
                           hipStream_t st) {
  PAMD_DISPATCH(launch_batch_t, m, b, it, n, ctr, s, L, st)
}

hipError_t launch_lj_finalize(const PathArgs& a, double* action, hipStream_t st) {
  const int grid = (a.mode & MODE_GRAD) ? a.n_tiles : 1;
  PathArgs b = a;
  if (!(a.mode & MODE_GRAD)) b.n_tiles = 1;
  hipLaunchKernelGGL(lj_finalize_kernel, dim3(grid), dim3(256), 0, st, b, action);
  return hipGetLastError();
}

hipError_t launch_batch_finalize(const BatchMember* m, const BatchBase& b, const int32_t* slot,
                                 int n_members, double* actions, int max_tiles, hipStream_t st) {
  hipLaunchKernelGGL(batch_finalize_kernel, dim3(max_tiles, n_members), dim3(256), 0, st, m, b,
                     slot, actions);
  return hipGetLastError();
}

hipError_t launch_reset_counter(int* c, hipStream_t st) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, st, c);
  return hipGetLastError();
}

}  // namespace pamd
