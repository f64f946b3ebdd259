// Plain (unfused) Lennard-Jones path action + gradient: the straightforward
// GPU form, one kernel per stage, every intermediate in device memory.
//   list   : per-slice cell list -> exact-cutoff neighbour list   (N x kmax x n_atoms)
//   force  : F(x_n)                                                (N x 3 x n_atoms)
//   resid  : rho_n = w_n (Delta_n - (dt/gamma) F_n), s_n, e_n      (N x 3 x n_atoms)
//   hv     : q_n = H(x_n) rho_n                                    (N x 3 x n_atoms)
//   grad   : g_m = c [rho_{m-1} - rho_m + (dt/gamma) q_m]
//   sum    : S = sum_n s_n (fixed order)
#include "lj_pair.hpp"

namespace pamd {

size_t plain_lds_bytes(int n_atoms, int nc) {
  const size_t ncell = (size_t)nc * nc * nc;
  return sizeof(double) * 6 * (size_t)n_atoms + sizeof(double) * 32 + sizeof(int) * 16 +
         sizeof(int) * (2 * ncell + 1) + sizeof(int) * (size_t)n_atoms;
}

struct PlainLDS {
  double* X;
  double* R;
  double* red;
  CellLDS cells;
};

__device__ inline PlainLDS plain_carve(char* base, int n_atoms, int ncell) {
  PlainLDS t;
  size_t off = 0;
  t.X = reinterpret_cast<double*>(base + off);
  off += sizeof(double) * 3 * (size_t)n_atoms;
  t.R = reinterpret_cast<double*>(base + off);
  off += sizeof(double) * 3 * (size_t)n_atoms;
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

__device__ inline void load_slice(double* X, const double* x, int n_atoms) {
  for (int e = threadIdx.x; e < 3 * n_atoms; e += blockDim.x) {
    const int c = e / n_atoms, i = e - c * n_atoms;
    X[3 * i + c] = x[e];
  }
}

__global__ void __launch_bounds__(1024) plain_list_kernel(PlainArgs a) {
  extern __shared__ __align__(16) char lds[];
  const PathArgs& p = a.p;
  const int N = p.n_atoms;
  const int64_t n = blockIdx.x;
  PlainLDS L = plain_carve(lds, N, p.nc * p.nc * p.nc);
  load_slice(L.X, p.x + (size_t)n * 3 * N, N);
  __syncthreads();
  if (p.nc > 0) build_cells(p.lj, L.X, N, p.nc, L.cells);
  uint16_t* nbr = a.nbr + (size_t)n * p.kmax * N;
  for (int i = threadIdx.x; i < N; i += blockDim.x)
    a.cnt[(size_t)n * N + i] =
        build_list(p.lj, L.X, N, p.nc, p.reach, L.cells, p.lj.rc2, p.kmax, nbr + i, i);
}

template <bool F32>
__global__ void __launch_bounds__(1024) plain_force_kernel(PlainArgs a) {
  extern __shared__ __align__(16) char lds[];
  const PathArgs& p = a.p;
  const int N = p.n_atoms;
  const int64_t n = blockIdx.x;
  PlainLDS L = plain_carve(lds, N, 0);
  load_slice(L.X, p.x + (size_t)n * 3 * N, N);
  __syncthreads();
  const uint16_t* nbr = a.nbr + (size_t)n * p.kmax * N;
  double* F = a.F + (size_t)n * 3 * N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    double fx, fy, fz;
    force_on<F32>(p.lj, L.X, N, nbr + i, a.cnt[(size_t)n * N + i], i, L.X[3 * i],
                  L.X[3 * i + 1], L.X[3 * i + 2], fx, fy, fz);
    F[i] = fx;
    F[N + i] = fy;
    F[2 * N + i] = fz;
  }
}

__global__ void __launch_bounds__(1024) plain_residual_kernel(PlainArgs a) {
  __shared__ double red[32];
  const PathArgs& p = a.p;
  const int N = p.n_atoms;
  const int64_t n = blockIdx.x;
  const size_t sl = (size_t)3 * N;
  const double w = p.weights ? p.weights[n] : 1.0;
  double s_loc = 0.0, e_loc = 0.0;
  for (int e = threadIdx.x; e < 3 * N; e += blockDim.x) {
    const double d = min_image(p.x[(size_t)(n + 1) * sl + e] - p.x[(size_t)n * sl + e], p.lj.box,
                               p.lj.inv_box);
    const double r = fma(-p.mu_dt, a.F[(size_t)n * sl + e], d);
    s_loc = fma(r, r, s_loc);
    e_loc = fma(r - d, r + d, e_loc);
    a.R[(size_t)n * sl + e] = w * r;
  }
  const double s = block_sum(s_loc, red);
  if (threadIdx.x == 0) p.per_step[n] = s * p.inv4Ddt;
  if (p.mode & MODE_EXCESS) {
    const double ex = block_sum(e_loc, red);
    if (threadIdx.x == 0) p.excess[n] = ex * p.inv4Ddt;
  }
}

template <bool F32>
__global__ void __launch_bounds__(1024) plain_hv_kernel(PlainArgs a) {
  extern __shared__ __align__(16) char lds[];
  const PathArgs& p = a.p;
  const int N = p.n_atoms;
  const int64_t n = blockIdx.x;
  PlainLDS L = plain_carve(lds, N, 0);
  load_slice(L.X, p.x + (size_t)n * 3 * N, N);
  load_slice(L.R, a.R + (size_t)n * 3 * N, N);
  __syncthreads();
  const uint16_t* nbr = a.nbr + (size_t)n * p.kmax * N;
  double* Q = a.Q + (size_t)n * 3 * N;
  for (int i = threadIdx.x; i < N; i += blockDim.x) {
    double qx, qy, qz;
    hv_on<F32>(p.lj, L.X, L.R, N, nbr + i, a.cnt[(size_t)n * N + i], i, L.X[3 * i],
               L.X[3 * i + 1], L.X[3 * i + 2], L.R[3 * i], L.R[3 * i + 1], L.R[3 * i + 2], qx,
               qy, qz);
    Q[i] = qx;
    Q[N + i] = qy;
    Q[2 * N + i] = qz;
  }
}

__global__ void plain_grad_kernel(PlainArgs a) {
  const PathArgs& p = a.p;
  const size_t sl = (size_t)3 * p.n_atoms;
  const size_t total = (size_t)(p.n_steps + 1) * sl;
  for (size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (size_t)gridDim.x * blockDim.x) {
    const int64_t m = (int64_t)(e / sl);
    double g = 0.0;
    if (m >= 1) g += a.R[e - sl];
    if (m < p.n_steps) g += fma(p.mu_dt, a.Q[e], -a.R[e]);
    p.grad[e] = p.c * g;
  }
}

__global__ void sum_kernel(const double* v, int64_t n, double* out) {
  __shared__ double red[32];
  double s = 0.0;
  for (int64_t k = threadIdx.x; k < n; k += blockDim.x) s += v[k];
  s = block_sum(s, red);
  if (threadIdx.x == 0 && out) *out = s;
}

hipError_t launch_sum(const double* v, int64_t n, double* out, hipStream_t st) {
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, v, n, out);
  return hipGetLastError();
}

hipError_t launch_lj_plain(const PlainArgs& a, int block, bool f32, double* action,
                           hipStream_t st) {
  const PathArgs& p = a.p;
  const int N = p.n_atoms;
  const unsigned grid = (unsigned)p.n_steps;
  const size_t lds_list = plain_lds_bytes(N, p.nc);
  const size_t lds_pair = plain_lds_bytes(N, 0);
  hipError_t e;
#define PAMD_SETLDS(K, B)                                                                        \
  e = hipFuncSetAttribute((const void*)(K), hipFuncAttributeMaxDynamicSharedMemorySize, (int)(B)); \
  if (e != hipSuccess) return e;
  PAMD_SETLDS(plain_list_kernel, lds_list)
  hipLaunchKernelGGL(plain_list_kernel, dim3(grid), dim3(block), lds_list, st, a);
  if (f32) {
    PAMD_SETLDS(plain_force_kernel<true>, lds_pair)
    hipLaunchKernelGGL(plain_force_kernel<true>, dim3(grid), dim3(block), lds_pair, st, a);
  } else {
    PAMD_SETLDS(plain_force_kernel<false>, lds_pair)
    hipLaunchKernelGGL(plain_force_kernel<false>, dim3(grid), dim3(block), lds_pair, st, a);
  }
  hipLaunchKernelGGL(plain_residual_kernel, dim3(grid), dim3(256), 0, st, a);
  if (p.mode & MODE_GRAD) {
    if (f32) {
      PAMD_SETLDS(plain_hv_kernel<true>, lds_pair)
      hipLaunchKernelGGL(plain_hv_kernel<true>, dim3(grid), dim3(block), lds_pair, st, a);
    } else {
      PAMD_SETLDS(plain_hv_kernel<false>, lds_pair)
      hipLaunchKernelGGL(plain_hv_kernel<false>, dim3(grid), dim3(block), lds_pair, st, a);
    }
    const size_t total = (size_t)(p.n_steps + 1) * 3 * N;
    const unsigned g2 = (unsigned)std::min<size_t>((total + 255) / 256, 65536);
    hipLaunchKernelGGL(plain_grad_kernel, dim3(g2), dim3(256), 0, st, a);
  }
#undef PAMD_SETLDS
  hipLaunchKernelGGL(sum_kernel, dim3(1), dim3(256), 0, st, p.per_step, p.n_steps, action);
  return hipGetLastError();
}

}  // namespace pamd
