// Device-side helpers shared by the path-action kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

namespace pamd {

constexpr int WAVE = 64;

// ---------------------------------------------------------------------------
// Reciprocal square root: the hardware estimate (v_rsq_f64, measured relative
// error <= 5.2e-8 on [0.5, 7.5]) refined by one Newton-Raphson step on
// f(y) = 1/y^2 - x, y <- y + y (1 - x y^2) / 2, whose quadratic convergence
// leaves <= 4.3e-15 (measured; a second step would reach 2.6e-16).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  return y;
}


// Minimum-image displacement in a cubic box: d - L * rint(d / L), round half to even.
__device__ __forceinline__ double min_image(double d, double box, double inv_box) {
  return fma(-box, __builtin_rint(d * inv_box), d);
}

// ---------------------------------------------------------------------------
// Deterministic reductions: fixed butterfly order inside a wave, then wave
// partials summed in wave order by thread 0.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = fmax(v, __shfl_xor(v, off, WAVE));
  return v;
}

__device__ __forceinline__ int wave_min_int(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = min(v, __shfl_xor(v, off, WAVE));
  return v;
}

__device__ __forceinline__ int wave_max_int(int v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v = max(v, __shfl_xor(v, off, WAVE));
  return v;
}

// Block-wide sum; result valid in thread 0 only.  `scratch` (LDS, generic or
// LDS-typed pointer) holds >= 16 doubles.
template <typename P>
__device__ __forceinline__ double block_sum(double v, P scratch) {
  v = wave_sum(v);
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = threadIdx.x / WAVE;
  const int nw = (blockDim.x + WAVE - 1) / WAVE;
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < nw; ++w) s += scratch[w];
  return s;
}

// Block-wide max broadcast to every thread.  `scratch` holds >= 17 doubles.
template <typename P>
__device__ __forceinline__ double block_max_all(double v, P scratch) {
  v = wave_max(v);
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = threadIdx.x / WAVE;
  const int nw = (blockDim.x + WAVE - 1) / WAVE;
  __syncthreads();
  if (lane == 0) scratch[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = scratch[0];
    for (int w = 1; w < nw; ++w) m = fmax(m, scratch[w]);
    scratch[16] = m;
  }
  __syncthreads();
  return scratch[16];
}

// Block-wide exclusive scan of n ints in LDS (in place); writes the total to
// data[n].  `tmp` holds >= 16 ints.  All threads must call.
template <typename P>
__device__ inline void block_exclusive_scan(P data, int n, P tmp) {
  const int nt = blockDim.x;
  const int per = (n + nt - 1) / nt;
  const int lo = threadIdx.x * per;
  const int hi = min(lo + per, n);
  int local = 0;
  for (int k = lo; k < hi; ++k) local += data[k];
  // inclusive scan of `local` across the block
  const int lane = threadIdx.x & (WAVE - 1);
  const int wid = threadIdx.x / WAVE;
  int v = local;
#pragma unroll
  for (int off = 1; off < WAVE; off <<= 1) {
    int o = __shfl_up(v, off, WAVE);
    if (lane >= off) v += o;
  }
  __syncthreads();
  if (lane == WAVE - 1) tmp[wid] = v;
  __syncthreads();
  int base = 0;
  for (int w = 0; w < wid; ++w) base += tmp[w];
  int run = base + v - local;  // exclusive prefix of this thread's chunk
  __syncthreads();
  for (int k = lo; k < hi; ++k) {
    int c = data[k];
    data[k] = run;
    run += c;
  }
  if (threadIdx.x == nt - 1) data[n] = base + v;
  __syncthreads();
}

}  // namespace pamd
