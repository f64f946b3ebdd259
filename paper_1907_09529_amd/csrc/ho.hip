// Harmonic-oscillator path action and gradient (V = k x^2 / 2 per degree of
// freedom, Sec. IV A).  Streaming kernel: every element needs x_{n-1}, x_n,
// x_{n+1} of the same degree of freedom, so one pass over the path computes
//   r_n = x_{n+1} - x_n + (dt/gamma) k x_n,   s_n = sum r_n^2 / (4 D dt),
//   g_n = c [w_{n-1} r_{n-1} - w_n r_n (1 - (dt/gamma) k)].
// `seg` lanes (a power of two <= 64) share a slice; per-slice sums use a
// fixed xor-butterfly inside the segment.  A path that one workgroup covers
// in at most two rounds is done by a single workgroup (ONE), which also sums
// the per-step terms into the action in a fixed order (each thread over its
// slices in slice order, then the block sum), so no second launch is needed.
#include "device.hpp"
#include "internal.hpp"

namespace pamd {

template <bool ONE>
__global__ void __launch_bounds__(1024) ho_kernel(HOArgs a, double* action) {
  const int lane = threadIdx.x & (WAVE - 1);
  const int seg = a.seg;
  const int per_wave = WAVE / seg;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / WAVE;
  const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) / WAVE;
  const int sub = lane / seg, sl = lane % seg;
  const double kmu = a.k * a.mu_dt;
  double acc = 0.0;  // ONE: this thread's per-step terms, in slice order
  for (int64_t base = wave * per_wave; base <= a.n_steps; base += n_waves * per_wave) {
    const int64_t n = base + sub;
    const bool valid = n <= a.n_steps;
    double s_loc = 0.0, e_loc = 0.0;
    if (valid) {
      const double w = (a.weights && n < a.n_steps) ? a.weights[n] : 1.0;
      const double wp = (a.weights && n >= 1) ? a.weights[n - 1] : 1.0;
      for (int64_t e = sl; e < a.n_dof; e += seg) {
        const double xn = a.x[n * a.n_dof + e];
        double g = 0.0;
        if (n < a.n_steps) {
          const double d = a.x[(n + 1) * a.n_dof + e] - xn;
          const double r = fma(kmu, xn, d);
          s_loc = fma(r, r, s_loc);
          e_loc = fma(r - d, r + d, e_loc);
          g = -w * r * (1.0 - kmu);
        }
        if (n >= 1) {
          const double xp = a.x[(n - 1) * a.n_dof + e];
          const double rp = fma(kmu, xp, xn - xp);
          g = fma(wp, rp, g);
        }
        if (a.mode & MODE_GRAD) a.grad[n * a.n_dof + e] = a.c * g;
      }
    }
    for (int off = seg >> 1; off >= 1; off >>= 1) {
      s_loc += __shfl_xor(s_loc, off, WAVE);
      e_loc += __shfl_xor(e_loc, off, WAVE);
    }
    if (valid && sl == 0 && n < a.n_steps) {
      const double v = s_loc * a.inv4Ddt;
      a.per_step[n] = v;
      if constexpr (ONE) acc += v;
      if (a.mode & MODE_EXCESS) a.excess[n] = e_loc * a.inv4Ddt;
    }
  }
  if constexpr (ONE) {
    __shared__ double red[32];
    const double t = block_sum(acc, red);
    if (threadIdx.x == 0 && action) *action = t;
  }
}

// Sequential Euler-Maruyama integration (Eq. 2) of the harmonic oscillator:
// each thread steps one degree of freedom, x_{n+1} = x_n - (dt/gamma) k x_n +
// sqrt(2 D dt) xi_n.
__global__ void ho_em_kernel(const double* x0, const double* xi, double* xout, int64_t n_steps,
                             int64_t n_dof, double kmu, double amp) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_dof) return;
  double x = x0[e];
  xout[e] = x;
  for (int64_t n = 0; n < n_steps; ++n) {
    x = fma(amp, xi[n * n_dof + e], fma(-kmu, x, x));
    xout[(n + 1) * n_dof + e] = x;
  }
}

hipError_t launch_ho_em(const double* x0, const double* xi, double* xout, int64_t n_steps,
                        int64_t n_dof, double kmu, double amp, hipStream_t st) {
  const int64_t blocks = (n_dof + 255) / 256;
  hipLaunchKernelGGL(ho_em_kernel, dim3((unsigned)blocks), dim3(256), 0, st, x0, xi, xout, n_steps,
                     n_dof, kmu, amp);
  return hipGetLastError();
}

hipError_t launch_ho(const HOArgs& a, double* action, hipStream_t st) {
  const int per_wave = WAVE / a.seg;
  const int64_t waves = (a.n_steps + 1 + per_wave - 1) / per_wave;
  if (waves <= 32) {  // one workgroup of 16 waves, at most two rounds each
    hipLaunchKernelGGL(ho_kernel<true>, dim3(1), dim3(1024), 0, st, a, action);
    return hipGetLastError();
  }
  const int64_t blocks = std::min<int64_t>((waves + 3) / 4, 8192);
  hipLaunchKernelGGL(ho_kernel<false>, dim3((unsigned)blocks), dim3(256), 0, st, a, nullptr);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_sum(a.per_step, a.n_steps, action, st);
}

}  // namespace pamd
