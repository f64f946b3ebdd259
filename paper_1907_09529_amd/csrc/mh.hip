// One Monte Carlo step of the multilevel sliding-and-sampling path move (Sec. III):
// random level and offset, free-particle trial fragments with fixed endpoints,
// fragment-wise Metropolis-Hastings test on the excess action, commit.
// Random numbers: Philox4x32-10 (Salmon et al., SC'11) with the stream layout
// documented in pamd.h; trial normals by Box-Muller.
#include <algorithm>

#include "device.hpp"
#include "internal.hpp"

namespace pamd {

struct U4 {
  uint32_t v[4];
};

// Philox4x32-10: 10 rounds of (c0,c1,c2,c3) <- (hi(M1 c2)^c1^k0, lo(M1 c2), hi(M0 c0)^c3^k1, lo(M0 c0)),
// key bumped by the Weyl constants before every round but the first.
__device__ __forceinline__ U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                     uint32_t k0, uint32_t k1) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
    const uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
    const uint32_t n0 = hi1 ^ c1 ^ k0, n2 = hi0 ^ c3 ^ k1;
    c0 = n0;
    c1 = lo1;
    c2 = n2;
    c3 = lo0;
  }
  U4 o;
  o.v[0] = c0;
  o.v[1] = c1;
  o.v[2] = c2;
  o.v[3] = c3;
  return o;
}

// Exact double in (0, 1): ((a >> 6) 2^26 + (b >> 6) + 1/2) 2^-52.
__device__ __forceinline__ double uniform52(uint32_t a, uint32_t b) {
  const double k = (double)(a >> 6) * 67108864.0 + (double)(b >> 6);
  return (k + 0.5) * (1.0 / 4503599627370496.0);
}

// Normal variates of flat elements 2p (cosine output) and 2p + 1 (sine output)
// from stream `purpose` (3: trial moves of sweep `ctr`, 4: regrowth after
// shifting event `ctr`).
__device__ __forceinline__ void stream_normal_pair(uint64_t p, uint32_t ctr, uint32_t purpose,
                                                   uint32_t k0, uint32_t k1, double& even,
                                                   double& odd) {
  const U4 w = philox((uint32_t)p, (uint32_t)(p >> 32), ctr, purpose, k0, k1);
  const double u1 = uniform52(w.v[0], w.v[1]);
  const double u2 = uniform52(w.v[2], w.v[3]);
  const double rad = sqrt(-2.0 * log(u1));
  double sn, cs;
  sincos(2.0 * M_PI * u2, &sn, &cs);
  even = rad * cs;
  odd = rad * sn;
}

// Writes the variates of flat elements lo .. hi - 1 to out[e - lo], one
// Box-Muller pair per thread.
__device__ __forceinline__ void fill_normals(double* out, uint64_t lo, uint64_t hi, uint32_t ctr,
                                             uint32_t purpose, uint32_t k0, uint32_t k1) {
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t p = (lo >> 1) + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; 2 * p < hi;
       p += stride) {
    double a, b;
    stream_normal_pair(p, ctr, purpose, k0, k1, a, b);
    if (2 * p >= lo) out[2 * p - lo] = a;
    if (2 * p + 1 < hi) out[2 * p + 1 - lo] = b;
  }
}

// Level and offset of the sweep (into state), and the trial variates of
// every element, stored in `trial` where the trial kernel consumes them.
__global__ void mh_normals_kernel(MHArgs m) {
  const uint32_t s = (uint32_t)(*m.sweep_counter);
  fill_normals(m.trial, 0, (uint64_t)(m.n_steps + 1) * m.n_dof, s, 3u, m.key0, m.key1);
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const U4 w = philox(0u, 0u, s, 1u, m.key0, m.key1);
  const int l = m.l_min + (int)(w.v[0] % (uint32_t)(m.l_max - m.l_min + 1));
  const int64_t span = (int64_t)1 << l;
  const int64_t u = 1 + (int64_t)(w.v[1] % (uint32_t)span);
  const int64_t n_end = (m.n_steps - u) / span + 1;           // endpoints u + k span <= N
  const int64_t last = u + (n_end - 1) * span;
  const int64_t n_frag = n_end + (last < m.n_steps ? 1 : 0);
  m.state[0] = l;
  m.state[1] = (int32_t)u;
  m.state[2] = (int32_t)n_frag;
  m.state[3] = 0;
}

// Fragment f spans [a, b]; f = 0 is the tail [0, u]; the nose (if any) ends at N.
__device__ __forceinline__ void frag_range(int f, int l, int64_t u, int n_frag, int64_t N,
                                           int64_t& a, int64_t& b, bool& nose) {
  const int64_t span = (int64_t)1 << l;
  if (f == 0) {
    a = 0;
    b = u;
  } else {
    a = u + (int64_t)(f - 1) * span;
    b = std::min(a + span, N);
  }
  nose = (f == n_frag - 1) && (b == N) && ((N - u) % span != 0);
}

// One thread per fragment and degree of freedom runs the fragment's trial
// recurrence; the variate of slice k sits in trial[k] until the thread
// overwrites it (each slot is read only by the thread that writes it).
constexpr int RUN = 8;  // variates loaded per batch by the serial recurrences

__global__ void mh_trial_kernel(MHArgs m) {
  const int l = m.state[0];
  const int64_t u = m.state[1];
  const int n_frag = m.state[2];
  const int64_t total = (int64_t)n_frag * m.n_dof;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int f = (int)(t / m.n_dof);
    const int64_t e = t - (int64_t)f * m.n_dof;
    int64_t a, b;
    bool nose;
    frag_range(f, l, u, n_frag, m.n_steps, a, b, nose);
    double y = m.x[a * m.n_dof + e];
    m.trial[a * m.n_dof + e] = y;
    // the variates are read RUN at a time ahead of the serial recurrence, so
    // that their loads overlap
    double* col = m.trial + e;
    if (nose) {
      for (int64_t k0 = a; k0 < b; k0 += RUN) {
        double z[RUN];
#pragma unroll
        for (int j = 0; j < RUN; ++j)
          if (k0 + j < b) z[j] = col[(k0 + j + 1) * m.n_dof];
#pragma unroll
        for (int j = 0; j < RUN; ++j)
          if (k0 + j < b) {
            y = fma(m.sig, z[j], y);
            col[(k0 + j + 1) * m.n_dof] = y;
          }
      }
    } else {
      const double xb = m.x[b * m.n_dof + e];
      for (int64_t k0 = a; k0 < b - 1; k0 += RUN) {
        double z[RUN];
#pragma unroll
        for (int j = 0; j < RUN; ++j)
          if (k0 + j < b - 1) z[j] = col[(k0 + j + 1) * m.n_dof];
#pragma unroll
        for (int j = 0; j < RUN; ++j)
          if (k0 + j < b - 1) {
            const double rem = (double)(b - (k0 + j));
            y = y + (xb - y) / rem + m.sig * sqrt((rem - 1.0) / rem) * z[j];
            col[(k0 + j + 1) * m.n_dof] = y;
          }
      }
      if (b == m.n_steps) m.trial[b * m.n_dof + e] = xb;
    }
  }
}

__global__ void mh_accept_kernel(MHArgs m) {
  __shared__ double red[32];
  const int l = m.state[0];
  const int64_t u = m.state[1];
  const int n_frag = m.state[2];
  const uint32_t s = (uint32_t)(*m.sweep_counter);
  double n_acc = 0.0;
  for (int f = threadIdx.x; f < n_frag; f += blockDim.x) {
    int64_t a, b;
    bool nose;
    frag_range(f, l, u, n_frag, m.n_steps, a, b, nose);
    double delta = 0.0;
    for (int64_t n = a; n < b; ++n) delta += m.excess_trial[n] - m.excess[n];
    const U4 w = philox((uint32_t)f, 0u, s, 2u, m.key0, m.key1);
    const double uf = uniform52(w.v[0], w.v[1]);
    const int acc = (uf < exp(-delta)) ? 1 : 0;
    m.acc_ws[f] = acc;
    if (m.frag_delta) m.frag_delta[f] = delta;
    if (m.frag_accept) m.frag_accept[f] = acc;
    n_acc += acc;
  }
  const double tot = block_sum(n_acc, red);
  if (threadIdx.x == 0) {
    m.state[3] = (int)tot;
    if (m.step_info) {
      m.step_info[0] = l;
      m.step_info[1] = (int32_t)u;
      m.step_info[2] = n_frag;
      m.step_info[3] = (int)tot;
    }
    if (m.level_stats) {
      atomicAdd(m.level_stats + 2 * l, (unsigned long long)n_frag);
      atomicAdd(m.level_stats + 2 * l + 1, (unsigned long long)tot);
    }
  }
}

// Copies accepted fragments into x and their excess actions into `excess`,
// and advances the sweep counter (no kernel of this sweep reads it later).
__global__ void mh_commit_kernel(MHArgs m) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *m.sweep_counter += 1;
  const int l = m.state[0];
  const int64_t u = m.state[1];
  const int64_t total = (m.n_steps + 1) * m.n_dof;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t n = t / m.n_dof;
    if (n == 0) continue;
    bool endpoint = false;
    int f;
    if (n < u) {
      f = 0;
    } else {
      const int64_t k = n - u;
      endpoint = (k & (((int64_t)1 << l) - 1)) == 0;
      f = 1 + (int)(k >> l);
    }
    if (!endpoint && m.acc_ws[f]) m.x[t] = m.trial[t];
  }
  for (int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; n < m.n_steps;
       n += (int64_t)gridDim.x * blockDim.x) {
    const int f = (n < u) ? 0 : 1 + (int)((n - u) >> l);
    if (m.acc_ws[f]) m.excess[n] = m.excess_trial[n];
  }
}

hipError_t launch_mh_prepare(const MHArgs& m, hipStream_t st) {
  const int64_t pairs = ((m.n_steps + 1) * m.n_dof + 1) / 2;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((pairs + 255) / 256, 16384));
  hipLaunchKernelGGL(mh_normals_kernel, dim3((unsigned)blocks), dim3(256), 0, st, m);
  return hipGetLastError();
}

hipError_t launch_mh_trial(const MHArgs& m, hipStream_t st) {
  const int64_t max_frag = m.n_steps / ((int64_t)1 << m.l_min) + 2;
  const int64_t total = max_frag * m.n_dof;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 16384);
  hipLaunchKernelGGL(mh_trial_kernel, dim3((unsigned)blocks), dim3(256), 0, st, m);
  return hipGetLastError();
}

hipError_t launch_mh_accept(const MHArgs& m, hipStream_t st) {
  hipLaunchKernelGGL(mh_accept_kernel, dim3(1), dim3(1024), 0, st, m);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = (m.n_steps + 1) * m.n_dof;
  const int64_t blocks = std::min<int64_t>((total + 255) / 256, 16384);
  hipLaunchKernelGGL(mh_commit_kernel, dim3((unsigned)blocks), dim3(256), 0, st, m);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Shifting event of the path-based integrator (Sec. II B, Fig. 2B)
// ---------------------------------------------------------------------------
// x_out[n] = x_in[n + s] for n = 0 .. N - s, the kept excess terms move along,
// x_in[1 .. s] leave as trajectory, and the regrowth variates are stored in
// the regrown slices of x_out.
__global__ void shift_copy_kernel(ShiftArgs a) {
  const int64_t keep = a.n_steps - a.n_shift;
  fill_normals(a.x_out + (keep + 1) * a.n_dof, (uint64_t)(keep + 1) * a.n_dof,
               (uint64_t)(a.n_steps + 1) * a.n_dof, (uint32_t)(*a.event_counter), 4u, a.key0,
               a.key1);
  const int64_t off = (int64_t)a.n_shift * a.n_dof;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t t = t0; t < (keep + 1) * a.n_dof; t += stride) a.x_out[t] = a.x_in[t + off];
  if (a.ex_out)
    for (int64_t n = t0; n < keep; n += stride) a.ex_out[n] = a.ex_in[n + a.n_shift];
  if (a.traj)
    for (int64_t t = t0; t < off; t += stride) a.traj[t] = a.x_in[t + a.n_dof];
}

// Slices N - s + 1 .. N regrown from the new slice N - s (= x_in[N]) by free
// Brownian continuation over the stored variates, one thread per degree of
// freedom; then the event counter advances (the copy kernel has read it).
__global__ void shift_regrow_kernel(ShiftArgs a) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k == 0) *a.event_counter += 1;
  if (k >= a.n_dof) return;
  double y = a.x_in[a.n_steps * a.n_dof + k];
  double* col = a.x_out + k;
  for (int64_t n0 = a.n_steps - a.n_shift + 1; n0 <= a.n_steps; n0 += RUN) {
    double z[RUN];
#pragma unroll
    for (int j = 0; j < RUN; ++j)
      if (n0 + j <= a.n_steps) z[j] = col[(n0 + j) * a.n_dof];
#pragma unroll
    for (int j = 0; j < RUN; ++j)
      if (n0 + j <= a.n_steps) {
        y = fma(a.sig, z[j], y);
        col[(n0 + j) * a.n_dof] = y;
      }
  }
}

__global__ void copy_kernel(const double* src, double* dst, int64_t n) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n;
       t += (int64_t)gridDim.x * blockDim.x)
    dst[t] = src[t];
}

hipError_t launch_shift(const ShiftArgs& a, hipStream_t st) {
  const int64_t total = (a.n_steps - a.n_shift + 1) * a.n_dof;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 16384));
  hipLaunchKernelGGL(shift_copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(shift_regrow_kernel, dim3((unsigned)((a.n_dof + 255) / 256)), dim3(256), 0,
                     st, a);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Gradient-informed (Metropolis-adjusted Langevin) path move
// ---------------------------------------------------------------------------
// y = x - tau g + sqrt(2 tau) z on slices 1..N (stream 5 of move t), y_0 = x_0.
__global__ void langevin_propose_kernel(LangevinArgs a) {
  const uint32_t t = (uint32_t)(*a.counter);
  const uint64_t total = (uint64_t)(a.n_steps + 1) * a.n_dof;
  const double amp = sqrt(2.0 * a.tau);
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t p = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; 2 * p < total; p += stride) {
    double z[2];
    stream_normal_pair(p, t, 5u, a.key0, a.key1, z[0], z[1]);
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const uint64_t e = 2 * p + j;
      if (e >= total) break;
      a.y[e] = e < (uint64_t)a.n_dof ? a.x[e] : a.x[e] - a.tau * a.grad[e] + amp * z[j];
    }
  }
}

// Per-block sums of |y - x + tau g|^2 and |x - y + tau g_y|^2 over slices 1..N.
__global__ void langevin_partial_kernel(LangevinArgs a) {
  __shared__ double red[32];
  const int64_t total = (a.n_steps + 1) * a.n_dof;
  double f2 = 0.0, b2 = 0.0;
  for (int64_t e = a.n_dof + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const double d = a.y[e] - a.x[e];
    const double f = d + a.tau * a.grad[e];
    const double b = a.tau * a.grad_y[e] - d;
    f2 = fma(f, f, f2);
    b2 = fma(b, b, b2);
  }
  f2 = block_sum(f2, red);
  b2 = block_sum(b2, red);
  if (threadIdx.x == 0) {
    a.partial[2 * blockIdx.x] = f2;
    a.partial[2 * blockIdx.x + 1] = b2;
  }
}

// One block: the log ratio, the uniform of move t (stream 6) and the decision.
__global__ void langevin_decide_kernel(LangevinArgs a) {
  __shared__ double red[32];
  double f2 = 0.0, b2 = 0.0;
  for (int k = threadIdx.x; k < a.blocks; k += blockDim.x) {
    f2 += a.partial[2 * k];
    b2 += a.partial[2 * k + 1];
  }
  f2 = block_sum(f2, red);
  b2 = block_sum(b2, red);
  if (threadIdx.x == 0) {
    const uint32_t t = (uint32_t)(*a.counter);
    const double la = (*a.action - *a.action_y) + (f2 - b2) / (4.0 * a.tau);
    const U4 w = philox(0u, 0u, t, 6u, a.key0, a.key1);
    const double u = uniform52(w.v[0], w.v[1]);
    const int acc = u < exp(la) ? 1 : 0;
    *a.flag = acc;
    if (a.accepted) *a.accepted = acc;
    if (a.log_alpha) *a.log_alpha = la;
  }
}

// On acceptance the proposal becomes the state; the move counter advances.
__global__ void langevin_commit_kernel(LangevinArgs a) {
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t0 == 0) {
    *a.counter += 1;
    if (*a.flag) *a.action = *a.action_y;
  }
  if (!*a.flag) return;
  const int64_t total = (a.n_steps + 1) * a.n_dof;
  for (int64_t e = t0; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    a.x[e] = a.y[e];
    a.grad[e] = a.grad_y[e];
  }
}

hipError_t launch_langevin_propose(const LangevinArgs& a, hipStream_t st) {
  const int64_t pairs = ((a.n_steps + 1) * a.n_dof + 1) / 2;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((pairs + 255) / 256, 16384));
  hipLaunchKernelGGL(langevin_propose_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_langevin_accept(const LangevinArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(langevin_partial_kernel, dim3(a.blocks), dim3(256), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(langevin_decide_kernel, dim3(1), dim3(256), 0, st, a);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t total = (a.n_steps + 1) * a.n_dof;
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 16384));
  hipLaunchKernelGGL(langevin_commit_kernel, dim3((unsigned)blocks), dim3(256), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_copy(const double* src, double* dst, int64_t n, hipStream_t st) {
  const int64_t blocks = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 16384));
  hipLaunchKernelGGL(copy_kernel, dim3((unsigned)blocks), dim3(256), 0, st, src, dst, n);
  return hipGetLastError();
}

}  // namespace pamd
