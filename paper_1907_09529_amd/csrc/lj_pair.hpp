// Lennard-Jones pair terms (Eq. 16) and neighbour-list construction in LDS.
#pragma once
#include "device.hpp"
#include "internal.hpp"

namespace pamd {

// ---------------------------------------------------------------------------
// Pair terms of the cut-and-force-shifted potential U(r) = u(r) - u(rc) - (r - rc) u'(rc),
// u = 4 eps [(sigma/r)^12 - (sigma/r)^6]:
//   fs = -U'(r)/r = 24 eps r^-2 [2 (s/r)^12 - (s/r)^6] + u'(rc)/r     (force on i: fs * d_ij)
//   U''(r)      = 24 eps r^-2 [26 (s/r)^12 - 7 (s/r)^6]
//   K_ij w = a w + b (d.w) d  with a = U'/r = -fs, b = (U'' - a)/r^2
// ---------------------------------------------------------------------------
template <bool F32>
struct PairMath;

template <>
struct PairMath<false> {
  // Force scalar fs for r^2 = r2 (caller guarantees r2 <= rc^2).
  static __device__ __forceinline__ void force(const LJConst& lj, double r2, double& fs,
                                               double& ir2, double& sr6) {
    const double ir = rsqrt_nr(r2);
    ir2 = ir * ir;
    const double sr2 = lj.sig2 * ir2;
    sr6 = sr2 * sr2 * sr2;
    fs = fma(lj.a24 * ir2 * sr6, fma(2.0, sr6, -1.0), lj.duc * ir);
  }
  static __device__ __forceinline__ void accum_force(const LJConst& lj, double dx, double dy,
                                                     double dz, double r2, double& fx,
                                                     double& fy, double& fz) {
    double fs, ir2, sr6;
    force(lj, r2, fs, ir2, sr6);
    fx = fma(fs, dx, fx);
    fy = fma(fs, dy, fy);
    fz = fma(fs, dz, fz);
  }
  static __device__ __forceinline__ void accum_hv(const LJConst& lj, double dx, double dy,
                                                  double dz, double r2, double wx, double wy,
                                                  double wz, double& qx, double& qy,
                                                  double& qz) {
    double fs, ir2, sr6;
    force(lj, r2, fs, ir2, sr6);
    const double a = -fs;
    const double upp = lj.a24 * ir2 * sr6 * fma(26.0, sr6, -7.0);
    const double b = (upp - a) * ir2;
    const double dw = fma(dx, wx, fma(dy, wy, dz * wz));
    const double t = b * dw;
    qx = fma(a, wx, fma(t, dx, qx));
    qy = fma(a, wy, fma(t, dy, qy));
    qz = fma(a, wz, fma(t, dz, qz));
  }
};

template <>
struct PairMath<true> {
  // Float32 pair products in the Hessian-vector pass: the pair functions
  // (r^-2, the r^-6 / r^-12 chain, U'/r, U'') stay in float64, since their
  // powers amplify float32 rounding about twelvefold, and the products of the
  // pair scalars with w and d (a w + b (d.w) d) are formed in float32 and
  // summed in float64.  The force pass stays float64: its products, rounded
  // to float32, alone move the gradient by ~1.7e-8 of its largest entry.
  static __device__ __forceinline__ void accum_force(const LJConst& lj, double dx, double dy,
                                                     double dz, double r2, double& fx,
                                                     double& fy, double& fz) {
    PairMath<false>::accum_force(lj, dx, dy, dz, r2, fx, fy, fz);
  }
  static __device__ __forceinline__ void accum_hv(const LJConst& lj, double dx, double dy,
                                                  double dz, double r2, double wx, double wy,
                                                  double wz, double& qx, double& qy,
                                                  double& qz) {
    double fs, ir2, sr6;
    PairMath<false>::force(lj, r2, fs, ir2, sr6);
    const double upp = lj.a24 * ir2 * sr6 * fma(26.0, sr6, -7.0);
    const float a = (float)(-fs);
    const float t = (float)((upp + fs) * ir2 * fma(dx, wx, fma(dy, wy, dz * wz)));
    qx += (double)fmaf(a, (float)wx, t * (float)dx);
    qy += (double)fmaf(a, (float)wy, t * (float)dy);
    qz += (double)fmaf(a, (float)wz, t * (float)dz);
  }
};

// Force on atom i (position xi) from its neighbour list (or from every atom
// when the list overflowed, cnt < 0).  X is the slice in LDS, AoS (3 per atom).
template <bool F32>
__device__ __forceinline__ void force_on(const LJConst& lj, const double* X, int n_atoms,
                                         const uint16_t* nbr, int cnt, int i, double xi,
                                         double yi, double zi, double& fx, double& fy,
                                         double& fz) {
  fx = fy = fz = 0.0;
  if (cnt >= 0) {
    for (int k = 0; k < cnt; ++k) {
      const int j = nbr[(size_t)k * n_atoms];
      const double dx = min_image(xi - X[3 * j + 0], lj.box, lj.inv_box);
      const double dy = min_image(yi - X[3 * j + 1], lj.box, lj.inv_box);
      const double dz = min_image(zi - X[3 * j + 2], lj.box, lj.inv_box);
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      if (r2 <= lj.rc2) PairMath<F32>::accum_force(lj, dx, dy, dz, r2, fx, fy, fz);
    }
  } else {
    for (int j = 0; j < n_atoms; ++j) {
      if (j == i) continue;
      const double dx = min_image(xi - X[3 * j + 0], lj.box, lj.inv_box);
      const double dy = min_image(yi - X[3 * j + 1], lj.box, lj.inv_box);
      const double dz = min_image(zi - X[3 * j + 2], lj.box, lj.inv_box);
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      if (r2 <= lj.rc2) PairMath<F32>::accum_force(lj, dx, dy, dz, r2, fx, fy, fz);
    }
  }
}

// (H(x) rho)_i from the neighbour list; R holds rho for every atom (AoS, LDS or global).
template <bool F32>
__device__ __forceinline__ void hv_on(const LJConst& lj, const double* X, const double* R,
                                      int n_atoms, const uint16_t* nbr, int cnt, int i,
                                      double xi, double yi, double zi, double rx, double ry,
                                      double rz, double& qx, double& qy, double& qz) {
  qx = qy = qz = 0.0;
  if (cnt >= 0) {
    for (int k = 0; k < cnt; ++k) {
      const int j = nbr[(size_t)k * n_atoms];
      const double dx = min_image(xi - X[3 * j + 0], lj.box, lj.inv_box);
      const double dy = min_image(yi - X[3 * j + 1], lj.box, lj.inv_box);
      const double dz = min_image(zi - X[3 * j + 2], lj.box, lj.inv_box);
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      if (r2 <= lj.rc2)
        PairMath<F32>::accum_hv(lj, dx, dy, dz, r2, rx - R[3 * j + 0], ry - R[3 * j + 1],
                                rz - R[3 * j + 2], qx, qy, qz);
    }
  } else {
    for (int j = 0; j < n_atoms; ++j) {
      if (j == i) continue;
      const double dx = min_image(xi - X[3 * j + 0], lj.box, lj.inv_box);
      const double dy = min_image(yi - X[3 * j + 1], lj.box, lj.inv_box);
      const double dz = min_image(zi - X[3 * j + 2], lj.box, lj.inv_box);
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      if (r2 <= lj.rc2)
        PairMath<F32>::accum_hv(lj, dx, dy, dz, r2, rx - R[3 * j + 0], ry - R[3 * j + 1],
                                rz - R[3 * j + 2], qx, qy, qz);
    }
  }
}

// ---------------------------------------------------------------------------
// Cell list of one slice in LDS: counting sort of atoms into nc^3 cells (edge
// L/nc), then each cell's members sorted by atom index so that list order -
// and hence every floating-point sum - is independent of thread timing.
// ---------------------------------------------------------------------------
struct CellLDS {
  int* start;   // ncell + 1
  int* fill;    // ncell
  int* atoms;   // n_atoms
  int* tmp;     // 16
};

__device__ __forceinline__ int cell_coord(double v, double box, double inv_box, int nc) {
  double w = v - box * floor(v * inv_box);  // wrap into [0, L)
  int c = (int)(w * inv_box * (double)nc);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

// Builds the cell list of the slice in X (all threads participate).
__device__ inline void build_cells(const LJConst& lj, const double* X, int n_atoms, int nc,
                                   CellLDS cl) {
  const int ncell = nc * nc * nc;
  for (int c = threadIdx.x; c < ncell; c += blockDim.x) cl.start[c] = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < n_atoms; i += blockDim.x) {
    const int cx = cell_coord(X[3 * i + 0], lj.box, lj.inv_box, nc);
    const int cy = cell_coord(X[3 * i + 1], lj.box, lj.inv_box, nc);
    const int cz = cell_coord(X[3 * i + 2], lj.box, lj.inv_box, nc);
    atomicAdd(&cl.start[(cz * nc + cy) * nc + cx], 1);
  }
  __syncthreads();
  block_exclusive_scan(cl.start, ncell, cl.tmp);
  for (int c = threadIdx.x; c < ncell; c += blockDim.x) cl.fill[c] = cl.start[c];
  __syncthreads();
  for (int i = threadIdx.x; i < n_atoms; i += blockDim.x) {
    const int cx = cell_coord(X[3 * i + 0], lj.box, lj.inv_box, nc);
    const int cy = cell_coord(X[3 * i + 1], lj.box, lj.inv_box, nc);
    const int cz = cell_coord(X[3 * i + 2], lj.box, lj.inv_box, nc);
    const int slot = atomicAdd(&cl.fill[(cz * nc + cy) * nc + cx], 1);
    cl.atoms[slot] = i;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
    const int lo = cl.start[c], hi = cl.start[c + 1];
    for (int a = lo + 1; a < hi; ++a) {  // insertion sort by atom index
      const int v = cl.atoms[a];
      int b = a - 1;
      while (b >= lo && cl.atoms[b] > v) {
        cl.atoms[b + 1] = cl.atoms[b];
        --b;
      }
      cl.atoms[b + 1] = v;
    }
  }
  __syncthreads();
}

// Neighbour list of atom i within radius^2 = rlist2 (minimum image).  Writes
// nbr[k * n_atoms] for k < count and returns count, or -1 when count would
// exceed kmax (the caller then scans all atoms).
__device__ inline int build_list(const LJConst& lj, const double* X, int n_atoms, int nc,
                                 int reach, const CellLDS& cl, double rlist2, int kmax,
                                 uint16_t* nbr, int i) {
  const double xi = X[3 * i + 0], yi = X[3 * i + 1], zi = X[3 * i + 2];
  int cnt = 0;
  bool over = false;
  auto visit = [&](int j) {
    const double dx = min_image(xi - X[3 * j + 0], lj.box, lj.inv_box);
    const double dy = min_image(yi - X[3 * j + 1], lj.box, lj.inv_box);
    const double dz = min_image(zi - X[3 * j + 2], lj.box, lj.inv_box);
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    if (r2 <= rlist2) {
      if (cnt < kmax)
        nbr[(size_t)cnt * n_atoms] = (uint16_t)j;
      else
        over = true;
      ++cnt;
    }
  };
  if (nc == 0) {
    for (int j = 0; j < n_atoms; ++j)
      if (j != i) visit(j);
  } else {
    const int cx = cell_coord(xi, lj.box, lj.inv_box, nc);
    const int cy = cell_coord(yi, lj.box, lj.inv_box, nc);
    const int cz = cell_coord(zi, lj.box, lj.inv_box, nc);
    for (int oz = -reach; oz <= reach; ++oz) {
      const int z = (cz + oz + nc) % nc;
      for (int oy = -reach; oy <= reach; ++oy) {
        const int y = (cy + oy + nc) % nc;
        for (int ox = -reach; ox <= reach; ++ox) {
          const int x = (cx + ox + nc) % nc;
          const int c = (z * nc + y) * nc + x;
          const int lo = cl.start[c], hi = cl.start[c + 1];
          for (int s = lo; s < hi; ++s) {
            const int j = cl.atoms[s];
            if (j != i) visit(j);
          }
        }
      }
    }
  }
  return over ? -1 : cnt;
}

}  // namespace pamd
