// Fused Lennard-Jones path action + adjoint gradient (gfx950).
//
// One workgroup owns a tile of consecutive time steps [n0, n1).  For each step
// n it holds slice x_n in LDS, evaluates F(x_n) from a neighbour list,
// forms r_n = Delta_n - (dt/gamma) F(x_n) and the per-step action
// s_n = |r_n|^2/(4 D dt) (Eq. 3), stores rho_n = w_n r_n for the whole slice,
// then applies the Hessian K-sum to rho_n and writes
//     g_n = c [rho_{n-1} - rho_n + (dt/gamma) H(x_n) rho_n],  c = 1/(2 D dt).
// rho_{n-1} is kept per atom in block-private memory; at the tile's first step
// it belongs to the previous tile, which writes c rho_{n0-1} to a boundary
// buffer that the finalize kernel adds (fixed order, no atomics).
//
// Positions in LDS are in box units (u = x / L), so that the minimum image of
// a displacement is du - rint(du) and the pair terms use constants scaled
// once on the host (BoxUnits).  Delta_n is taken from the unscaled positions
// in HBM.
//
// Neighbour lists (radius r_c + skin) are built at the tile start from a cell
// list in LDS and reused while no atom has moved more than skin/2 from where
// the list was built (then every pair with r <= r_c at the current slice is
// in the list); otherwise the list is rebuilt on the spot.  The cutoff test
// itself is exact at every slice.  At every build the atoms are re-sorted in
// cell order inside LDS, so that threads of a wave handle neighbouring atoms
// and read largely the same neighbour positions (LDS broadcast, few bank
// conflicts).  Pass 1 records the partners it finds within r_c (the slice's
// exact list, about 60% of the neighbour list at the default skin), and
// pass 2 visits only those.
//
// Two list kinds:
//   full  every atom lists all its partners; each pair is evaluated twice and
//         every sum has a fixed order (bitwise repeatable);
//   half  each pair is listed once (half-space rule on the build-time
//         displacement); the partner's share is added with LDS float64 atomics
//         (half the pair arithmetic; sums are order-dependent at rounding level).
#include <type_traits>

#include "device.hpp"
#include "internal.hpp"

namespace pamd {

// LDS-typed pointers: 32-bit addressing for every shared-memory access.
typedef __attribute__((address_space(3))) double lds_f64;
typedef __attribute__((address_space(3))) int lds_i32;
typedef __attribute__((address_space(3))) uint16_t lds_u16;
typedef __attribute__((address_space(3))) int16_t lds_i16;
typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) f64x2 lds_f64x2;
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) f32x4 lds_f32x4;

// 16-byte LDS load (ds_read_b128) of two doubles at a 16-byte aligned address.
__device__ __forceinline__ f64x2 lds_ld2(const lds_f64* p) { return *(const lds_f64x2*)p; }

constexpr int HALF_SLOTS = 2;  // atoms per thread supported by the half-list kernel
constexpr int EX_PAD = 32;     // exact-list entries per atom beyond kmax (see TileScratch)

// Shared-memory layout of one tile.  With rho in LDS every slot holds
// XS_R = 6 doubles, its position u (0..2) and rho (3..5), read as three
// 16-byte loads, and there are two slot arrays when they fit: slice n + 1 is
// loaded into one while pass 2 of slice n reads the other; with one array the
// next slice is loaded after pass 2.  (16-byte LDS loads move about 1.6x the
// bytes per clock of 8-byte ones at scattered addresses on gfx950.)
// Otherwise a slot holds 3 doubles (positions only; rho lives in global
// scratch) and there is one array.
constexpr int XS_R = 6;
struct TileLDS {
  lds_f64* X;     // stride XS: slice x_n / L, sorted slots (the array in use)
  lds_f64* X2;    // the other slot array (== X when there is one)
  lds_f64* ACC;   // 3 * n_atoms, partner-share accumulator (half lists)
  lds_f64* red;   // 32 doubles
  lds_i32* tmp;   // 16
  lds_i32* flag;  // 2: slice m needs a list rebuild (flag[m & 1] != 0)
  lds_u16* perm;  // n_atoms: slot -> original atom index
  lds_i16* ecnt;  // 2 n_atoms: exact-list lengths this slice (-1: not recorded)
  // Pass 1 and the list build never run at the same time, so their scratch
  // shares one region:
  lds_u16* stage; // pass 1: 16 per thread, ring of exact-list entries not yet stored
  lds_i32* start; // build: ncell + 1, first slot of each cell
  lds_i32* fill;  // build: ncell
  lds_u16* perm2; // build: n_atoms, scratch for re-sorting
  lds_u16* atoms; // build: n_atoms, slots in cell order
  // LDS position of slot t.  With full lists the even slots come first and
  // the odd ones after them (H = number of even slots): each lane reads
  // partners of one slot parity, which then sit at consecutive positions and
  // spread over all LDS banks.  Half lists keep slot order (H = 0).  List
  // entries hold positions.
  int H;
  __device__ __forceinline__ int pos(int t) const { return H ? (t >> 1) + (t & 1) * H : t; }
};

// Shared-memory bytes of one tile (see carve_lds).
constexpr uint32_t STAGE = 16;  // exact-list staging entries per thread

__host__ __device__ inline uint32_t lds_shared_region(int n_atoms, int ncell, int block) {
  const uint32_t ring = 2u * STAGE * (uint32_t)block;
  const uint32_t build = 4u * (2u * (uint32_t)ncell + 1u) + 4u * (uint32_t)n_atoms;
  return ring > build ? ring : build;
}

__device__ inline TileLDS carve_lds(char* base_generic, int n_atoms, int ncell, bool r_in_lds,
                                    bool half, bool two) {
  typedef __attribute__((address_space(3))) char lds_char;
  lds_char* base = (lds_char*)base_generic;
  TileLDS t;
  uint32_t off = 0;
  auto f64 = [&](uint32_t n) {
    lds_f64* p = (lds_f64*)(base + off);
    off += 8u * n;
    return p;
  };
  t.X = f64((uint32_t)(r_in_lds ? XS_R : 3) * n_atoms);
  t.X2 = r_in_lds && two ? f64((uint32_t)XS_R * n_atoms) : t.X;
  t.ACC = half ? f64(3u * n_atoms) : nullptr;
  t.red = f64(32);
  t.tmp = (lds_i32*)(base + off);
  t.flag = t.tmp + 16;
  off += 4u * 18u;
  t.perm = (lds_u16*)(base + off);
  off += 2u * n_atoms;
  t.ecnt = (lds_i16*)(base + off);
  off += 4u * n_atoms;
  off = (off + 15u) & ~15u;
  t.stage = (lds_u16*)(base + off);
  t.start = (lds_i32*)(base + off);
  t.fill = t.start + ncell + 1;
  t.perm2 = (lds_u16*)(t.fill + ncell);
  t.atoms = t.perm2 + n_atoms;
  t.H = half ? 0 : (n_atoms + 1) / 2;
  return t;
}

size_t fused_lds_bytes(int n_atoms, int nc, bool r_in_lds, bool half, int block, bool two) {
  const size_t ncell = (size_t)nc * nc * nc;
  const size_t slots = r_in_lds ? (two ? 2 * XS_R : XS_R) : 3;
  size_t b = sizeof(double) * (size_t)n_atoms * (slots + (half ? 3 : 0));
  b += sizeof(double) * 32 + sizeof(int) * 18 + 6 * (size_t)n_atoms + 16;
  b += lds_shared_region(n_atoms, (int)ncell, block);
  return b;
}

size_t fused_lds_stage_bytes(int block) { return 2 * STAGE * (size_t)block; }

int fused_half_slots() { return HALF_SLOTS; }

// Per-block global scratch for one tile: lists and per-atom state that only
// the owning thread touches.
struct TileScratch {
  uint16_t* nbr;   // (kmax + EX_PAD) * n_atoms: R rows (R = n_atoms for half lists, 2 n_atoms
                   // for full ones) in chunks of 8 entries, entry k of row r at [(k/8) R + r] * 8 + k%8
  uint16_t* ex;    // 2 n_atoms rows in chunks of 4: the partners within r_c at the current slice
  int* cnt;        // R: entries per row
  double* xref;    // 3 * n_atoms: positions u (sorted slots) at the last list build
  double* rprev;   // 3 * n_atoms: rho_{n-1}, by original atom index
  double* rglob;   // 3 * n_atoms: rho_n (sorted slots) when not in LDS; sort scratch
};

// Minimum image in box units.
__device__ __forceinline__ double wrap_u(double du) { return du - __builtin_rint(du); }

// Half-space rule: the pair is stored by the atom whose displacement to its
// partner points "up" (z, then y, then x); exact ties fall back to slot order.
__device__ __forceinline__ bool upper_half(double dx, double dy, double dz, int s, int t) {
  if (dz != 0.0) return dz > 0.0;
  if (dy != 0.0) return dy > 0.0;
  if (dx != 0.0) return dx > 0.0;
  return s < t;
}

// Cell of a box-unit coordinate: floor(frac(u) nc), clamped.
__device__ __forceinline__ int cell_of(double u, int nc) {
  const double w = u - floor(u);
  const int c = (int)(w * (double)nc);
  return c < 0 ? 0 : (c >= nc ? nc - 1 : c);
}

template <int XS>
__device__ __forceinline__ int cell_of_slot(const lds_f64* X, int s, int nc) {
  return (cell_of(X[XS * s + 2], nc) * nc + cell_of(X[XS * s + 1], nc)) * nc +
         cell_of(X[XS * s + 0], nc);
}

// Counting sort of the slots into nc^3 cells (z-major); members of a cell
// keep their slot order, so the result does not depend on thread timing.
template <int XS>
__device__ void sort_cells(int N, int nc, const TileLDS& L) {
  auto cell = [&](int s) { return cell_of_slot<XS>(L.X, L.pos(s), nc); };
  const int ncell = nc * nc * nc;
  const int B = blockDim.x;
  for (int c = threadIdx.x; c < ncell; c += B) L.start[c] = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < N; s += B)
    atomicAdd((int*)&L.start[cell(s)], 1);
  __syncthreads();
  block_exclusive_scan(L.start, ncell, L.tmp);
  for (int c = threadIdx.x; c < ncell; c += B) L.fill[c] = L.start[c];
  __syncthreads();
  for (int s = threadIdx.x; s < N; s += B)
    L.atoms[atomicAdd((int*)&L.fill[cell(s)], 1)] = (uint16_t)s;
  __syncthreads();
  for (int c = threadIdx.x; c < ncell; c += B) {
    const int lo = L.start[c], hi = L.start[c + 1];
    for (int a = lo + 1; a < hi; ++a) {  // insertion sort by slot
      const int v = L.atoms[a];
      int b = a - 1;
      while (b >= lo && L.atoms[b] > v) {
        L.atoms[b + 1] = L.atoms[b];
        --b;
      }
      L.atoms[b + 1] = (uint16_t)v;
    }
  }
  __syncthreads();
}

// Evens out the two rows of an atom (lanes l and l + 32 of a wave, rows
// `mine` and `other` of a list in chunks of CH entries, entry k of row r at
// [(k / CH) rows + r] CH + k % CH): the longer row moves the surplus from its
// tail to the other row's tail, and both pad their new last chunks with
// `pad`.  A wave runs as long as its longest row, so this shortens the wave
// by up to half the difference.  Rows of length -1 (overflow) stay as they
// are.  Every lane of the wave must call; `live` lanes take part.  (Used for
// the neighbour lists at each build; evening out the exact lists every slice
// costs more in pass 1 than it saves in pass 2.)
template <int CH>
__device__ __forceinline__ int balance_rows(uint16_t* list, int rows, int mine, int other_row,
                                            int cnt, bool live, uint16_t pad) {
  const int other = __shfl_xor(cnt, 32, WAVE);
  if (!live || cnt < 0 || other < 0) return cnt;
  const int k = (cnt - other) / 2;  // > 0: give k entries; < 0: receive -k
  auto at = [&](int r, int e) { return ((size_t)(e / CH) * rows + r) * CH + e % CH; };
  if (k > 0) {
    for (int i = 0; i < k; ++i) list[at(other_row, other + i)] = list[at(mine, cnt - k + i)];
    // the moved entries must not be read again from this row's last chunk
    for (int e = cnt - k; e % CH; ++e) list[at(mine, e)] = pad;
    return cnt - k;
  }
  if (k < 0) {
    const int n = cnt - k;
    for (int e = n; e % CH; ++e) list[at(mine, e)] = pad;
    return n;
  }
  return cnt;
}

// Entries per list row: one row per atom for half lists; for full lists two
// rows per atom (parts 0 and 1: partners of even and odd slot index), each
// with room for half of kmax plus a spare chunk.
template <bool HALF>
__device__ __forceinline__ int row_capacity(int kmax) {
  return HALF ? kmax : ((kmax / 2 + 15) & ~7);
}

// (Re)builds the neighbour lists of the slice in L.X (box units).  With cells,
// atoms are first re-sorted into cell order (slots and perm are rewritten).
// With rho in LDS (XS == XS_R) a pair is listed when its distance is at most
// rcm + d_i + d_j, with the per-atom reach d taken from dsrc (by original atom
// index) or, when dsrc is null, dconst for every atom; the reaches are
// parked in slot element 3 for the scan (free until pass 1 stores rho).
// Otherwise the radius^2 is rl2.  scan_radius() of the caller keeps both forms
// conservative (a relative 1e-12 margin).
//
// With rho in LDS and full lists the scan tests candidates in float32: a
// float copy of each slot (position wrapped into [0, 1) box units, reach)
// goes to the slot's last 16 bytes, free until pass 1 stores rho, and a pair
// is listed when the float distance is within the float limit plus
// SCAN_MARGIN.  The float rounding of the wrapped positions, of r^2 and of the
// limit is below 1e-6 box units, so every pair the float64 test would list is
// listed (a few more may be); the cutoff itself is tested in float64 in the
// passes.
constexpr float SCAN_MARGIN = 1e-5f;  // box units

template <int XS, bool HALF>
__device__ void rebuild(const PathArgs& a, const TileLDS& L, const TileScratch& ts, double rl2,
                        double rcm, const double* dsrc, double dconst) {
  constexpr int PARTS = HALF ? 1 : 2;
  constexpr int SPAN = WAVE / PARTS;  // slots per wave
  constexpr bool F32S = XS == XS_R && !HALF;
  auto c32 = [&](int p) { return (lds_f32x4*)(L.X + XS * p + 4); };  // elements 4, 5 of slot p
  const int N = a.n_atoms;
  const int B = blockDim.x;
  if (a.nc > 0) {
    sort_cells<XS>(N, a.nc, L);
    // gather into cell order through scratch: the rho half of each slot
    // (dead at this point) when rho is in LDS, else global scratch
    for (int s = threadIdx.x; s < N; s += B) {
      const int old = L.atoms[s];
      const int ps = L.pos(s), po = L.pos(old);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double v = L.X[XS * po + c];
        if constexpr (XS == XS_R)
          L.X[XS * ps + 3 + c] = v;
        else
          ts.rglob[3 * ps + c] = v;
      }
      L.perm2[s] = L.perm[old];
    }
    __syncthreads();
    for (int s = threadIdx.x; s < N; s += B) {
      const int ps = L.pos(s);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        if constexpr (XS == XS_R)
          L.X[XS * ps + c] = L.X[XS * ps + 3 + c];
        else
          L.X[XS * ps + c] = ts.rglob[3 * ps + c];
      }
      L.perm[s] = L.perm2[s];
    }
    __syncthreads();
  }
  if constexpr (XS == XS_R) {
    for (int s = threadIdx.x; s < N; s += B) {
      const int p = L.pos(s);
      const double d = dsrc ? dsrc[L.perm[s]] : dconst;
      L.X[XS * p + 3] = d;
      if constexpr (F32S) {
        const double x = L.X[XS * p], y = L.X[XS * p + 1], z = L.X[XS * p + 2];
        *c32(p) = f32x4{(float)(x - floor(x)), (float)(y - floor(y)), (float)(z - floor(z)),
                        (float)d};
      }
    }
    __syncthreads();  // every reach parked
  }
  const int nc = a.nc, reach = a.reach;
  const int lane = threadIdx.x & (WAVE - 1);
  const int part = PARTS == 1 ? 0 : lane / SPAN;
  const int R = PARTS * N;  // list rows
  // entry k of row r lives at nbr[((k >> 3) * R + r) * 8 + (k & 7)]; woff
  // tracks that offset as entries are appended (woff & 7 == k & 7)
  const uint32_t step8 = 8u * R - 7u;
  const uint32_t cap = (uint32_t)row_capacity<HALF>(a.kmax) * (uint32_t)R;  // offset span of a row
  const int wv = threadIdx.x / WAVE, nwv = B / WAVE;
  // Each wave takes SPAN consecutive slots and scans the union of their cell
  // stencils: the candidate pair index is wave-uniform (LDS broadcast reads,
  // no divergent loop bounds); part p of a slot tests the candidates of slot
  // parity p against its atom, so the two rows of an atom split its partners
  // evenly and the wave's scan is half as long as one lane per atom would
  // make it.
  for (int base = wv * SPAN; base < N; base += nwv * SPAN) {
    const int s = base + (lane % SPAN);
    const bool live = s < N;
    const int sc = live ? s : base;
    const int me = L.pos(sc);
    const double xs = L.X[XS * me], ys = L.X[XS * me + 1], zs = L.X[XS * me + 2];
    const double rme = XS == XS_R ? rcm + L.X[XS * me + 3] : 0.0;  // rc + own reach
    const float xs32 = (float)(xs - floor(xs)), ys32 = (float)(ys - floor(ys)),
                zs32 = (float)(zs - floor(zs)), rme32 = (float)rme + SCAN_MARGIN;
    uint16_t* nb = ts.nbr;
    const uint32_t wbase = 8u * (uint32_t)(PARTS * sc + part);
    const uint32_t wcap = wbase + cap;
    // a lane past the last slot never appends
    uint32_t woff = live ? wbase : wcap;
    bool over = false;
    auto append = [&](int t) {
      const bool room = woff < wcap;
      if (room) nb[woff] = (uint16_t)t;
      over |= !room;
      woff += room ? ((woff & 7u) == 7u ? step8 : 1u) : 0u;
    };
    // Candidates are the slots [t0, t1) (wave-uniform).  Each lane tests
    // those of its parity, which sit at consecutive LDS positions [p0,
    // p0 + np), in groups of up to 32, collecting the accepted ones in a bit
    // mask, then appends their positions in a short loop over the set bits,
    // so the test loop itself has no stores and no branches.
    auto scan = [&](int t0, int t1) {
      t0 = __builtin_amdgcn_readfirstlane(t0);
      t1 = __builtin_amdgcn_readfirstlane(t1);
      int p0, np, nmax;
      if constexpr (PARTS == 1) {
        p0 = t0;
        np = nmax = t1 - t0;
      } else {
        const int e0 = (t0 + 1) >> 1, e1 = (t1 + 1) >> 1;  // even slots 2k: k in [e0, e1)
        const int o0 = t0 >> 1, o1 = t1 >> 1;              // odd slots 2k + 1: k in [o0, o1)
        p0 = part ? L.H + o0 : e0;
        np = part ? o1 - o0 : e1 - e0;
        nmax = max(e1 - e0, o1 - o0);
      }
      const int plast = max(p0 + np - 1, 0);  // in-range position for padded lanes
      // every test is computed in full (no lane branches); slot positions
      // are 16-bit, as in the lists, which the mask tells the compiler so
      // that the address takes a 24-bit multiply
      auto cand = [&](int p) { return *c32((int)((uint32_t)min(p, plast) & 0xffffu)); };
      for (int g = 0; g < nmax; g += 32) {
        uint32_t bits = 0;
        if constexpr (F32S) {
          for (int j = 0; j < 32; j += 2) {
            if (g + j >= nmax) break;
            f32x4 c[2];
#pragma unroll
            for (int u = 0; u < 2; ++u) c[u] = cand(p0 + g + j + u);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              const int k = g + j + u;
              float dx = xs32 - c[u].x, dy = ys32 - c[u].y, dz = zs32 - c[u].z;
              dx -= __builtin_rintf(dx);
              dy -= __builtin_rintf(dy);
              dz -= __builtin_rintf(dz);
              const float r2 = fmaf(dx, dx, fmaf(dy, dy, dz * dz));
              const float lim = rme32 + c[u].w;
              const bool pass = (k < np) & (p0 + k != me) & (r2 <= lim * lim);
              bits |= pass ? (1u << (j + u)) : 0u;
            }
          }
        } else {
        for (int j = 0; j < 32; j += 4) {
          if (g + j >= nmax) break;
          double px[4], py[4], pz[4], pd[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int p = (int)((uint32_t)min(p0 + g + j + u, plast) & 0xffffu);
            if constexpr (XS == XS_R) {
              const f64x2 xy = lds_ld2(L.X + XS * p), zd = lds_ld2(L.X + XS * p + 2);
              px[u] = xy.x;
              py[u] = xy.y;
              pz[u] = zd.x;
              pd[u] = zd.y;
            } else {
              px[u] = L.X[XS * p + 0];
              py[u] = L.X[XS * p + 1];
              pz[u] = L.X[XS * p + 2];
            }
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int k = g + j + u;
            const double dx = wrap_u(xs - px[u]);
            const double dy = wrap_u(ys - py[u]);
            const double dz = wrap_u(zs - pz[u]);
            const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
            double lim2 = rl2;
            if constexpr (XS == XS_R) {
              const double lim = rme + pd[u];
              lim2 = lim * lim;
            }
            const bool pass = (k < np) & (p0 + k != me) & (r2 <= lim2) &
                              (!HALF || upper_half(dx, dy, dz, s, p0 + k));
            bits |= pass ? (1u << (j + u)) : 0u;
          }
        }
        }
        if (!live) bits = 0;
        while (bits) {
          const int j = __builtin_ctz(bits);
          bits &= bits - 1u;
          append(p0 + g + j);
        }
      }
    };
    if (nc == 0) {
      scan(0, N);
    } else {
      const int cx = cell_of(xs, nc), cy = cell_of(ys, nc), cz = cell_of(zs, nc);
      // slots are in z-major cell order, so the wave's z range is contiguous;
      // y (x) ranges are exact only when the wave lies in one z plane (one row)
      const int zlo = wave_min_int(live ? cz : nc), zhi = wave_max_int(live ? cz : -1);
      int ylo = 0, yhi = nc - 1, xlo = 0, xhi = nc - 1;
      if (zlo == zhi) {
        ylo = wave_min_int(live ? cy : nc);
        yhi = wave_max_int(live ? cy : -1);
        if (ylo == yhi) {
          xlo = wave_min_int(live ? cx : nc);
          xhi = wave_max_int(live ? cx : -1);
        }
      }
      // stencil extent per axis (start, count), wrapped periodically
      auto extent = [&](int l, int h, int& st, int& n) {
        n = h - l + 1 + 2 * reach;
        if (n >= nc) {
          st = 0;
          n = nc;
        } else {
          st = l - reach;
          st += st < 0 ? nc : 0;
        }
      };
      int zs0, zn, ys0, yn, xs0, xn;
      extent(zlo, zhi, zs0, zn);
      extent(ylo, yhi, ys0, yn);
      extent(xlo, xhi, xs0, xn);
      // cells lo .. lo + n - 1 (mod m) of a run of m consecutive runs of
      // `unit` cells starting at cell `base` are one or two contiguous slot
      // ranges
      auto scan_cells = [&](int base, int unit, int lo, int n, int m) {
        const int hi = lo + n;
        if (hi <= m) {
          scan(L.start[base + lo * unit], L.start[base + hi * unit]);
        } else {
          scan(L.start[base + lo * unit], L.start[base + m * unit]);
          scan(L.start[base], L.start[base + (hi - m) * unit]);
        }
      };
      const int plane = nc * nc;
      if (xn == nc && yn == nc) {
        scan_cells(0, plane, zs0, zn, nc);  // whole planes
      } else {
        for (int iz = 0; iz < zn; ++iz) {
          int z = zs0 + iz;
          z -= z >= nc ? nc : 0;
          if (xn == nc) {
            scan_cells(z * plane, nc, ys0, yn, nc);  // whole rows of plane z
          } else {
            for (int iy = 0; iy < yn; ++iy) {
              int y = ys0 + iy;
              y -= y >= nc ? nc : 0;
              scan_cells((z * nc + y) * nc, 1, xs0, xn, nc);
            }
          }
        }
      }
    }
    int cnt = 0;
    if (live) {
      // pad the last chunk with the slot's own position (read as invalid)
      for (uint32_t o = woff; (o & 7u) != 0u; ++o) nb[o] = (uint16_t)me;
      const uint32_t rel = woff - wbase;
      cnt = over ? -1 : (int)((rel & ~7u) / (uint32_t)R + (rel & 7u));
    }
    if constexpr (PARTS == 2)
      cnt = balance_rows<8>(nb, R, 2 * sc + part, 2 * sc + 1 - part, cnt, live, (uint16_t)me);
    if (live) {
      ts.cnt[PARTS * s + part] = cnt;
      if (part == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) ts.xref[3 * s + c] = L.X[XS * me + c];
      }
    }
  }
}

// Build-time half-space membership of pair (s, t) for the overflow scan.
__device__ __forceinline__ bool ref_upper(const double* xref, int s, int t) {
  return upper_half(wrap_u(xref[3 * s] - xref[3 * t]), wrap_u(xref[3 * s + 1] - xref[3 * t + 1]),
                    wrap_u(xref[3 * s + 2] - xref[3 * t + 2]), s, t);
}

// List chunks: CH uint16 entries read with one load (neighbour lists: 8,
// exact lists: 4, which halves the padding of their shorter rows).
template <int CH>
struct ChunkOf;
template <>
struct ChunkOf<8> {
  typedef uint4 T;
  static __device__ __forceinline__ T zero() { return make_uint4(0u, 0u, 0u, 0u); }
  static __device__ __forceinline__ int entry(const T& c, int e) {
    const uint32_t w = e < 2 ? c.x : e < 4 ? c.y : e < 6 ? c.z : c.w;
    return (int)((w >> (16 * (e & 1))) & 0xffffu);
  }
};
template <>
struct ChunkOf<4> {
  typedef uint2 T;
  static __device__ __forceinline__ T zero() { return make_uint2(0u, 0u); }
  static __device__ __forceinline__ int entry(const T& c, int e) {
    const uint32_t w = e < 2 ? c.x : c.y;
    return (int)((w >> (16 * (e & 1))) & 0xffffu);
  }
};
constexpr int EX_CH = 4;  // entries per exact-list chunk

// Chunks of a list fetched ahead of use: the chunk loads come from HBM (the
// lists of all workgroups do not fit in L2), so several are kept in flight.
#ifndef PAMD_LIST_PREFETCH
#define PAMD_LIST_PREFETCH 2
#endif
constexpr int LIST_PREFETCH = PAMD_LIST_PREFETCH;

// Visits chunks first, first + STEP, ... of row `row` of a list in chunks of
// CH entries (chunk c at list[(c * rows + row) * CH]) with LIST_PREFETCH
// chunk loads in flight, calling after_chunk() after each chunk.  The row's
// last chunk is padded with slot indices; entries past cnt are passed with
// valid = false.
template <int CH, int STEP, typename Pair, typename After>
__device__ __forceinline__ void for_each_listed(const uint16_t* list, int rows, int row, int cnt,
                                                int first, Pair&& pair, After&& after_chunk) {
  typedef ChunkOf<CH> C;
  typedef typename C::T T;
  const T* nb = reinterpret_cast<const T*>(list) + row;
  const int nch = (cnt + CH - 1) / CH;
  T q[LIST_PREFETCH];
#pragma unroll
  for (int i = 0; i < LIST_PREFETCH; ++i) {
    const int c = first + i * STEP;
    q[i] = c < nch ? nb[(size_t)c * rows] : C::zero();
  }
  for (int ch = first; ch < nch; ch += STEP) {
    const T cur = q[0];
#pragma unroll
    for (int i = 0; i + 1 < LIST_PREFETCH; ++i) q[i] = q[i + 1];
    const int ahead = ch + LIST_PREFETCH * STEP;
    q[LIST_PREFETCH - 1] = ahead < nch ? nb[(size_t)ahead * rows] : cur;
    const int left = cnt - ch * CH;  // valid entries from this chunk on
#pragma unroll
    for (int e = 0; e < CH; ++e) pair(C::entry(cur, e), e < left);
    after_chunk();
  }
}

// Scan of all atoms (the list did not fit, or the path keeps no lists):
// atoms first, first + STEP, ... of the slot's half (half lists) or of all
// other atoms (full lists).
template <bool HALF, int STEP, typename Pair>
__device__ __forceinline__ void for_each_atom(const PathArgs& a, const TileLDS& L,
                                              const TileScratch& ts, int s, int first,
                                              Pair&& pair) {
  for (int t = first; t < a.n_atoms; t += STEP) {
    if (t == s) continue;
    if (HALF && !ref_upper(ts.xref, s, t)) continue;
    pair(L.pos(t), true);
  }
}

// Pass 1 for slot s, part `part` of STEP: the force on s from list row
// STEP s + part (the caller adds the STEP partial forces).
// The partners found within r_c are recorded, in list order, as exact-list
// row `er` of `erows` (ts.ex, padded with the slot itself to a whole chunk;
// length in L.ecnt[er]) for pass 2; after an overflow scan no exact list is
// recorded (-1).  With half lists the partners' shares are added into ACC.
// REC = false computes the force alone (no exact list).
template <int XS, bool F32, bool HALF, int STEP, bool REC = true>
__device__ __forceinline__ void pass1_part(const PathArgs& a, const TileLDS& L,
                                           const TileScratch& ts, int s, int part, int er,
                                           int erows, double& fx, double& fy, double& fz) {
  const BoxUnits& k = a.bu;
  const int N = a.n_atoms;
  const int ps = L.pos(s);
  const double xs = L.X[XS * ps], ys = L.X[XS * ps + 1], zs = L.X[XS * ps + 2];
  fx = fy = fz = 0.0;
  // accepted partners go to a 16-entry ring in LDS (a rejected entry's write
  // lands on the next free position and is overwritten); whole chunks of 8
  // are stored to the exact list with one 16-byte store
  lds_u16* ring = L.stage + STAGE * threadIdx.x;
  uint2* exr = reinterpret_cast<uint2*>(ts.ex) + er;
  uint32_t acc = 0, done = 0;  // entries accepted / stored
  auto body = [&](int t, bool valid, auto record) {
    double ux, uy;  // partner position
    if constexpr (XS == XS_R) {
      const f64x2 uxy = lds_ld2(L.X + XS * t);
      ux = uxy.x;
      uy = uxy.y;
    } else {
      ux = L.X[XS * t + 0];
      uy = L.X[XS * t + 1];
    }
    const double dx = wrap_u(xs - ux);
    const double dy = wrap_u(ys - uy);
    const double dz = wrap_u(zs - L.X[XS * t + 2]);
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const bool ok = valid && r2 <= k.rc2;
    if constexpr (decltype(record)::value) {
      ring[acc & (STAGE - 1)] = (uint16_t)t;
      acc += ok ? 1u : 0u;
    }
    // a rejected pair gets iru = 0, which zeroes every term below
    double px = 0.0, py = 0.0, pz = 0.0;
    double iru = rsqrt_nr(r2);
    iru = ok ? iru : 0.0;
    const double ir2 = iru * iru;
    const double ir6 = ir2 * ir2 * ir2;
    const double fsl = fma(ir2 * ir6, fma(k.f12, ir6, -k.f6), k.duc * iru);
    {  // the force pass is float64 in both precisions
      fx = fma(fsl, dx, fx);
      fy = fma(fsl, dy, fy);
      fz = fma(fsl, dz, fz);
      if constexpr (HALF) {
        px = fsl * dx;
        py = fsl * dy;
        pz = fsl * dz;
      }
    }
    if constexpr (HALF) {
      if (ok) {
        unsafeAtomicAdd((double*)&L.ACC[3 * t + 0], -px);
        unsafeAtomicAdd((double*)&L.ACC[3 * t + 1], -py);
        unsafeAtomicAdd((double*)&L.ACC[3 * t + 2], -pz);
      }
    }
  };
  // Stores the ring's oldest 4-entry chunk when it is complete (at most 11
  // entries are pending after a list chunk); otherwise the same store goes
  // to the row's last (spare) chunk, never read, which keeps the loop free
  // of branches.
  const uint32_t spare = (uint32_t)(a.kmax + EX_PAD) / (EX_CH * STEP) - 1u;  // erows = STEP N
  auto flush = [&](bool full) {
    const uint32_t c = full ? (done >> 2) : spare;
    exr[(size_t)c * erows] = *(const uint2*)(ring + (done & (STAGE - 1)));
    done += full ? 4u : 0u;
  };
  const int cnt = ts.cnt[STEP * s + part];
  if (cnt >= 0) {
    if constexpr (REC) {
      for_each_listed<8, 1>(
          ts.nbr, STEP * N, STEP * s + part, cnt, 0,
          [&](int t, bool valid) { body(t, valid, std::true_type{}); },
          [&]() {
            flush(acc - done >= 4u);
            flush(acc - done >= 4u);
          });
      if (acc > done) {  // pad the last chunk with the slot itself
        for (uint32_t k = acc; k & 3u; ++k) ring[k & (STAGE - 1)] = (uint16_t)ps;
        flush(true);
      }
      L.ecnt[er] = (int16_t)acc;
    } else {
      for_each_listed<8, 1>(
          ts.nbr, STEP * N, STEP * s + part, cnt, 0,
          [&](int t, bool valid) { body(t, valid, std::false_type{}); }, [&]() {});
    }
  } else {
    for_each_atom<HALF, STEP>(a, L, ts, s, part,
                              [&](int t, bool valid) { body(t, valid, std::false_type{}); });
    if constexpr (REC) L.ecnt[er] = -1;
  }
}

// Pass 2 for slot s, part `part` of STEP: q_s = sum_t K_st (rho_s - rho_t),
// physical units, from box-unit geometry (see BoxUnits), over exact-list row
// `er` of `erows` recorded by the same part in pass 1 (no cutoff test: every
// entry is within r_c at this slice), or over the part's share of an
// overflow scan with the cutoff test.  R holds rho with stride RS.
template <int XS, int RS, bool F32, bool HALF, int STEP, typename RPtr>
__device__ __forceinline__ void pass2_part(const PathArgs& a, const TileLDS& L, RPtr R,
                                           const TileScratch& ts, int s, int part, int er,
                                           int erows, double& qx, double& qy, double& qz) {
  const BoxUnits& k = a.bu;
  const int ps = L.pos(s);
  const double xs = L.X[XS * ps], ys = L.X[XS * ps + 1], zs = L.X[XS * ps + 2];
  const double rx = R[RS * ps], ry = R[RS * ps + 1], rz = R[RS * ps + 2];
  qx = qy = qz = 0.0;
  auto body = [&](int t, bool valid, auto check) {
    double px, py, pz, qtx, qty, qtz;  // partner position and rho
    if constexpr (XS == XS_R && RS == XS_R) {
      // one slot: u (0..2) and rho (3..5) as three 16-byte loads
      const f64x2 a0 = lds_ld2(L.X + XS * t), a1 = lds_ld2(L.X + XS * t + 2),
                  a2 = lds_ld2(L.X + XS * t + 4);
      px = a0.x;
      py = a0.y;
      pz = a1.x;
      qtx = a1.y;
      qty = a2.x;
      qtz = a2.y;
    } else {
      px = L.X[XS * t + 0];
      py = L.X[XS * t + 1];
      pz = L.X[XS * t + 2];
      qtx = R[RS * t + 0];
      qty = R[RS * t + 1];
      qtz = R[RS * t + 2];
    }
    const double dx = wrap_u(xs - px);
    const double dy = wrap_u(ys - py);
    const double dz = wrap_u(zs - pz);
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    bool ok = valid;
    if constexpr (decltype(check)::value) ok = ok && r2 <= k.rc2;
    const double wx = rx - qtx, wy = ry - qty, wz = rz - qtz;
    if constexpr (F32) {
      // pair functions in float64 (as below), the products with w and d in
      // float32, the sums in float64.  Padding entries are masked: their
      // clamped r^2 gives pair scalars that overflow float32, and inf * 0 is
      // not 0.
      const double iru = ok ? rsqrt_nr(fmax(r2, 1e-30)) : 0.0;
      const double ir2 = iru * iru;
      const double ir6 = ir2 * ir2 * ir2;
      const double ir8 = ir2 * ir6;
      const double ducir = k.duc_L * iru;
      const double fs = fma(ir8, fma(k.s12, ir6, -k.s6), ducir);
      const double bv = fma(ir8, fma(k.b12, ir6, -k.b6), ducir) * ir2;
      const float a = (float)(-fs);
      const float tt = (float)(bv * fma(dx, wx, fma(dy, wy, dz * wz)));
      const double kx = (double)fmaf(a, (float)wx, tt * (float)dx);
      const double ky = (double)fmaf(a, (float)wy, tt * (float)dy);
      const double kz = (double)fmaf(a, (float)wz, tt * (float)dz);
      qx += kx;
      qy += ky;
      qz += kz;
      if constexpr (HALF) {
        if (ok) {
          unsafeAtomicAdd((double*)&L.ACC[3 * t + 0], -kx);
          unsafeAtomicAdd((double*)&L.ACC[3 * t + 1], -ky);
          unsafeAtomicAdd((double*)&L.ACC[3 * t + 2], -kz);
        }
      }
    } else {
      // Exact-list entries need no mask: the padding entries name the slot
      // itself (d = w = 0), and 1e-30 added to r^2 (far below one ulp of any
      // pair's r^2, so no pair's value changes) keeps every term finite, so
      // they add exactly 0.
      double iru;
      if constexpr (decltype(check)::value)
        iru = ok ? rsqrt_nr(r2) : 0.0;
      else
        iru = rsqrt_nr(fma(dx, dx, fma(dy, dy, fma(dz, dz, 1e-30))));
      const double ir2 = iru * iru;
      const double ir6 = ir2 * ir2 * ir2;
      const double ir8 = ir2 * ir6;
      const double ducir = k.duc_L * iru;
      // fs = -U'(r)/r;  bv = (U'' - U'/r) L^2 / r^2
      const double fs = fma(ir8, fma(k.s12, ir6, -k.s6), ducir);
      const double bv = fma(ir8, fma(k.b12, ir6, -k.b6), ducir) * ir2;
      const double tt = bv * fma(dx, wx, fma(dy, wy, dz * wz));
      if constexpr (HALF) {
        const double kx = fma(-fs, wx, tt * dx);
        const double ky = fma(-fs, wy, tt * dy);
        const double kz = fma(-fs, wz, tt * dz);
        qx += kx;
        qy += ky;
        qz += kz;
        if (ok) {
          unsafeAtomicAdd((double*)&L.ACC[3 * t + 0], -kx);
          unsafeAtomicAdd((double*)&L.ACC[3 * t + 1], -ky);
          unsafeAtomicAdd((double*)&L.ACC[3 * t + 2], -kz);
        }
      } else {
        qx = fma(tt, dx, fma(-fs, wx, qx));
        qy = fma(tt, dy, fma(-fs, wy, qy));
        qz = fma(tt, dz, fma(-fs, wz, qz));
      }
    }
  };
  const int ec = L.ecnt[er];
  if (ec >= 0)
    for_each_listed<EX_CH, 1>(
        ts.ex, erows, er, ec, 0, [&](int t, bool valid) { body(t, valid, std::false_type{}); },
        [] {});
  else
    for_each_atom<HALF, STEP>(a, L, ts, s, part,
                              [&](int t, bool valid) { body(t, valid, std::true_type{}); });
}

// GRAD = false compiles the action-only form: no Hessian-vector pass and no
// exact-list recording (the mode's gradient bit is then ignored).
template <bool F32, bool RLDS, bool HALF, bool GRAD = true>
__device__ __forceinline__ void tile_body(const PathArgs& a, int tile, const TileScratch& ts,
                                          char* lds_base) {
  constexpr int XS = RLDS ? XS_R : 3;  // LDS doubles per slot
  const bool DB = RLDS && a.lds2;      // two slot arrays (see TileLDS)
  const int N = a.n_atoms;
  const int ncell = a.nc * a.nc * a.nc;
  TileLDS L = carve_lds(lds_base, N, ncell, RLDS, HALF, DB);
  const int64_t n0 = (int64_t)tile * a.tile;
  const int64_t n1 = min(n0 + (int64_t)a.tile, a.n_steps);
  const size_t slice = (size_t)3 * N;
  const bool grad = GRAD && (a.mode & MODE_GRAD) != 0;
  const bool excess = (a.mode & MODE_EXCESS) != 0;
  const int B = blockDim.x;
  const int lane = threadIdx.x & (WAVE - 1);
  const int part = lane >> 5;  // list part of this lane (full lists)
  const int wv = threadIdx.x / WAVE, nwv = B / WAVE;
  const double box = a.lj.box, ib = a.lj.inv_box;
  // rho_n of slot s, component c
  auto rho_get = [&](int s, int c) -> double {
    if constexpr (RLDS)
      return L.X[XS * L.pos(s) + 3 + c];
    else
      return ts.rglob[3 * L.pos(s) + c];
  };
  auto rho_set = [&](int s, int c, double v) {
    if constexpr (RLDS)
      L.X[XS * L.pos(s) + 3 + c] = v;
    else
      ts.rglob[3 * L.pos(s) + c] = v;
  };
  // This tile's displacement bound (hs2, squared) and list radius^2 (rl2),
  // set below; box units.
  double hs2 = a.bu.half_skin2, rl2 = a.bu.rlist2;
  // Loads slice m into slot array X (slot order of the current lists) and
  // raises flag[m & 1] when an atom has moved further than sqrt(hs2) from
  // where the lists were built (then slice m needs new lists).
  auto load_slice = [&](lds_f64* X, int64_t m) {
    double dmax = 0.0;
    for (int s = threadIdx.x; s < N; s += B) {
      const int o = L.perm[s], ps = L.pos(s);
      double d2 = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double u = a.x[(size_t)m * slice + (size_t)c * N + o] * ib;
        X[XS * ps + c] = u;
        const double du = wrap_u(u - ts.xref[3 * s + c]);
        d2 = fma(du, du, d2);
      }
      dmax = fmax(dmax, d2);
    }
    if (!(dmax <= hs2)) L.flag[m & 1] = 1;
  };

  // The tile's first lists are built around each atom's centre: the middle
  // of the box that bounds its positions over the force-evaluated slices
  // n0 .. n1 - 1 (box units, coordinates unwrapped).  Every position of
  // atom i then lies within d_i, half the box's diagonal, of that centre, so
  // a pair's distance differs from the distance of the centres by at most
  // d_i + d_j.  D2 = max d_i^2 bounds the displacement test of load_slice:
  // lists of radius r_c + 2 sqrt(D2) hold every pair that comes within r_c
  // anywhere in the tile, and no slice asks for new lists.  When D2 exceeds
  // (skin/2)^2 the configured skin applies instead and slices that move
  // further get new lists.
  //
  // With rho in LDS the bound is per atom: a pair is listed when its centres
  // are at most r_c + d_i + d_j apart (the reaches wait in the second slot
  // array, which the first slice load has not used yet, or with one array in
  // global scratch).
  double d2max = 0.0;
  for (int i = threadIdx.x; i < N; i += B) {
    L.perm[i] = (uint16_t)i;
    double lo[3], hi[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      lo[c] = hi[c] = a.x[(size_t)n0 * slice + (size_t)c * N + i] * ib;
      ts.rprev[3 * i + c] = 0.0;
    }
    for (int64_t m = n0 + 1; m < n1; ++m) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double u = a.x[(size_t)m * slice + (size_t)c * N + i] * ib;
        lo[c] = fmin(lo[c], u);
        hi[c] = fmax(hi[c], u);
      }
    }
    double di2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double h = 0.5 * (hi[c] - lo[c]);
      di2 = fma(h, h, di2);
      L.X[XS * L.pos(i) + c] = 0.5 * (hi[c] + lo[c]);
    }
    if constexpr (RLDS) {
      if (DB)
        L.X2[i] = di2;
      else
        ts.rglob[i] = di2;
    }
    d2max = fmax(d2max, di2);
  }
  if (threadIdx.x == 0) L.flag[0] = L.flag[1] = 0;
  // (rounding of the centres and of the test's differences stays far inside
  // the relative 1e-10 on D2 and 1e-12 on the reaches)
  d2max = block_max_all(d2max, L.red) * (1.0 + 1e-10);
  const double rcm = sqrt(a.bu.rc2) * (1.0 + 1e-12);
  const double* reach = nullptr;
  if (d2max <= hs2) {
    hs2 = d2max;
    const double r = sqrt(a.bu.rc2) + 2.0 * sqrt(d2max);
    rl2 = r * r * (1.0 + 1e-12);
    if constexpr (RLDS) {
      if (DB) {
        for (int i = threadIdx.x; i < N; i += B) L.X2[i] = sqrt(L.X2[i]) * (1.0 + 1e-12);
        reach = (const double*)L.X2;
      } else {
        for (int i = threadIdx.x; i < N; i += B) ts.rglob[i] = sqrt(ts.rglob[i]) * (1.0 + 1e-12);
        reach = ts.rglob;
      }
    }
  }
  const double reach_all = 0.5 * (sqrt(rl2) - rcm);  // every atom's reach at radius sqrt(rl2)
  bool first = true;  // X holds the centres, whose lists come first

  for (int64_t n = n0; n < n1;) {
    __syncthreads();  // X holds x_n (or the centres); flag[n & 1] is final
    if (first || L.flag[n & 1]) {
      rebuild<XS, HALF>(a, L, ts, rl2, rcm, first ? reach : nullptr, reach_all);
      __syncthreads();  // lists and slots ready
      if (first) {
        // x_n0 in the new slot order; it may itself need new lists
        first = false;
        load_slice(L.X, n0);
        continue;
      }
    }
    const double w = a.weights ? a.weights[n] : 1.0;
    const double* xcur = a.x + (size_t)n * slice;
    const double* xnext = xcur + slice;
    if constexpr (HALF) {
      for (int e = threadIdx.x; e < 3 * N; e += B) L.ACC[e] = 0.0;
      __syncthreads();  // ACC cleared
    }

    // ---- pass 1: force, residual, per-step action ----
    double s_loc = 0.0, e_loc = 0.0;
    auto residual = [&](int s, const double* f) {
      const int o = L.perm[s];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const size_t e = (size_t)c * N + o;
        const double d = min_image(xnext[e] - xcur[e], box, ib);
        const double r = fma(-a.mu_dt, f[c], d);
        s_loc = fma(r, r, s_loc);
        e_loc = fma(r - d, r + d, e_loc);
        if (grad) rho_set(s, c, w * r);
      }
    };
    if constexpr (!HALF) {
      // two lanes per atom (lanes l and l + 32 of a wave), each taking every
      // other list chunk: the block's work comes in half-atom pieces that
      // spread evenly over the four SIMDs
      for (int base = wv * 32; base < N; base += nwv * 32) {
        const int s = base + (lane & 31);
        const bool live = s < N;
        double f[3] = {0.0, 0.0, 0.0};
        if (live)
          pass1_part<XS, F32, false, 2, GRAD>(a, L, ts, s, part, 2 * s + part, 2 * N, f[0], f[1],
                                              f[2]);
#pragma unroll
        for (int c = 0; c < 3; ++c) f[c] += __shfl_xor(f[c], 32, WAVE);
        if (live && part == 0) residual(s, f);
      }
    } else {
      for (int s = threadIdx.x; s < N; s += B) {
        double f[3];
        pass1_part<XS, F32, true, 1, GRAD>(a, L, ts, s, 0, s, N, f[0], f[1], f[2]);
        // own partial force waits in rho until every partner share has arrived
#pragma unroll
        for (int c = 0; c < 3; ++c) rho_set(s, c, f[c]);
      }
      __syncthreads();  // every partner share is in ACC
      for (int s = threadIdx.x; s < N; s += B) {
        double f[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) f[c] = rho_get(s, c) + L.ACC[3 * s + c];
        residual(s, f);
      }
    }
    // per-wave partial sums; the block total is formed after the barrier
    {
      const double ws_ = wave_sum(s_loc);
      const double we_ = excess ? wave_sum(e_loc) : 0.0;
      if (lane == 0) {
        L.red[wv] = ws_;
        L.red[16 + wv] = we_;
      }
    }
    __syncthreads();  // rho_n of every atom is stored; partial sums are in red
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int k = 0; k < nwv; ++k) t += L.red[k];
      a.per_step[n] = t * a.inv4Ddt;
      if (excess) {
        double e = 0.0;
        for (int k = 0; k < nwv; ++k) e += L.red[16 + k];
        a.excess[n] = e * a.inv4Ddt;
      }
      L.flag[n & 1] = 0;  // every thread has read it; next raised by slice n + 2
    }
    // slice n + 1 goes into the other slot array while pass 2 reads this one
    if (DB && n + 1 < n1) load_slice(L.X2, n + 1);

    // ---- pass 2: Hessian-vector product and gradient ----
    if (grad) {
      if constexpr (HALF) {
        for (int e = threadIdx.x; e < 3 * N; e += B) L.ACC[e] = 0.0;
        __syncthreads();  // ACC cleared
      }
      const double cq = a.c * a.mu_dt;
      if constexpr (!HALF) {
        for (int base = wv * 32; base < N; base += nwv * 32) {
          const int s = base + (lane & 31);
          const bool live = s < N;
          double q[3] = {0.0, 0.0, 0.0};
          if (live) {
            if constexpr (RLDS)
              pass2_part<XS, XS, F32, false, 2>(a, L, L.X + 3, ts, s, part, 2 * s + part, 2 * N,
                                               q[0], q[1], q[2]);
            else
              pass2_part<XS, 3, F32, false, 2>(a, L, (const double*)ts.rglob, ts, s, part,
                                               2 * s + part, 2 * N, q[0], q[1], q[2]);
          }
#pragma unroll
          for (int c = 0; c < 3; ++c) q[c] += __shfl_xor(q[c], 32, WAVE);
          if (live && part == 0) {
            const int o = L.perm[s];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const double rho = rho_get(s, c);
              const double g = fma(cq, q[c], a.c * (ts.rprev[3 * o + c] - rho));
              a.grad[(size_t)n * slice + (size_t)c * N + o] = g;
              ts.rprev[3 * o + c] = rho;
            }
          }
        }
      } else {
        // own partial q stays in registers until the partner shares arrive
        double q[HALF_SLOTS][3];
#pragma unroll
        for (int kk = 0; kk < HALF_SLOTS; ++kk) {
          const int s = threadIdx.x + kk * B;
          q[kk][0] = q[kk][1] = q[kk][2] = 0.0;
          if (s < N) {
            if constexpr (RLDS)
              pass2_part<XS, XS, F32, true, 1>(a, L, L.X + 3, ts, s, 0, s, N, q[kk][0], q[kk][1],
                                              q[kk][2]);
            else
              pass2_part<XS, 3, F32, true, 1>(a, L, (const double*)ts.rglob, ts, s, 0, s, N,
                                              q[kk][0], q[kk][1], q[kk][2]);
          }
        }
        __syncthreads();  // every partner share is in ACC
#pragma unroll
        for (int kk = 0; kk < HALF_SLOTS; ++kk) {
          const int s = threadIdx.x + kk * B;
          if (s < N) {
            const int o = L.perm[s];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
              const double rho = rho_get(s, c);
              const double g =
                  fma(cq, q[kk][c] + L.ACC[3 * s + c], a.c * (ts.rprev[3 * o + c] - rho));
              a.grad[(size_t)n * slice + (size_t)c * N + o] = g;
              ts.rprev[3 * o + c] = rho;
            }
          }
        }
      }
    }
    if (DB) {
      lds_f64* t = L.X;
      L.X = L.X2;
      L.X2 = t;
    } else if (n + 1 < n1) {
      __syncthreads();  // every read of X (and rho, ACC) for slice n is done
      load_slice(L.X, n + 1);
    }
    ++n;
  }

  if (grad) {
    __syncthreads();
    for (int o = threadIdx.x; o < N; o += B) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double v = a.c * ts.rprev[3 * o + c];
        if (n1 == a.n_steps)
          a.grad[(size_t)a.n_steps * slice + (size_t)c * N + o] = v;
        else
          a.bnd[(size_t)tile * slice + (size_t)c * N + o] = v;
      }
    }
  }
  __syncthreads();  // LDS is reused by the next tile of this block
}

__device__ __forceinline__ TileScratch block_scratch(const BlockScratch& s) {
  TileScratch t;
  t.nbr = s.nbr + (size_t)blockIdx.x * s.nbr_stride;
  t.ex = s.ex_off ? t.nbr + s.ex_off : nullptr;
  t.cnt = s.cnt + (size_t)blockIdx.x * s.cnt_stride;
  t.xref = s.xref + (size_t)blockIdx.x * s.xref_stride;
  t.rprev = t.xref + s.xref_stride / 2;
  t.rglob = s.rglob ? s.rglob + (size_t)blockIdx.x * s.rglob_stride : nullptr;
  return t;
}

// ===========================================================================
// Exact lists in LDS.  The partners found within r_c in pass 1 are kept in
// shared memory for pass 2, so no per-slice list traffic reaches device
// memory.  Each atom owns EXL_ROW entries: the lane of part 0 appends its
// partners from the front, the lane of part 1 from the back, so the region
// overflows only when the atom has more than EXL_ROW partners in all (then
// pass 2 walks the candidate rows again with the cutoff test).  Before
// pass 2 the lane with more partners hands the ones nearest the gap to the
// other lane, so both walk about half, each from its own end of the region
// in whole chunks of four.  The slice has one slot array (position and rho),
// and the next slice is fetched into registers during pass 2 and stored after
// it.  The candidate rows are walked four entries at a time.
// ===========================================================================
constexpr int EXL_ROW = 64;  // LDS entries per atom (both parts)

size_t exl_lds_bytes(int n_atoms, int nc, int block) {
  const size_t ncell = (size_t)nc * nc * nc;
  size_t b = sizeof(double) * (size_t)n_atoms * XS_R;
  b += sizeof(double) * 32 + sizeof(int) * 18 + 6 * (size_t)n_atoms + 16;
  // the atoms' regions, then one discard entry per thread (the build's
  // scratch shares the space)
  const size_t rows = ((size_t)n_atoms * EXL_ROW + (size_t)block) * sizeof(uint16_t);
  return b + std::max<size_t>(rows, lds_shared_region(n_atoms, (int)ncell, block));
}


// Entries of row `row` of a list stored in chunks of 8 (entry k at
// [(k / 8) rows + row] 8 + k % 8), visited four at a time with PF quarter
// chunks in flight; entries past cnt are passed with valid = false.
template <typename Pair>
__device__ __forceinline__ void for_each_listed4(const uint16_t* list, int rows, int row, int cnt,
                                                 Pair&& pair) {
  constexpr int PF = 3;
  const uint2* nb = reinterpret_cast<const uint2*>(list);
  auto at = [&](int q) { return ((size_t)(q >> 1) * rows + row) * 2 + (q & 1); };
  const int nq = (cnt + 3) >> 2;
  uint2 buf[PF];
#pragma unroll
  for (int i = 0; i < PF; ++i) buf[i] = i < nq ? nb[at(i)] : make_uint2(0u, 0u);
  for (int q = 0; q < nq; ++q) {
    const uint2 cur = buf[0];
#pragma unroll
    for (int i = 0; i + 1 < PF; ++i) buf[i] = buf[i + 1];
    buf[PF - 1] = q + PF < nq ? nb[at(q + PF)] : cur;
    const int left = cnt - 4 * q;
#pragma unroll
    for (int e = 0; e < 4; ++e) pair(ChunkOf<4>::entry(cur, e), e < left);
  }
}

// Pass 1 of slot s, part `part`: force from candidate row 2 s + part, with
// the partners within r_c written to the atom's region `reg` (part 0 from
// entry 0 upwards, part 1 from entry EXL_ROW - 1 downwards, each entry e at
// (e + rot) mod EXL_ROW; a candidate that is not kept goes to the lane's
// discard entry).  Returns their number (which
// may exceed what the region holds), or -1 after an overflow scan (then
// nothing is recorded).
template <bool REC>
__device__ __forceinline__ int pass1_exl(const PathArgs& a, const TileLDS& L, const TileScratch& ts,
                                         int s, int part, lds_u16* reg, int rot, lds_u16* discard,
                                         double& fx, double& fy, double& fz) {
  const BoxUnits& k = a.bu;
  const int N = a.n_atoms;
  const int ps = L.pos(s);
  const double xs = L.X[XS_R * ps], ys = L.X[XS_R * ps + 1], zs = L.X[XS_R * ps + 2];
  const int first = part ? EXL_ROW - 1 : 0, dir = part ? -1 : 1;
  fx = fy = fz = 0.0;
  uint32_t acc = 0;
  auto body = [&](int t, bool valid, auto record) {
    const f64x2 uxy = lds_ld2(L.X + XS_R * t);
    const double dx = wrap_u(xs - uxy.x);
    const double dy = wrap_u(ys - uxy.y);
    const double dz = wrap_u(zs - L.X[XS_R * t + 2]);
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const bool ok = valid && r2 <= k.rc2;
    if constexpr (decltype(record)::value) {
      const bool keep = ok && acc < (uint32_t)EXL_ROW;
      lds_u16* dst = keep ? reg + ((first + dir * (int)acc + rot) & (EXL_ROW - 1)) : discard;
      *dst = (uint16_t)t;
      acc += ok ? 1u : 0u;
    }
    double iru = rsqrt_nr(r2);
    iru = ok ? iru : 0.0;
    const double ir2 = iru * iru;
    const double ir6 = ir2 * ir2 * ir2;
    const double fsl = fma(ir2 * ir6, fma(k.f12, ir6, -k.f6), k.duc * iru);
    fx = fma(fsl, dx, fx);
    fy = fma(fsl, dy, fy);
    fz = fma(fsl, dz, fz);
  };
  const int cnt = a.reach < 0 ? -1 : ts.cnt[2 * s + part];  // reach -1: no lists
  if (cnt >= 0) {
    for_each_listed4(ts.nbr, 2 * N, 2 * s + part, cnt, [&](int t, bool valid) {
      body(t, valid, std::integral_constant<bool, REC>{});
    });
    return (int)acc;
  }
  for_each_atom<false, 2>(a, L, ts, s, part,
                          [&](int t, bool valid) { body(t, valid, std::false_type{}); });
  return -1;
}

// Pass 2 of slot s, part `part`: q_s from the part's ec entries of the
// atom's region (part 0 from the front, part 1 from the back, padded with the
// slot itself to whole chunks of 4), from the candidate row with the cutoff
// test when the region overflowed (ec == -2), or from the part's share of an
// overflow scan when the candidate rows did (ec == -1).
template <bool F32>
__device__ __forceinline__ void pass2_exl(const PathArgs& a, const TileLDS& L, const TileScratch& ts,
                                          int s, int part, int ec, const lds_u16* reg, int rot,
                                          double& qx, double& qy, double& qz) {
  const BoxUnits& k = a.bu;
  const int ps = L.pos(s);
  const f64x2 o0 = lds_ld2(L.X + XS_R * ps), o1 = lds_ld2(L.X + XS_R * ps + 2),
              o2 = lds_ld2(L.X + XS_R * ps + 4);
  const double xs = o0.x, ys = o0.y, zs = o1.x, rx = o1.y, ry = o2.x, rz = o2.y;
  qx = qy = qz = 0.0;
  auto body = [&](int t, bool ok) {
    const f64x2 a0 = lds_ld2(L.X + XS_R * t), a1 = lds_ld2(L.X + XS_R * t + 2),
                a2 = lds_ld2(L.X + XS_R * t + 4);
    const double dx = wrap_u(xs - a0.x);
    const double dy = wrap_u(ys - a0.y);
    const double dz = wrap_u(zs - a1.x);
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const double wx = rx - a1.y, wy = ry - a2.x, wz = rz - a2.y;
    if constexpr (F32) {
      // pair functions float64, products with w and d float32, sums float64;
      // the padding entries (r^2 = 0) are masked
      const double iru = ok && r2 > 0.0 ? rsqrt_nr(r2) : 0.0;
      const double ir2 = iru * iru;
      const double ir6 = ir2 * ir2 * ir2;
      const double ir8 = ir2 * ir6;
      const double ducir = k.duc_L * iru;
      const double fs = fma(ir8, fma(k.s12, ir6, -k.s6), ducir);
      const double bv = fma(ir8, fma(k.b12, ir6, -k.b6), ducir) * ir2;
      const float af = (float)(-fs);
      const float tt = (float)(bv * fma(dx, wx, fma(dy, wy, dz * wz)));
      qx += (double)fmaf(af, (float)wx, tt * (float)dx);
      qy += (double)fmaf(af, (float)wy, tt * (float)dy);
      qz += (double)fmaf(af, (float)wz, tt * (float)dz);
    } else {
      // padding entries name the slot itself (d = w = 0); 1e-30 added to r^2
      // (far below one ulp of any pair's r^2) keeps their terms finite, so
      // they add exactly 0; `ok` is false only where the overflow paths below
      // test the cutoff
      double iru = rsqrt_nr(fma(dx, dx, fma(dy, dy, fma(dz, dz, 1e-30))));
      iru = ok ? iru : 0.0;
      const double ir2 = iru * iru;
      const double ir6 = ir2 * ir2 * ir2;
      const double ir8 = ir2 * ir6;
      const double ducir = k.duc_L * iru;
      const double fs = fma(ir8, fma(k.s12, ir6, -k.s6), ducir);
      const double bv = fma(ir8, fma(k.b12, ir6, -k.b6), ducir) * ir2;
      const double tt = bv * fma(dx, wx, fma(dy, wy, dz * wz));
      qx = fma(tt, dx, fma(-fs, wx, qx));
      qy = fma(tt, dy, fma(-fs, wy, qy));
      qz = fma(tt, dz, fma(-fs, wz, qz));
    }
  };
  if (ec >= 0) {
    typedef __attribute__((address_space(3))) const unsigned long long lds_u64;
    // chunk q: entries [4 q, 4 q + 4) for part 0, [EXL_ROW - 4 q - 4, EXL_ROW - 4 q) for
    // part 1, stored rotated by rot (a multiple of 4, so a chunk stays whole)
    const lds_u64* ch = (const lds_u64*)reg;
    const int c0 = part ? EXL_ROW / 4 - 1 : 0, step = part ? -1 : 1, r4 = rot >> 2;
    const int nq = (ec + 3) >> 2;
    for (int q = 0; q < nq; ++q) {
      const unsigned long long v = ch[(c0 + step * q + r4) & (EXL_ROW / 4 - 1)];  // 8-byte read
      const uint2 c = make_uint2((uint32_t)v, (uint32_t)(v >> 32));
#pragma unroll
      for (int e = 0; e < 4; ++e) body(ChunkOf<4>::entry(c, e), true);
    }
  } else if (ec == -2) {
    // rare: one entry at a time, so that this path adds no registers to the
    // common one (candidate entry j of row r is at [(j / 8) 2 N + r] 8 + j % 8)
    const int r = 2 * s + part;
    const size_t rows = (size_t)2 * a.n_atoms;
    const int cnt = ts.cnt[r];
    for (int j = 0; j < cnt; ++j) {
      const int t = ts.nbr[((size_t)(j >> 3) * rows + r) * 8 + (j & 7)];
      const double dx = wrap_u(xs - L.X[XS_R * t]);
      const double dy = wrap_u(ys - L.X[XS_R * t + 1]);
      const double dz = wrap_u(zs - L.X[XS_R * t + 2]);
      body(t, fma(dx, dx, fma(dy, dy, dz * dz)) <= k.rc2);
    }
  } else {
    for_each_atom<false, 2>(a, L, ts, s, part, [&](int t, bool) {
      const double dx = wrap_u(xs - L.X[XS_R * t]);
      const double dy = wrap_u(ys - L.X[XS_R * t + 1]);
      const double dz = wrap_u(zs - L.X[XS_R * t + 2]);
      body(t, fma(dx, dx, fma(dy, dy, dz * dz)) <= k.rc2);
    });
  }
}

// One tile with the exact lists in LDS (see above).  Full lists, rho in LDS,
// one slot array; n_atoms <= blockDim.x (one slot per thread in the
// next-slice fetch).
template <bool F32, bool GRAD = true>
__device__ void tile_body_exl(const PathArgs& a, int tile, const TileScratch& ts, char* lds_base) {
  constexpr int XS = XS_R;
  const int N = a.n_atoms;
  const int ncell = a.nc * a.nc * a.nc;
  TileLDS L = carve_lds(lds_base, N, ncell, true, false, false);
  lds_u16* const EXR = L.stage;  // N regions of EXL_ROW entries (shares the build's region)
  lds_u16* const discard = EXR + (size_t)N * EXL_ROW + threadIdx.x;
  const int64_t n0 = (int64_t)tile * a.tile;
  const int64_t n1 = min(n0 + (int64_t)a.tile, a.n_steps);
  const size_t slice = (size_t)3 * N;
  const bool grad = GRAD && (a.mode & MODE_GRAD) != 0;
  const bool excess = (a.mode & MODE_EXCESS) != 0;
  const int B = blockDim.x;
  const int lane = threadIdx.x & (WAVE - 1);
  const int part = lane >> 5;
  const int wv = threadIdx.x / WAVE, nwv = B / WAVE;
  const double box = a.lj.box, ib = a.lj.inv_box;
  double hs2 = a.bu.half_skin2, rl2 = a.bu.rlist2;

  // reach -1: no lists (the list sphere would hold most of the box); both
  // passes scan all atoms, so nothing is built and no skin is watched
  const bool nolist = a.reach < 0;

  // Initial lists around each atom's centre over the tile (see tile_body);
  // the per-atom reaches wait in global scratch.
  double d2max = 0.0;
  for (int i = threadIdx.x; i < N; i += B) {
    L.perm[i] = (uint16_t)i;
#pragma unroll
    for (int c = 0; c < 3; ++c) ts.rprev[3 * i + c] = 0.0;
    if (nolist) continue;
    double lo[3], hi[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) lo[c] = hi[c] = a.x[(size_t)n0 * slice + (size_t)c * N + i] * ib;
    for (int64_t m = n0 + 1; m < n1; ++m) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double u = a.x[(size_t)m * slice + (size_t)c * N + i] * ib;
        lo[c] = fmin(lo[c], u);
        hi[c] = fmax(hi[c], u);
      }
    }
    double di2 = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double h = 0.5 * (hi[c] - lo[c]);
      di2 = fma(h, h, di2);
      L.X[XS * L.pos(i) + c] = 0.5 * (hi[c] + lo[c]);
    }
    ts.rglob[i] = di2;
    d2max = fmax(d2max, di2);
  }
  if (threadIdx.x == 0) L.flag[0] = L.flag[1] = 0;
  if (!nolist) d2max = block_max_all(d2max, L.red) * (1.0 + 1e-10);
  const double rcm = sqrt(a.bu.rc2) * (1.0 + 1e-12);
  const double* reach = nullptr;
  if (!nolist && d2max <= hs2) {
    hs2 = d2max;
    const double r = sqrt(a.bu.rc2) + 2.0 * sqrt(d2max);
    rl2 = r * r * (1.0 + 1e-12);
    for (int i = threadIdx.x; i < N; i += B) ts.rglob[i] = sqrt(ts.rglob[i]) * (1.0 + 1e-12);
    reach = ts.rglob;
  }
  const double reach_all = 0.5 * (sqrt(rl2) - rcm);
  bool first = true;

  // the next slice, fetched during pass 2 (slot threadIdx.x) and stored after it
  double nx[3] = {0.0, 0.0, 0.0}, nref[3] = {0.0, 0.0, 0.0};
  const int my = threadIdx.x;
  auto store_next = [&](int64_t m) {
    if (my < N) {
      double d2 = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double u = nx[c] * ib;
        L.X[XS * L.pos(my) + c] = u;
        const double du = wrap_u(u - nref[c]);
        d2 = fma(du, du, d2);
      }
      if (!nolist && !(d2 <= hs2)) L.flag[m & 1] = 1;
    }
  };
  auto fetch_next = [&](int64_t m) {
    if (my < N) {
      const int o = L.perm[my];
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        nx[c] = a.x[(size_t)m * slice + (size_t)c * N + o];
        nref[c] = nolist ? 0.0 : ts.xref[3 * my + c];
      }
    }
  };

  for (int64_t n = n0; n < n1;) {
    __syncthreads();  // X holds x_n (or the centres); flag[n & 1] is final
    if (first || L.flag[n & 1]) {
      if (!nolist) {
        rebuild<XS, false>(a, L, ts, rl2, rcm, first ? reach : nullptr, reach_all);
        __syncthreads();  // lists and slots ready
      }
      if (first) {
        first = false;
        fetch_next(n0);
        store_next(n0);
        continue;
      }
    }
    const double w = a.weights ? a.weights[n] : 1.0;
    const double* xcur = a.x + (size_t)n * slice;
    const double* xnext = xcur + slice;

    // ---- pass 1: force, exact rows, residual, per-step action ----
    double s_loc = 0.0, e_loc = 0.0;
    for (int base = wv * 32; base < N; base += nwv * 32) {
      const int s = base + (lane & 31);
      const bool live = s < N;
      const int r = 2 * (live ? s : 0) + part;
      lds_u16* reg = EXR + (size_t)(live ? s : 0) * EXL_ROW;
      // the regions of consecutive atoms lie EXL_ROW entries (128 bytes)
      // apart, so each is rotated by 4 (s mod 16) entries: the 32 lanes of a
      // part then reach different LDS banks
      const int rot = 4 * (s & 15);
      auto at = [&](int e) { return (e + rot) & (EXL_ROW - 1); };
      double f[3] = {0.0, 0.0, 0.0};
      int c = 0;
      if (live) c = pass1_exl<GRAD>(a, L, ts, s, part, reg, rot, discard, f[0], f[1], f[2]);
#pragma unroll
      for (int k = 0; k < 3; ++k) f[k] += __shfl_xor(f[k], 32, WAVE);
      // split the atom's partners evenly between its two lanes, then pad each
      // part to whole chunks
      const int co = __shfl_xor(c, 32, WAVE);
      if (live && GRAD) {
        int ec = -1;  // candidate rows overflowed: scan
        if (c >= 0 && co >= 0) {
          if (c + co > EXL_ROW) {
            ec = -2;  // the region overflowed: candidate rows again
          } else {
            const int E = c + co;
            const int h = part == 0 ? (E + 1) >> 1 : E >> 1;
            const int ho = E - h;
            // This part's entries are [0, c) (part 0) or [EXL_ROW - c, EXL_ROW)
            // (part 1); it keeps [0, h) or [EXL_ROW - h, EXL_ROW).  Surplus
            // entries that already lie in the other part's final segment stay;
            // the rest move to the other part's free entries next to the gap
            // (source and destination ranges are disjoint).
            if (c > h) {
              int src, dst, n;
              if (part == 0) {
                src = h;
                n = min(c, EXL_ROW - ho) - h;
                dst = max(c, EXL_ROW - ho);
              } else {
                src = max(EXL_ROW - c, ho);
                n = EXL_ROW - h - src;
                dst = co;
              }
              for (int j = 0; j < n; ++j) reg[at(dst + j)] = reg[at(src + j)];
            }
            // the padding may overwrite surplus the other lane has just moved:
            // both lanes are in this wave, and the barrier keeps the moves
            // ahead of the padding in the instruction stream
            __builtin_amdgcn_wave_barrier();
            const uint16_t self = (uint16_t)L.pos(s);
            for (int i = h; i & 3; ++i) reg[at(part == 0 ? i : EXL_ROW - 1 - i)] = self;
            ec = h;
          }
        }
        L.ecnt[r] = (int16_t)ec;
      }
      if (live && part == 0) {
        const int o = L.perm[s];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const size_t e = (size_t)k * N + o;
          const double d = min_image(xnext[e] - xcur[e], box, ib);
          const double rr = fma(-a.mu_dt, f[k], d);
          s_loc = fma(rr, rr, s_loc);
          e_loc = fma(rr - d, rr + d, e_loc);
          if (grad) L.X[XS * L.pos(s) + 3 + k] = w * rr;
        }
      }
    }
    {
      const double ws_ = wave_sum(s_loc);
      const double we_ = excess ? wave_sum(e_loc) : 0.0;
      if (lane == 0) {
        L.red[wv] = ws_;
        L.red[16 + wv] = we_;
      }
    }
    __syncthreads();  // rho_n of every atom and every exact row are stored
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int k = 0; k < nwv; ++k) t += L.red[k];
      a.per_step[n] = t * a.inv4Ddt;
      if (excess) {
        double e = 0.0;
        for (int k = 0; k < nwv; ++k) e += L.red[16 + k];
        a.excess[n] = e * a.inv4Ddt;
      }
      L.flag[n & 1] = 0;
    }
    const bool more = n + 1 < n1;
    if (more) fetch_next(n + 1);

    // ---- pass 2: Hessian-vector product and gradient ----
    if (grad) {
      const double cq = a.c * a.mu_dt;
      for (int base = wv * 32; base < N; base += nwv * 32) {
        const int s = base + (lane & 31);
        const bool live = s < N;
        double q[3] = {0.0, 0.0, 0.0};
        if (live) {
          pass2_exl<F32>(a, L, ts, s, part, L.ecnt[2 * s + part], EXR + (size_t)s * EXL_ROW,
                         4 * (s & 15), q[0], q[1], q[2]);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) q[k] += __shfl_xor(q[k], 32, WAVE);
        if (live && part == 0) {
          const int o = L.perm[s];
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            const double rho = L.X[XS * L.pos(s) + 3 + k];
            const double g = fma(cq, q[k], a.c * (ts.rprev[3 * o + k] - rho));
            a.grad[(size_t)n * slice + (size_t)k * N + o] = g;
            ts.rprev[3 * o + k] = rho;
          }
        }
      }
    }
    __syncthreads();  // every read of slice n in X is done
    if (more) store_next(n + 1);
    ++n;
  }

  if (grad) {
    __syncthreads();
    for (int o = threadIdx.x; o < N; o += B) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const double v = a.c * ts.rprev[3 * o + c];
        if (n1 == a.n_steps)
          a.grad[(size_t)a.n_steps * slice + (size_t)c * N + o] = v;
        else
          a.bnd[(size_t)tile * slice + (size_t)c * N + o] = v;
      }
    }
  }
  __syncthreads();  // LDS is reused by the next tile of this block
}

template <bool F32>
__global__ void __launch_bounds__(1024) lj_fused_exl_kernel(PathArgs a, BlockScratch s) {
  extern __shared__ __align__(16) char lds[];
  const TileScratch ts = block_scratch(s);
  for (int t = blockIdx.x; t < a.n_tiles; t += gridDim.x) tile_body_exl<F32>(a, t, ts, lds);
}

template <bool F32>
__global__ void __launch_bounds__(1024) lj_action_exl_kernel(PathArgs a, BlockScratch s) {
  extern __shared__ __align__(16) char lds[];
  const TileScratch ts = block_scratch(s);
  for (int t = blockIdx.x; t < a.n_tiles; t += gridDim.x) tile_body_exl<F32, false>(a, t, ts, lds);
}

template <bool F32, bool RLDS, bool HALF>
__global__ void __launch_bounds__(1024) lj_fused_kernel(PathArgs a, BlockScratch s) {
  extern __shared__ __align__(16) char lds[];
  const TileScratch ts = block_scratch(s);
  for (int t = blockIdx.x; t < a.n_tiles; t += gridDim.x)
    tile_body<F32, RLDS, HALF>(a, t, ts, lds);
}

// Action (and excess) without the gradient.
template <bool F32, bool RLDS, bool HALF>
__global__ void __launch_bounds__(1024) lj_action_kernel(PathArgs a, BlockScratch s) {
  extern __shared__ __align__(16) char lds[];
  const TileScratch ts = block_scratch(s);
  for (int t = blockIdx.x; t < a.n_tiles; t += gridDim.x)
    tile_body<F32, RLDS, HALF, false>(a, t, ts, lds);
}

__device__ __forceinline__ PathArgs member_args(const BatchMember& m, const BatchBase& b) {
  PathArgs a = m.a;
  a.x = m.x_abs ? m.x_abs : b.x + m.x_off;
  a.weights = b.weights ? b.weights + m.step_off : nullptr;
  a.grad = m.x_abs ? m.grad_abs : (b.grad ? b.grad + m.x_off : nullptr);
  a.per_step = b.per_step + m.step_off;
  a.bnd = b.bnd + m.bnd_off;
  a.excess = nullptr;
  a.mode = (b.mode | MODE_GRAD) & ~MODE_EXCESS;
  if (!a.grad) a.mode &= ~MODE_GRAD;
  return a;
}

// Persistent batch kernel: workgroups pull (path, tile) items, largest first.
template <bool F32, bool RLDS, bool HALF>
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
    tile_body<F32, RLDS, HALF>(a, item.tile, ts, lds);
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

// Sequential Euler-Maruyama integration (Eq. 2) of one Lennard-Jones system:
// one workgroup steps x_{n+1} = x_n + (dt/gamma) F(x_n) + sqrt(2 D dt) xi_n
// with the path kernel's force pass, slot layout and neighbour lists (new
// lists when an atom has moved more than skin/2 since the last build).  x_n
// in physical units is read back from x_out, where the previous step stored
// it.  With DB the next slice goes straight into the second slot array;
// otherwise it is reloaded from x_out after the step (one array, 3 doubles
// per slot, sort scratch in global memory).
template <bool DB>
__global__ void __launch_bounds__(1024) lj_em_kernel(PathArgs a, const double* xi, double amp,
                                                     double* xout, BlockScratch sc) {
  extern __shared__ __align__(16) char lds[];
  constexpr int XS = DB ? XS_R : 3;
  const TileScratch ts = block_scratch(sc);
  const int N = a.n_atoms;
  TileLDS L = carve_lds(lds, N, a.nc * a.nc * a.nc, DB, false, DB);
  const size_t slice = (size_t)3 * N;
  const double ib = a.lj.inv_box;
  const int B = blockDim.x;
  const int lane = threadIdx.x & (WAVE - 1);
  const int part = lane >> 5;
  const int wv = threadIdx.x / WAVE, nwv = B / WAVE;
  for (int i = threadIdx.x; i < N; i += B) {
    L.perm[i] = (uint16_t)i;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const double v = a.x[(size_t)c * N + i];
      xout[(size_t)c * N + i] = v;
      L.X[XS * L.pos(i) + c] = v * ib;
    }
  }
  if (threadIdx.x == 0) L.flag[0] = L.flag[1] = 0;
  const double hs2 = a.bu.half_skin2, rl2 = a.bu.rlist2;
  bool first = true;
  for (int64_t n = 0; n < a.n_steps; ++n) {
    __syncthreads();  // X and x_out hold x_n; flag[n & 1] is final
    if (first || L.flag[n & 1]) {
      const double rcm = sqrt(a.bu.rc2) * (1.0 + 1e-12);
      rebuild<XS, false>(a, L, ts, rl2, rcm, nullptr, 0.5 * (sqrt(rl2) - rcm));
      __syncthreads();  // lists and slots ready
      first = false;
    }
    const double* xcur = xout + (size_t)n * slice;
    double* xnext = xout + (size_t)(n + 1) * slice;
    const double* xin = xi + (size_t)n * slice;
    bool moved = false;
    for (int base = wv * 32; base < N; base += nwv * 32) {
      const int s = base + (lane & 31);
      const bool live = s < N;
      const bool own = live && part == 0;  // this lane steps atom perm[s]
      // x_n and xi_n are fetched before the force pass so that their latency
      // overlaps it
      const int o = own ? (int)L.perm[s] : 0;
      double xc[3] = {0.0, 0.0, 0.0}, xr[3] = {0.0, 0.0, 0.0};
      if (own) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          xc[c] = xcur[(size_t)c * N + o];
          xr[c] = xin[(size_t)c * N + o];
        }
      }
      double f[3] = {0.0, 0.0, 0.0};
      if (live)
        pass1_part<XS, false, false, 2, false>(a, L, ts, s, part, 2 * s + part, 2 * N, f[0], f[1],
                                               f[2]);
#pragma unroll
      for (int c = 0; c < 3; ++c) f[c] += __shfl_xor(f[c], 32, WAVE);
      if (own) {
        double d2 = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          const size_t e = (size_t)c * N + o;
          const double x1 = fma(amp, xr[c], fma(a.mu_dt, f[c], xc[c]));
          xnext[e] = x1;
          const double u = x1 * ib;
          if constexpr (DB) L.X2[XS * L.pos(s) + c] = u;
          const double du = wrap_u(u - ts.xref[3 * s + c]);
          d2 = fma(du, du, d2);
        }
        moved = moved || !(d2 <= hs2);
      }
    }
    if (moved) L.flag[(n + 1) & 1] = 1;
    __syncthreads();  // x_{n+1} is stored; every read of X for step n is done
    if (threadIdx.x == 0) L.flag[n & 1] = 0;
    if constexpr (DB) {
      lds_f64* t = L.X;
      L.X = L.X2;
      L.X2 = t;
    } else {
      for (int s = threadIdx.x; s < N; s += B) {
        const int o = L.perm[s];
#pragma unroll
        for (int c = 0; c < 3; ++c) L.X[XS * L.pos(s) + c] = xnext[(size_t)c * N + o] * ib;
      }
    }
  }
}

hipError_t launch_lj_em(const PathArgs& a, const double* xi, double amp, double* xout,
                        const BlockScratch& s, const FusedLaunch& L, hipStream_t st) {
  const bool db = L.r_in_lds && L.lds2;  // else one array of positions (3 doubles per slot)
  const void* k = db ? (const void*)lj_em_kernel<true> : (const void*)lj_em_kernel<false>;
  hipError_t e =
      hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_bytes);
  if (e != hipSuccess) return e;
  if (db)
    hipLaunchKernelGGL(lj_em_kernel<true>, dim3(1), dim3(L.block), L.lds_bytes, st, a, xi, amp,
                       xout, s);
  else
    hipLaunchKernelGGL(lj_em_kernel<false>, dim3(1), dim3(L.block), L.lds_bytes, st, a, xi, amp,
                       xout, s);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------
template <bool F32>
static hipError_t launch_exl_t(const PathArgs& a, const BlockScratch& s, const FusedLaunch& L,
                               hipStream_t st) {
  auto kern = (a.mode & MODE_GRAD) ? lj_fused_exl_kernel<F32> : lj_action_exl_kernel<F32>;
  hipError_t e = hipFuncSetAttribute((const void*)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)L.lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(L.grid), dim3(L.block), L.lds_bytes, st, a, s);
  return hipGetLastError();
}

template <bool F32, bool RLDS, bool HALF>
static hipError_t launch_fused_t(const PathArgs& a, const BlockScratch& s, const FusedLaunch& L,
                                 hipStream_t st) {
  auto kern = (a.mode & MODE_GRAD) ? lj_fused_kernel<F32, RLDS, HALF>
                                   : lj_action_kernel<F32, RLDS, HALF>;
  hipError_t e = hipFuncSetAttribute((const void*)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)L.lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(L.grid), dim3(L.block), L.lds_bytes, st, a, s);
  return hipGetLastError();
}

template <bool F32, bool RLDS, bool HALF>
static hipError_t launch_batch_t(const BatchMember* m, const BatchBase& b, const BatchItem* it,
                                 int n, int* ctr, const BlockScratch& s, const FusedLaunch& L,
                                 hipStream_t st) {
  auto kern = lj_batch_kernel<F32, RLDS, HALF>;
  hipError_t e = hipFuncSetAttribute((const void*)kern,
                                     hipFuncAttributeMaxDynamicSharedMemorySize,
                                     (int)L.lds_bytes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(kern, dim3(L.grid), dim3(L.block), L.lds_bytes, st, m, b, it, n, ctr, s);
  return hipGetLastError();
}

#define PAMD_DISPATCH3(FN, F32, ...)                                                      \
  if (L.half)                                                                             \
    return L.r_in_lds ? FN<F32, true, true>(__VA_ARGS__) : FN<F32, false, true>(__VA_ARGS__); \
  return L.r_in_lds ? FN<F32, true, false>(__VA_ARGS__) : FN<F32, false, false>(__VA_ARGS__);

#define PAMD_DISPATCH(FN, ...)             \
  if (L.f32) {                             \
    PAMD_DISPATCH3(FN, true, __VA_ARGS__)  \
  } else {                                 \
    PAMD_DISPATCH3(FN, false, __VA_ARGS__) \
  }

hipError_t launch_lj_fused(const PathArgs& a, const BlockScratch& s, const FusedLaunch& L,
                           hipStream_t st) {
  if (L.exl) return L.f32 ? launch_exl_t<true>(a, s, L, st) : launch_exl_t<false>(a, s, L, st);
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
