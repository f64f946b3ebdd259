/*
 * pamd.h -- C ABI of libpamd, the MI355X (gfx950) implementation of the
 * discretized Brownian path action and its gradient.
 *
 * Method: Rosa-Raices, Zhang, Miller, "Path-accelerated molecular dynamics:
 * parallel-in-time integration using path integrals", arXiv:1907.09529.
 *
 * A path is X = {x_0, ..., x_N} (Sec. II A, above Eq. 4): N time steps of
 * length dt and N + 1 configurations ("slices").  For overdamped Langevin
 * dynamics (Eq. 1) discretized by Euler-Maruyama (Eq. 2), each step has the
 * Gaussian transition density of Eq. 3 and the path likelihood is
 * prod_n K(x_{n+1} | x_n; dt) = exp(-S[X]) (Eq. 4).  This library evaluates,
 * for all steps at once,
 *
 *     r_n = Delta_n - (dt / gamma) F(x_n),      Delta_n = x_{n+1} - x_n (minimum image),
 *     s_n = |r_n|^2 / (4 D dt),                 S = sum_{n<N} s_n,
 *
 * with F = -V' (harmonic, or the cut-and-force-shifted Lennard-Jones pair
 * potential of Eq. 16 under cubic periodic boundaries), and the gradient
 *
 *     g_m = dS/dx_m = c [ w_{m-1} r_{m-1} - w_m r_m + (dt/gamma) H(x_m) w_m r_m ],  c = 1/(2 D dt),
 *
 * (terms with an index outside 0..N-1 vanish; H is the potential-energy
 * Hessian, applied as a Hessian-vector product and never formed; w_n are
 * optional per-step weights, all 1 by default, giving the gradient of
 * sum_n w_n s_n).  S excludes the normalisation of the N Gaussian densities;
 * pamd_log_norm() returns it.
 *
 * Conventions for every entry point
 *   - Memory layout: a path is float64, contiguous, slice-major with the
 *     coordinates of one slice grouped by component:
 *         x[(n * n_dim + c) * n_atoms + i],  n = 0..N, c = 0..n_dim-1.
 *     Coordinates are unwrapped (no periodic folding is required or applied).
 *   - Pointers named "device" must be device memory of the current HIP device
 *     (e.g. torch tensors' data_ptr()); "host" pointers are host memory.
 *     The caller owns all buffers.  The library never allocates device memory.
 *   - Every call is asynchronous on `stream` (a hipStream_t; NULL = the null
 *     stream).  Results are valid once the stream has reached them.
 *   - Workspace: `ws` is caller-provided device memory of at least the size
 *     reported by the matching *_workspace_size call, 256-byte aligned.  Its
 *     contents need no initialisation and are not meaningful after a call.
 *     Two calls that overlap in time must not share a workspace.
 *   - Errors: 0 on success, a negative PAMD_E* code otherwise; then
 *     pamd_last_error() returns a message (thread-local).  All arguments are
 *     validated on the host before any device work is enqueued, so a failed
 *     call has no device side effects.  Non-finite coordinates are not
 *     checked: they propagate as IEEE NaN/Inf.
 *   - Calls enqueue kernels only (no memset, no host synchronisation), so they
 *     may be captured into a HIP graph (see pamd_graph_*).  pamd_autotune is
 *     the exception: it synchronises and must not be captured.
 */
#ifndef PAMD_H
#define PAMD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes ---- */
#define PAMD_OK 0
#define PAMD_EINVAL (-1)          /* malformed argument (null pointer, bad size, bad value) */
#define PAMD_EUNSUPPORTED (-2)    /* well-formed but outside what the library implements */
#define PAMD_EWORKSPACE (-3)      /* ws_bytes smaller than required, or ws misaligned */
#define PAMD_EHIP (-4)            /* a HIP runtime call failed (message has the HIP error) */

/* ---- potential kinds (pamd_potential.kind) ---- */
#define PAMD_HARMONIC 0           /* V = k/2 sum x^2 over all degrees of freedom (Sec. IV A) */
#define PAMD_LJ 1                 /* cut-and-force-shifted LJ pair potential, Eq. 16 (Sec. IV B) */

/* ---- force precision (pamd_path.precision) ---- */
#define PAMD_FP64 0               /* all arithmetic in float64 */
#define PAMD_FP32_FORCE 1         /* LJ pair products of the Hessian-vector pass in float32: each
                                     pair's term a w + b (d.w) d is formed in float32 before it is
                                     summed in float64.  The pair functions of Eq. 16 (whose r^-12
                                     powers would amplify float32 rounding twelvefold), the force
                                     pass, displacements, cutoff test, sums, residuals, actions and
                                     gradients stay float64, so the action equals the float64 one
                                     and the gradient is within 1e-8 of it.  Harmonic paths ignore
                                     this. */

/* ---- algorithm choice (pamd_tuning.algo) ---- */
#define PAMD_ALGO_AUTO 0          /* fused */
#define PAMD_ALGO_FUSED 1         /* one pass per time tile: neighbour list, force, residual,
                                     action, Hessian-vector product and gradient on chip */
#define PAMD_ALGO_PLAIN 2         /* unfused reference form: per-slice cell list, then separate
                                     force, residual, Hessian-vector and gradient kernels with
                                     every intermediate in device memory */

/* Potential.  kind = PAMD_HARMONIC uses k; kind = PAMD_LJ uses eps, sigma,
 * rc and box (Eq. 16 with epsilon = eps, sigma = sigma, r_c = rc; periodic
 * cubic box of edge `box`, minimum-image convention, pair included when
 * r^2 <= rc^2).  Requirements: LJ: eps, sigma > 0, 0 < rc <= box/2, n_dim = 3.
 * Harmonic: box must be 0 (no periodic boundaries). */
typedef struct pamd_potential {
  int32_t kind;
  int32_t reserved0;
  double k;
  double eps;
  double sigma;
  double rc;
  double box;
} pamd_potential;

/* Path description (Eqs. 1-4).  n_steps = N >= 1 (the path holds N + 1
 * slices), n_atoms >= 1 (at most 65535 for LJ), n_dim in {1, 3}, dt > 0,
 * D > 0 (diffusion coefficient), gamma > 0 (friction; the Einstein relation
 * of Eq. 1, D = 1/(beta gamma), is the caller's to apply). */
typedef struct pamd_path {
  int64_t n_steps;
  int32_t n_atoms;
  int32_t n_dim;
  double dt;
  double D;
  double gamma;
  int32_t precision;
  int32_t reserved0;
} pamd_path;

/* ---- neighbour-list kind (pamd_tuning.neighbour_list) ---- */
#define PAMD_LIST_AUTO 0          /* library choice (currently full) */
#define PAMD_LIST_FULL 1          /* every atom lists all partners; fixed summation order,
                                     results bitwise repeatable run to run */
#define PAMD_LIST_HALF 2          /* every pair listed once; partner shares added with LDS
                                     float64 atomics: half the pair arithmetic, summation order
                                     (and so the last bits) may vary run to run */

/* Optional launch tuning; pass NULL (or a zeroed struct) for the library's
 * choice (the autotune cache when an entry exists, else built-in defaults).
 * Fields equal to 0 (skin <= 0) are chosen by the library.
 *   block          threads per workgroup, multiple of 64 in [64, 1024]
 *   tile           time steps per workgroup tile (fused)
 *   skin           neighbour-list skin in length units (fused): a list built
 *                  with radius rc + skin is reused while no atom has moved
 *                  more than skin/2 from where the list was built
 *   max_neighbours capacity of each atom's list; an atom whose list would
 *                  overflow falls back to a scan over all atoms (still exact)
 *   neighbour_list PAMD_LIST_* (fused); half lists need n_atoms <= 2 * block
 *   slot_arrays    LDS copies of the slice (fused): 2 = the next slice loads
 *                  into a second array while the current one is in use (the
 *                  per-slice lists of partners within r_c then live in device
 *                  memory), 1 = one array, which leaves room to keep those
 *                  lists in LDS when n_atoms <= block (else less shared memory
 *                  per workgroup), 0 = the library's choice (1 where the lists
 *                  fit in LDS, else 2) */
typedef struct pamd_tuning {
  int32_t algo;
  int32_t block;
  int32_t tile;
  int32_t max_neighbours;
  double skin;
  int32_t neighbour_list;
  int32_t slot_arrays;
} pamd_tuning;

/* Bytes of workspace needed by pamd_action / pamd_action_grad /
 * pamd_excess_action for this problem and tuning.  Host-only; no device
 * is touched. */
int pamd_workspace_size(const pamd_path* path, const pamd_potential* pot,
                        const pamd_tuning* tuning, size_t* bytes);

/* The launch the library would use for this problem and tuning (host-only;
 * no device is touched): the planner's choices, for callers that need to
 * know the time tiling (tests of tile edges, work accounting).  Fields that
 * do not apply are 0 (the harmonic kernel has no tiles, cells or lists). */
typedef struct pamd_launch {
  int32_t algo;             /* PAMD_ALGO_FUSED or PAMD_ALGO_PLAIN (Lennard-Jones), 0 (harmonic) */
  int32_t block;            /* threads per workgroup */
  int32_t tile;             /* time steps per workgroup tile (fused) */
  int32_t n_tiles;          /* ceil(n_steps / tile) */
  int32_t grid;             /* workgroups launched (tiles are taken in a grid-stride loop) */
  int32_t cells;            /* cells per axis of the list build (0: all pairs) */
  int32_t reach;            /* stencil half-width in cells; -1 (with cells 0): no lists,
                               both passes scan all atoms (a system whose list sphere
                               holds most of the box, tiles of one or two steps, default
                               list capacity and skin) */
  int32_t max_neighbours;   /* list capacity per atom */
  int32_t neighbour_list;   /* PAMD_LIST_FULL or PAMD_LIST_HALF */
  int32_t lds_bytes;        /* shared memory per workgroup */
  int32_t slot_arrays;      /* residual slot arrays in LDS: 1 or 2 (0: residuals in device memory) */
  int32_t exact_lists;      /* 1: each atom's partners within the cutoff, found in the force
                               pass, stay in LDS for the Hessian-vector pass (fused, full lists) */
  double skin;              /* list skin in length units */
} pamd_launch;

int pamd_launch_info(const pamd_path* path, const pamd_potential* pot, const pamd_tuning* tuning,
                     pamd_launch* out);

/* Action S[X] (Eq. 4 without normalisation).
 *   x         device, (N+1) * n_dim * n_atoms float64, layout above
 *   action    device, 1 float64 (written)
 *   per_step  device, N float64 (written: s_n), or NULL */
int pamd_action(const pamd_path* path, const pamd_potential* pot, const pamd_tuning* tuning,
                const double* x, double* action, double* per_step,
                void* ws, size_t ws_bytes, void* stream);

/* Action and its gradient with respect to every slice (including the
 * fixed x_0; callers that hold slices fixed mask them).
 *   step_weights device, N float64, or NULL (= all ones): the gradient is
 *                that of sum_n w_n s_n; action and per_step stay unweighted
 *   action       device, 1 float64, or NULL
 *   per_step     device, N float64, or NULL
 *   grad         device, same shape as x (written) */
int pamd_action_grad(const pamd_path* path, const pamd_potential* pot, const pamd_tuning* tuning,
                     const double* x, const double* step_weights,
                     double* action, double* per_step, double* grad,
                     void* ws, size_t ws_bytes, void* stream);

/* Action and gradient for callers that cannot allocate: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  Same
 * arguments, results and errors as pamd_action_grad except that there is no
 * workspace: the scratch lives in a static device array of
 * PAMD_NOALLOC_SCRATCH_BYTES bytes that the library holds on every device it
 * runs on until the process ends (nothing is allocated or freed per call).
 * The caller still passes x, grad and the optional outputs.  When the usual
 * plan's workspace is larger, the call runs the same kernels on fewer
 * concurrent workgroups (same results, more time); a problem whose scratch
 * cannot fit even so (e.g. very many steps of a large system) fails with
 * PAMD_EWORKSPACE before any device work.  Every call on one device shares
 * that device's array: calls that overlap in time on one device (two streams,
 * two threads) race and must not be issued; calls in stream order are fine.
 * No scratch contents need to start at zero, and none survive a call in any
 * meaningful way. */
#define PAMD_NOALLOC_SCRATCH_BYTES (128ull << 20)
int pamd_action_grad_noalloc(const pamd_path* path, const pamd_potential* pot,
                             const pamd_tuning* tuning, const double* x,
                             const double* step_weights, double* action, double* per_step,
                             double* grad, void* stream);

/* Per-step excess action e_n = s_n - s0_n, where s0_n = |Delta_n|^2/(4 D dt)
 * is the force-free (free-particle) term: the quantity the fragment-wise
 * Metropolis-Hastings test needs (Sec. III).  e_n is evaluated as
 * sum (r - Delta)(r + Delta) / (4 D dt) to avoid cancellation.
 *   excess    device, N float64 (written)
 *   per_step  device, N float64 (written: s_n) or NULL */
int pamd_excess_action(const pamd_path* path, const pamd_potential* pot, const pamd_tuning* tuning,
                       const double* x, double* excess, double* per_step,
                       void* ws, size_t ws_bytes, void* stream);

/* Normalisation omitted from S: N * (n_dim * n_atoms / 2) * ln(4 pi D dt), so
 * that -ln prod_n K(x_{n+1}|x_n; dt) = S + pamd_log_norm(path) (Eq. 3 with its
 * Gaussian normalisation).  Returns NaN for an invalid path. */
double pamd_log_norm(const pamd_path* path);

/* Message of the calling thread's last failed call ("" if none). */
const char* pamd_last_error(void);

/* Library version string. */
const char* pamd_version(void);

/* ------------------------------------------------------------------------
 * Batches: many independent paths (different N, n_atoms, dt, potential) in
 * one persistent launch for all Lennard-Jones members plus one launch per
 * harmonic member (Eq. 4 evaluated for each path, as pamd_action_grad does
 * for one).  The work list holds every (path, time tile) pair, largest first;
 * workgroups take items from it until it is empty.  All members must share
 * one precision.  Each Lennard-Jones member's time tile holds about the same
 * work (tile = 16384 / n_atoms steps, within [4, 128], by default); the batch
 * autotuner below picks that budget and the list skin by timing the launch.
 *
 * Two forms:
 *   - pamd_batch_action_grad: the paths' own device buffers, passed as host
 *     arrays of device pointers.  Plans, uploads the work list into `ws` and
 *     synchronises `stream` before it launches, so it cannot be captured
 *     into a graph.
 *   - a batch handle (pamd_batch_create / _layout / _prepare / _run): the
 *     paths packed into one device array; the work list is uploaded once
 *     (pamd_batch_prepare), after which pamd_batch_run only enqueues kernels
 *     and can be captured and replayed (pamd_graph_*).
 * ---------------------------------------------------------------------- */

/* Workspace bytes of pamd_batch_action_grad for these paths (host-only). */
int pamd_batch_workspace_size(int32_t n_paths, const pamd_path* paths /* host, n_paths */,
                              const pamd_potential* pots /* host, n_paths */, size_t* bytes);

/* Actions and gradients of n_paths independent paths.
 *   paths, pots  host arrays of n_paths descriptors (validated as by pamd_action_grad)
 *   x            host array of n_paths device pointers: path p, layout as for one path
 *   actions      device, n_paths float64 (written: S of each path)
 *   grads        host array of n_paths device pointers (gradient p, same shape as x[p],
 *                written), or NULL for actions only; an entry may be NULL to skip
 *                that path's gradient
 *   ws           device workspace of pamd_batch_workspace_size bytes
 * Buffers of different paths must not overlap. */
int pamd_batch_action_grad(int32_t n_paths, const pamd_path* paths, const pamd_potential* pots,
                           const double* const* x, double* actions, double* const* grads,
                           void* ws, size_t ws_bytes, void* stream);

typedef struct pamd_batch pamd_batch;

int pamd_batch_create(int32_t n_paths, const pamd_path* paths /* host, n_paths */,
                      const pamd_potential* pots /* host, n_paths */,
                      const pamd_tuning* tuning, pamd_batch** out);
void pamd_batch_destroy(pamd_batch* batch);

/* Packed layout: member p's path starts at element x_offsets[p] of one device
 * array (offsets are multiples of 32 elements) and the same offsets index the
 * packed gradient; per-step arrays are packed at step_offsets[p].  x_offsets
 * and step_offsets are host arrays of n_paths + 1 int64 (the last entry is the
 * total), either may be NULL.  ws_bytes gets the workspace size. */
int pamd_batch_layout(const pamd_batch* batch, int64_t* x_offsets, int64_t* step_offsets,
                      size_t* ws_bytes);

/* Uploads the batch's work list into `ws` (one host-to-device copy, then a
 * stream synchronisation).  Call once per workspace before pamd_batch_run,
 * outside any graph capture; the workspace then stays valid for any number of
 * calls on this batch. */
int pamd_batch_prepare(const pamd_batch* batch, void* ws, size_t ws_bytes, void* stream);

/* Batch autotuning: times the prepared launch (pamd_batch_run on x_all, with
 * gradients into grad_all, which may be NULL) for each candidate member-tile
 * policy (tile = budget / n_atoms steps, within [4, 128], for budgets 2^13 ..
 * 2^18 atom-steps,
 * list skin 0.3 or 0.5 sigma; fields the batch's tuning fixes are kept) and
 * re-plans the batch with the fastest; when it fits `ws`, also prepares it
 * (else call pamd_batch_layout for the new size and pamd_batch_prepare).
 * Candidates whose workspace exceeds ws_bytes are skipped;
 * pamd_batch_autotune_workspace_size gives the size that admits them all.
 * Synchronises the stream; not capturable.  tile_budget and skin_frac (host,
 * may be NULL) receive the choice. */
int pamd_batch_autotune_workspace_size(pamd_batch* batch, size_t* bytes);
int pamd_batch_autotune(pamd_batch* batch, const double* x_all, double* grad_all, void* ws,
                        size_t ws_bytes, void* stream, double* tile_budget, double* skin_frac);

/* Actions (and gradients) of every member of a prepared batch.
 *   x_all        device, packed paths
 *   weights_all  device, packed per-step weights, or NULL (= all ones)
 *   actions      device, n_paths float64 (written)
 *   per_step_all device, packed per-step actions, or NULL
 *   grad_all     device, packed gradients, or NULL for actions only */
int pamd_batch_run(const pamd_batch* batch, const double* x_all, const double* weights_all,
                   double* actions, double* per_step_all, double* grad_all, void* ws,
                   size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Path sampling (Sec. III): one Monte Carlo step of the multilevel sliding-
 * and-sampling move with free-particle trial paths.
 *   1. level l uniform in [l_min, l_max], offset u uniform in [1, 2^l];
 *      fragment endpoints u, u + 2^l, ... <= N; the tail fragment is [0, u],
 *      internal fragments span 2^l steps, a nose fragment [e_last, N] exists
 *      when e_last < N (random fragmentation, Fig. 5);
 *   2. every fragment draws a free-particle trial with its endpoints fixed
 *      (Brownian bridge, per-step variance 2 D dt; the nose fragment continues
 *      freely and also moves x_N); x_0 never moves;
 *   3. fragment f is accepted when u_f < exp(-Delta_f),
 *      Delta_f = sum_{n in f} (e'_n - e_n), e = excess action (see
 *      pamd_excess_action), primes for the trial path;
 *   4. accepted fragments are copied into x and their e_n into `excess`.
 * Random numbers: Philox4x32-10 with key (seed mod 2^32, seed >> 32):
 *   level/offset    counter (0, 0, s, 1): l = l_min + w0 mod (l_max - l_min + 1),
 *                   u = 1 + w1 mod 2^l
 *   accept uniform  counter (f, 0, s, 2): ((w0 >> 6) 2^26 + (w1 >> 6) + 1/2) 2^-52
 *   trial normal    counter (p mod 2^32, p >> 32, s, 3), p = e >> 1 for flat element
 *                   index e = n * n_dim * n_atoms + k; Box-Muller of the two
 *                   uniforms (w0,w1), (w2,w3); even e takes the cosine output,
 *                   odd e the sine output
 * where s is the sweep index read from *sweep_counter (device int64), which
 * the call increments, so a captured graph replays successive sweeps.
 * ---------------------------------------------------------------------- */
int pamd_mh_workspace_size(const pamd_path* path, const pamd_potential* pot,
                           const pamd_tuning* tuning, size_t* bytes);

/*   x             device path (read and updated in place)
 *   excess        device, N float64: e_n of x on entry, updated on exit
 *   trial         device scratch, same shape as x (holds the trial path on exit)
 *   frag_delta    device, N + 2 float64 (Delta_f by fragment), or NULL
 *   frag_accept   device, N + 2 int32 (1 accepted, 0 rejected), or NULL
 *   step_info     device, 4 int32 {l, u, n_fragments, n_accepted}, or NULL
 *   requires 1 <= l_min <= l_max and 2^l_max <= N. */
int pamd_mh_step(const pamd_path* path, const pamd_potential* pot, const pamd_tuning* tuning,
                 uint64_t seed, int32_t l_min, int32_t l_max, int64_t* sweep_counter,
                 double* x, double* excess, double* trial,
                 double* frag_delta, int32_t* frag_accept, int32_t* step_info,
                 void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Path-based integration (Sec. II B, Figs. 1-2): sample the path, shift it
 * along itself, regrow it, repeat.
 *
 * pamd_shift performs one shifting event (Fig. 2B) with s = n_shift:
 *     x_out[n] = x_in[n + s]                      n = 0 .. N - s
 *     x_out[n] = x_out[n - 1] + sqrt(2 D dt) z_n   n = N - s + 1 .. N
 * (regrowth by free Brownian continuation, the trial distribution of Sec. III),
 * excess_out[n] = excess_in[n + s] for n < N - s (the last s entries are left
 * for the caller: pamd_excess_action on the sub-path x_out + (N - s) slices
 * with n_steps = s gives them), and traj_out (if not NULL) receives
 * x_in[1 .. s], the slices that join the integrated trajectory.
 * z_n: Philox4x32-10 with key (seed mod 2^32, seed >> 32), counter
 * (p mod 2^32, p >> 32, v, 4) with p = e >> 1 for flat element index
 * e = n * n_dim * n_atoms + k of x_out, Box-Muller as for trial normals, and v
 * read from *event_counter (device int64), which the call increments.
 *   x_in, x_out         device paths, must not overlap
 *   excess_in/out       device, N float64 each, both or neither, must not overlap
 *   traj_out            device, n_shift * n_dim * n_atoms float64, or NULL; must not
 *                       overlap x_in or x_out
 *   requires 1 <= n_shift <= N.
 * ---------------------------------------------------------------------- */
int pamd_shift(const pamd_path* path, uint64_t seed, int32_t n_shift, int64_t* event_counter,
               const double* x_in, double* x_out, const double* excess_in, double* excess_out,
               double* traj_out, void* stream);

/* The integration loop: n_events shifting events, each preceded by n_sample
 * Monte Carlo steps (pamd_mh_step with levels l_min..l_max), with the
 * regrown steps' excess evaluated after every shift.  x and excess hold the
 * path and its excess on entry and on exit; x_alt, excess_alt and trial are
 * scratch of the same sizes (the path moves between x and x_alt from event
 * to event).  counters (device int64[2]) = {sweep, event}, both advanced.
 * traj_out (device, n_events * n_shift slices, or NULL) receives the
 * integrated trajectory, x_1 .. x_{n_shift} of every event in time order.
 * level_stats (device uint64[62], or NULL) accumulates, for each level l,
 * the fragments proposed ([2 l]) and accepted ([2 l + 1]); the caller clears it.
 * Workspace: pamd_run_workspace_size.  Enqueues kernels only. */
int pamd_run_workspace_size(const pamd_path* path, const pamd_potential* pot,
                            const pamd_tuning* tuning, int32_t n_shift, size_t* bytes);
int pamd_run(const pamd_path* path, const pamd_potential* pot, const pamd_tuning* tuning,
             uint64_t seed, int32_t l_min, int32_t l_max, int32_t n_sample, int32_t n_shift,
             int32_t n_events, int64_t* counters, double* x, double* x_alt, double* trial,
             double* excess, double* excess_alt, double* traj_out, uint64_t* level_stats,
             void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Gradient-informed path move (an extension: the paper's moves, Sec. III, use
 * no gradient).  One Metropolis-adjusted Langevin step in path space targeting
 * exp(-S[X]) of Eq. 4 with x_0 fixed, using the adjoint gradient:
 *     y = x - tau g(x) + sqrt(2 tau) z    (slices 1..N; y_0 = x_0)
 *     log alpha = S(x) - S(y) + (|y - x + tau g(x)|^2 - |x - y + tau g(y)|^2) / (4 tau)
 * and y replaces x when u < exp(log alpha).  z: Philox4x32-10 counter
 * (p mod 2^32, p >> 32, t, 5), p = e >> 1 over flat element indices e of the
 * path, Box-Muller as for trial normals; u: counter (0, 0, t, 6) ->
 * uniform52(w0, w1); t read from *move_counter (device int64), which the call
 * increments.  The sums run in a fixed order.
 *   x, grad, action  device state: the path, dS/dx and S (action: 1 float64);
 *                    the caller initialises grad and action with
 *                    pamd_action_grad(x); on acceptance all three are updated
 *   y, grad_y        device scratch, path-sized (the proposal and its gradient)
 *   accepted         device int32 (1 accepted, 0 rejected), or NULL
 *   log_alpha        device float64, or NULL
 *   x, grad, y and grad_y must not overlap; tau > 0.
 * Workspace: pamd_langevin_workspace_size.
 * ---------------------------------------------------------------------- */
int pamd_langevin_workspace_size(const pamd_path* path, const pamd_potential* pot,
                                 const pamd_tuning* tuning, size_t* bytes);
int pamd_langevin_step(const pamd_path* path, const pamd_potential* pot,
                       const pamd_tuning* tuning, uint64_t seed, double tau,
                       int64_t* move_counter, double* x, double* grad, double* action,
                       double* y, double* grad_y, int32_t* accepted, double* log_alpha,
                       void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Sequential Euler-Maruyama integration (Eq. 2, Sec. II A): the time-stepping
 * baseline that path sampling parallelises.  Steps
 *     x_{n+1} = x_n + (dt / gamma) F(x_n) + sqrt(2 D dt) xi_n,   n = 0..N-1,
 * in order, with the same forces (and, for Lennard-Jones, the same cell and
 * neighbour lists) as the action kernels; coordinates stay unwrapped.  The
 * action of the resulting path is sum_n |xi_n|^2 / 2 up to rounding.
 * Lennard-Jones systems run as one workgroup stepping all atoms (float64
 * forces, full neighbour lists: PAMD_FP32_FORCE, PAMD_LIST_HALF and
 * PAMD_ALGO_PLAIN are rejected with PAMD_EUNSUPPORTED); harmonic systems run
 * one thread per degree of freedom.  tuning->block and tuning->skin apply;
 * tile and max_neighbours as for a one-step path.
 * ---------------------------------------------------------------------- */
int pamd_em_workspace_size(const pamd_path* path, const pamd_potential* pot,
                           const pamd_tuning* tuning, size_t* bytes);

/*   x0     device, n_dim * n_atoms float64: the first slice, layout of one slice
 *   noise  device, N * n_dim * n_atoms float64: xi_n, layout of slices 0..N-1
 *   x_out  device, (N + 1) * n_dim * n_atoms float64 (written: x_0 .. x_N);
 *          must not overlap noise (x0 may be x_out's first slice) */
int pamd_em_integrate(const pamd_path* path, const pamd_potential* pot,
                      const pamd_tuning* tuning, const double* x0, const double* noise,
                      double* x_out, void* ws, size_t ws_bytes, void* stream);

/* ------------------------------------------------------------------------
 * Autotuning: times candidate (block, tile, skin, list kind, slot arrays)
 * choices for this problem on the given inputs, the library's own choices
 * among them, and caches the fastest for later calls whose
 * key matches: potential kind, n_atoms, precision, floor(log2 n_steps), and
 * for Lennard-Jones the box edge and cutoff.  Single-path calls and batch
 * members made after it (pamd_batch_create) take their launch from the cache
 * when no tuning field overrides it.  Synchronises the stream.  `best` (host,
 * may be NULL) receives the choice.
 * ---------------------------------------------------------------------- */
int pamd_autotune(const pamd_path* path, const pamd_potential* pot, const double* x,
                  double* grad_scratch, void* ws, size_t ws_bytes, void* stream,
                  pamd_tuning* best);

/* ------------------------------------------------------------------------
 * Measurement hook: the next action evaluation or integration enqueued by
 * this thread records `start` (a hipEvent_t) on its stream just before its
 * main kernel and `stop` just after it, so that the events bracket that kernel
 * alone: pamd_action, pamd_action_grad, pamd_excess_action and
 * pamd_em_integrate bracket their own kernel; pamd_mh_step, pamd_run and
 * pamd_langevin_step bracket their first action evaluation.  Host-only; pass
 * NULLs to clear.
 * ---------------------------------------------------------------------- */
int pamd_profile_events(void* start, void* stop);

/* ------------------------------------------------------------------------
 * HIP graph helpers: capture any sequence of pamd_* calls enqueued on
 * `stream` between begin and end, then replay it.
 * ---------------------------------------------------------------------- */
typedef struct pamd_graph pamd_graph;
int pamd_graph_begin(void* stream);
int pamd_graph_end(void* stream, pamd_graph** out);
int pamd_graph_launch(const pamd_graph* graph, void* stream);
void pamd_graph_destroy(pamd_graph* graph);

#ifdef __cplusplus
}
#endif
#endif /* PAMD_H */
