"""GPU parity of the path-based integration loop (Sec. II B, Figs. 1-2).

* pamd_shift against the oracle's shift_path with the same regrowth
  variates: moved slices, excess terms and trajectory bit-exact; regrown
  slices within 1e-12 (Box-Muller's log/sin/cos on the two sides differ by
  a few ulps per variate, summed over the regrown steps);
* pamd_run against the oracle's loop (same Philox streams, so the same
  levels, offsets, trial paths and accept decisions) for a harmonic path and
  for the paper's 27-atom Lennard-Jones system: trajectories within 1e-10;
* the law of the emitted trajectory on the GPU alone: at dt = 0.4 the Euler
  chain of the harmonic oscillator has variance 1.25 and lag-1
  autocorrelation 0.6 (Eq. 2), which converged path sampling reproduces.
"""
import dataclasses
import math

import numpy as np
import pytest
import torch

import paper_1907_09529_amd as P
import workloads as W
from oracle import em as OE
from oracle import pamd as OP

from common import lib_descriptors, oracle_pot

pytestmark = pytest.mark.gpu


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_shift_matches_oracle(device):
    rng = np.random.default_rng(5)
    n_steps, n_shift, seed = 32, 5, 77
    path = P.make_path(n_steps, 5, 3, 0.01, 1.0, 1.0)
    X = rng.standard_normal((n_steps + 1, 3, 5))
    ex = rng.standard_normal(n_steps)
    x_in, ex_in = dev(X), dev(ex)
    x_out = torch.full_like(x_in, np.nan)
    ex_out = torch.full_like(ex_in, np.nan)
    traj = torch.empty((n_shift, 3, 5), dtype=torch.float64, device="cuda")
    counter = torch.tensor([9], dtype=torch.int64, device="cuda")
    P.pamd_shift(path, seed, n_shift, counter, x_in, x_out, ex_in, ex_out, traj)
    torch.cuda.synchronize()
    Y = x_out.cpu().numpy()
    keep = n_steps - n_shift
    ref = OP.shift_path(X, n_shift, OP.regrowth_normals(seed, 9, X.shape, n_shift), 1.0, 0.01)
    assert np.array_equal(Y[:keep + 1], X[n_shift:])
    assert np.max(np.abs(Y - ref)) <= 1e-12
    assert np.array_equal(traj.cpu().numpy(), X[1:n_shift + 1])
    e = ex_out.cpu().numpy()
    assert np.array_equal(e[:keep], ex[n_shift:])
    assert np.all(np.isnan(e[keep:]))        # left for the caller
    assert int(counter.item()) == 10


def run_gpu(w, X, seed, l_min, l_max, n_sample, n_shift, n_events, stats=None):
    path, pot = lib_descriptors(w)
    x = dev(X)
    ex = torch.empty(w.n_steps, dtype=torch.float64, device="cuda")
    P.pamd_excess_action(path, pot, x, ex)
    counters = torch.zeros(2, dtype=torch.int64, device="cuda")
    traj = torch.empty((n_events * n_shift,) + X.shape[1:], dtype=torch.float64, device="cuda")
    P.pamd_run(path, pot, seed, l_min, l_max, n_sample, n_shift, n_events, counters, x,
               torch.empty_like(x), torch.empty_like(x), ex, torch.empty_like(ex), traj,
               level_stats=stats)
    torch.cuda.synchronize()
    return traj.cpu().numpy(), x, ex, counters.cpu().numpy()


def check_final_excess(w, x, ex):
    path, pot = lib_descriptors(w)
    fresh = torch.empty_like(ex)
    P.pamd_excess_action(path, pot, x, fresh)
    torch.cuda.synchronize()
    a, b = ex.cpu().numpy(), fresh.cpu().numpy()
    assert np.max(np.abs(a - b)) <= 1e-10 * max(1.0, np.max(np.abs(b)))


def test_run_matches_oracle_harmonic(device):
    w = dataclasses.replace(W.workload("ho1d"), n_steps=16, dt=0.4)
    rng = np.random.default_rng(8)
    X = np.zeros((17, 1, 1))
    for n in range(16):
        X[n + 1] = 0.6 * X[n] + math.sqrt(0.8) * rng.standard_normal()
    T, x, ex, counters = run_gpu(w, X, 31, 3, 3, 2, 2, 20)
    T_ref, X_ref = OP.run(X, oracle_pot(w), w.dt, w.D, w.gamma, 31, 3, 3, 2, 2, 20)
    assert np.max(np.abs(T - T_ref)) <= 1e-10
    assert np.max(np.abs(x.cpu().numpy() - X_ref)) <= 1e-10
    assert list(counters) == [40, 20]
    check_final_excess(w, x, ex)


def test_run_matches_oracle_lj27(device):
    """The paper's Lennard-Jones system (27 atoms, rho 0.5, r_c = L/2): a
    32-step path integrated by Euler-Maruyama, then six events of one sweep
    (levels 2..4) and a shift of 4."""
    w = W.workload("lj27").with_steps(32)
    x0 = W.initial_lattice(w.n_atoms, w.box)
    xi, _ = W.draw_noise(w)
    X = OE.em_path(x0, xi, oracle_pot(w), w.dt, w.D, w.gamma)
    stats = torch.zeros(62, dtype=torch.int64, device="cuda")
    T, x, ex, _ = run_gpu(w, X, 5, 2, 4, 1, 4, 6, stats)
    ref_stats = np.zeros(62, dtype=np.int64)
    T_ref, X_ref = OP.run(X, oracle_pot(w), w.dt, w.D, w.gamma, 5, 2, 4, 1, 4, 6,
                          level_stats=ref_stats)
    assert np.max(np.abs(T - T_ref)) <= 1e-10 * w.box
    assert np.max(np.abs(x.cpu().numpy() - X_ref)) <= 1e-10 * w.box
    assert np.array_equal(stats.cpu().numpy(), ref_stats)      # same fragments, same decisions
    check_final_excess(w, x, ex)


def test_level_stats_free_particle(device):
    """V = 0: every proposed fragment is accepted; levels outside l_min..l_max
    see none; the counts match the oracle's fragmentations exactly."""
    w = dataclasses.replace(W.workload("ho1d"), n_steps=64, n_atoms=8, k=0.0, dt=0.05)
    X = np.cumsum(np.random.default_rng(2).standard_normal((65, 1, 8)) * math.sqrt(0.1), axis=0)
    stats = torch.zeros(62, dtype=torch.int64, device="cuda")
    run_gpu(w, X, 17, 2, 5, 3, 8, 10, stats)
    st = stats.cpu().numpy().reshape(31, 2)
    assert np.array_equal(st[:, 0], st[:, 1])
    assert st[2:6, 0].sum() == st[:, 0].sum() > 0
    ref = np.zeros(62, dtype=np.int64)
    OP.run(X, oracle_pot(w), w.dt, w.D, w.gamma, 17, 2, 5, 3, 8, 10, level_stats=ref)
    assert np.array_equal(stats.cpu().numpy(), ref)


def test_run_graph_replays_match_eager(device):
    """A captured two-event run replayed three times, with eager runs on a
    second set of buffers in between, matches them bit for bit each time."""
    w = W.workload("lj27").with_steps(64)
    x0 = W.initial_lattice(w.n_atoms, w.box)
    xi, _ = W.draw_noise(w)
    X = OE.em_path(x0, xi, oracle_pot(w), w.dt, w.D, w.gamma)
    path, pot = lib_descriptors(w)

    def buffers():
        x = dev(X)
        ex = torch.empty(w.n_steps, dtype=torch.float64, device="cuda")
        P.pamd_excess_action(path, pot, x, ex)
        return dict(counters=torch.zeros(2, dtype=torch.int64, device="cuda"), x=x,
                    x_alt=torch.empty_like(x), trial=torch.empty_like(x), excess=ex,
                    excess_alt=torch.empty_like(ex),
                    traj_out=torch.empty((8,) + X.shape[1:], dtype=torch.float64, device="cuda"),
                    level_stats=torch.zeros(62, dtype=torch.int64, device="cuda"))

    g_buf, e_buf = buffers(), buffers()
    ws = P.workspace(P.pamd_run_workspace_size(path, pot, 4))
    ws_e = P.workspace(P.pamd_run_workspace_size(path, pot, 4))
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = P.PamdGraph()
    with torch.cuda.stream(s):
        g.begin(s)
        P.pamd_run(path, pot, 9, 2, 4, 1, 4, 2, ws=ws, stream=s, **g_buf)
        g.end(s)
    try:
        for rep in range(3):
            with torch.cuda.stream(s):
                g.launch(s)
            s.synchronize()
            P.pamd_run(path, pot, 9, 2, 4, 1, 4, 2, ws=ws_e, **e_buf)
            torch.cuda.synchronize()
            for k in ("x", "excess", "traj_out", "counters", "level_stats"):
                assert torch.equal(g_buf[k], e_buf[k]), (rep, k)
    finally:
        g.close()


def test_run_harmonic_follows_the_euler_law(device):
    """20000 events of the paper's Simulation 1 schedule (N_path 16,
    N_sample = N_shift = 2, level 3) at dt = 0.4 from an exact start."""
    w = dataclasses.replace(W.workload("ho1d"), n_steps=16, dt=0.4)
    rng = np.random.default_rng(9)
    X = np.zeros((17, 1, 1))
    X[0] = rng.standard_normal() * math.sqrt(1.25)
    for n in range(16):
        X[n + 1] = 0.6 * X[n] + math.sqrt(0.8) * rng.standard_normal()
    T, x, ex, _ = run_gpu(w, X, 123, 3, 3, 2, 2, 20000)
    v = T[:, 0, 0]
    var = v.var()
    lag1 = np.mean(v[1:] * v[:-1]) / var
    # ~2e4 effective samples: sd(var) ~ 0.013, sd(lag1) ~ 0.006
    assert abs(var - 1.25) < 0.06, var
    assert abs(lag1 - 0.6) < 0.03, lag1
    check_final_excess(w, x, ex)


@pytest.mark.parametrize("n_sample,n_shift,n_events", [(0, 3, 5), (1, 16, 3), (2, 1, 4)])
def test_run_edge_schedules(device, n_sample, n_shift, n_events):
    """Shift-only events (no sampling), a shift of the whole path (the scheme
    of Fig. 1: every slice regrown) and single-step shifts."""
    w = dataclasses.replace(W.workload("ho1d"), n_steps=16, n_atoms=3, dt=0.4)
    X = exact_paths_ho(np.random.default_rng(12), 16, 3)
    T, x, ex, counters = run_gpu(w, X, 77, 2, 3, n_sample, n_shift, n_events)
    T_ref, X_ref = OP.run(X, oracle_pot(w), w.dt, w.D, w.gamma, 77, 2, 3, n_sample, n_shift,
                          n_events)
    assert np.max(np.abs(T - T_ref)) <= 1e-10
    assert np.max(np.abs(x.cpu().numpy() - X_ref)) <= 1e-10
    assert list(counters) == [n_sample * n_events, n_events]
    check_final_excess(w, x, ex)


def test_shift_without_excess_or_trajectory(device):
    path = P.make_path(8, 2, 1, 0.1, 1.0, 1.0)
    X = np.random.default_rng(3).standard_normal((9, 1, 2))
    x_in = dev(X)
    x_out = torch.empty_like(x_in)
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    P.pamd_shift(path, 5, 3, counter, x_in, x_out)
    torch.cuda.synchronize()
    ref = OP.shift_path(X, 3, OP.regrowth_normals(5, 0, X.shape, 3), 1.0, 0.1)
    assert np.max(np.abs(x_out.cpu().numpy() - ref)) <= 1e-12
    assert int(counter.item()) == 1


def exact_paths_ho(rng, n_steps, n_dof):
    X = np.zeros((n_steps + 1, 1, n_dof))
    for n in range(n_steps):
        X[n + 1] = 0.6 * X[n] + math.sqrt(0.8) * rng.standard_normal((1, n_dof))
    return X
