"""Pins of the oracle's Philox generator, fragmentation, trial paths and MH step (Sec. III)."""
import math
import os

import numpy as np

from oracle import action as A
from oracle import philox as P
from oracle import sampling as MC
from oracle.potentials import Harmonic, LennardJones

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_philox_known_answers():
    for line in open(os.path.join(GOLDEN, "philox_kat.txt")):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(t, 16) for t in line.split()]
        out = P.philox4x32_10(tuple(v[0:4]), tuple(v[4:6]))
        assert [int(o) for o in out] == v[6:10]


def test_uniform_and_normal_moments():
    u = P.uniform52(np.arange(1000, dtype=np.uint64) * 4294967, np.arange(1000, dtype=np.uint64))
    assert np.all((u > 0) & (u < 1))
    assert P.uniform52(0, 0) == 0.5 * 2.0 ** -52
    assert P.uniform52(0xFFFFFFFF, 0xFFFFFFFF) < 1.0
    z = P.trial_normals(1234, 7, 200000)
    assert abs(z.mean()) < 4.5 / math.sqrt(z.size)
    assert abs(z.var() - 1) < 4.5 * math.sqrt(2.0 / z.size)
    # first and second halves of the flat index come from the same words pairwise
    z2 = P.trial_normals(1234, 7, 10, first=100)
    assert np.array_equal(z2, z[100:110])


def test_fragments_cover_path():
    for n_steps, level in [(16, 2), (16, 3), (64, 4), (40, 3)]:
        span = 1 << level
        for off in range(1, span + 1):
            fr = MC.fragments(n_steps, level, off)
            assert fr[0][0] == 0 and fr[-1][1] == n_steps
            for (a, b, _), (c, d, _) in zip(fr, fr[1:]):
                assert b == c
            assert fr[0][1] == off
            for a, b, nose in fr[1:]:
                if not nose:
                    assert b - a == span
            if n_steps % span == 0:
                tail = fr[0][1] - fr[0][0]
                nose = (fr[-1][1] - fr[-1][0]) if fr[-1][2] else 0
                if off < span:
                    assert tail + nose == span
            assert sum(1 for f in fr if f[2]) <= 1


def test_bridge_moments():
    # Brownian bridge from 0 to B over m steps: mean k B / m, variance s^2 k (m-k)/m.
    D, dt, m, B = 0.5, 0.1, 8, 1.3
    n_dof = 40000
    X = np.zeros((m + 1, 1, n_dof))
    X[m] = B
    z = np.random.default_rng(5).standard_normal(X.shape)
    Y = MC.trial_path(X, [(0, m, False)], z, D, dt)
    s2 = 2 * D * dt
    for k in range(1, m):
        mean, var = k * B / m, s2 * k * (m - k) / m
        assert abs(Y[k].mean() - mean) / math.sqrt(var / n_dof) < 4.5
        assert abs(Y[k].var() - var) / (var * math.sqrt(2.0 / n_dof)) < 4.5
    assert np.all(Y[0] == 0) and np.all(Y[m] == B)
    # free continuation: variance grows as s^2 k
    Yn = MC.trial_path(X, [(0, m, True)], z, D, dt)
    assert abs(Yn[m].var() - s2 * m) / (s2 * m * math.sqrt(2.0 / n_dof)) < 4.5


def test_free_particle_trials_always_accepted():
    # With V = 0 the target equals the proposal: Delta_f = 0 for every fragment.
    ho = Harmonic(k=0.0)
    X = np.cumsum(np.random.default_rng(1).standard_normal((33, 1, 3)) * 0.1, axis=0)
    out = MC.mh_step(X, ho, 0.01, 1.0, 1.0, seed=77, sweep=3, l_min=2, l_max=4)
    assert np.max(np.abs(out["delta"])) < 1e-9
    assert out["accepted"].all()


def test_mh_stationary_moments_harmonic():
    # e^{-S} for the harmonic path with x_0 fixed is the AR(1) law of the EM chain
    # (mean a^n x_0, variance 2 D dt (1 - a^{2n})/(1 - a^2)).  Independent chains give
    # independent time averages, so a t-statistic across chains needs no
    # autocorrelation model.
    k, dt, D, gamma = 1.0, 0.4, 1.0, 1.0
    n_steps, x0, n_chain, n_sweep, burn = 8, 1.0, 8, 1700, 200
    ho = Harmonic(k=k)
    a = 1 - k * dt / gamma
    s2 = 2 * D * dt
    m1, m2 = [], []
    for c in range(n_chain):
        X = np.full((n_steps + 1, 1, 1), x0)
        samples = []
        for sweep in range(n_sweep):
            X = MC.mh_step(X, ho, dt, D, gamma, seed=100 + c, sweep=sweep, l_min=1, l_max=2)["path"]
            if sweep >= burn:
                samples.append(X[:, 0, 0].copy())
        S = np.array(samples)
        m1.append(S.mean(axis=0))
        m2.append((S * S).mean(axis=0))
    m1, m2 = np.array(m1), np.array(m2)
    for n in range(1, n_steps + 1):
        mean = a ** n * x0
        second = s2 * (1 - a ** (2 * n)) / (1 - a ** 2) + mean ** 2
        t1 = (m1[:, n].mean() - mean) / (m1[:, n].std(ddof=1) / math.sqrt(n_chain))
        t2 = (m2[:, n].mean() - second) / (m2[:, n].std(ddof=1) / math.sqrt(n_chain))
        assert abs(t1) < 6.0 and abs(t2) < 6.0, (n, t1, t2)


def test_mh_step_bookkeeping_lj():
    from oracle import em as E
    import workloads as W
    w = W.workload("lj108").with_atoms(32).with_steps(16)
    lj = LennardJones(rc=0.499 * w.box, box=w.box)
    x0 = W.initial_lattice(32, w.box)
    xi, _ = W.draw_noise(w, 16)
    X = E.em_path(x0, xi, lj, w.dt, w.D, w.gamma)
    out = MC.mh_step(X, lj, w.dt, w.D, w.gamma, seed=5, sweep=0, l_min=2, l_max=3)
    Xn = out["path"]
    assert np.array_equal(Xn[0], X[0])
    for (a, b, nose), acc in zip(out["fragments"], out["accepted"]):
        hi = b + 1 if nose else b
        src = out["trial"] if acc else X
        assert np.array_equal(Xn[a + 1:hi], src[a + 1:hi])
        if not nose:
            assert np.array_equal(Xn[b], X[b])
    s_chk = A.per_step_action(out["trial"], lj, w.dt, w.D, w.gamma)
    assert np.allclose(s_chk, out["s_new"], rtol=1e-14, atol=0)
