"""Pins of the oracle's path-based integration loop (Sec. II B, Figs. 1-2).

Both pins use the loop's defining property: if the path entering every
sampling stage is distributed as exp(-S) given x_0 (Eq. 4), and the sampler
preserves that law, the emitted trajectory is a realisation of the Euler
scheme (Eq. 2) at step dt.

* Free particle (V = 0): every trial is accepted (the excess action is 0),
  and from an exact Brownian start every path stays exactly Brownian, so the
  trajectory's increments are independent N(0, 2 D dt) variates.  Many
  independent degrees of freedom in one path make this a sharp test of the
  bridge, shift and regrowth bookkeeping.
* Harmonic oscillator at the paper's dt = 0.4 (k = gamma = D = 1): the Euler
  chain x_{n+1} = 0.6 x_n + sqrt(0.8) xi has stationary variance
  0.8 / (1 - 0.36) = 1.25 and lag-1 autocorrelation 0.6.  One degree of
  freedom (the sampler moves all degrees of freedom of a fragment together),
  the paper's Simulation 1 schedule (N_path 16, N_sample = N_shift = 2,
  level 3).
"""
import math

import numpy as np

from oracle import pamd as OP
from oracle.potentials import Harmonic


def free_start(rng, n_steps, n_dof, sig):
    steps = sig * rng.standard_normal((n_steps, 1, n_dof))
    X = np.zeros((n_steps + 1, 1, n_dof))
    X[1:] = np.cumsum(steps, axis=0)
    return X


def test_free_particle_trajectory_is_brownian():
    dt, D = 0.05, 1.0
    sig = math.sqrt(2 * D * dt)
    X = free_start(np.random.default_rng(11), 16, 2000, sig)
    T, Xf = OP.run(X, Harmonic(k=0.0), dt, D, 1.0, seed=21, l_min=1, l_max=4, n_sample=1,
                   n_shift=4, n_events=30)
    traj = np.concatenate([X[:1], T])[:, 0, :]          # x_0 then the emitted slices
    inc = np.diff(traj, axis=0) / sig                     # should be iid N(0, 1)
    assert T.shape == (120, 1, 2000)
    assert abs(inc.mean()) < 0.01
    assert abs(inc.var() - 1.0) < 0.015
    for lag in (1, 3, 4, 5):                              # 4 = one shifting event apart
        c = np.mean(inc[lag:] * inc[:-lag])
        assert abs(c) < 0.01, (lag, c)
    # the final path continues the trajectory
    np.testing.assert_array_equal(Xf[0], T[-1])


def test_harmonic_trajectory_follows_the_euler_law():
    dt = 0.4
    pot = Harmonic(k=1.0)
    xs = []
    for seed in (3, 4):
        rng = np.random.default_rng(seed)
        X = np.empty((17, 1, 1))
        X[0] = rng.standard_normal() * math.sqrt(1.25)
        for n in range(16):
            X[n + 1] = 0.6 * X[n] + math.sqrt(0.8) * rng.standard_normal()
        T, _ = OP.run(X, pot, dt, 1.0, 1.0, seed=100 + seed, l_min=3, l_max=3, n_sample=2,
                      n_shift=2, n_events=2500)
        xs.append(T[:, 0, 0])
    x = np.concatenate(xs)
    var = x.var()
    lag1 = np.mean(np.concatenate([v[1:] * v[:-1] for v in xs])) / var
    # ~1250 effective samples per chain: sd(var) ~ 0.05, sd(lag1) ~ 0.02
    assert abs(var - 1.25) < 0.15, var
    assert abs(lag1 - 0.6) < 0.06, lag1
    # the continuous-time law (variance 1, decay exp(-0.4) = 0.67) is excluded
    assert var > 1.1
