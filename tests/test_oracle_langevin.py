"""Pins of the oracle's gradient-informed (Langevin) path move.

* The Metropolis-Hastings log ratio equals one built independently: the
  harmonic action and gradient from their closed forms (the Euler chain
  x_{n+1} = a x_n + noise, a = 1 - k dt / gamma) and the Gaussian proposal
  densities from scipy.stats.multivariate_normal.
* The move leaves the path distribution exp(-S) with x_0 fixed invariant:
  from an exact sample of 256 independent harmonic chains (x_0 = 1, a = 0.6
  at dt = 0.4) the sampled x_n keep the conditional mean a^n, variance
  0.8 (1 - a^(2n)) / (1 - a^2) and lag covariance.
* As the step tau shrinks the proposal becomes reversible and nearly every
  move is accepted.
"""
import math

import numpy as np
from scipy.stats import multivariate_normal

from oracle import langevin as OL
from oracle.potentials import Harmonic

A = 0.6   # 1 - k dt / gamma at k = gamma = 1, dt = 0.4
DT = 0.4


def closed_action_grad(X):
    """S = sum_n (x_{n+1} - a x_n)^2 / (4 D dt) and its gradient (D = 1)."""
    x = X[:, 0, :]
    e = x[1:] - A * x[:-1]
    S = float(np.sum(e * e) / (4 * DT))
    g = np.zeros_like(x)
    g[1:] += e / (2 * DT)
    g[:-1] -= A * e / (2 * DT)
    return S, g[:, None, :]


def exact_paths(rng, n_steps, n_dof, x0=1.0):
    X = np.zeros((n_steps + 1, 1, n_dof))
    X[0] = x0
    for n in range(n_steps):
        X[n + 1] = A * X[n] + math.sqrt(0.8) * rng.standard_normal((1, n_dof))
    return X


def test_log_ratio_matches_independent_construction():
    rng = np.random.default_rng(4)
    X = exact_paths(rng, 6, 3)
    tau = 0.07
    S_x, g_x = closed_action_grad(X)
    Y = X - tau * g_x + math.sqrt(2 * tau) * rng.standard_normal(X.shape)
    Y[0] = X[0]
    S_y, g_y = closed_action_grad(Y)
    cov = 2 * tau * np.eye(X[1:].size)
    log_q_fwd = multivariate_normal.logpdf(Y[1:].ravel(), (X - tau * g_x)[1:].ravel(), cov)
    log_q_bwd = multivariate_normal.logpdf(X[1:].ravel(), (Y - tau * g_y)[1:].ravel(), cov)
    expect = (S_x - S_y) + log_q_bwd - log_q_fwd
    got = OL.log_ratio(X, Y, S_x, S_y, g_x, g_y, tau)
    assert abs(got - expect) <= 1e-9 * max(1.0, abs(expect))
    # and through the oracle's own action and gradient
    pot = Harmonic(k=1.0)
    r = OL.langevin_step(X, pot, DT, 1.0, 1.0, tau, seed=3, move=0)
    Sp, gp = closed_action_grad(r["proposal"])
    ref = OL.log_ratio(X, r["proposal"], S_x, Sp, g_x, gp, tau)
    assert abs(r["log_alpha"] - ref) <= 1e-9 * max(1.0, abs(ref))


def test_move_keeps_the_path_distribution():
    X = exact_paths(np.random.default_rng(1), 8, 256)
    pot = Harmonic(k=1.0)
    xs, acc = [], 0
    for m in range(1500):
        r = OL.langevin_step(X, pot, DT, 1.0, 1.0, 0.05, seed=5, move=m)
        X = r["path"]
        acc += r["accepted"]
        if m % 5 == 0:
            xs.append(X[:, 0, :].copy())
    xs = np.array(xs)
    assert 0.4 < acc / 1500 < 0.8
    for n in (4, 8):
        mean = A ** n
        var = 0.8 * (1 - A ** (2 * n)) / (1 - A * A)
        assert abs(xs[:, n].mean() - mean) < 0.06, n
        assert abs(xs[:, n].var() / var - 1) < 0.06, n
    cov34 = np.mean((xs[:, 3] - A ** 3) * (xs[:, 4] - A ** 4))
    assert abs(cov34 / (A * 0.8 * (1 - A ** 6) / (1 - A * A)) - 1) < 0.08


def test_small_steps_are_accepted():
    X = exact_paths(np.random.default_rng(2), 8, 4)
    pot = Harmonic(k=1.0)
    acc = sum(OL.langevin_step(X, pot, DT, 1.0, 1.0, 1e-5, seed=9, move=m)["accepted"]
              for m in range(50))
    assert acc >= 49
