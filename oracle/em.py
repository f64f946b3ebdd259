"""Euler-Maruyama paths of overdamped Langevin dynamics (Sec. II A, Eqs. 1-2).

    x(t + dt) = x(t) - gamma^{-1} V'(x(t)) dt + sqrt(2 D dt) xi,
i.e. x_{n+1} = x_n + mu dt F(x_n) + sqrt(2 D dt) xi_n with mu = 1/gamma and
xi_n a standard Gaussian variate per degree of freedom.  Coordinates are
left unwrapped (no periodic folding).
"""
from __future__ import annotations

import math

import numpy as np

from . import forces as _f


def em_path(x0, xi, pot, dt: float, D: float, gamma: float, method: str = "brute"):
    """Path (N + 1, n_dim, n_atoms) from x0 (n_dim, n_atoms) and noise xi (N, n_dim, n_atoms)."""
    mu = 1.0 / gamma
    amp = math.sqrt(2.0 * D * dt)
    n_steps = xi.shape[0]
    X = np.empty((n_steps + 1,) + np.shape(x0), dtype=np.float64)
    X[0] = x0
    for n in range(n_steps):
        X[n + 1] = X[n] + mu * dt * _f.forces(X[n], pot, method) + amp * xi[n]
    return X


def perturbed_em_path(x0, xi, eta, eta_sd: float, pot, dt, D, gamma, method: str = "brute"):
    """EM path with slices 1..N displaced by eta_sd * eta afterwards (x_0 stays fixed)."""
    X = em_path(x0, xi, pot, dt, D, gamma, method)
    X[1:] += eta_sd * eta
    return X
