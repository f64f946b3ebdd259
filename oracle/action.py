"""Discretized path action and its gradient (Sec. II A, Eqs. 2-4).

A path is an array X of shape (N + 1, n_dim, n_atoms) holding x_0 .. x_N
(Eq. 4: X = {x(t_0), ..., x(t_N)}, t_n = t + n dt); N is the number of time
steps (N_path in Sec. II, one force evaluation per step, Eq. 9).

Per-step term (the exponent of Eq. 3, dropping its normalisation):
    r_n = Delta_n + (dt/gamma) V'(x_n) = Delta_n - mu dt F(x_n),   mu = 1/gamma,
    s_n = |r_n|^2 / (4 D dt),
with Delta_n = x_{n+1} - x_n taken as the minimum image under periodic
boundaries.  The action is S[X] = sum_{n=0}^{N-1} s_n (Eq. 4).  The omitted
normalisation of the N Gaussian transition densities adds
N (n_dim n_atoms / 2) ln(4 pi D dt) to -ln prod K (``log_norm``).

Gradient (derived from the above; the paper itself evaluates only S):
    d r_n / d x_m = delta_{n+1,m} I + delta_{n,m} (-I + mu dt H(x_m)),
so with c = 1/(2 D dt) and H symmetric
    g_m = c [ r_{m-1} [m >= 1] - r_m [m < N] + mu dt H(x_m) r_m [m < N] ].
With per-step weights w_n the same expression with r_n replaced by w_n r_n
is the gradient of sum_n w_n s_n.
"""
from __future__ import annotations

import math

import numpy as np

from . import forces as _f
from .potentials import Harmonic, LennardJones


def _box(pot) -> float:
    return pot.box if isinstance(pot, LennardJones) else 0.0


def residuals(X, pot, dt: float, D: float, gamma: float, method: str = "brute"):
    """r_n for n = 0..N-1, shape (N, n_dim, n_atoms)."""
    mu = 1.0 / gamma
    n_steps = X.shape[0] - 1
    r = np.empty((n_steps,) + X.shape[1:], dtype=X.dtype)
    for n in range(n_steps):
        delta = _f.minimum_image(X[n + 1] - X[n], _box(pot))
        r[n] = delta - mu * dt * _f.forces(X[n], pot, method)
    return r


def per_step_action(X, pot, dt, D, gamma, method: str = "brute"):
    """s_n = |r_n|^2 / (4 D dt), n = 0..N-1 (Eq. 3 exponent)."""
    r = residuals(X, pot, dt, D, gamma, method)
    return np.sum((r * r).reshape(r.shape[0], -1), axis=1) / (4.0 * D * dt)


def path_action(X, pot, dt, D, gamma, method: str = "brute"):
    """S[X] = sum_n s_n (Eq. 4), summed with math.fsum for real paths."""
    s = per_step_action(X, pot, dt, D, gamma, method)
    if np.iscomplexobj(s):
        return np.sum(s)
    return math.fsum(s.tolist())


def path_gradient(X, pot, dt, D, gamma, step_weights=None, method: str = "brute"):
    """dS/dX (or d(sum w_n s_n)/dX), shape (N + 1, n_dim, n_atoms)."""
    mu = 1.0 / gamma
    c = 1.0 / (2.0 * D * dt)
    n_steps = X.shape[0] - 1
    r = residuals(X, pot, dt, D, gamma, method)
    if step_weights is not None:
        r = r * np.asarray(step_weights, dtype=np.float64)[:, None, None]
    g = np.zeros(X.shape, dtype=np.result_type(X, r))
    for m in range(n_steps + 1):
        if m >= 1:
            g[m] += r[m - 1]
        if m < n_steps:
            g[m] += -r[m] + mu * dt * _f.hessian_vec(X[m], r[m], pot, method)
    return c * g


def log_norm(n_steps: int, n_dim: int, n_atoms: int, D: float, dt: float) -> float:
    """Normalisation of the N Gaussian transition densities of Eq. 3: -ln prod K = S + this."""
    return n_steps * (n_dim * n_atoms / 2.0) * math.log(4.0 * math.pi * D * dt)


def slice_terms(X, m: int, pot, dt, D, gamma, method: str = "brute", step_weights=None):
    """Terms touching slice m only, for spot checks of long paths.

    Returns (s_m or None, g_m): the per-step action of step m (when m < N)
    and the gradient row of slice m, using only x_{m-1}, x_m, x_{m+1}.
    """
    mu = 1.0 / gamma
    c = 1.0 / (2.0 * D * dt)
    n_steps = X.shape[0] - 1
    box = _box(pot)

    def res(n):
        delta = _f.minimum_image(X[n + 1] - X[n], box)
        w = 1.0 if step_weights is None else float(step_weights[n])
        r = delta - mu * dt * _f.forces(X[n], pot, method)
        return r, w

    g = np.zeros(X.shape[1:])
    s = None
    if m >= 1:
        r_prev, w_prev = res(m - 1)
        g += w_prev * r_prev
    if m < n_steps:
        r_m, w_m = res(m)
        s = float(np.sum(r_m * r_m) / (4.0 * D * dt))
        g += -w_m * r_m + mu * dt * _f.hessian_vec(X[m], w_m * r_m, pot, method)
    return s, c * g
