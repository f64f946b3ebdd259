"""A gradient-informed path move: Metropolis-adjusted Langevin dynamics in path space.

Test infrastructure.  The paper samples paths with force-free trial moves
(Sec. III) and never uses the gradient of the action; this move is an
extension that does, targeting the same path distribution exp(-S[X]) of
Eq. 4 with x_0 fixed.  With g = dS/dX (rows 1..N; row 0 is held fixed) and
step tau:

    Y = X - tau g(X) + sqrt(2 tau) z,     z ~ N(0, I)
    log alpha = S(X) - S(Y) + |z|^2 / 2 - |X - Y + tau g(Y)|^2 / (4 tau)

(the second pair of terms is log q(X | Y) - log q(Y | X) for the Gaussian
proposal q), and Y replaces X when u < exp(log alpha).  The normals z and
the uniform u come from the Philox streams 5 and 6 (``philox``).
"""
from __future__ import annotations

import math

import numpy as np

from . import action as _a
from . import philox as _p


def log_ratio(X, Y, S_x, S_y, g_x, g_y, tau: float):
    """log alpha of the move X -> Y (rows 0 of X and Y are equal and ignored)."""
    f = (Y[1:] - X[1:] + tau * g_x[1:])
    b = (X[1:] - Y[1:] + tau * g_y[1:])
    return (S_x - S_y) + (math.fsum((f * f).ravel().tolist())
                          - math.fsum((b * b).ravel().tolist())) / (4.0 * tau)


def langevin_step(X, pot, dt, D, gamma, tau: float, seed: int, move: int,
                  method: str = "brute"):
    """One move; returns dict(path, accepted, log_alpha, proposal)."""
    S_x = _a.path_action(X, pot, dt, D, gamma, method)
    g_x = _a.path_gradient(X, pot, dt, D, gamma, method=method)
    z = _p.langevin_normals(seed, move, X.size).reshape(X.shape)
    Y = X - tau * g_x + math.sqrt(2.0 * tau) * z
    Y[0] = X[0]
    S_y = _a.path_action(Y, pot, dt, D, gamma, method)
    g_y = _a.path_gradient(Y, pot, dt, D, gamma, method=method)
    la = log_ratio(X, Y, S_x, S_y, g_x, g_y, tau)
    u = _p.langevin_uniform(seed, move)
    acc = la >= 0.0 or u < math.exp(la)
    return dict(path=Y if acc else X.copy(), accepted=acc, log_alpha=la, proposal=Y)
