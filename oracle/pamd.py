"""The path-based integration loop of Sec. II B (Figs. 1-2).

Test infrastructure: a plain CPU statement of the loop that the GPU tests
compare against.  Per shifting event, in the paper's order:

1. sample: N_sample Monte Carlo steps of the path sampler (Sec. III, here
   ``sampling.mh_step``) on the path X = {x_0 .. x_N}, x_0 fixed;
2. shift: the slices x_1 .. x_{N_shift} join the integrated trajectory and
   the path is moved along itself, so that x_{N_shift} becomes its first slice
   (Fig. 2B);
3. regenerate: the path is grown back to N steps from its new last slice
   with the trial distribution (Sec. III: regeneration uses the same
   distribution as the trial moves), here free Brownian continuation,
   y_{k+1} = y_k + sqrt(2 D dt) z_k.

If every sampling stage left the path distributed as exp(-S) (Eq. 4) given
x_0, the trajectory would be a realisation of the Euler scheme (Eq. 2) at
step dt.
"""
from __future__ import annotations

import math

import numpy as np

from . import philox as _p
from . import sampling as _s


def shift_path(X, n_shift: int, normals, D: float, dt: float):
    """Shifted and regrown path; normals[k] is the variate of new slice k."""
    n_steps = X.shape[0] - 1
    keep = n_steps - n_shift
    Y = np.empty_like(X)
    Y[:keep + 1] = X[n_shift:]
    sig = math.sqrt(2.0 * D * dt)
    for k in range(keep + 1, n_steps + 1):
        Y[k] = Y[k - 1] + sig * normals[k]
    return Y


def regrowth_normals(seed: int, event: int, shape, n_shift: int):
    """Variates of the regrown slices after shifting event `event` (zeros elsewhere)."""
    n_dof = int(np.prod(shape[1:]))
    n_steps = shape[0] - 1
    first = (n_steps - n_shift + 1) * n_dof
    z = np.zeros(shape)
    z[n_steps - n_shift + 1:] = _p.regrow_normals(seed, event, n_shift * n_dof,
                                                  first).reshape((n_shift,) + tuple(shape[1:]))
    return z


def run(X, pot, dt, D, gamma, seed: int, l_min: int, l_max: int, n_sample: int, n_shift: int,
        n_events: int, sweep0: int = 0, event0: int = 0, method: str = "brute",
        level_stats=None):
    """n_events shifting events from path X; returns (trajectory, final path).

    The trajectory holds x_1 .. x_{N_shift} of every event, in time order
    (n_events * n_shift slices); sweeps and events number from sweep0, event0.
    level_stats, if given (an integer array of 2 * 31), accumulates the
    fragments proposed ([2 l]) and accepted ([2 l + 1]) at each level l.
    """
    traj = []
    sweep = sweep0
    for v in range(n_events):
        for _ in range(n_sample):
            r = _s.mh_step(X, pot, dt, D, gamma, seed, sweep, l_min, l_max, method)
            X = r["path"]
            if level_stats is not None:
                level_stats[2 * r["level"]] += len(r["accepted"])
                level_stats[2 * r["level"] + 1] += int(np.sum(r["accepted"]))
            sweep += 1
        traj.append(X[1:n_shift + 1].copy())
        X = shift_path(X, n_shift, regrowth_normals(seed, event0 + v, X.shape, n_shift), D, dt)
    return np.concatenate(traj), X
