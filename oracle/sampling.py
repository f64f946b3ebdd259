"""One Monte Carlo step of the multilevel sliding-and-sampling path sampler (Sec. III).

Steps, in the order the paper describes them:

1. A level l is drawn uniformly in [l_min, l_max] (Sec. III, below Table I).
2. Random fragmentation at level l: neighbouring fragments share endpoints;
   internal fragments span 2^l steps, the two terminal fragments together
   2^l (Sec. III, Fig. 5).  Here the first shared endpoint sits at a uniform
   offset u in [1, 2^l]; endpoints are u, u + 2^l, ... up to N.  The tail
   fragment is [0, u]; the nose fragment [e_last, N] exists when e_last < N.
3. Shared endpoints and the tail x_0 stay fixed; the nose endpoint x_N is
   sampled with the nose fragment (Sec. III).
4. Trial configurations come from the free-particle path distribution with
   the fragment's boundary conditions (Sec. III: harmonic-oscillator trials;
   here used for every potential): a Brownian bridge between two fixed
   endpoints, or free Brownian continuation for the nose, with per-step
   variance 2 D dt per degree of freedom.
5. Each fragment is accepted with the Metropolis-Hastings probability
   min(1, exp(-Delta_f)), where, with s_n the per-step action (Eq. 3) and
   s0_n its force-free (free-particle) counterpart |Delta_n|^2/(4 D dt),
       Delta_f = sum_{n in f} [(s'_n - s0'_n) - (s_n - s0_n)]
   over the steps n = a .. b-1 of fragment [a, b] (primes: trial path).  The
   proposal density is proportional to exp(-sum s0), so this is the MH ratio
   of the target exp(-S) (Eq. 4) to the proposal.

Random numbers come from the Philox streams documented in ``philox``.
"""
from __future__ import annotations

import math

import numpy as np

from . import action as _a
from . import forces as _f
from . import philox as _p
from .potentials import LennardJones


def fragments(n_steps: int, level: int, offset: int):
    """List of (a, b, is_nose) covering [0, N] for a random fragmentation."""
    span = 1 << level
    ends = list(range(offset, n_steps + 1, span))
    out = []
    a = 0
    for e in ends:
        out.append((a, e, False))
        a = e
    if a < n_steps:
        out.append((a, n_steps, True))
    return out


def free_step_action(X, D: float, dt: float, box: float):
    """s0_n = |Delta_n|^2 / (4 D dt): the per-step action with V' = 0."""
    d = _f.minimum_image(X[1:] - X[:-1], box)
    return np.sum((d * d).reshape(d.shape[0], -1), axis=1) / (4.0 * D * dt)


def trial_path(X, frags, normals, D: float, dt: float):
    """Free-particle trial path: bridges inside fragments, free continuation at the nose.

    normals has the shape of X; the variate for slice k is normals[k].
    """
    sig = math.sqrt(2.0 * D * dt)
    Y = X.copy()
    for a, b, nose in frags:
        if nose:
            for k in range(a, b):
                Y[k + 1] = Y[k] + sig * normals[k + 1]
        else:
            for k in range(a, b - 1):
                rem = b - k
                Y[k + 1] = (Y[k] + (X[b] - Y[k]) / rem
                            + sig * math.sqrt((rem - 1) / rem) * normals[k + 1])
    return Y


def mh_step(X, pot, dt, D, gamma, seed: int, sweep: int, l_min: int, l_max: int,
            method: str = "brute"):
    """One MC step; returns a dict with the new path and the step's bookkeeping."""
    n_steps = X.shape[0] - 1
    box = pot.box if isinstance(pot, LennardJones) else 0.0
    level, offset = _p.level_and_offset(seed, sweep, l_min, l_max)
    frags = fragments(n_steps, level, offset)
    normals = _p.trial_normals(seed, sweep, X.size).reshape(X.shape)
    Y = trial_path(X, frags, normals, D, dt)
    s_old = _a.per_step_action(X, pot, dt, D, gamma, method)
    s_new = _a.per_step_action(Y, pot, dt, D, gamma, method)
    f_old = free_step_action(X, D, dt, box)
    f_new = free_step_action(Y, D, dt, box)
    u = _p.accept_uniforms(seed, sweep, len(frags))
    Xn = X.copy()
    deltas, accepted = [], []
    for fi, (a, b, nose) in enumerate(frags):
        delta = math.fsum(((s_new[a:b] - f_new[a:b]) - (s_old[a:b] - f_old[a:b])).tolist())
        acc = bool(u[fi] < math.exp(-delta)) if delta > -700 else True
        deltas.append(delta)
        accepted.append(acc)
        if acc:
            hi = b + 1 if nose else b
            Xn[a + 1:hi] = Y[a + 1:hi]
    return dict(path=Xn, trial=Y, level=level, offset=offset, fragments=frags,
                delta=np.array(deltas), accepted=np.array(accepted), uniforms=u,
                s_old=s_old, s_new=s_new)
