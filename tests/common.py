"""Shared helpers for the GPU tests: oracle-built inputs and comparison norms."""
from __future__ import annotations

import functools

import numpy as np

import workloads as W
from oracle import action as OA
from oracle import em as OE
from oracle.potentials import Harmonic, LennardJones


def rel_inf(a, b) -> float:
    """||a - b||_inf / ||b||_inf (normwise relative error of a against reference b)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (den if den > 0 else 1.0))


def rel(a: float, b: float) -> float:
    return abs(a - b) / abs(b) if b != 0 else abs(a)


def oracle_pot(w: W.Workload):
    if w.potential == "harmonic":
        return Harmonic(k=w.k)
    return LennardJones(eps=w.eps, sigma=w.sigma, rc=w.cutoff, box=w.box)


@functools.lru_cache(maxsize=16)
def em_input(name: str, n_atoms: int = 0, n_steps: int = 0):
    """Perturbed Euler-Maruyama path of a workload, built by the oracle (cached)."""
    w = W.workload(name)
    if n_atoms:
        w = w.with_atoms(n_atoms)
    if n_steps:
        w = w.with_steps(n_steps)
    pot = oracle_pot(w)
    if w.potential == "harmonic":
        x0 = np.zeros((w.n_dim, w.n_atoms))
    else:
        x0 = W.initial_lattice(w.n_atoms, w.box)
    xi, eta = W.draw_noise(w)
    X = OE.perturbed_em_path(x0, xi, eta, w.perturb_sd, pot, w.dt, w.D, w.gamma)
    X.setflags(write=False)
    return w, X


def lib_descriptors(w: W.Workload, precision: str = "fp64"):
    import paper_1907_09529_amd as P
    path = P.make_path(w.n_steps, w.n_atoms, w.n_dim, w.dt, w.D, w.gamma, precision)
    if w.potential == "harmonic":
        pot = P.make_potential("harmonic", k=w.k)
    else:
        pot = P.make_potential("lj", eps=w.eps, sigma=w.sigma, rc=w.cutoff, box=w.box)
    return path, pot


def oracle_full(w: W.Workload, X, weights=None):
    pot = oracle_pot(w)
    s = OA.per_step_action(X, pot, w.dt, w.D, w.gamma)
    g = OA.path_gradient(X, pot, w.dt, w.D, w.gamma, step_weights=weights)
    return s, g


def pairs_at_the_cutoff(n_steps, period=16, alpha=0.004, rel_eps=1e-11):
    """27 pairs of atoms, the pairs 10 sigma apart in a 30-sigma box (pairs
    centred on a face straddle the periodic boundary); pair k moves along its
    own random axis with separation D(n) = D* + alpha |n - n*|, where n* is
    slice k mod period of every block of `period` slices and D* is
    r_c (1 - rel_eps) for even k, r_c (1 + rel_eps) for odd k.  The motion is
    collinear, so at n* the distance of the two atoms' bounding-box centres
    over any tile holding n* minus both half-diagonals is exactly D*."""
    import dataclasses
    w = dataclasses.replace(W.workload("lj108").with_steps(n_steps), n_atoms=54,
                            density=54 / 30.0 ** 3)
    rng = np.random.default_rng(190701)
    rc, L = w.cutoff, w.box
    X = np.empty((n_steps + 1, 3, 54))
    n = np.arange(n_steps + 1)
    for k in range(27):
        centre = (L / 3.0) * np.array([k % 3, (k // 3) % 3, k // 9])
        u = rng.normal(size=3)
        u /= np.linalg.norm(u)
        d_star = rc * (1.0 - rel_eps if k % 2 == 0 else 1.0 + rel_eps)
        n_star = (n // period) * period + k % period
        sep = d_star + alpha * np.abs(n - n_star)
        X[:, :, 2 * k] = centre + 0.5 * sep[:, None] * u
        X[:, :, 2 * k + 1] = centre - 0.5 * sep[:, None] * u
    return w, X
