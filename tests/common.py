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
