"""Seeded draws and geometry for the synthetic workloads.

Nothing here evaluates a potential, a force or an action.  Paths that follow a
real Euler-Maruyama run are built by the oracle from these draws; the
``tethered_path`` recipe below is a force-free stand-in with the same sizes,
density, neighbour counts and per-step displacement scale, used where the
oracle cannot afford a sequential run (the full-size workloads).
"""
from __future__ import annotations

import math

import numpy as np

from .configs import Workload, n_fcc_cells


def rng_for(w: Workload, stream: int = 0) -> np.random.Generator:
    """Generator for workload w; stream > 0 gives independent side streams."""
    if stream == 0:
        return np.random.default_rng(w.seed)
    return np.random.default_rng([w.seed, stream])


def fcc_lattice(n_atoms: int, box: float) -> np.ndarray:
    """FCC sites, SoA layout (3, n_atoms), cubic box of edge ``box``.

    n = (n_atoms/4)^(1/3) cells per edge, lattice constant a = box/n, basis
    (0,0,0), (1/2,1/2,0), (1/2,0,1/2), (0,1/2,1/2).
    """
    n = n_fcc_cells(n_atoms)
    a = box / n
    basis = np.array([[0.0, 0.0, 0.0], [0.5, 0.5, 0.0], [0.5, 0.0, 0.5], [0.0, 0.5, 0.5]])
    sites = []
    for ix in range(n):
        for iy in range(n):
            for iz in range(n):
                for b in basis:
                    sites.append((np.array([ix, iy, iz], dtype=np.float64) + b) * a)
    return np.ascontiguousarray(np.array(sites).T)


def cubic_lattice(n_atoms: int, box: float) -> np.ndarray:
    """Simple-cubic sites (3, n_atoms) for n_atoms = n^3 (the paper's 27-atom system)."""
    n = int(round(n_atoms ** (1.0 / 3.0)))
    if n ** 3 != n_atoms:
        raise ValueError(f"{n_atoms} atoms is not n^3")
    a = box / n
    g = (np.arange(n, dtype=np.float64) + 0.5) * a
    X, Y, Z = np.meshgrid(g, g, g, indexing="ij")
    return np.ascontiguousarray(np.stack([X.ravel(), Y.ravel(), Z.ravel()]))


def initial_lattice(n_atoms: int, box: float) -> np.ndarray:
    """FCC when n_atoms = 4 n^3, else simple cubic when n_atoms = n^3."""
    n = int(round((n_atoms / 4) ** (1.0 / 3.0)))
    if 4 * n ** 3 == n_atoms:
        return fcc_lattice(n_atoms, box)
    return cubic_lattice(n_atoms, box)


def draw_noise(w: Workload, n_steps: int | None = None):
    """(xi, eta): two standard-normal arrays of shape (n_steps, n_dim, n_atoms), C order.

    xi drives the dynamics (Eq. 2's Gaussian variate), eta is scaled by
    ``w.perturb_sd`` and added to slices 1..N afterwards.
    """
    n = w.n_steps if n_steps is None else n_steps
    rng = rng_for(w)
    shape = (n, w.n_dim, w.n_atoms)
    xi = rng.standard_normal(shape)
    eta = rng.standard_normal(shape)
    return xi, eta


def ho_noise(w: Workload, n_steps: int | None = None):
    """Same as draw_noise; named for the harmonic workload."""
    return draw_noise(w, n_steps)


def tethered_path(w: Workload, n_steps: int | None = None, vib_sd: float = 0.08,
                  dtype=np.float64) -> np.ndarray:
    """Force-free stand-in for an equilibrated LJ path near its lattice, (N+1, 3, n_atoms).

    Each coordinate is its FCC site plus a stationary Gaussian AR(1) sequence
    whose per-step innovation is sqrt(2 D dt) (the free-diffusion step of the
    workload) and whose stationary sd is ``vib_sd``; slice 0 is the bare
    lattice and slices 1..N receive the workload's perturbation eta.
    """
    n = w.n_steps if n_steps is None else n_steps
    box = w.box
    sites = initial_lattice(w.n_atoms, box)
    step_sd = math.sqrt(2.0 * w.D * w.dt)
    rho = math.sqrt(max(0.0, 1.0 - step_sd ** 2 / vib_sd ** 2))
    rng = rng_for(w, stream=7)
    shape = (w.n_dim, w.n_atoms)
    out = np.empty((n + 1,) + shape, dtype=dtype)
    out[0] = sites
    u = np.zeros(shape)
    for t in range(1, n + 1):
        u = rho * u + step_sd * rng.standard_normal(shape)
        out[t] = sites + u + w.perturb_sd * rng.standard_normal(shape)
    return out


def free_walk_path(w: Workload, n_steps: int | None = None) -> np.ndarray:
    """Force-free stand-in path, (N+1, n_dim, n_atoms): a Gaussian random walk
    from the origin with per-step sd sqrt(2 D dt) (the free-diffusion step),
    slices 1..N then perturbed by N(0, perturb_sd^2)."""
    n = w.n_steps if n_steps is None else n_steps
    step_sd = math.sqrt(2.0 * w.D * w.dt)
    rng = rng_for(w, stream=7)
    shape = (n, w.n_dim, w.n_atoms)
    steps = step_sd * rng.standard_normal(shape)
    out = np.zeros((n + 1, w.n_dim, w.n_atoms))
    out[1:] = np.cumsum(steps, axis=0) + w.perturb_sd * rng.standard_normal(shape)
    return out
