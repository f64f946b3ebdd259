"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds random draws, lattice geometry and workload sizes only.  It
computes no potential, force, action or gradient: the physics of the path
action lives on each side separately (the CPU oracle and the HIP library).

Workloads (all in reduced Lennard-Jones units, epsilon = sigma = 1):

* ``ho1d``      1-D harmonic oscillator, k = beta = D = 1, dt = 0.01, 1024 steps.
* ``lj108``     LJ, N = 108, density 0.8442, T = 1, r_c = 2.5, dt = 1e-4, 256 steps.
* ``lj864``     LJ, N = 864, same state point, 4096 steps (the headline workload).
* ``batch64``   64 independent LJ paths, N in {108, 256, 500, 864, 2048},
                step counts log-uniform in [128, 8192].
* ``sweep4000`` LJ, N = 4000, 16384 steps, path-sampling levels 4..7.
* ``lj27``      the paper's own LJ state point (Sec. IV B): N = 27, density 0.5,
                beta*eps = 0.74, r_c = L/2, dt = 5e-4.

Einstein relation (Sec. II A, Eq. 1): gamma = 1/(beta D).
"""
from .configs import (WORKLOADS, Workload, BatchWorkload, SEED_BASE, workload, batch_members,
                      box_length, n_fcc_cells)
from .generate import (fcc_lattice, cubic_lattice, initial_lattice, draw_noise, tethered_path,
                       ho_noise, free_walk_path, rng_for)

__all__ = [
    "WORKLOADS", "Workload", "BatchWorkload", "SEED_BASE", "workload", "batch_members",
    "box_length", "n_fcc_cells", "fcc_lattice", "cubic_lattice", "initial_lattice", "draw_noise", "tethered_path", "ho_noise",
    "free_walk_path", "rng_for",
]
