"""Workload sizes and parameters (no arithmetic of the method here)."""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional

import numpy as np

SEED_BASE = 190709529  # seed_i = SEED_BASE + i for the i-th workload below


@dataclasses.dataclass(frozen=True)
class Workload:
    name: str
    seed: int
    potential: str            # "harmonic" or "lj"
    n_atoms: int
    n_dim: int
    n_steps: int              # N_path: number of time steps; the path holds n_steps + 1 slices
    dt: float
    D: float
    beta: float
    k: float = 1.0            # harmonic force constant
    density: float = 0.0      # LJ reduced density
    rc: float = 2.5           # LJ cutoff (sigma units); 0 means half the box
    eps: float = 1.0
    sigma: float = 1.0
    perturb_sd: float = 0.0   # sd of the Gaussian perturbation added to slices 1..N
    l_min: int = 0            # path-sampling levels (sweep workload only)
    l_max: int = 0
    n_sweeps: int = 0

    @property
    def gamma(self) -> float:
        # Einstein relation D = 1/(beta gamma), Sec. II A under Eq. 1.
        return 1.0 / (self.beta * self.D)

    @property
    def box(self) -> float:
        if self.potential != "lj":
            return 0.0
        return box_length(self.n_atoms, self.density)

    @property
    def cutoff(self) -> float:
        if self.potential != "lj":
            return 0.0
        return self.rc if self.rc > 0 else 0.5 * self.box

    def with_steps(self, n_steps: int) -> "Workload":
        return dataclasses.replace(self, n_steps=n_steps)

    def with_atoms(self, n_atoms: int) -> "Workload":
        return dataclasses.replace(self, n_atoms=n_atoms)


@dataclasses.dataclass(frozen=True)
class BatchWorkload:
    name: str
    seed: int
    n_paths: int
    atom_choices: tuple
    min_steps: int
    max_steps: int
    base: Workload


def box_length(n_atoms: int, density: float) -> float:
    """Cubic box edge for n_atoms at reduced number density."""
    return (n_atoms / density) ** (1.0 / 3.0)


def n_fcc_cells(n_atoms: int) -> int:
    """FCC unit cells per edge for n_atoms = 4 n^3 atoms."""
    n = int(round((n_atoms / 4) ** (1.0 / 3.0)))
    if 4 * n ** 3 != n_atoms:
        raise ValueError(f"{n_atoms} atoms is not 4 n^3")
    return n


_LJ = dict(potential="lj", n_dim=3, D=1.0, beta=1.0, density=0.8442, rc=2.5, perturb_sd=0.01)

WORKLOADS: Dict[str, Workload] = {
    "ho1d": Workload("ho1d", SEED_BASE + 1, "harmonic", n_atoms=1, n_dim=1, n_steps=1024,
                     dt=0.01, D=1.0, beta=1.0, k=1.0, perturb_sd=0.1),
    "lj108": Workload("lj108", SEED_BASE + 2, n_atoms=108, n_steps=256, dt=1e-4, **_LJ),
    "lj864": Workload("lj864", SEED_BASE + 3, n_atoms=864, n_steps=4096, dt=1e-4, **_LJ),
    "sweep4000": Workload("sweep4000", SEED_BASE + 5, n_atoms=4000, n_steps=16384, dt=1e-4,
                          l_min=4, l_max=7, n_sweeps=100, **_LJ),
    # The paper's LJ system (Sec. IV B, Table III): N = 27, rho = 0.5, beta eps = 0.74,
    # cutoff at half the box; D = 1/(beta gamma) with gamma = 1.
    "lj27": Workload("lj27", SEED_BASE + 6, "lj", n_atoms=27, n_dim=3, n_steps=128, dt=5e-4,
                     D=1.0 / 0.74, beta=0.74, density=0.5, rc=0.0, perturb_sd=0.01),
}

BATCH = BatchWorkload("batch64", SEED_BASE + 4, n_paths=64,
                      atom_choices=(108, 256, 500, 864, 2048), min_steps=128, max_steps=8192,
                      base=WORKLOADS["lj864"])


def workload(name: str) -> Workload:
    return WORKLOADS[name]


def batch_members(b: BatchWorkload = BATCH, n_paths: Optional[int] = None) -> List[Workload]:
    """The batch's member paths: atoms uniform over the choices, steps log-uniform."""
    rng = np.random.default_rng(b.seed)
    n = b.n_paths if n_paths is None else n_paths
    atoms = rng.choice(np.asarray(b.atom_choices), size=b.n_paths)
    steps = np.floor(np.exp(rng.uniform(math.log(b.min_steps), math.log(b.max_steps),
                                        size=b.n_paths))).astype(np.int64)
    seeds = np.random.SeedSequence(b.seed).spawn(b.n_paths)
    out = []
    for p in range(n):
        w = dataclasses.replace(b.base, name=f"{b.name}[{p}]", n_atoms=int(atoms[p]),
                                n_steps=int(steps[p]),
                                seed=int(seeds[p].generate_state(1)[0]))
        out.append(w)
    return out
