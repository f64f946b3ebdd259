"""Potentials of the paper's two model systems.

Harmonic oscillator: V(x) = k x^2 / 2 for every Cartesian degree of freedom
(Sec. II A below Eq. 7; Sec. IV A uses k = 1).

Lennard-Jones liquid: the cut-and-force-shifted pair potential of Eq. 16,
    U(r) = u(r) - u(r_c) - (r - r_c) u'(r_c)   for r <= r_c,   0 otherwise,
    u(r) = 4 eps [ (sigma/r)^12 - (sigma/r)^6 ],
so U and U' both vanish at r_c (Sec. IV B).  The derivatives used by the
force and the Hessian follow by differentiating that expression once and
twice in r:
    u'(r)  = -(24 eps / r)   [ 2 (sigma/r)^12 -     (sigma/r)^6 ]
    u''(r) =  (24 eps / r^2) [26 (sigma/r)^12 - 7   (sigma/r)^6 ]
    U'(r)  = u'(r) - u'(r_c),   U''(r) = u''(r).
All functions accept real or complex r (complex for complex-step pins).
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass(frozen=True)
class Harmonic:
    k: float = 1.0


@dataclasses.dataclass(frozen=True)
class LennardJones:
    eps: float = 1.0
    sigma: float = 1.0
    rc: float = 2.5
    box: float = 0.0          # cubic periodic box edge (Sec. IV B: PBC at constant volume)

    def u(self, r):
        sr6 = (self.sigma / r) ** 6
        return 4.0 * self.eps * (sr6 * sr6 - sr6)

    def du(self, r):
        sr6 = (self.sigma / r) ** 6
        return -(24.0 * self.eps / r) * (2.0 * sr6 * sr6 - sr6)

    def d2u(self, r):
        sr6 = (self.sigma / r) ** 6
        return (24.0 * self.eps / r ** 2) * (26.0 * sr6 * sr6 - 7.0 * sr6)

    def U(self, r):
        """Eq. 16 for r <= r_c (caller applies the cutoff)."""
        rc = self.rc
        return self.u(r) - self.u(rc) - (r - rc) * self.du(rc)

    def dU(self, r):
        return self.du(r) - self.du(self.rc)

    def d2U(self, r):
        return self.d2u(r)
