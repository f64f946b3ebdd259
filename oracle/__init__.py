"""Plain, slow FP64 CPU oracle for the discretized Brownian path action and its gradient.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this package; only
the test suite, the smoke check and the benchmark's CPU-baseline leg may
import or call it.  It shares no code with the HIP path: it is written from
the paper's equations (Rosa-Raices, Zhang, Miller, "Path-accelerated
molecular dynamics", arXiv:1907.09529) and from textbook definitions, in
float64 (complex128 where a pin differentiates it by complex step).

Modules
  potentials : harmonic and cut-and-force-shifted LJ pair functions (Eq. 16)
  forces     : pair sets (brute force, cell list), energy, force, Hessian-vector
  action     : per-step action (Eq. 3), total action (Eq. 4), gradient, log norm
  em         : Euler-Maruyama paths (Eq. 2)
  philox     : Philox4x32-10 counter-based generator, uniforms, Box-Muller normals
  sampling   : random fragmentation, free-particle trial paths and the
               fragment-wise Metropolis-Hastings step (Sec. III)
  pamd       : the sample-shift-regrow integration loop (Sec. II B, Figs. 1-2)
  langevin   : a gradient-informed (Metropolis-adjusted Langevin) path move, an
               extension targeting exp(-S) of Eq. 4

Parity status: every function here is pinned by a test in tests/test_oracle_*.py
against closed forms, invariants, finite or complex-step differences, brute
force, or published known-answer values.
"""
from . import potentials, forces, action, em, philox, sampling, pamd, langevin  # noqa: F401
from .potentials import Harmonic, LennardJones  # noqa: F401
from .action import (residuals, per_step_action, path_action, path_gradient,  # noqa: F401
                     log_norm, slice_terms)
