"""MI355X (gfx950) implementation of the discretized Brownian path action and
its adjoint gradient (Rosa-Raices, Zhang, Miller, arXiv:1907.09529, Sec. II-III).

The work runs in the HIP library libpamd.so behind the C ABI of include/pamd.h;
this package is its Python binding (``api``, same names as the C entry points)
plus torch.autograd wrappers (``autograd``).  Importing the binding does not
load the library; the first call does, and fails loudly if it is missing.

Typical use (device tensors, float64, path layout x[n, component, atom])::

    import paper_1907_09529_amd as P
    path = P.make_path(n_steps, n_atoms, 3, dt, D, gamma)
    pot = P.make_potential("lj", eps=1.0, sigma=1.0, rc=2.5, box=L)
    P.pamd_action_grad(path, pot, x, grad, action=S)        # S[X] and dS/dX
    S = P.path_action(x, path, pot)                          # autograd form

    # path sampling (Sec. III) and the integration loop (Sec. II B)
    P.pamd_excess_action(path, pot, x, excess)
    P.pamd_run(path, pot, seed, l_min, l_max, n_sample, n_shift, n_events,
               counters, x, x_alt, trial, excess, excess_alt, trajectory)

    # sequential Euler-Maruyama (Eq. 2) and a gradient-informed path move
    P.pamd_em_integrate(path, pot, x0, noise, x_out)
    P.pamd_langevin_step(path, pot, seed, tau, counter, x, grad, S, y, grad_y)
"""
from . import _lib  # noqa: F401
from .api import *  # noqa: F401,F403
from .autograd import PamdAction, PamdPerStepAction, path_action, per_step_action  # noqa: F401

LIB_PATH = _lib.LIB_PATH


def load():
    """Loads libpamd.so (raises ImportError when it has not been built)."""
    return _lib.load()
