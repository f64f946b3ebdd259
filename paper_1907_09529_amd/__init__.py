"""MI355X (gfx950) implementation of the discretized Brownian path action and
its adjoint gradient (Rosa-Raices, Zhang, Miller, arXiv:1907.09529, Sec. II-III).

The work runs in the HIP library libpamd.so behind the C ABI of include/pamd.h;
this package is its Python binding (``api``, same names as the C entry points)
plus torch.autograd wrappers (``autograd``).  Importing the binding does not
load the library; the first call does, and fails loudly if it is missing.
"""
from . import _lib  # noqa: F401
from .api import *  # noqa: F401,F403
from .autograd import PamdAction, PamdPerStepAction, path_action, per_step_action  # noqa: F401

LIB_PATH = _lib.LIB_PATH


def load():
    """Loads libpamd.so (raises ImportError when it has not been built)."""
    return _lib.load()
