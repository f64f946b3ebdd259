"""The Python binding refuses tensors of the wrong type, layout, size or device
before it calls the library (the C ABI takes bare pointers and cannot check
them).  Runs without a GPU: every case raises before any device work."""
import os

import pytest
import torch

import paper_1907_09529_amd as P
from paper_1907_09529_amd import _lib

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH),
                                reason="libpamd.so not built (run __graft_entry__.build())")

BOX = (108 / 0.8442) ** (1 / 3)


def lj(n_steps=8, n_atoms=108):
    path = P.make_path(n_steps, n_atoms, 3, 1e-4, 1.0, 1.0)
    pot = P.make_potential("lj", rc=2.5, box=BOX)
    return path, pot


def f64(*shape):
    return torch.zeros(*shape, dtype=torch.float64)


WS = torch.zeros(256, dtype=torch.uint8)


def test_undersized_path_is_refused():
    path, pot = lj()
    x = f64(8, 3, 108)          # one slice short of (N + 1) slices
    with pytest.raises(ValueError, match="elements"):
        P.pamd_action_grad(path, pot, x, f64(9, 3, 108), ws=WS)


def test_undersized_gradient_is_refused():
    path, pot = lj()
    with pytest.raises(ValueError, match="grad has"):
        P.pamd_action_grad(path, pot, f64(9, 3, 108), f64(9, 3, 100), ws=WS)


def test_undersized_per_step_and_weights_are_refused():
    path, pot = lj()
    x, g = f64(9, 3, 108), f64(9, 3, 108)
    with pytest.raises(ValueError, match="per_step has"):
        P.pamd_action_grad(path, pot, x, g, per_step=f64(7), ws=WS)
    with pytest.raises(ValueError, match="step_weights has"):
        P.pamd_action_grad(path, pot, x, g, step_weights=f64(3), ws=WS)
    with pytest.raises(ValueError, match="excess has"):
        P.pamd_excess_action(path, pot, x, f64(2), ws=WS)


def test_wrong_dtype_and_layout_are_refused():
    path, pot = lj()
    with pytest.raises(ValueError, match="float64"):
        P.pamd_action(path, pot, torch.zeros(9, 3, 108, dtype=torch.float32), f64(1), ws=WS)
    xt = f64(108, 3, 9).permute(2, 1, 0)  # right shape, not contiguous
    with pytest.raises(ValueError, match="contiguous"):
        P.pamd_action(path, pot, xt, f64(1), ws=WS)


def test_host_tensor_of_the_right_size_is_refused():
    path, pot = lj()
    with pytest.raises(ValueError, match="device tensor"):
        P.pamd_action(path, pot, f64(9, 3, 108), f64(1), ws=WS)


def test_sampler_and_integrator_buffers_are_sized():
    path, pot = lj()
    x = f64(9, 3, 108)
    with pytest.raises(ValueError, match="sweep_counter has"):
        P.pamd_mh_step(path, pot, 1, 1, 2, torch.zeros(0, dtype=torch.int64), x, f64(8), x,
                       ws=WS)
    with pytest.raises(ValueError, match="noise has"):
        P.pamd_em_integrate(path, pot, f64(3, 108), f64(7, 3, 108), x, ws=WS)
    with pytest.raises(ValueError, match="traj_out has"):
        P.pamd_shift(path, 1, 4, torch.zeros(1, dtype=torch.int64), x, f64(9, 3, 108),
                     traj_out=f64(3, 3, 108))


def test_autograd_forward_checks_through_the_binding():
    path, pot = lj()
    with pytest.raises(ValueError, match="x has"):
        P.path_action(f64(4, 3, 108), path, pot, retain=True)
