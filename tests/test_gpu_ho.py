"""GPU parity of the harmonic-oscillator path action and gradient (Sec. IV A)."""
import math

import numpy as np
import pytest
import torch

import paper_1907_09529_amd as P
import workloads as W
from oracle import em as OE
from oracle.potentials import Harmonic

from common import em_input, lib_descriptors, oracle_full, rel, rel_inf

pytestmark = pytest.mark.gpu


def run(w, X, weights=None, excess=False):
    path, pot = lib_descriptors(w)
    x = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    grad = torch.empty_like(x)
    act = torch.empty(1, dtype=torch.float64, device="cuda")
    ps = torch.empty(w.n_steps, dtype=torch.float64, device="cuda")
    wt = None if weights is None else torch.from_numpy(np.asarray(weights, dtype=np.float64)).cuda()
    P.pamd_action_grad(path, pot, x, grad, action=act, per_step=ps, step_weights=wt)
    torch.cuda.synchronize()
    return float(act.item()), ps.cpu().numpy(), grad.cpu().numpy()


def test_ho1d_full(device):
    w, X = em_input("ho1d")
    s_ref, g_ref = oracle_full(w, X)
    S, s, g = run(w, X)
    assert rel(S, math.fsum(s_ref.tolist())) <= 1e-12
    assert np.max(np.abs(s - s_ref) / s_ref) <= 1e-12
    assert rel_inf(g, g_ref) <= 1e-10


def test_ho1d_closed_form_and_weights(device):
    w, X = em_input("ho1d")
    a = 1 - w.k * w.dt / w.gamma
    x = X[:, 0, 0]
    closed = np.sum((x[1:] - a * x[:-1]) ** 2) / (4 * w.D * w.dt)
    S, _, _ = run(w, X)
    assert rel(S, closed) <= 1e-12
    wts = np.random.default_rng(3).uniform(0.0, 3.0, size=w.n_steps)
    _, g_ref = oracle_full(w, X, weights=wts)
    _, _, g = run(w, X, weights=wts)
    assert rel_inf(g, g_ref) <= 1e-10


@pytest.mark.parametrize("n_dim,n_atoms,n_steps", [(3, 1, 17), (1, 5, 33), (3, 40, 65),
                                                   (3, 500, 9), (1, 1, 1), (1, 1, 2047),
                                                   (1, 1, 2048), (3, 40, 1000)])
def test_ho_shapes(device, n_dim, n_atoms, n_steps):
    """Paths that one workgroup covers (up to 2047 steps of one degree of
    freedom: the action is summed in the same launch) and larger ones (2048
    steps, 120 degrees of freedom x 1000 steps: many workgroups and a separate
    sum), against the oracle."""
    w = W.workload("ho1d")
    w = w.__class__(**{**w.__dict__, "n_dim": n_dim, "n_atoms": n_atoms, "n_steps": n_steps})
    xi, eta = W.draw_noise(w)
    X = OE.perturbed_em_path(np.zeros((n_dim, n_atoms)), xi, eta, w.perturb_sd, Harmonic(w.k),
                             w.dt, w.D, w.gamma)
    s_ref, g_ref = oracle_full(w, X)
    S, s, g = run(w, X)
    assert rel(S, math.fsum(s_ref.tolist())) <= 1e-12
    assert rel_inf(g, g_ref) <= 1e-10


def test_em_identity_on_gpu(device):
    # an unperturbed EM path returns sum |xi|^2 / 2 (Eq. 2 -> Eq. 3)
    w = W.workload("ho1d")
    xi, _ = W.draw_noise(w)
    X = OE.em_path(np.zeros((1, 1)), xi, Harmonic(w.k), w.dt, w.D, w.gamma)
    S, _, _ = run(w, X)
    assert rel(S, 0.5 * math.fsum((xi ** 2).ravel().tolist())) <= 1e-12
