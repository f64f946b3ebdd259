"""GPU parity of the gradient-informed (Metropolis-adjusted Langevin) path move.

* Against the oracle's langevin_step with the same Philox streams: the same
  decisions move by move, log alpha within 1e-9 (relative to max(1, |log
  alpha|): sums of squares over the path in a different order), and the
  final paths within 1e-10 (harmonic) and 1e-10 L (Lennard-Jones, 108 atoms).
* On the GPU alone: from an exact sample of 256 independent harmonic chains
  the move keeps the conditional law of the Euler chain (Eq. 2) at
  dt = 0.4.
"""
import dataclasses
import math

import numpy as np
import pytest
import torch

import paper_1907_09529_amd as P
import workloads as W
from oracle import em as OE
from oracle import langevin as OL

from common import lib_descriptors, oracle_pot

pytestmark = pytest.mark.gpu

A = 0.6


def exact_paths(rng, n_steps, n_dof, x0=1.0):
    X = np.zeros((n_steps + 1, 1, n_dof))
    X[0] = x0
    for n in range(n_steps):
        X[n + 1] = A * X[n] + math.sqrt(0.8) * rng.standard_normal((1, n_dof))
    return X


class Chain:
    def __init__(self, w, X, tau, seed):
        self.path, self.pot = lib_descriptors(w)
        self.x = torch.from_numpy(np.ascontiguousarray(X)).cuda()
        self.g = torch.empty_like(self.x)
        self.S = torch.empty(1, dtype=torch.float64, device="cuda")
        P.pamd_action_grad(self.path, self.pot, self.x, self.g, action=self.S)
        self.y, self.gy = torch.empty_like(self.x), torch.empty_like(self.x)
        self.counter = torch.zeros(1, dtype=torch.int64, device="cuda")
        self.acc = torch.empty(1, dtype=torch.int32, device="cuda")
        self.la = torch.empty(1, dtype=torch.float64, device="cuda")
        self.ws = P.workspace(P.pamd_langevin_workspace_size(self.path, self.pot))
        self.tau, self.seed = tau, seed

    def step(self):
        P.pamd_langevin_step(self.path, self.pot, self.seed, self.tau, self.counter, self.x,
                             self.g, self.S, self.y, self.gy, self.acc, self.la, ws=self.ws)


def compare_with_oracle(w, X, tau, seed, moves, tol):
    c = Chain(w, X, tau, seed)
    pot = oracle_pot(w)
    Xo = X.copy()
    n_acc = 0
    for m in range(moves):
        c.step()
        torch.cuda.synchronize()
        r = OL.langevin_step(Xo, pot, w.dt, w.D, w.gamma, tau, seed, m)
        Xo = r["path"]
        assert bool(c.acc.item()) == r["accepted"], m
        la = float(c.la.item())
        assert abs(la - r["log_alpha"]) <= 1e-9 * max(1.0, abs(r["log_alpha"])), m
        n_acc += r["accepted"]
    assert np.max(np.abs(c.x.cpu().numpy() - Xo)) <= tol
    assert int(c.counter.item()) == moves
    return n_acc


def test_harmonic_matches_oracle(device):
    w = dataclasses.replace(W.workload("ho1d"), n_steps=8, n_atoms=6, dt=0.4)
    X = exact_paths(np.random.default_rng(3), 8, 6)
    n_acc = compare_with_oracle(w, X, 0.1, 41, 40, 1e-10)
    assert 0 < n_acc < 40


def test_lj108_matches_oracle(device):
    w = W.workload("lj108").with_steps(32)
    x0 = W.initial_lattice(w.n_atoms, w.box)
    xi, _ = W.draw_noise(w)
    X = OE.em_path(x0, xi, oracle_pot(w), w.dt, w.D, w.gamma)
    n_acc = compare_with_oracle(w, X, 5e-6, 7, 8, 1e-10 * w.box)
    assert 0 < n_acc < 8      # both branches of the decision


def test_move_keeps_the_path_distribution(device):
    w = dataclasses.replace(W.workload("ho1d"), n_steps=8, n_atoms=256, dt=0.4)
    X = exact_paths(np.random.default_rng(1), 8, 256)
    c = Chain(w, X, 0.05, 5)
    xs, acc = [], 0
    for m in range(3000):
        c.step()
        acc += int(c.acc.item()) if m % 50 == 0 else 0
        if m % 5 == 0:
            xs.append(c.x[:, 0, :].clone())
    xs = torch.stack(xs).cpu().numpy()
    for n in (4, 8):
        mean = A ** n
        var = 0.8 * (1 - A ** (2 * n)) / (1 - A * A)
        assert abs(xs[:, n].mean() - mean) < 0.04, n
        assert abs(xs[:, n].var() / var - 1) < 0.04, n
    # the gradient and action kept with the path stay those of the path
    g = torch.empty_like(c.x)
    S = torch.empty(1, dtype=torch.float64, device="cuda")
    P.pamd_action_grad(c.path, c.pot, c.x, g, action=S)
    torch.cuda.synchronize()
    assert torch.allclose(g, c.g, rtol=0, atol=1e-12 * float(g.abs().max()))
    assert abs(float(S.item()) - float(c.S.item())) <= 1e-12 * abs(float(S.item()))
