"""GPU parity of the sequential Euler-Maruyama integrator (Eq. 2).

Three checks, each independent of trajectory divergence:

* elementwise against the oracle's em_path where the dynamics does not
  amplify rounding (harmonic: a contraction; Lennard-Jones: 200 steps of
  dt = 1e-4, far below the time over which chaos grows a 1e-16 difference);
* per step: the force the GPU applied, (x_{n+1} - x_n - sqrt(2 D dt) xi_n)
  gamma / dt, against the oracle's F(x_n) at the GPU's own x_n (normwise
  relative 1e-9: the subtraction loses about ulp(x) / (dt/gamma) ~ 1e-11 in
  force units against forces of order 10-100);
* the action identity: a path made from noise xi has r_n = sqrt(2 D dt) xi_n,
  so its per-step action (computed by the path kernel) is |xi_n|^2 / 2
  (relative 1e-9 per step: r_n keeps about 1e-14 relative after the
  cancellation in x_{n+1} - x_n - (dt/gamma) F).
"""
import dataclasses
import math

import numpy as np
import pytest
import torch

import paper_1907_09529_amd as P
import workloads as W
from oracle import em as OE
from oracle import forces as OF

from common import lib_descriptors, oracle_pot, rel

pytestmark = pytest.mark.gpu

FORCE_TOL = 1e-9
STEP_TOL = 1e-9


def integrate(w, x0, xi, tuning=None):
    path, pot = lib_descriptors(w)
    x0_d = torch.from_numpy(np.ascontiguousarray(x0)).cuda()
    xi_d = torch.from_numpy(np.ascontiguousarray(xi)).cuda()
    out = torch.empty((w.n_steps + 1,) + x0.shape, dtype=torch.float64, device="cuda")
    P.pamd_em_integrate(path, pot, x0_d, xi_d, out, tuning=tuning)
    torch.cuda.synchronize()
    return out


def per_step_action(w, X_d):
    path, pot = lib_descriptors(w)
    act = torch.empty(1, dtype=torch.float64, device="cuda")
    s = torch.empty(w.n_steps, dtype=torch.float64, device="cuda")
    P.pamd_action(path, pot, X_d, act, per_step=s)
    torch.cuda.synchronize()
    return float(act.item()), s.cpu().numpy()


def lj_inputs(name, n_steps=None, n_atoms=None):
    w = W.workload(name)
    if n_atoms:
        w = w.with_atoms(n_atoms)
    if n_steps:
        w = w.with_steps(n_steps)
    x0 = W.initial_lattice(w.n_atoms, w.box)
    xi, _ = W.draw_noise(w)
    return w, x0, xi


def check_forces(w, X, xi, picks, method="brute"):
    pot = oracle_pot(w)
    mu_dt = w.dt / w.gamma
    amp = math.sqrt(2.0 * w.D * w.dt)
    for n in picks:
        applied = (X[n + 1] - X[n] - amp * xi[n]) / mu_dt
        ref = OF.forces(X[n], pot, method)
        err = np.max(np.abs(applied - ref)) / max(np.max(np.abs(ref)), 1.0)
        assert err <= FORCE_TOL, (n, err)


def check_action_identity(w, X_d, xi):
    S, s = per_step_action(w, X_d)
    half = 0.5 * np.sum(xi.reshape(w.n_steps, -1) ** 2, axis=1)
    assert np.max(np.abs(s - half) / half) <= STEP_TOL
    assert rel(S, math.fsum(half.tolist())) <= STEP_TOL


def test_harmonic_matches_oracle(device):
    for n_atoms, n_dim in [(1, 1), (300, 3)]:   # one dof; 900 dofs (ragged over blocks)
        w = dataclasses.replace(W.workload("ho1d"), n_atoms=n_atoms, n_dim=n_dim)
        xi = np.random.default_rng(w.seed + 5).standard_normal((w.n_steps, n_dim, n_atoms))
        x0 = np.random.default_rng(w.seed + 6).standard_normal((n_dim, n_atoms))
        X = integrate(w, x0, xi).cpu().numpy()
        ref = OE.em_path(x0, xi, oracle_pot(w), w.dt, w.D, w.gamma)
        assert np.max(np.abs(X - ref)) <= 1e-13 * np.max(np.abs(ref)), (n_atoms, n_dim)
        assert np.array_equal(X[0], x0)


@pytest.mark.parametrize("name", ["lj108", "lj27"])
def test_lj_matches_oracle(device, name):
    """200 steps: atoms cross skin/2 and the lists are rebuilt several times
    (lj27: r_c = L/2, every pair in one list)."""
    w, x0, xi = lj_inputs(name, n_steps=200)
    X_d = integrate(w, x0, xi)
    X = X_d.cpu().numpy()
    ref = OE.em_path(x0, xi, oracle_pot(w), w.dt, w.D, w.gamma)
    assert np.max(np.abs(X - ref)) <= 1e-11 * w.box
    check_forces(w, X, xi, [0, 1, 99, 199])
    check_action_identity(w, X_d, xi)


def test_lj_skin_rebuild_every_step_and_determinism(device):
    w, x0, xi = lj_inputs("lj108", n_steps=64)
    t = P.make_tuning("fused", skin=0.01)   # skin/2 = 0.005: nearly every step rebuilds
    X1 = integrate(w, x0, xi, t)
    X2 = integrate(w, x0, xi, t)
    assert torch.equal(X1, X2)
    X = X1.cpu().numpy()
    check_forces(w, X, xi, range(0, 64, 7))
    ref = integrate(w, x0, xi).cpu().numpy()    # default skin, other list history
    assert np.max(np.abs(X - ref)) <= 1e-11 * w.box


def test_lj_one_step(device):
    w, x0, xi = lj_inputs("lj108", n_steps=1)
    X = integrate(w, x0, xi).cpu().numpy()
    ref = OE.em_path(x0, xi, oracle_pot(w), w.dt, w.D, w.gamma)
    assert np.max(np.abs(X - ref)) <= 1e-13 * w.box


def test_lj864_full_size(device):
    """The headline system at its full path length (864 atoms x 4096 steps)
    in the default launch configuration."""
    w, x0, xi = lj_inputs("lj864")
    X_d = integrate(w, x0, xi)
    X = X_d.cpu().numpy()
    assert np.all(np.isfinite(X))
    rng = np.random.default_rng(w.seed + 17)
    picks = {0, 1, w.n_steps - 1} | set(int(v) for v in rng.integers(0, w.n_steps, size=4))
    check_forces(w, X, xi, sorted(picks))
    check_action_identity(w, X_d, xi)


def test_lj4000_residuals_in_global_scratch(device):
    """4000 atoms: one slot array in LDS (x_{n+1} reloaded from x_out)."""
    w, x0, xi = lj_inputs("sweep4000", n_steps=48)
    X_d = integrate(w, x0, xi)
    X = X_d.cpu().numpy()
    check_forces(w, X, xi, [0, 1, 23, 47], method="cells")
    check_action_identity(w, X_d, xi)
