"""Pins of the oracle's path action and gradient (Eqs. 2-4 and the derived adjoint).

* Euler-Maruyama identity: a path built by Eq. 2 from recorded noise xi has
  r_n = sqrt(2 D dt) xi_n, so S = sum |xi|^2 / 2 exactly (up to rounding).
* Harmonic closed form: S = sum (x_{n+1} - a x_n)^2 / (4 D dt), a = 1 - k dt/gamma,
  with a tridiagonal gradient.
* AR(1) law of the harmonic EM chain (mean a^n x_0, variance 2 D dt (1-a^{2n})/(1-a^2)).
* Normalisation: S + log_norm equals -sum log N(x_{n+1}; x_n + mu dt F, 2 D dt)
  evaluated with scipy's Gaussian density.
* Gradient: complex-step derivatives of S (independent of the adjoint code),
  central differences of the local action, translation invariance.
"""
import math

import numpy as np
import pytest
from scipy import stats

import workloads as W
from oracle import action as A
from oracle import em as E
from oracle import forces as F
from oracle.potentials import Harmonic, LennardJones


def _lj_em_path(n_atoms=108, n_steps=16, eta_sd=0.01, seed=5, dt=1e-4):
    w = W.workload("lj108").with_atoms(n_atoms).with_steps(n_steps)
    box = w.box
    lj = LennardJones(rc=min(2.5, 0.499 * box), box=box)
    x0 = W.initial_lattice(n_atoms, box)
    rng = np.random.default_rng(seed)
    xi = rng.standard_normal((n_steps, 3, n_atoms))
    eta = rng.standard_normal((n_steps, 3, n_atoms))
    X = E.em_path(x0, xi, lj, dt, w.D, w.gamma)
    Xp = X.copy()
    Xp[1:] += eta_sd * eta
    return X, Xp, xi, lj, w


def test_em_identity_lj():
    X, _, xi, lj, w = _lj_em_path(n_steps=24)
    S = A.path_action(X, lj, w.dt, w.D, w.gamma)
    ref = 0.5 * math.fsum((xi * xi).ravel().tolist())
    assert abs(S - ref) <= 1e-12 * ref


def test_em_identity_harmonic_and_closed_form():
    w = W.workload("ho1d")
    ho = Harmonic(k=w.k)
    xi, eta = W.draw_noise(w)
    X = E.em_path(np.zeros((1, 1)), xi, ho, w.dt, w.D, w.gamma)
    S = A.path_action(X, ho, w.dt, w.D, w.gamma)
    assert abs(S - 0.5 * np.sum(xi ** 2)) <= 1e-12 * S
    Xp = X.copy()
    Xp[1:] += w.perturb_sd * eta
    a = 1.0 - w.k * w.dt / w.gamma
    x = Xp[:, 0, 0]
    closed = np.sum((x[1:] - a * x[:-1]) ** 2) / (4 * w.D * w.dt)
    assert abs(A.path_action(Xp, ho, w.dt, w.D, w.gamma) - closed) <= 1e-12 * closed
    # tridiagonal gradient: g_m = c[(x_m - a x_{m-1}) - a (x_{m+1} - a x_m)], truncated at the ends
    c = 1.0 / (2 * w.D * w.dt)
    e = x[1:] - a * x[:-1]
    g = np.zeros_like(x)
    g[1:] += c * e
    g[:-1] += -c * a * e
    go = A.path_gradient(Xp, ho, w.dt, w.D, w.gamma)[:, 0, 0]
    assert np.max(np.abs(go - g)) <= 1e-10 * np.max(np.abs(g))


def test_ar1_law_of_harmonic_em_chain():
    # Many independent 1-D chains; z-scores of mean and variance at a few times.
    ho = Harmonic(k=1.0)
    dt, D, gamma = 0.05, 1.0, 1.0
    n_chain, n_steps, x0 = 20000, 40, 1.5
    rng = np.random.default_rng(99)
    xi = rng.standard_normal((n_steps, 1, n_chain))
    X = E.em_path(np.full((1, n_chain), x0), xi, ho, dt, D, gamma)
    a = 1 - dt / gamma
    for n in (1, 5, 20, 40):
        mean = a ** n * x0
        var = 2 * D * dt * (1 - a ** (2 * n)) / (1 - a ** 2)
        xs = X[n, 0]
        assert abs(xs.mean() - mean) / math.sqrt(var / n_chain) < 4.5
        assert abs(xs.var() - var) / (var * math.sqrt(2.0 / n_chain)) < 4.5
    # stationary variance 2 D dt/(1 - a^2) at dt = 0.01 is 1.0050251...
    a1 = 0.99
    assert abs(2 * 0.01 / (1 - a1 ** 2) - 1.0050251256281406) < 1e-12


def test_log_norm_against_gaussian_density():
    X, Xp, _, lj, w = _lj_em_path(n_atoms=32, n_steps=6)
    S = A.path_action(Xp, lj, w.dt, w.D, w.gamma)
    nll = 0.0
    for n in range(Xp.shape[0] - 1):
        mean = Xp[n] + w.dt / w.gamma * F.forces(Xp[n], lj)
        d = F.minimum_image(Xp[n + 1] - mean, lj.box)
        nll -= np.sum(stats.norm.logpdf(d, scale=math.sqrt(2 * w.D * w.dt)))
    assert abs(S + A.log_norm(6, 3, 32, w.D, w.dt) - nll) <= 1e-10 * abs(nll)


def test_gradient_complex_step():
    _, Xp, _, lj, w = _lj_em_path(n_atoms=32, n_steps=6, seed=8)
    g = A.path_gradient(Xp, lj, w.dt, w.D, w.gamma)
    rng = np.random.default_rng(3)
    h = 1e-30
    gmax = np.max(np.abs(g))
    for _ in range(16):
        idx = tuple(int(rng.integers(0, s)) for s in Xp.shape)
        Xc = Xp.astype(np.complex128)
        Xc[idx] += 1j * h
        cs = np.imag(A.path_action(Xc, lj, w.dt, w.D, w.gamma)) / h
        assert abs(cs - g[idx]) <= 1e-10 * gmax, idx


def test_weighted_gradient_complex_step():
    _, Xp, _, lj, w = _lj_em_path(n_atoms=32, n_steps=5, seed=9)
    wts = np.random.default_rng(4).uniform(0.5, 2.0, size=5)
    g = A.path_gradient(Xp, lj, w.dt, w.D, w.gamma, step_weights=wts)
    h = 1e-30
    for idx in [(0, 1, 3), (2, 0, 7), (5, 2, 31), (3, 1, 0)]:
        Xc = Xp.astype(np.complex128)
        Xc[idx] += 1j * h
        s = A.per_step_action(Xc, lj, w.dt, w.D, w.gamma)
        cs = np.imag(np.sum(wts * s)) / h
        assert abs(cs - g[idx]) <= 1e-10 * np.max(np.abs(g))


def test_gradient_local_central_difference_and_translation():
    _, Xp, _, lj, w = _lj_em_path(n_atoms=108, n_steps=8, seed=10)
    g = A.path_gradient(Xp, lj, w.dt, w.D, w.gamma)
    s = A.per_step_action(Xp, lj, w.dt, w.D, w.gamma)
    m, c, a = 4, 1, 17
    h = 1e-6

    def local(X):
        return np.sum(A.per_step_action(X[m - 1:m + 2], lj, w.dt, w.D, w.gamma))

    Xa, Xb = Xp.copy(), Xp.copy()
    Xa[m, c, a] += h
    Xb[m, c, a] -= h
    fd = (local(Xa) - local(Xb)) / (2 * h)
    assert abs(fd - g[m, c, a]) <= 1e-6 * np.max(np.abs(g[m]))
    # translation invariance: sum over atoms of g_m = c sum (r_{m-1} - r_m)
    r = A.residuals(Xp, lj, w.dt, w.D, w.gamma)
    cc = 1.0 / (2 * w.D * w.dt)
    lhs = g[m].sum(axis=1)
    rhs = cc * (r[m - 1] - r[m]).sum(axis=1)
    assert np.max(np.abs(lhs - rhs)) <= 1e-9 * np.max(np.abs(g[m]))
    assert s.shape == (8,)


def test_em_path_gradient_identity():
    # r_n = sqrt(2 D dt) xi_n on an unperturbed EM path, so
    # g_m = [xi_{m-1} - xi_m + mu dt H(x_m) xi_m] / sqrt(2 D dt)
    X, _, xi, lj, w = _lj_em_path(n_atoms=32, n_steps=4, seed=12)
    g = A.path_gradient(X, lj, w.dt, w.D, w.gamma)
    amp = math.sqrt(2 * w.D * w.dt)
    m = 2
    ref = (xi[m - 1] - xi[m] + w.dt / w.gamma * F.hessian_vec(X[m], xi[m], lj)) / amp
    assert np.max(np.abs(g[m] - ref)) <= 1e-10 * np.max(np.abs(ref))


def test_slice_terms_match_full():
    _, Xp, _, lj, w = _lj_em_path(n_atoms=32, n_steps=5, seed=13)
    g = A.path_gradient(Xp, lj, w.dt, w.D, w.gamma)
    s = A.per_step_action(Xp, lj, w.dt, w.D, w.gamma)
    for m in range(6):
        sm, gm = A.slice_terms(Xp, m, lj, w.dt, w.D, w.gamma)
        assert np.max(np.abs(gm - g[m])) <= 1e-13 * np.max(np.abs(g))
        if m < 5:
            assert abs(sm - s[m]) <= 1e-14 * s[m]


def test_paper_lj27_state_point():
    # Sec. IV B: 27 atoms, rho = 0.5, beta eps = 0.74, r_c = L/2 (one cell per axis)
    w = W.workload("lj27")
    lj = LennardJones(rc=w.cutoff, box=w.box)
    assert abs(w.cutoff - 0.5 * (27 / 0.5) ** (1 / 3)) < 1e-12
    x0 = W.initial_lattice(27, w.box)
    xi, eta = W.draw_noise(w, 8)
    X = E.em_path(x0, xi, lj, w.dt, w.D, w.gamma)
    S = A.path_action(X, lj, w.dt, w.D, w.gamma)
    assert abs(S - 0.5 * np.sum(xi ** 2)) <= 1e-12 * S
