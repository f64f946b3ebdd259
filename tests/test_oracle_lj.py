"""Pins of the oracle's potentials, forces and Hessian-vector products.

Each check ties the oracle to something other than itself: hand-evaluated
closed forms of Eq. 16, complex-step derivatives (exact to rounding, no
truncation error), Newton's third law, lattice symmetry, and brute-force
versus cell-list enumeration.
"""
import os

import numpy as np
import pytest

import workloads as W
from oracle import forces as F
from oracle.potentials import LennardJones, Harmonic

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    out = {}
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith("#") or not line.strip():
            continue
        k, r, v = line.split()
        out[k] = (float(r), float(v))
    return out


def test_closed_form_values_eq16():
    g = _golden("lj_closed_forms.txt")
    lj = LennardJones(rc=2.5)
    checks = {"u_at_sigma": lj.u, "u_at_min": lj.u, "du_at_min": lj.du, "u_at_2": lj.u,
              "du_at_2": lj.du, "d2u_at_2": lj.d2u, "u_at_rc": lj.u, "du_at_rc": lj.du,
              "U_at_min_rc25": lj.U, "U_at_2_rc25": lj.U}
    for k, fn in checks.items():
        r, v = g[k]
        assert abs(fn(r) - v) <= 1e-14 * max(1.0, abs(v)), k


def test_shifted_potential_vanishes_at_cutoff():
    lj = LennardJones(rc=2.5)
    assert abs(lj.U(2.5)) < 1e-17
    assert abs(lj.dU(2.5)) < 1e-17


@pytest.mark.parametrize("r", [0.95, 1.1, 1.5, 2.2, 2.49])
def test_pair_derivatives_complex_step(r):
    lj = LennardJones(rc=2.5)
    h = 1e-30
    assert abs(np.imag(lj.U(r + 1j * h)) / h - lj.dU(r)) <= 1e-13 * max(1, abs(lj.dU(r)))
    assert abs(np.imag(lj.dU(r + 1j * h)) / h - lj.d2U(r)) <= 1e-13 * max(1, abs(lj.d2U(r)))


def _disordered(n_atoms, density, seed, sd=0.12):
    box = W.box_length(n_atoms, density)
    x = W.initial_lattice(n_atoms, box)
    rng = np.random.default_rng(seed)
    return x + sd * rng.standard_normal(x.shape), box


def test_force_is_minus_energy_gradient_complex_step():
    x, box = _disordered(32, 0.8442, 11)
    lj = LennardJones(rc=0.5 * box * 0.999, box=box)
    f = F.forces(x, lj)
    h = 1e-30
    g = np.zeros_like(x)
    for c in range(3):
        for a in range(x.shape[1]):
            xc = x.astype(np.complex128)
            xc[c, a] += 1j * h
            g[c, a] = np.imag(F.energy(xc, lj)) / h
    assert np.max(np.abs(f + g)) <= 1e-12 * np.max(np.abs(f))


def test_newton_third_law_and_lattice_zero():
    x, box = _disordered(108, 0.8442, 12)
    lj = LennardJones(rc=2.5, box=box)
    f = F.forces(x, lj)
    assert np.max(np.abs(f.sum(axis=1))) <= 1e-12 * np.max(np.abs(f))
    for n in (108, 256, 500):
        box = W.box_length(n, 0.8442)
        xl = W.fcc_lattice(n, box)
        fl = F.forces(xl, LennardJones(rc=2.5, box=box))
        assert np.max(np.abs(fl)) < 1e-12


def test_hessian_vector_complex_step_and_symmetry():
    x, box = _disordered(32, 0.8442, 13)
    lj = LennardJones(rc=0.5 * box * 0.999, box=box)
    rng = np.random.default_rng(14)
    v = rng.standard_normal(x.shape)
    w = rng.standard_normal(x.shape)
    hv = F.hessian_vec(x, v, lj)
    h = 1e-30
    fd = -np.imag(F.forces(x + 1j * h * v, lj)) / h   # H v = -dF/dx . v
    assert np.max(np.abs(hv - fd)) <= 1e-12 * np.max(np.abs(hv))
    hw = F.hessian_vec(x, w, lj)
    assert abs(np.sum(w * hv) - np.sum(v * hw)) <= 1e-12 * abs(np.sum(w * hv))
    # rows of H sum to zero: a uniform translation is a null vector
    t = np.ones_like(x) * np.array([[0.3], [-0.7], [1.1]])
    assert np.max(np.abs(F.hessian_vec(x, t, lj))) <= 1e-10


def test_hessian_vector_central_difference():
    x, box = _disordered(108, 0.8442, 15)
    lj = LennardJones(rc=2.5, box=box)
    v = np.random.default_rng(16).standard_normal(x.shape)
    h = 1e-6
    fd = -(F.forces(x + h * v, lj) - F.forces(x - h * v, lj)) / (2 * h)
    hv = F.hessian_vec(x, v, lj)
    assert np.max(np.abs(hv - fd)) <= 1e-5 * np.max(np.abs(hv))


@pytest.mark.parametrize("n_atoms,rc", [(500, 2.5), (108, 1.5), (256, 2.0)])
def test_brute_force_equals_cell_list(n_atoms, rc):
    x, box = _disordered(n_atoms, 0.8442, 17 + n_atoms)
    lj = LennardJones(rc=rc, box=box)
    assert int(np.floor(box / rc)) >= 3
    ib, jb, _ = F.pairs_brute(x, lj)
    ic, jc, _ = F.pairs_cells(x, lj)
    assert sorted(zip(ib.tolist(), jb.tolist())) == sorted(zip(ic.tolist(), jc.tolist()))
    fb = F.forces(x, lj, "brute")
    fc = F.forces(x, lj, "cells")
    assert np.max(np.abs(fb - fc)) <= 1e-13 * np.max(np.abs(fb))
    v = np.random.default_rng(3).standard_normal(x.shape)
    qb = F.hessian_vec(x, v, lj, "brute")
    qc = F.hessian_vec(x, v, lj, "cells")
    assert np.max(np.abs(qb - qc)) <= 1e-13 * np.max(np.abs(qb))


def test_neighbour_count_matches_density():
    # mean partners within r_c is rho * 4/3 pi r_c^3 (55.25 at rho = 0.8442, r_c = 2.5)
    x, box = _disordered(500, 0.8442, 21, sd=0.15)
    cnt = F.neighbour_counts(x, LennardJones(rc=2.5, box=box))
    expect = 0.8442 * 4.0 / 3.0 * np.pi * 2.5 ** 3
    assert abs(cnt.mean() - expect) < 2.0


def test_harmonic_forces():
    x = np.random.default_rng(1).standard_normal((3, 5))
    ho = Harmonic(k=2.0)
    assert np.allclose(F.forces(x, ho), -2.0 * x, rtol=0, atol=0)
    assert np.allclose(F.hessian_vec(x, x, ho), 2.0 * x, rtol=0, atol=0)


def test_minimum_image_half_even():
    d = np.array([0.5, -0.5, 1.5, 2.49, -2.51]) * 2.0
    out = F.minimum_image(d, 2.0)
    assert np.allclose(out, np.array([1.0, -1.0, -1.0, 0.98, 0.98]), atol=1e-12)


def test_cutoff_edge_pairs_decide_the_gradient():
    """The pairs that the GPU list-limit test runs (common.pairs_at_the_cutoff,
    closest approaches at r_c (1 -/+ 1e-11)) make the oracle's gradient
    depend on each pair's cutoff decision far above the 1e-10 parity bound:
    moving r_c by 2e-11 relative, which drops the inner pairs at their closest
    approach or admits the outer ones, changes it by more than 1e-7 of its
    largest entry.  Atoms of different pairs stay more than r_c + 1 apart, so
    only the designed pairs interact."""
    import dataclasses

    from common import oracle_full, pairs_at_the_cutoff, rel_inf
    w, X = pairs_at_the_cutoff(48)
    L = w.box
    for n in range(X.shape[0]):
        d = X[n].T[:, None, :] - X[n].T[None, :, :]
        d -= L * np.rint(d / L)
        r = np.sqrt(np.sum(d * d, axis=-1))
        other = np.arange(54)[:, None] // 2 != np.arange(54)[None, :] // 2
        assert r[other].min() > w.cutoff + 1.0
    _, g0 = oracle_full(w, X)
    for f in (1.0 - 2e-11, 1.0 + 2e-11):
        _, g1 = oracle_full(dataclasses.replace(w, rc=w.cutoff * f), X)
        assert rel_inf(g1, g0) > 1e-7
