"""GPU parity of the Lennard-Jones path action and adjoint gradient against the oracle.

Tolerances (FP64 path): action and every per-step term within 1e-12 relative;
gradient within 1e-10 in the normwise sense ||g - g_ref||_inf / ||g_ref||_inf.

FP32-force variant: the pair products of the Hessian-vector pass
(a w + b (d.w) d) are rounded to float32 before the float64 sums; the pair
functions and the force pass stay float64, so the action is the float64
one.  The gradient is held to the variant's bound of 1e-8 and the action to
1e-12; both measured errors are printed.
"""
import math

import numpy as np
import pytest
import torch

import paper_1907_09529_amd as P
import workloads as W
from oracle import action as OA
from oracle import sampling as OS

from common import (em_input, lib_descriptors, oracle_full, oracle_pot, pairs_at_the_cutoff, rel,
                    rel_inf)

pytestmark = pytest.mark.gpu

ACTION_TOL = 1e-12
GRAD_TOL = 1e-10
GRAD_TOL_F32 = 1e-8
ACTION_TOL_F32 = 1e-12


def run(w, X, precision="fp64", tuning=None, weights=None):
    path, pot = lib_descriptors(w, precision)
    x = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    grad = torch.empty_like(x)
    act = torch.empty(1, dtype=torch.float64, device="cuda")
    per_step = torch.empty(w.n_steps, dtype=torch.float64, device="cuda")
    wt = None if weights is None else torch.from_numpy(np.asarray(weights, dtype=np.float64)).cuda()
    P.pamd_action_grad(path, pot, x, grad, action=act, per_step=per_step, step_weights=wt,
                       tuning=tuning)
    torch.cuda.synchronize()
    return float(act.item()), per_step.cpu().numpy(), grad.cpu().numpy()


def check(w, X, tuning=None, precision="fp64", weights=None, ref=None):
    s_ref, g_ref = ref if ref is not None else oracle_full(w, X, weights)
    S, s, g = run(w, X, precision, tuning, weights)
    S_ref = math.fsum(s_ref.tolist())
    gtol = GRAD_TOL if precision == "fp64" else GRAD_TOL_F32
    err_s = rel(S, S_ref)
    err_g = rel_inf(g, g_ref)
    if precision == "fp64":
        assert err_s <= ACTION_TOL, err_s
        assert np.max(np.abs(s - s_ref) / np.abs(s_ref)) <= ACTION_TOL
    else:
        print(f"FP32-force vs FP64 oracle: action {err_s:.3e}, gradient {err_g:.3e}")
        assert err_s <= ACTION_TOL_F32
    assert err_g <= gtol, err_g
    return err_s, err_g


@pytest.fixture(scope="module")
def lj108():
    return em_input("lj108")


@pytest.fixture(scope="module")
def lj108_ref(lj108):
    w, X = lj108
    return oracle_full(w, X)


def test_lj108_fused_fp64(device, lj108, lj108_ref):
    w, X = lj108
    check(w, X, ref=lj108_ref)


def test_lj108_plain_fp64(device, lj108, lj108_ref):
    w, X = lj108
    check(w, X, tuning=P.make_tuning("plain"), ref=lj108_ref)


def test_lj108_fp32_force(device, lj108, lj108_ref):
    w, X = lj108
    e_s, e_g = check(w, X, precision="fp32_force", ref=lj108_ref)
    print(f"lj108 FP32-force: action rel {e_s:.2e}, grad rel {e_g:.2e}")


def test_lj108_fp32_force_plain(device, lj108, lj108_ref):
    w, X = lj108
    check(w, X, precision="fp32_force", tuning=P.make_tuning("plain"), ref=lj108_ref)


@pytest.mark.parametrize("nlist", ["full", "half"])
@pytest.mark.parametrize("tile,skin,kmax", [(1, 0.3, 0), (7, 0.3, 0), (16, 1e-6, 0),
                                            (32, 0.9, 0), (5, 0.3, 4), (300, 0.3, 0)])
def test_lj108_tiles_skins_overflow(device, lj108, lj108_ref, tile, skin, kmax, nlist):
    w, X = lj108
    check(w, X, tuning=P.make_tuning("fused", tile=tile, skin=skin, max_neighbours=kmax,
                                     neighbour_list=nlist), ref=lj108_ref)


@pytest.mark.parametrize("block,nlist", [(64, "half"), (128, "half"), (192, "full"),
                                         (1024, "half"), (64, "full")])
def test_lj108_block_sizes(device, lj108, lj108_ref, block, nlist):
    w, X = lj108
    check(w, X, tuning=P.make_tuning("fused", block=block, neighbour_list=nlist), ref=lj108_ref)


def test_lj108_without_lists(device, lj108, lj108_ref):
    """108 atoms: the list sphere holds most of the 5.04-sigma box, so with
    one- and two-step tiles the plan builds no lists (reach -1) and both
    passes scan all atoms; longer tiles or a skin given in the tuning keep
    the lists.  All against the oracle."""
    w, X = lj108
    path, pot = lib_descriptors(w)
    assert P.pamd_launch_info(path, pot).reach == -1
    assert P.pamd_launch_info(path, pot, P.make_tuning("fused", tile=2)).reach == -1
    assert P.pamd_launch_info(path, pot, P.make_tuning("fused", tile=16)).reach >= 0
    assert P.pamd_launch_info(path, pot, P.make_tuning("fused", skin=0.5)).reach >= 0
    for tuning in (None, P.make_tuning("fused", tile=2), P.make_tuning("fused", tile=16),
                   P.make_tuning("fused", skin=0.5)):
        check(w, X, tuning=tuning, ref=lj108_ref)
    check(w, X, precision="fp32_force", tuning=P.make_tuning("fused", tile=2), ref=lj108_ref)


def test_lj108_step_weights(device, lj108):
    w, X = lj108
    wts = np.random.default_rng(5).uniform(-1.0, 2.0, size=w.n_steps)
    check(w, X, weights=wts)
    check(w, X, weights=wts, tuning=P.make_tuning("plain"))


def test_lj108_excess_action(device, lj108, lj108_ref):
    w, X = lj108
    path, pot = lib_descriptors(w)
    x = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    ex = torch.empty(w.n_steps, dtype=torch.float64, device="cuda")
    ps = torch.empty_like(ex)
    for tun in (None, P.make_tuning("plain")):
        P.pamd_excess_action(path, pot, x, ex, per_step=ps, tuning=tun)
        torch.cuda.synchronize()
        s0 = OS.free_step_action(X, w.D, w.dt, w.box)
        ref = lj108_ref[0] - s0
        # e_n is small against s_n: compare against the scale of s_n
        assert np.max(np.abs(ex.cpu().numpy() - ref)) <= 1e-11 * np.max(np.abs(lj108_ref[0]))
        assert np.max(np.abs(ps.cpu().numpy() - lj108_ref[0]) / lj108_ref[0]) <= ACTION_TOL


def test_lj108_action_only_matches(device, lj108, lj108_ref):
    w, X = lj108
    path, pot = lib_descriptors(w)
    x = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    act = torch.empty(1, dtype=torch.float64, device="cuda")
    ps = torch.empty(w.n_steps, dtype=torch.float64, device="cuda")
    P.pamd_action(path, pot, x, act, per_step=ps)
    torch.cuda.synchronize()
    assert rel(float(act.item()), math.fsum(lj108_ref[0].tolist())) <= ACTION_TOL


def test_bitwise_repeatable_full_lists(device, lj108):
    w, X = lj108
    t = P.make_tuning("fused", neighbour_list="full")
    a1 = run(w, X, tuning=t)
    a2 = run(w, X, tuning=t)
    assert a1[0] == a2[0]
    assert np.array_equal(a1[1], a2[1]) and np.array_equal(a1[2], a2[2])


def test_paper_lj27_state_point(device):
    w, X = em_input("lj27")
    check(w, X)
    check(w, X, tuning=P.make_tuning("plain"))


def test_single_step_and_short_paths(device):
    for n in (1, 2, 3):
        w, X = em_input("lj108", n_steps=n)
        check(w, X)
        check(w, X, tuning=P.make_tuning("plain"))


@pytest.mark.parametrize("n_atoms,box", [(1, 6.0), (2, 6.0), (3, 6.0), (3, 4.0)])
def test_tiny_systems(device, n_atoms, box):
    """One to three atoms: no pair at all (one atom: the action is the free
    Brownian one, sum |x_{n+1} - x_n|^2 / (4 D dt)), a single pair, and three
    atoms with lists (6-sigma box, r_c 2.5) and without (4-sigma box, r_c = L/2:
    the list sphere fills the box).  Seeded positions at least 1.1 sigma apart,
    then a seeded Euler-Maruyama path of the oracle; fused and unfused forms."""
    import dataclasses
    from oracle import em as OE
    w = dataclasses.replace(W.workload("lj108").with_steps(20), n_atoms=n_atoms,
                            density=n_atoms / box ** 3, rc=2.5 if box > 5.0 else 0.0)
    rng = np.random.default_rng(1900 + 10 * n_atoms + int(box))
    pts = []
    while len(pts) < n_atoms:
        p = rng.uniform(0.0, w.box, 3)
        if all(np.linalg.norm((p - q) - w.box * np.rint((p - q) / w.box)) >= 1.1 for q in pts):
            pts.append(p)
    x0 = np.ascontiguousarray(np.array(pts).T)
    xi, eta = W.draw_noise(w)
    X = OE.perturbed_em_path(x0, xi, eta, w.perturb_sd, oracle_pot(w), w.dt, w.D, w.gamma)
    ref = oracle_full(w, X)
    if box < 5.0:
        assert P.pamd_launch_info(*lib_descriptors(w)).reach == -1
    check(w, X, ref=ref)
    check(w, X, tuning=P.make_tuning("plain"), ref=ref)
    if n_atoms == 1:
        S, _, _ = run(w, X)
        free = math.fsum((np.diff(X, axis=0) ** 2).ravel().tolist()) / (4 * w.D * w.dt)
        assert rel(S, free) <= ACTION_TOL


def test_lj864_em_ragged_tiles(device):
    w, X = em_input("lj864", n_steps=40)
    ref = oracle_full(w, X)
    check(w, X, ref=ref)
    check(w, X, tuning=P.make_tuning("fused", tile=7), ref=ref)
    check(w, X, tuning=P.make_tuning("fused", tile=6, neighbour_list="full"), ref=ref)
    check(w, X, tuning=P.make_tuning("fused", tile=9, block=448), ref=ref)
    check(w, X, tuning=P.make_tuning("plain"), ref=ref)
    check(w, X, precision="fp32_force", ref=ref)


@pytest.mark.parametrize("rc", [2.6, 3.2])
def test_lj500_long_exact_rows(device, rc):
    """Cutoffs at which atoms have more partners within r_c than the 64
    shared-memory entries an atom's two lanes share (about 62 per atom on
    average at r_c = 2.6, so some atoms overflow and most do not; about 116
    at 3.2, so every atom does and pass 2 walks its candidate rows again with
    the cutoff test); against the oracle and the form with the exact lists in
    device memory (two slot arrays)."""
    import dataclasses
    from oracle import em as OE
    w = dataclasses.replace(W.workload("lj108").with_atoms(500).with_steps(12), rc=rc)
    pot = oracle_pot(w)
    xi, eta = W.draw_noise(w)
    X = OE.perturbed_em_path(W.initial_lattice(w.n_atoms, w.box), xi, eta, w.perturb_sd, pot,
                             w.dt, w.D, w.gamma)
    ref = oracle_full(w, X)
    path, lpot = lib_descriptors(w)
    assert P.pamd_launch_info(path, lpot).lds_bytes > 0
    check(w, X, ref=ref)
    check(w, X, tuning=P.make_tuning("fused", slot_arrays=2), ref=ref)
    check(w, X, tuning=P.make_tuning("fused", tile=3, skin=0.05), ref=ref)
    check(w, X, precision="fp32_force", ref=ref)


def test_lj108_dilute_few_partners(device):
    """A dilute gas (density 0.05, about three partners within r_c per atom,
    many atoms with none or one) from seeded random positions at least one
    sigma apart: the exact rows hold empty, single and odd splits between an
    atom's two lanes; against the oracle in the default form (exact lists in
    LDS), the two-array form and the unfused form."""
    import dataclasses
    from oracle import em as OE
    w = dataclasses.replace(W.workload("lj108").with_steps(24), density=0.05)
    rng = np.random.default_rng(1907)
    pts = []
    while len(pts) < w.n_atoms:                 # random sequential placement
        p = rng.uniform(0.0, w.box, 3)
        if all(np.sum((d := (p - q) - w.box * np.rint((p - q) / w.box)) * d) >= 1.0 for q in pts):
            pts.append(p)
    x0 = np.ascontiguousarray(np.array(pts).T)
    pot = oracle_pot(w)
    xi, eta = W.draw_noise(w)
    X = OE.perturbed_em_path(x0, xi, eta, w.perturb_sd, pot, w.dt, w.D, w.gamma)
    ref = oracle_full(w, X)
    path, lpot = lib_descriptors(w)
    assert P.pamd_launch_info(path, lpot).exact_lists == 1
    check(w, X, ref=ref)
    check(w, X, tuning=P.make_tuning("fused", slot_arrays=2), ref=ref)
    check(w, X, tuning=P.make_tuning("plain"), ref=ref)


def test_pairs_at_the_list_limit(device):
    """Pairs that reach r_c (1 -/+ 1e-11) at one slice of every 16 (see
    common.pairs_at_the_cutoff): with one-step tiles (no reach, so only the float32
    scan's margin keeps the inner pairs), 16-step tiles aligned with the
    closest approaches (the per-atom reach test at its limiting case), ragged
    5-step tiles with a small skin, the two-array form and the unfused form.
    The force-shifted pair force vanishes at r_c but its Hessian does not:
    an inner pair dropped, or an outer one kept, moves the gradient by ~1e-5
    of its largest entry."""
    w, X = pairs_at_the_cutoff(48)
    ref = oracle_full(w, X)
    path, lpot = lib_descriptors(w)
    assert P.pamd_launch_info(path, lpot).exact_lists == 1
    for tuning in (None, P.make_tuning("fused", tile=1), P.make_tuning("fused", tile=16),
                   P.make_tuning("fused", tile=5, skin=0.05),
                   P.make_tuning("fused", tile=16, slot_arrays=2),
                   P.make_tuning("plain")):
        check(w, X, tuning=tuning, ref=ref)


def test_largest_exact_list_system(device):
    """887 atoms, the largest system whose exact lists fit in LDS (its plan
    uses all but 14 of the 163840 bytes; 888 atoms take the two-array form):
    one-step, 8-step and ragged 5-step tiles against the oracle.  The start is
    887 of the 1000 sites of a simple-cubic lattice of spacing 1.07 sigma
    filling the box (density 0.724; r_c lies between the fifth and sixth
    shells, so about 50 partners per atom and few overflowing rows), then a
    seeded Euler-Maruyama path of the oracle."""
    import dataclasses
    from oracle import em as OE
    w = dataclasses.replace(W.workload("lj108").with_atoms(887).with_steps(24),
                            density=887 / 10.7 ** 3)
    g = (np.arange(10) + 0.5) * (w.box / 10)
    x0 = np.ascontiguousarray(np.stack(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)[:, :887])
    xi, eta = W.draw_noise(w)
    X = OE.perturbed_em_path(x0, xi, eta, w.perturb_sd, oracle_pot(w), w.dt, w.D, w.gamma)
    path, lpot = lib_descriptors(w)
    info = P.pamd_launch_info(path, lpot)
    assert info.exact_lists == 1 and 163840 - 64 < info.lds_bytes <= 163840
    w888 = dataclasses.replace(w.with_atoms(888), density=888 / 10.7 ** 3)
    assert P.pamd_launch_info(*lib_descriptors(w888)).exact_lists == 0
    ref = oracle_full(w, X)
    for tuning in (None, P.make_tuning("fused", tile=8), P.make_tuning("fused", tile=5)):
        check(w, X, tuning=tuning, ref=ref)


def test_lj500_cell_list_path(device):
    # 500 atoms: n_c = 3 cells of edge >= 2.8 (reach 1) or 5 with reach 2
    w, X = em_input("lj108", n_atoms=500, n_steps=24)
    ref = oracle_full(w, X)
    check(w, X, ref=ref)
    check(w, X, tuning=P.make_tuning("fused", skin=0.05), ref=ref)
    check(w, X, tuning=P.make_tuning("plain"), ref=ref)


# ---------------------------------------------------------------------------
# Full-size headline workload (864 atoms x 4096 steps), default launch shape.
# The oracle checks sampled slices one by one; the rest is checked through
# properties that hold at any size.
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def lj864_full():
    w = W.workload("lj864")
    X = W.tethered_path(w)
    return w, X


def _sample_slices(w, tile):
    """Slices on both sides of the first two tile edges and of the last one,
    the path's ends, and six random slices."""
    rng = np.random.default_rng(w.seed + 11)
    last_edge = (w.n_steps - 1) // tile * tile
    picks = {0, 1, w.n_steps - 1, w.n_steps, tile - 1, tile, tile + 1, 2 * tile - 1, 2 * tile,
             2 * tile + 1, last_edge - 1, last_edge, last_edge + 1}
    picks |= set(int(v) for v in rng.integers(0, w.n_steps + 1, size=6))
    return sorted(p for p in picks if 0 <= p <= w.n_steps)


def test_lj864_full_size_sampled(device, lj864_full):
    w, X = lj864_full
    S, s, g = run(w, X)
    assert np.all(s > 0) and np.all(np.isfinite(g))
    assert rel(S, math.fsum(s.tolist())) <= 1e-13
    pot = oracle_pot(w)
    path, lpot = lib_descriptors(w)
    tile = P.pamd_launch_info(path, lpot).tile   # the launch run() used (default tuning)
    assert 1 <= tile < w.n_steps
    picks = _sample_slices(w, tile)
    print(f"lj864 full size: tile {tile}, sampled slices {picks}")
    for m in picks:
        sm, gm = OA.slice_terms(X, m, pot, w.dt, w.D, w.gamma)
        assert rel_inf(g[m], gm) <= GRAD_TOL, m
        if sm is not None:
            assert rel(s[m], sm) <= ACTION_TOL, m


def test_lj864_full_size_fused_equals_plain(device, lj864_full):
    w, X = lj864_full
    S1, s1, g1 = run(w, X)
    S2, s2, g2 = run(w, X, tuning=P.make_tuning("plain"))
    assert rel(S1, S2) <= ACTION_TOL
    assert rel_inf(g1, g2) <= GRAD_TOL
    S4, s4, g4 = run(w, X, tuning=P.make_tuning("fused", neighbour_list="full"))
    assert rel(S1, S4) <= ACTION_TOL
    assert rel_inf(g1, g4) <= GRAD_TOL


@pytest.mark.xfail(strict=True, reason="float32 Hessian-vector pair products move the gradient "
                   "of the 864 x 4096 path by ~5e-8 of its largest entry, above the 1e-8 bound "
                   "(which holds on the shorter and smaller paths); no float32 split of the pair "
                   "arithmetic meets it at this size")
def test_lj864_full_size_fp32_force_bound(device, lj864_full):
    w, X = lj864_full
    S1, s1, g1 = run(w, X)
    S3, s3, g3 = run(w, X, precision="fp32_force")
    e_s, e_g = rel(S3, S1), rel_inf(g3, g1)
    print(f"lj864 full FP32-force vs FP64: action rel {e_s:.2e}, grad rel {e_g:.2e}")
    assert e_s <= ACTION_TOL_F32
    assert e_g <= GRAD_TOL_F32


def test_lj864_fd_gradient_16_coordinates(device, lj864_full):
    """Central differences of the local action s_{m-1} + s_m (library-evaluated on
    the 3-slice sub-path) against the adjoint gradient at 16 random coordinates."""
    w, X = lj864_full
    _, _, g = run(w, X)
    rng = np.random.default_rng(w.seed + 1)
    h = 1e-6
    for _ in range(16):
        m = int(rng.integers(0, w.n_steps + 1))
        c = int(rng.integers(0, 3))
        a = int(rng.integers(0, w.n_atoms))
        lo, hi = max(0, m - 1), min(w.n_steps, m + 1)
        sub = np.ascontiguousarray(X[lo:hi + 1]).copy()
        vals = []
        for sgn in (+1, -1):
            Y = sub.copy()
            Y[m - lo, c, a] += sgn * h
            ws = w.with_steps(hi - lo)
            path, pot = lib_descriptors(ws)
            act = torch.empty(1, dtype=torch.float64, device="cuda")
            P.pamd_action(path, pot, torch.from_numpy(Y).cuda(), act)
            torch.cuda.synchronize()
            vals.append(float(act.item()))
        fd = (vals[0] - vals[1]) / (2 * h)
        scale = max(abs(g[m, c, a]), 1e-3 * np.max(np.abs(g[m])))
        assert abs(fd - g[m, c, a]) <= 2e-5 * scale + 1e-6 * np.max(np.abs(g[m])), (m, c, a)


# ---------------------------------------------------------------------------
# Path-sampling size: 4000 atoms.  A slice does not fit the workgroup's LDS
# with its residuals, so they live in global scratch and the cell grid is the
# finest that fits; the oracle (cell-list mode) checks sampled slices.
# ---------------------------------------------------------------------------
def _check_sampled(w, X, S, s, g, picks):
    assert np.all(s > 0) and np.all(np.isfinite(g))
    assert rel(S, math.fsum(s.tolist())) <= 1e-13
    pot = oracle_pot(w)
    for m in picks:
        sm, gm = OA.slice_terms(X, m, pot, w.dt, w.D, w.gamma, method="cells")
        assert rel_inf(g[m], gm) <= GRAD_TOL, m
        if sm is not None:
            assert rel(s[m], sm) <= ACTION_TOL, m


def test_lj4000_ragged_tiles_sampled(device):
    w = W.workload("sweep4000").with_steps(100)
    X = W.tethered_path(w)
    S, s, g = run(w, X, tuning=P.make_tuning("fused", tile=32))
    # tile edges (32, 64, 96), the ragged last tile (96..99) and both ends
    _check_sampled(w, X, S, s, g, [0, 1, 31, 32, 33, 64, 95, 96, 99, 100])


@pytest.mark.parametrize("nlist", ["full", "half"])
def test_lj2048_one_slot_array_sampled(device, nlist):
    """2048 atoms: rho in LDS with one slot array (two do not fit), so the
    next slice loads after pass 2 and the per-atom list reaches wait in
    global scratch; 16-step tiles and a ragged last tile."""
    w = W.workload("lj864").with_atoms(2048).with_steps(70)
    X = W.tethered_path(w)
    S, s, g = run(w, X, tuning=P.make_tuning("fused", tile=16, neighbour_list=nlist))
    _check_sampled(w, X, S, s, g, [0, 1, 15, 16, 17, 47, 48, 63, 64, 69, 70])


def test_sweep4000_full_size_sampled(device):
    """The path-sampling workload at full size (4000 atoms x 16384 steps,
    1.6 GB of coordinates) in the default launch configuration."""
    w = W.workload("sweep4000")
    X = W.tethered_path(w)
    S, s, g = run(w, X)
    tile = max(1, min(32, w.n_steps // 256))
    rng = np.random.default_rng(w.seed + 11)
    picks = {0, tile - 1, tile, w.n_steps - 1, w.n_steps}
    picks |= set(int(v) for v in rng.integers(0, w.n_steps + 1, size=3))
    _check_sampled(w, X, S, s, g, sorted(picks))


@pytest.mark.parametrize("variant", ["default", "half", "skin", "ragged_tile", "fp32", "n4000"])
def test_action_kernel_matches_gradient_kernel(device, variant):
    """The action-only kernel (pamd_action, pamd_excess_action) runs the same
    force pass as the gradient kernel without recording exact lists: its
    per-step terms equal the gradient call's bit for bit with full lists, and
    to rounding with half lists (whose LDS atomics add in arrival order)."""
    name, steps, tuning, precision = "lj108", 256, None, "fp64"
    if variant == "half":
        tuning = P.make_tuning("fused", block=448, neighbour_list="half")
    elif variant == "skin":
        tuning = P.make_tuning("fused", skin=0.05, tile=16)     # rebuilds inside tiles
    elif variant == "ragged_tile":
        tuning = P.make_tuning("fused", tile=7)
    elif variant == "fp32":
        precision = "fp32_force"
    elif variant == "n4000":
        name, steps = "sweep4000", 40
    w = W.workload(name).with_steps(steps)
    X = W.tethered_path(w)
    path, pot = lib_descriptors(w, precision)
    x = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    ps_a = torch.empty(w.n_steps, dtype=torch.float64, device="cuda")
    ps_g = torch.empty_like(ps_a)
    ex = torch.empty_like(ps_a)
    act = torch.empty(1, dtype=torch.float64, device="cuda")
    P.pamd_action(path, pot, x, act, per_step=ps_a, tuning=tuning)
    P.pamd_excess_action(path, pot, x, ex, tuning=tuning)
    P.pamd_action_grad(path, pot, x, torch.empty_like(x), per_step=ps_g, tuning=tuning)
    torch.cuda.synchronize()
    if variant == "half":
        assert float(((ps_a - ps_g).abs() / ps_g).max()) <= 1e-13
    else:
        assert torch.equal(ps_a, ps_g)
    s0 = OS.free_step_action(X, w.D, w.dt, w.box)
    assert np.max(np.abs(ex.cpu().numpy() - (ps_g.cpu().numpy() - s0))) <= \
        1e-11 * float(ps_g.max())
    assert rel(float(act.item()), math.fsum(ps_g.cpu().numpy().tolist())) <= 1e-13
