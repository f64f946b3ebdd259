"""Invariants of the launch planner over many problem shapes, checked on the
host through pamd_launch_info and pamd_workspace_size (no device is touched):
shared memory within a workgroup's 160 KB, tiles that cover every step, the
exact-list form only where one thread holds each atom, its workspace without
room for exact lists, and the unfused form's thread-per-atom workgroups."""
import os

import pytest

import paper_1907_09529_amd as P
from paper_1907_09529_amd import _lib

pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH),
                                reason="libpamd.so not built (run __graft_entry__.build())")

LDS_MAX = 160 * 1024


def lj(n_atoms, n_steps, density=0.8442, rc=2.5, precision="fp64"):
    box = (n_atoms / density) ** (1.0 / 3.0)
    rc = min(rc, 0.5 * box)
    return (P.make_path(n_steps, n_atoms, 3, 1e-4, 1.0, 1.0, precision),
            P.make_potential("lj", rc=rc, box=box))


SHAPES = [(n, s) for n in (2, 27, 64, 108, 256, 500, 864, 900, 1000, 2048, 4000)
          for s in (1, 3, 17, 256, 4096)]


@pytest.mark.parametrize("n_atoms,n_steps", SHAPES)
def test_fused_plan_invariants(n_atoms, n_steps):
    path, pot = lj(n_atoms, n_steps)
    info = P.pamd_launch_info(path, pot)
    assert info.algo == _lib.PAMD_ALGO_FUSED
    assert 0 < info.lds_bytes <= LDS_MAX
    assert info.block % 64 == 0 and 64 <= info.block <= 1024
    assert info.tile >= 1 and info.tile * info.n_tiles >= n_steps
    assert (info.tile * (info.n_tiles - 1)) < n_steps            # no empty tile
    assert 1 <= info.grid <= min(info.n_tiles, 2048)
    if info.exact_lists:
        assert n_atoms <= info.block and info.slot_arrays == 1
        two = P.make_tuning("fused", slot_arrays=2)
        two_info = P.pamd_launch_info(path, pot, two)
        assert two_info.exact_lists == 0
        if two_info.grid == info.grid and two_info.block == info.block:
            # the exact-list plan keeps no exact lists in device memory (for
            # tiny systems the aligned sizes can coincide)
            ws, ws2 = P.pamd_workspace_size(path, pot), P.pamd_workspace_size(path, pot, two)
            assert ws < ws2 if n_atoms >= 64 else ws <= ws2


@pytest.mark.parametrize("n_atoms", [2, 27, 108, 500, 864, 1000, 2048])
def test_plain_plan_invariants(n_atoms):
    path, pot = lj(n_atoms, 64)
    info = P.pamd_launch_info(path, pot, P.make_tuning("plain"))
    assert info.algo == _lib.PAMD_ALGO_PLAIN
    assert info.block == min(1024, -(-n_atoms // 64) * 64)        # one thread per atom
    assert 0 < info.lds_bytes <= LDS_MAX
    assert info.tile == 1 and info.n_tiles == 64


def test_headline_plan():
    # 864 atoms x 4096 steps: one 16-step tile per compute unit, exact lists in LDS
    path, pot = lj(864, 4096)
    info = P.pamd_launch_info(path, pot)
    assert (info.block, info.tile, info.n_tiles, info.grid) == (1024, 16, 256, 256)
    assert info.exact_lists == 1 and info.cells == 10 and info.reach == 3
    assert P.pamd_workspace_size(path, pot) < _lib.PAMD_NOALLOC_SCRATCH_BYTES


def test_fp32_force_plans_like_fp64():
    a = P.pamd_launch_info(*lj(864, 4096))
    b = P.pamd_launch_info(*lj(864, 4096, precision="fp32_force"))
    assert (a.block, a.tile, a.exact_lists, a.lds_bytes) == (b.block, b.tile, b.exact_lists,
                                                             b.lds_bytes)


def test_no_lists_only_for_short_tiles_of_boxes_the_list_sphere_fills():
    # 108 atoms (box 5.04) and the paper's 27 atoms (box 3.78, r_c = L/2):
    # the sphere of r_c + skin holds >= 60% of the box, and these paths get
    # one-step tiles, so no lists (reach -1)
    for n, dens, half, steps in ((108, 0.8442, False, 256), (27, 0.5, True, 4096)):
        box = (n / dens) ** (1.0 / 3.0)
        path = P.make_path(steps, n, 3, 1e-4, 1.0, 1.0)
        pot = P.make_potential("lj", rc=0.5 * box if half else 2.5, box=box)
        info = P.pamd_launch_info(path, pot)
        assert info.exact_lists == 1 and info.cells == 0 and info.tile == 1 and info.reach == -1
        assert P.pamd_launch_info(path, pot, P.make_tuning("fused", tile=2)).reach == -1
        # longer tiles amortise a list build; a skin or a list capacity asked
        # for keeps the lists
        for t in (P.make_tuning("fused", tile=3), P.make_tuning("fused", skin=0.3),
                  P.make_tuning("fused", max_neighbours=64)):
            assert P.pamd_launch_info(path, pot, t).reach == 0
        long_path = P.make_path(100000, n, 3, 1e-4, 1.0, 1.0)
        assert P.pamd_launch_info(long_path, pot).reach == 0
    # 256 atoms (box 6.72): no cell grid, but the sphere holds 37% of the box
    path, pot = lj(256, 256)
    info = P.pamd_launch_info(path, pot)
    assert info.cells == 0 and info.reach == 0
