"""Host-side checks of the C ABI (no GPU needed).

The library validates every argument before any device work, so error
returns can be exercised on a machine without a GPU.  Device pointers here are
fake non-null addresses that are never dereferenced.
"""
import ctypes
import math
import os
import re

import pytest

import paper_1907_09529_amd as P
from paper_1907_09529_amd import _lib
from oracle import action as OA

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pamd.h")


def _gpu_visible() -> bool:
    """True when a HIP device is visible (counting devices does not initialise one)."""
    import torch
    return torch.cuda.device_count() > 0


pytestmark = pytest.mark.skipif(not os.path.exists(_lib.LIB_PATH),
                                reason="libpamd.so not built (run __graft_entry__.build())")

# The error-path tests below hand the library fake device addresses that its
# host-side validation must refuse.  Where a GPU is visible, a regressed check
# would enqueue a kernel on unmapped memory, so those tests run only on hosts
# without one (the CPU suite); the export check runs everywhere.
cpu_only = pytest.mark.skipif(_gpu_visible(), reason="fake device addresses must never reach a GPU")

FAKE = ctypes.c_void_p(0x100000)        # aligned, never dereferenced
FAKE_BAD = ctypes.c_void_p(0x100010)    # not 256-byte aligned
BOX864 = (864 / 0.8442) ** (1 / 3)


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pamd_[a-z_0-9]+)\s*\(", text)))


def test_exports_every_declared_symbol():
    lib = P.load()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(_lib.EXPORTED)


def lj_path(**kw):
    d = dict(n_steps=64, n_atoms=864, n_dim=3, dt=1e-4, D=1.0, gamma=1.0)
    d.update(kw)
    return P.make_path(**d)


def lj_pot(**kw):
    d = dict(eps=1.0, sigma=1.0, rc=2.5, box=BOX864)
    d.update(kw)
    return P.make_potential("lj", **d)


def ws_size(path, pot, tuning=None):
    n = ctypes.c_size_t(0)
    code = P.load().pamd_workspace_size(ctypes.byref(path), ctypes.byref(pot),
                                        ctypes.byref(tuning) if tuning else None, ctypes.byref(n))
    return code, n.value


def action_call(path, pot, x=FAKE, action=FAKE, ws=FAKE, ws_bytes=None, tuning=None):
    if ws_bytes is None:
        ws_bytes = ws_size(path, pot, tuning)[1]
    return P.load().pamd_action(ctypes.byref(path), ctypes.byref(pot),
                                ctypes.byref(tuning) if tuning else None, x, action, None, ws,
                                ctypes.c_size_t(ws_bytes), None)


@pytest.mark.parametrize("bad,code", [
    (dict(n_steps=0), _lib.PAMD_EINVAL),
    (dict(n_atoms=0), _lib.PAMD_EINVAL),
    (dict(n_dim=2), _lib.PAMD_EUNSUPPORTED),
    (dict(n_dim=1), _lib.PAMD_EUNSUPPORTED),     # LJ needs 3 dimensions
    (dict(dt=0.0), _lib.PAMD_EINVAL),
    (dict(dt=float("nan")), _lib.PAMD_EINVAL),
    (dict(D=-1.0), _lib.PAMD_EINVAL),
    (dict(gamma=0.0), _lib.PAMD_EINVAL),
    (dict(n_atoms=70000), _lib.PAMD_EUNSUPPORTED),
])
@cpu_only
def test_path_validation(bad, code):
    c, _ = ws_size(lj_path(**bad), lj_pot())
    assert c == code
    assert P.load().pamd_last_error()


@cpu_only
def test_precision_validation():
    p = lj_path()
    p.precision = 7
    assert ws_size(p, lj_pot())[0] == _lib.PAMD_EINVAL


@pytest.mark.parametrize("bad,code", [
    (dict(rc=6.0), _lib.PAMD_EUNSUPPORTED),      # r_c > L/2
    (dict(box=0.0), _lib.PAMD_EINVAL),
    (dict(eps=0.0), _lib.PAMD_EINVAL),
    (dict(sigma=-1.0), _lib.PAMD_EINVAL),
    (dict(rc=float("inf")), _lib.PAMD_EINVAL),
])
@cpu_only
def test_potential_validation(bad, code):
    assert ws_size(lj_path(), lj_pot(**bad))[0] == code


@cpu_only
def test_harmonic_rejects_box_and_unknown_kind():
    p = P.make_path(16, 1, 1, 0.01, 1.0, 1.0)
    h = P.make_potential("harmonic")
    h.box = 3.0
    assert ws_size(p, h)[0] == _lib.PAMD_EUNSUPPORTED
    h.box = 0.0
    h.kind = 9
    assert ws_size(p, h)[0] == _lib.PAMD_EINVAL


@pytest.mark.parametrize("field,value", [("algo", 5), ("block", 100), ("block", 2048),
                                         ("tile", -1), ("max_neighbours", -3),
                                         ("neighbour_list", 7)])
@cpu_only
def test_tuning_validation(field, value):
    t = P.make_tuning()
    setattr(t, field, value)
    assert ws_size(lj_path(), lj_pot(), t)[0] == _lib.PAMD_EINVAL


@cpu_only
def test_null_pointers_and_workspace():
    path, pot = lj_path(), lj_pot()
    assert action_call(path, pot, x=None) == _lib.PAMD_EINVAL
    assert action_call(path, pot, action=None) == _lib.PAMD_EINVAL
    need = ws_size(path, pot)[1]
    assert need > 0
    assert action_call(path, pot, ws_bytes=need - 1) == _lib.PAMD_EWORKSPACE
    assert action_call(path, pot, ws=FAKE_BAD) == _lib.PAMD_EWORKSPACE
    assert action_call(path, pot, ws=None) == _lib.PAMD_EINVAL
    lib = P.load()
    code = lib.pamd_action_grad(ctypes.byref(path), ctypes.byref(pot), None, FAKE, None, None,
                                None, None, FAKE, ctypes.c_size_t(need), None)
    assert code == _lib.PAMD_EINVAL and b"grad" in lib.pamd_last_error()
    code = lib.pamd_excess_action(ctypes.byref(path), ctypes.byref(pot), None, FAKE, None, None,
                                  FAKE, ctypes.c_size_t(need), None)
    assert code == _lib.PAMD_EINVAL


@cpu_only
def test_half_list_needs_room():
    # 864 atoms with 64-thread blocks cannot hold two slots per thread
    t = P.make_tuning("fused", block=64, neighbour_list="half")
    assert ws_size(lj_path(), lj_pot(), t)[0] == _lib.PAMD_EUNSUPPORTED
    t = P.make_tuning("fused", block=448, neighbour_list="half")
    assert ws_size(lj_path(), lj_pot(), t)[0] == 0


@cpu_only
def test_workspace_grows_with_problem_and_plain_form():
    small = ws_size(lj_path(n_steps=64), lj_pot())[1]
    big = ws_size(lj_path(n_steps=4096), lj_pot())[1]
    plain = ws_size(lj_path(n_steps=4096), lj_pot(), P.make_tuning("plain"))[1]
    assert 0 < small < big < plain
    assert big % 256 == 0


@cpu_only
def test_mh_validation():
    path, pot = lj_path(n_steps=64), lj_pot()
    lib = P.load()
    n = ctypes.c_size_t(0)
    assert lib.pamd_mh_workspace_size(ctypes.byref(path), ctypes.byref(pot), None,
                                      ctypes.byref(n)) == 0

    def step(l_min, l_max, counter=FAKE):
        return lib.pamd_mh_step(ctypes.byref(path), ctypes.byref(pot), None, 1, l_min, l_max,
                                counter, FAKE, FAKE, FAKE, None, None, None, FAKE,
                                ctypes.c_size_t(n.value), None)

    assert step(0, 2) == _lib.PAMD_EINVAL
    assert step(3, 2) == _lib.PAMD_EINVAL
    assert step(2, 7) == _lib.PAMD_EINVAL          # 2^7 > 64 steps
    assert step(2, 3, counter=None) == _lib.PAMD_EINVAL


@cpu_only
def test_batch_validation_and_layout():
    paths = [lj_path(n_steps=100, n_atoms=108, ), lj_path(n_steps=37, n_atoms=256),
             P.make_path(50, 4, 3, 0.01, 1.0, 1.0)]
    paths[0].n_atoms = 108
    pots = [lj_pot(box=(108 / 0.8442) ** (1 / 3)), lj_pot(box=(256 / 0.8442) ** (1 / 3)),
            P.make_potential("harmonic")]
    b = P.PamdBatch(paths, pots)
    assert b.x_offsets[0] == 0
    for p in range(3):
        n = (paths[p].n_steps + 1) * paths[p].n_dim * paths[p].n_atoms
        assert b.x_offsets[p + 1] - b.x_offsets[p] >= n
        assert b.x_offsets[p] % 32 == 0
    assert b.ws_bytes > 0
    b.close()
    bad = [lj_path(n_steps=10, n_atoms=108)]
    bad[0].precision = 1
    with pytest.raises(P.PamdError):
        P.PamdBatch(bad + [lj_path(n_steps=10, n_atoms=108)], [pots[0], pots[0]])
    with pytest.raises(P.PamdError):
        P.PamdBatch([lj_path()], [lj_pot(rc=9.0)])


@cpu_only
def test_log_norm_matches_oracle():
    path = lj_path(n_steps=4096)
    ref = OA.log_norm(4096, 3, 864, 1.0, 1e-4)
    assert abs(P.pamd_log_norm(path) - ref) <= 1e-12 * abs(ref)
    bad = lj_path(n_steps=0)
    assert math.isnan(P.pamd_log_norm(bad))


@cpu_only
def test_graph_begin_rejects_null_stream():
    assert P.load().pamd_graph_begin(None) == _lib.PAMD_EINVAL


@cpu_only
def test_em_validation():
    lib = P.load()

    def size(path, pot, tuning=None):
        n = ctypes.c_size_t(0)
        code = lib.pamd_em_workspace_size(ctypes.byref(path), ctypes.byref(pot),
                                          ctypes.byref(tuning) if tuning else None,
                                          ctypes.byref(n))
        return code, n.value

    path, pot = lj_path(n_steps=1000), lj_pot()
    code, need = size(path, pot)
    assert code == 0 and need > 0 and need % 256 == 0
    # one workgroup's scratch, whatever the path length
    assert need == size(lj_path(n_steps=5), pot)[1]
    assert need < ws_size(path, pot)[1]
    assert size(path, pot, P.make_tuning("plain"))[0] == _lib.PAMD_EUNSUPPORTED
    assert size(path, pot, P.make_tuning("fused", block=448, neighbour_list="half"))[0] == \
        _lib.PAMD_EUNSUPPORTED
    p32 = lj_path(n_steps=1000)
    p32.precision = _lib.PAMD_FP32_FORCE
    assert size(p32, pot)[0] == _lib.PAMD_EUNSUPPORTED
    assert size(lj_path(n_steps=0), pot)[0] == _lib.PAMD_EINVAL
    assert size(P.make_path(16, 2, 1, 0.01, 1.0, 1.0), P.make_potential("harmonic"))[0] == 0

    def integrate(x0=FAKE, noise=ctypes.c_void_p(0x10000000), x_out=ctypes.c_void_p(0x20000000),
                  ws=FAKE, ws_bytes=need):
        return lib.pamd_em_integrate(ctypes.byref(path), ctypes.byref(pot), None, x0, noise,
                                     x_out, ws, ctypes.c_size_t(ws_bytes), None)

    assert integrate(x0=None) == _lib.PAMD_EINVAL
    assert integrate(noise=None) == _lib.PAMD_EINVAL
    assert integrate(x_out=None) == _lib.PAMD_EINVAL
    # noise (1000 slices of 2592 doubles) starting inside x_out
    assert integrate(noise=ctypes.c_void_p(0x20000000 + 8 * 2592 * 999)) == _lib.PAMD_EINVAL
    assert b"overlaps" in lib.pamd_last_error()
    assert integrate(ws_bytes=need - 1) == _lib.PAMD_EWORKSPACE
    assert integrate(ws=FAKE_BAD) == _lib.PAMD_EWORKSPACE


@cpu_only
def test_shift_and_run_validation():
    lib = P.load()
    path = P.make_path(16, 1, 1, 0.4, 1.0, 1.0)
    pot = P.make_potential("harmonic")
    A, B = ctypes.c_void_p(0x10000000), ctypes.c_void_p(0x20000000)
    EA, EB = ctypes.c_void_p(0x30000000), ctypes.c_void_p(0x40000000)

    def shift(n_shift=2, x_in=A, x_out=B, e_in=EA, e_out=EB, counter=FAKE):
        return lib.pamd_shift(ctypes.byref(path), 1, n_shift, counter, x_in, x_out, e_in, e_out,
                              None, None)

    for bad in (0, 17):
        assert shift(n_shift=bad) == _lib.PAMD_EINVAL
    assert shift(counter=None) == _lib.PAMD_EINVAL
    assert shift(x_out=ctypes.c_void_p(0x10000000 + 8)) == _lib.PAMD_EINVAL      # overlaps x_in
    assert shift(e_out=None) == _lib.PAMD_EINVAL                                 # one of two
    n = ctypes.c_size_t(0)
    assert lib.pamd_run_workspace_size(ctypes.byref(path), ctypes.byref(pot), None, 2,
                                       ctypes.byref(n)) == 0 and n.value > 0
    assert lib.pamd_run_workspace_size(ctypes.byref(path), ctypes.byref(pot), None, 0,
                                       ctypes.byref(n)) == _lib.PAMD_EINVAL

    def run(l_min=3, l_max=3, n_sample=2, n_shift=2, n_events=1, x_alt=B, ws_bytes=None):
        need = ctypes.c_size_t(0)
        lib.pamd_run_workspace_size(ctypes.byref(path), ctypes.byref(pot), None, n_shift,
                                    ctypes.byref(need))
        return lib.pamd_run(ctypes.byref(path), ctypes.byref(pot), None, 1, l_min, l_max,
                            n_sample, n_shift, n_events, FAKE, A, x_alt,
                            ctypes.c_void_p(0x50000000), EA, EB, None, None, FAKE,
                            ctypes.c_size_t(need.value if ws_bytes is None else ws_bytes), None)

    assert run(l_max=5) == _lib.PAMD_EINVAL            # 2^5 > 16 steps
    assert run(n_sample=-1) == _lib.PAMD_EINVAL
    assert run(x_alt=A) == _lib.PAMD_EINVAL
    assert run(ws_bytes=8) == _lib.PAMD_EWORKSPACE


@cpu_only
def test_langevin_validation():
    lib = P.load()
    path, pot = lj_path(), lj_pot()
    n = ctypes.c_size_t(0)
    assert lib.pamd_langevin_workspace_size(ctypes.byref(path), ctypes.byref(pot), None,
                                            ctypes.byref(n)) == 0
    assert n.value >= ws_size(path, pot)[1]
    bufs = [ctypes.c_void_p(0x10000000 * k) for k in range(1, 5)]

    def step(tau=1e-6, counter=FAKE, x=bufs[0], y=bufs[2], ws_bytes=n.value):
        return lib.pamd_langevin_step(ctypes.byref(path), ctypes.byref(pot), None, 1,
                                      ctypes.c_double(tau), counter, x, bufs[1], FAKE, y,
                                      bufs[3], None, None, FAKE, ctypes.c_size_t(ws_bytes), None)

    assert step(tau=0.0) == _lib.PAMD_EINVAL
    assert step(tau=float("nan")) == _lib.PAMD_EINVAL
    assert step(counter=None) == _lib.PAMD_EINVAL
    assert step(y=bufs[0]) == _lib.PAMD_EINVAL
    assert step(ws_bytes=n.value - 1) == _lib.PAMD_EWORKSPACE


@cpu_only
def test_launch_info_reports_the_plan():
    lib = P.load()
    path = lj_path(n_steps=4096)
    pot = lj_pot()
    info = P.pamd_launch_info(path, pot)
    assert info.algo == _lib.PAMD_ALGO_FUSED
    assert 1 <= info.tile <= 32 and info.n_tiles == -(-4096 // info.tile)
    assert info.block % 64 == 0 and 64 <= info.block <= 1024
    assert info.grid == min(info.n_tiles, 2048)
    assert info.neighbour_list == _lib.PAMD_LIST_FULL and info.skin > 0
    # default: exact partner lists kept in LDS, with one residual slot array
    assert info.exact_lists == 1 and info.slot_arrays == 1
    two = P.pamd_launch_info(path, pot, P.make_tuning("fused", slot_arrays=2))
    assert two.exact_lists == 0 and two.slot_arrays == 2 and two.lds_bytes > 0
    t = P.make_tuning("fused", tile=7)
    assert P.pamd_launch_info(path, pot, t).tile == 7
    assert P.pamd_launch_info(path, pot, P.make_tuning("plain")).algo == _lib.PAMD_ALGO_PLAIN
    h = P.pamd_launch_info(P.make_path(64, 1, 1, 0.01, 1.0, 1.0), P.make_potential("harmonic"))
    assert h.algo == 0 and h.tile == 0
    bad = lj_path(n_steps=0)
    assert lib.pamd_launch_info(ctypes.byref(bad), ctypes.byref(pot), None,
                                ctypes.byref(_lib.PamdLaunch())) == _lib.PAMD_EINVAL


@cpu_only
def test_noalloc_refuses_problems_beyond_its_static_scratch():
    lib = P.load()
    path = lj_path(n_steps=1 << 22, n_atoms=4000)
    pot = lj_pot(box=(4000 / 0.8442) ** (1 / 3))
    code = lib.pamd_action_grad_noalloc(ctypes.byref(path), ctypes.byref(pot), None, FAKE, None,
                                        None, None, FAKE, None)
    assert code == _lib.PAMD_EWORKSPACE
    assert b"static" in lib.pamd_last_error()
    # invalid arguments are refused as by pamd_action_grad
    small = lj_path(n_steps=4)
    assert lib.pamd_action_grad_noalloc(ctypes.byref(small), ctypes.byref(pot), None, None, None,
                                        None, None, FAKE, None) == _lib.PAMD_EINVAL


@cpu_only
def test_pointer_array_batch_validation():
    lib = P.load()
    paths = (_lib.PamdPath * 2)(lj_path(n_steps=8, n_atoms=108),
                                lj_path(n_steps=5, n_atoms=108))
    pots = (_lib.PamdPotential * 2)(lj_pot(box=(108 / 0.8442) ** (1 / 3)),
                                    lj_pot(box=(108 / 0.8442) ** (1 / 3)))
    need = ctypes.c_size_t(0)
    assert lib.pamd_batch_workspace_size(2, paths, pots, ctypes.byref(need)) == _lib.PAMD_OK
    assert need.value > 0
    xs = (ctypes.c_void_p * 2)(0x10000000, 0x20000000)
    gs = (ctypes.c_void_p * 2)(0x30000000, None)
    def call(x=xs, act=FAKE, g=gs, ws=FAKE, nbytes=need.value, n=2):
        return lib.pamd_batch_action_grad(n, paths, pots, x, act, g, ws, ctypes.c_size_t(nbytes),
                                          None)
    assert call(x=None) == _lib.PAMD_EINVAL
    assert call(act=None) == _lib.PAMD_EINVAL
    assert call(x=(ctypes.c_void_p * 2)(0x10000000, None)) == _lib.PAMD_EINVAL
    assert call(nbytes=need.value - 1) == _lib.PAMD_EWORKSPACE
    assert call(ws=FAKE_BAD) == _lib.PAMD_EWORKSPACE
    assert call(n=0) == _lib.PAMD_EINVAL
    bad = (_lib.PamdPath * 2)(lj_path(n_steps=8, n_atoms=108), lj_path(n_steps=0, n_atoms=108))
    assert lib.pamd_batch_workspace_size(2, bad, pots, ctypes.byref(need)) == _lib.PAMD_EINVAL
