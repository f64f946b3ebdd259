"""pamd_action_grad_noalloc (static scratch, no workspace) against
pamd_action_grad on the same inputs, called through the C ABI: two calls in a
row, the second on a smaller problem, plus a problem whose usual workspace
exceeds the static array (the call then runs fewer workgroups at once)."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1907_09529_amd as P
import workloads as W
from paper_1907_09529_amd import _lib

from common import em_input, lib_descriptors, rel, rel_inf

pytestmark = pytest.mark.gpu

ACTION_TOL = 1e-12
GRAD_TOL = 1e-10


def _vp(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _compare(w, X, tuning=None):
    path, pot = lib_descriptors(w)
    x = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    g_ref = torch.empty_like(x)
    a_ref = torch.empty(1, dtype=torch.float64, device="cuda")
    s_ref = torch.empty(w.n_steps, dtype=torch.float64, device="cuda")
    P.pamd_action_grad(path, pot, x, g_ref, action=a_ref, per_step=s_ref, tuning=tuning)
    g = torch.full_like(x, float("nan"))
    a = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    s = torch.full((w.n_steps,), float("nan"), dtype=torch.float64, device="cuda")
    lib = P.load()
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    code = lib.pamd_action_grad_noalloc(ctypes.byref(path), ctypes.byref(pot),
                                        ctypes.byref(tuning) if tuning is not None else None,
                                        _vp(x), None, _vp(a), _vp(s), _vp(g), stream)
    assert code == _lib.PAMD_OK, lib.pamd_last_error()
    torch.cuda.synchronize()
    A, A_ref = float(a.item()), float(a_ref.item())
    assert rel(A, A_ref) <= ACTION_TOL
    sn, sr = s.cpu().numpy(), s_ref.cpu().numpy()
    assert np.all(np.abs(sn - sr) <= ACTION_TOL * np.abs(sr))
    assert rel_inf(g.cpu().numpy(), g_ref.cpu().numpy()) <= GRAD_TOL
    return A


def test_noalloc_matches_workspace_call_twice_smaller_second(device):
    w1, X1 = em_input("lj108", n_steps=64)
    _compare(w1, X1)
    w2, X2 = em_input("lj108", n_steps=12)       # second call: smaller, same static scratch
    _compare(w2, X2)
    wh, Xh = em_input("ho1d")
    _compare(wh, Xh)
    _compare(wh.with_steps(100), np.ascontiguousarray(Xh[:101]))


def test_noalloc_shrinks_the_grid_when_the_workspace_is_larger(device):
    # the 864 x 4096 path with its exact lists in device memory (two slot
    # arrays) plans more scratch than the static array holds
    w = W.workload("lj864")
    path, pot = lib_descriptors(w)
    two = P.make_tuning("fused", slot_arrays=2)
    need = P.pamd_workspace_size(path, pot, two)
    assert need > _lib.PAMD_NOALLOC_SCRATCH_BYTES   # the usual plan would not fit
    X = W.tethered_path(w)
    _compare(w, X, tuning=two)
    _compare(w, X)                                  # the default launch fits as planned
    w2 = w.with_steps(256)                          # then a smaller problem again
    _compare(w2, np.ascontiguousarray(X[:257]), tuning=two)


def test_noalloc_refuses_what_cannot_fit(device):
    path = P.make_path(1 << 22, 4000, 3, 1e-4, 1.0, 1.0)
    pot = P.make_potential("lj", rc=2.5, box=(4000 / 0.8442) ** (1 / 3))
    lib = P.load()
    fake = ctypes.c_void_p(0x100000)   # refused on the host before any device work
    code = lib.pamd_action_grad_noalloc(ctypes.byref(path), ctypes.byref(pot), None, fake, None,
                                        None, None, fake, None)
    assert code == _lib.PAMD_EWORKSPACE
    assert b"static" in lib.pamd_last_error()
