"""autograd wrappers, graph capture and autotuning on the GPU."""
import math

import numpy as np
import pytest
import torch

import paper_1907_09529_amd as P
from oracle import action as OA

from common import em_input, lib_descriptors, oracle_full, oracle_pot, rel, rel_inf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case():
    w, X = em_input("lj108", n_steps=48)
    return w, X, oracle_full(w, X)


@pytest.mark.parametrize("retain", [True, False])
def test_action_backward(device, case, retain):
    w, X, (s_ref, g_ref) = case
    path, pot = lib_descriptors(w)
    x = torch.from_numpy(X.copy()).cuda().requires_grad_(True)
    S = P.path_action(x, path, pot, retain=retain)
    assert rel(float(S), math.fsum(s_ref.tolist())) <= 1e-12
    (2.5 * S).backward()
    assert rel_inf(x.grad.cpu().numpy(), 2.5 * g_ref) <= 1e-10


def test_per_step_backward_uses_weights(device, case):
    w, X, _ = case
    path, pot = lib_descriptors(w)
    x = torch.from_numpy(X.copy()).cuda().requires_grad_(True)
    s = P.per_step_action(x, path, pot)
    v = torch.from_numpy(np.random.default_rng(1).standard_normal(w.n_steps)).cuda()
    (s * v).sum().backward()
    _, g_ref = oracle_full(w, X, weights=v.cpu().numpy())
    assert rel_inf(x.grad.cpu().numpy(), g_ref) <= 1e-10


def test_gradcheck_tiny(device):
    w, X = em_input("lj27", n_steps=3)
    path, pot = lib_descriptors(w)
    x = torch.from_numpy(X.copy()).cuda().requires_grad_(True)
    assert torch.autograd.gradcheck(lambda t: P.path_action(t, path, pot, retain=False), (x,),
                                    eps=1e-6, atol=1e-4, rtol=1e-6)


# Graph replays are compared bit for bit, so these use the repeatable (full-list) form.
FULL = P.make_tuning("fused", neighbour_list="full")


def test_library_graph_replays_match_eager(device, case):
    w, X, _ = case
    path, pot = lib_descriptors(w)
    x = torch.from_numpy(X.copy()).cuda()
    ws = P.workspace(P.pamd_workspace_size(path, pot, FULL))
    g_e = torch.empty_like(x)
    a_e = torch.empty(1, dtype=torch.float64, device="cuda")
    P.pamd_action_grad(path, pot, x, g_e, action=a_e, ws=ws, tuning=FULL)
    torch.cuda.synchronize()
    g_c = torch.zeros_like(x)
    a_c = torch.zeros(1, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    graph = P.PamdGraph()
    with torch.cuda.stream(s):
        graph.begin(s)
        P.pamd_action_grad(path, pot, x, g_c, action=a_c, ws=ws, stream=s, tuning=FULL)
        graph.end(s)
    for rep in range(3):
        g_c.zero_()
        a_c.zero_()
        junk = torch.randn(1000, device="cuda").sum()  # eager work between replays
        torch.cuda.synchronize()
        graph.launch(s)
        s.synchronize()
        assert torch.equal(g_c, g_e) and torch.equal(a_c, a_e), rep
        del junk
    graph.close()


def test_torch_cuda_graph_capture(device, case):
    w, X, _ = case
    path, pot = lib_descriptors(w)
    x = torch.from_numpy(X.copy()).cuda()
    ws = P.workspace(P.pamd_workspace_size(path, pot, FULL))
    g_e = torch.empty_like(x)
    a_e = torch.empty(1, dtype=torch.float64, device="cuda")
    P.pamd_action_grad(path, pot, x, g_e, action=a_e, ws=ws, tuning=FULL)
    torch.cuda.synchronize()
    g_c = torch.empty_like(x)
    a_c = torch.empty(1, dtype=torch.float64, device="cuda")
    cg = torch.cuda.CUDAGraph()
    with torch.cuda.graph(cg):
        P.pamd_action_grad(path, pot, x, g_c, action=a_c, ws=ws, tuning=FULL)
    for rep in range(3):
        g_c.fill_(0.0)
        torch.cuda.synchronize()
        cg.replay()
        torch.cuda.synchronize()
        assert torch.equal(g_c, g_e) and torch.equal(a_c, a_e), rep


def test_half_list_graph_replays_within_rounding(device, case):
    w, X, (s_ref, g_ref) = case
    path, pot = lib_descriptors(w)
    half = P.make_tuning("fused", neighbour_list="half")
    x = torch.from_numpy(X.copy()).cuda()
    ws = P.workspace(P.pamd_workspace_size(path, pot, half))
    g_c = torch.zeros_like(x)
    a_c = torch.zeros(1, dtype=torch.float64, device="cuda")
    s = torch.cuda.Stream()
    graph = P.PamdGraph()
    with torch.cuda.stream(s):
        graph.begin(s)
        P.pamd_action_grad(path, pot, x, g_c, action=a_c, ws=ws, stream=s, tuning=half)
        graph.end(s)
    for rep in range(3):
        g_c.zero_()
        torch.cuda.synchronize()
        graph.launch(s)
        s.synchronize()
        assert rel(float(a_c.item()), math.fsum(s_ref.tolist())) <= 1e-12, rep
        assert rel_inf(g_c.cpu().numpy(), g_ref) <= 1e-10, rep
    graph.close()


def test_autotune_then_cached_choice_is_exact(device, case):
    w, X, (s_ref, g_ref) = case
    path, pot = lib_descriptors(w)
    x = torch.from_numpy(X.copy()).cuda()
    scratch = torch.empty_like(x)
    big = max(P.pamd_workspace_size(path, pot, P.make_tuning("fused", tile=2, skin=0.45, block=b))
              for b in (64, 128, 256, 512, 1024))
    ws = P.workspace(big)
    best = P.pamd_autotune(path, pot, x, scratch, ws)
    assert best.block % 64 == 0 and best.tile >= 1
    grad = torch.empty_like(x)
    act = torch.empty(1, dtype=torch.float64, device="cuda")
    P.pamd_action_grad(path, pot, x, grad, action=act)   # uses the cached choice
    torch.cuda.synchronize()
    assert rel(float(act.item()), math.fsum(s_ref.tolist())) <= 1e-12
    assert rel_inf(grad.cpu().numpy(), g_ref) <= 1e-10
