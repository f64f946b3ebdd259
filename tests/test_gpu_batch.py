"""GPU parity of the persistent batched launch against the oracle and single-path calls."""
import math

import numpy as np
import pytest
import torch

import paper_1907_09529_amd as P
import workloads as W
from oracle import action as OA

from common import em_input, lib_descriptors, oracle_full, oracle_pot, rel, rel_inf

pytestmark = pytest.mark.gpu


def pack(batch, arrays):
    total = batch.x_offsets[-1]
    buf = np.zeros(total)
    for p, X in enumerate(arrays):
        o = batch.x_offsets[p]
        buf[o:o + X.size] = X.ravel()
    return torch.from_numpy(buf).cuda()


def test_small_mixed_batch_vs_oracle(device):
    members = [em_input("lj108", n_steps=40), em_input("lj27", n_steps=21),
               em_input("lj108", n_atoms=256, n_steps=13), em_input("ho1d", n_steps=50),
               em_input("lj108", n_steps=1)]
    paths, pots = zip(*(lib_descriptors(w) for w, _ in members))
    b = P.PamdBatch(list(paths), list(pots))
    x = pack(b, [X for _, X in members])
    grad = torch.zeros_like(x)
    act = torch.empty(len(members), dtype=torch.float64, device="cuda")
    ps = torch.empty(b.step_offsets[-1], dtype=torch.float64, device="cuda")
    b.pamd_batch_run(x, act, grad_all=grad, per_step_all=ps)
    torch.cuda.synchronize()
    for p, (w, X) in enumerate(members):
        s_ref, g_ref = oracle_full(w, X)
        assert rel(float(act[p]), math.fsum(s_ref.tolist())) <= 1e-12, p
        assert np.max(np.abs(b.steps_view(ps, p).cpu().numpy() - s_ref) / s_ref) <= 1e-12, p
        assert rel_inf(b.view(grad, p).cpu().numpy(), g_ref) <= 1e-10, p
    # repeated calls reuse the prepared workspace and give identical results
    act2 = torch.empty_like(act)
    b.pamd_batch_run(x, act2)
    torch.cuda.synchronize()
    assert torch.equal(act, act2)


def test_pointer_array_form_vs_oracle(device):
    """pamd_batch_action_grad: each path in its own buffer (host arrays of
    device pointers), one member without a gradient; against the oracle."""
    members = [em_input("lj108", n_steps=40), em_input("ho1d", n_steps=50),
               em_input("lj108", n_atoms=256, n_steps=13), em_input("lj27", n_steps=21)]
    paths, pots = zip(*(lib_descriptors(w) for w, _ in members))
    xs = [torch.from_numpy(np.ascontiguousarray(X)).cuda() for _, X in members]
    grads = [torch.full_like(x, float("nan")) for x in xs]
    grads[2] = None
    act = torch.empty(len(members), dtype=torch.float64, device="cuda")
    P.pamd_batch_action_grad(list(paths), list(pots), xs, act, grads)
    torch.cuda.synchronize()
    for p, (w, X) in enumerate(members):
        s_ref, g_ref = oracle_full(w, X)
        assert rel(float(act[p]), math.fsum(s_ref.tolist())) <= 1e-12, p
        if grads[p] is not None:
            assert rel_inf(grads[p].cpu().numpy(), g_ref) <= 1e-10, p
    # actions only
    act2 = torch.empty_like(act)
    P.pamd_batch_action_grad(list(paths), list(pots), xs, act2)
    torch.cuda.synchronize()
    assert torch.allclose(act, act2, rtol=1e-13, atol=0.0)


def test_batch_autotune_keeps_results(device):
    """After pamd_batch_autotune re-plans the member tiles, the batch still
    matches the oracle."""
    members = [em_input("lj108", n_steps=40), em_input("lj108", n_atoms=256, n_steps=13),
               em_input("lj27", n_steps=21), em_input("ho1d", n_steps=50)]
    paths, pots = zip(*(lib_descriptors(w) for w, _ in members))
    b = P.PamdBatch(list(paths), list(pots))
    x = pack(b, [X for _, X in members])
    grad = torch.zeros_like(x)
    budget, skin = b.autotune(x, grad)
    assert budget in (8192, 16384, 32768, 65536, 131072, 262144) and skin in (0.3, 0.5)
    act = torch.empty(len(members), dtype=torch.float64, device="cuda")
    grad.zero_()
    b.pamd_batch_run(x, act, grad_all=grad)
    torch.cuda.synchronize()
    for p, (w, X) in enumerate(members):
        s_ref, g_ref = oracle_full(w, X)
        assert rel(float(act[p]), math.fsum(s_ref.tolist())) <= 1e-12, p
        assert rel_inf(b.view(grad, p).cpu().numpy(), g_ref) <= 1e-10, p


def test_batch64_full_workload(device):
    """The 64-path workload: every member against the single-path call, sampled
    slices of three members against the oracle."""
    ws = W.batch_members()
    paths, pots, arrays = [], [], []
    for w in ws:
        X = W.tethered_path(w)
        arrays.append(X)
        pa, po = lib_descriptors(w)
        paths.append(pa)
        pots.append(po)
    b = P.PamdBatch(paths, pots)
    x = pack(b, arrays)
    grad = torch.zeros_like(x)
    act = torch.empty(len(ws), dtype=torch.float64, device="cuda")
    b.pamd_batch_run(x, act, grad_all=grad)
    torch.cuda.synchronize()
    for p, w in enumerate(ws):
        g1 = torch.empty_like(b.view(x, p))
        a1 = torch.empty(1, dtype=torch.float64, device="cuda")
        P.pamd_action_grad(paths[p], pots[p], b.view(x, p).contiguous(), g1, action=a1)
        torch.cuda.synchronize()
        assert rel(float(act[p]), float(a1)) <= 1e-12, p
        assert rel_inf(b.view(grad, p).cpu().numpy(), g1.cpu().numpy()) <= 1e-10, p
    rng = np.random.default_rng(0)
    for p in rng.choice(len(ws), size=3, replace=False):
        w, X = ws[p], arrays[p]
        pot = oracle_pot(w)
        gp = b.view(grad, int(p)).cpu().numpy()
        for m in sorted({0, int(rng.integers(1, w.n_steps)), w.n_steps}):
            _, gm = OA.slice_terms(X, m, pot, w.dt, w.D, w.gamma)
            assert rel_inf(gp[m], gm) <= 1e-10, (p, m)


def test_batch_graph_replays_match_eager(device):
    """The persistent batched launch captured once and replayed, with eager work
    and synchronisations between replays: every replay equals the eager result."""
    members = [em_input("lj108", n_steps=40), em_input("lj108", n_atoms=256, n_steps=13),
               em_input("ho1d", n_steps=50)]
    paths, pots = zip(*(lib_descriptors(w) for w, _ in members))
    b = P.PamdBatch(list(paths), list(pots))
    x = pack(b, [X for _, X in members])
    ref_g = torch.zeros_like(x)
    ref_a = torch.empty(len(members), dtype=torch.float64, device="cuda")
    b.pamd_batch_run(x, ref_a, grad_all=ref_g)
    torch.cuda.synchronize()
    grad = torch.zeros_like(x)
    act = torch.empty_like(ref_a)
    s = torch.cuda.Stream()
    g = P.PamdGraph()
    with torch.cuda.stream(s):
        g.begin(s)
        b.pamd_batch_run(x, act, grad_all=grad, stream=s)
        g.end(s)
    for _ in range(3):
        grad.zero_()
        act.zero_()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.launch(s)
        s.synchronize()
        assert torch.equal(act, ref_a) and torch.equal(grad, ref_g)
    g.close()
