"""GPU parity of the fragment-wise Metropolis-Hastings path move (Sec. III).

Both sides draw from the same Philox4x32-10 streams.  Level, offset and
fragmentation are integers and must match exactly; the trial path and the
per-fragment Delta_f agree to rounding; accept decisions must agree except at
near ties (|ln u_f + Delta_f| tiny), where either outcome is valid.
"""
import math

import numpy as np
import pytest
import torch

import paper_1907_09529_amd as P
from oracle import sampling as OS

from common import em_input, lib_descriptors, oracle_pot, rel_inf

pytestmark = pytest.mark.gpu

SEED = 0x5EED1907


def gpu_state(w, X):
    path, pot = lib_descriptors(w)
    x = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    ex = torch.empty(w.n_steps, dtype=torch.float64, device="cuda")
    P.pamd_excess_action(path, pot, x, ex)
    return path, pot, x, ex


@pytest.mark.parametrize("name,kw,levels", [("lj108", dict(n_steps=64), (1, 3)),
                                            ("lj27", dict(n_steps=32), (2, 4)),
                                            ("ho1d", dict(n_steps=128), (2, 5))])
def test_mh_steps_match_oracle(device, name, kw, levels):
    w, X0 = em_input(name, **kw)
    pot_o = oracle_pot(w)
    path, pot, x, ex = gpu_state(w, X0)
    trial = torch.empty_like(x)
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    fd = torch.empty(w.n_steps + 2, dtype=torch.float64, device="cuda")
    fa = torch.empty(w.n_steps + 2, dtype=torch.int32, device="cuda")
    info = torch.empty(4, dtype=torch.int32, device="cuda")
    X = X0.copy()
    accepted_total = 0
    for sweep in range(6):
        P.pamd_mh_step(path, pot, SEED, levels[0], levels[1], counter, x, ex, trial,
                       frag_delta=fd, frag_accept=fa, step_info=info)
        torch.cuda.synchronize()
        ref = OS.mh_step(X, pot_o, w.dt, w.D, w.gamma, SEED, sweep, levels[0], levels[1])
        l, u, nf, na = info.cpu().tolist()
        assert (l, u, nf) == (ref["level"], ref["offset"], len(ref["fragments"]))
        assert int(counter.item()) == sweep + 1
        scale = np.max(np.abs(ref["trial"]))
        assert np.max(np.abs(trial.cpu().numpy() - ref["trial"])) <= 1e-13 * scale
        d_gpu = fd.cpu().numpy()[:nf]
        s_scale = np.abs(ref["s_old"]).sum()
        assert np.max(np.abs(d_gpu - ref["delta"])) <= 1e-10 * s_scale
        acc_gpu = fa.cpu().numpy()[:nf].astype(bool)
        margin = np.abs(np.log(ref["uniforms"]) + ref["delta"])
        decided = margin > 1e-6
        assert np.array_equal(acc_gpu[decided], ref["accepted"][decided])
        assert na == int(acc_gpu.sum())
        accepted_total += na
        # continue both chains from the GPU's decisions (identical unless a near tie)
        Xn = X.copy()
        for (a, b, nose), acc in zip(ref["fragments"], acc_gpu):
            hi = b + 1 if nose else b
            if acc:
                Xn[a + 1:hi] = ref["trial"][a + 1:hi]
        X = Xn
        assert rel_inf(x.cpu().numpy(), X) <= 1e-13
        # the carried excess action equals a fresh evaluation of the committed path
        fresh = torch.empty_like(ex)
        P.pamd_excess_action(path, pot, x, fresh)
        torch.cuda.synchronize()
        assert np.max(np.abs(ex.cpu().numpy() - fresh.cpu().numpy())) <= 1e-10 * s_scale
    print(f"{name}: {accepted_total} fragments accepted over 6 sweeps")


def test_mh_graph_replay_advances_sweeps(device):
    """A captured MH step replays successive sweeps (the counter lives on the device)."""
    w, X0 = em_input("ho1d", n_steps=64)
    path, pot, x, ex = gpu_state(w, X0)
    trial = torch.empty_like(x)
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    ws = P.workspace(P.pamd_mh_workspace_size(path, pot))
    # eager reference chain
    xe, exe = x.clone(), ex.clone()
    ce = torch.zeros_like(counter)
    for _ in range(4):
        P.pamd_mh_step(path, pot, SEED, 2, 4, ce, xe, exe, trial, ws=ws)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = P.PamdGraph()
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        g.begin(s)
        P.pamd_mh_step(path, pot, SEED, 2, 4, counter, x, ex, trial, ws=ws, stream=s)
        g.end(s)
        for _ in range(4):
            g.launch(s)
    s.synchronize()
    assert int(counter.item()) == 4
    assert torch.equal(x, xe) and torch.equal(ex, exe)
    g.close()


def test_sweep4000_full_size_graph(device):
    """The path-sampling workload at full size (4000 atoms x 16384 steps): two
    graph-replayed sweeps (MH move, then action + gradient of the committed
    path).  Checked: the sweep counter, the move's bookkeeping, that only
    accepted fragments changed, the carried excess action against a fresh
    evaluation, and sampled gradient rows against the oracle."""
    import workloads as W
    from oracle import action as OA
    w = W.workload("sweep4000")
    X0 = W.tethered_path(w)
    path, pot = lib_descriptors(w)
    x = torch.from_numpy(X0).cuda()
    ex = torch.empty(w.n_steps, dtype=torch.float64, device="cuda")
    P.pamd_excess_action(path, pot, x, ex)
    trial = torch.empty_like(x)
    grad = torch.empty_like(x)
    act = torch.empty(1, dtype=torch.float64, device="cuda")
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    info = torch.empty(4, dtype=torch.int32, device="cuda")
    fa = torch.empty(w.n_steps + 2, dtype=torch.int32, device="cuda")
    ws_mh = P.workspace(P.pamd_mh_workspace_size(path, pot))
    ws = P.workspace(P.pamd_workspace_size(path, pot))
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = P.PamdGraph()
    with torch.cuda.stream(s):
        g.begin(s)
        P.pamd_mh_step(path, pot, SEED, w.l_min, w.l_max, counter, x, ex, trial,
                       frag_accept=fa, step_info=info, ws=ws_mh, stream=s)
        P.pamd_action_grad(path, pot, x, grad, action=act, ws=ws, stream=s)
        g.end(s)
    X = X0
    for sweep in range(2):
        with torch.cuda.stream(s):
            g.launch(s)
        s.synchronize()
        assert int(counter.item()) == sweep + 1
        l, u, nf, na = info.cpu().tolist()
        assert w.l_min <= l <= w.l_max and 1 <= u <= 2 ** l and nf >= 1
        acc = fa.cpu().numpy()[:nf].astype(bool)
        assert na == int(acc.sum())
        Xn = x.cpu().numpy()
        T = trial.cpu().numpy()
        frags = OS.fragments(w.n_steps, l, u)
        assert len(frags) == nf
        for f, (a, b, nose) in enumerate(frags):
            hi = b + 1 if nose else b  # the nose moves its endpoint too
            src = T if acc[f] else X
            assert np.array_equal(Xn[a + 1:hi], src[a + 1:hi]), (sweep, f)
            assert np.array_equal(Xn[a], X[a]), (sweep, f)  # shared endpoints stay
        X = Xn
        fresh = torch.empty_like(ex)
        P.pamd_excess_action(path, pot, x, fresh)
        torch.cuda.synchronize()
        scale = float(np.abs(ex.cpu().numpy()).sum())
        assert np.max(np.abs(ex.cpu().numpy() - fresh.cpu().numpy())) <= 1e-10 * scale
    pot_o = oracle_pot(w)
    gp = grad.cpu().numpy()
    for m in (0, 7777, w.n_steps):
        _, gm = OA.slice_terms(X, m, pot_o, w.dt, w.D, w.gamma, method="cells")
        assert rel_inf(gp[m], gm) <= 1e-10, m
    g.close()
