"""Benchmark: slice-atom action+gradient evaluations per second on one MI355X.

Workload (default): Lennard-Jones path, 864 atoms at reduced density 0.8442,
T = 1, r_c = 2.5 sigma, cubic periodic box, dt = 1e-4, D = gamma = 1, 4096
time steps; seeded synthetic path (FCC lattice plus a tethered Gaussian random
walk with the free-diffusion step size, plus N(0, 0.01^2) per-slice noise),
resident in device memory before timing.  One benchmark step = one
pamd_action_grad call (FP64): action, per-step terms and the gradient of
every slice.

Prints one JSON line with the metric, the roofline of the dominant kernel
(measured with HIP events around that kernel inside the timed region) and a
CPU baseline (the oracle, timed on a bounded sample on this host's cores).
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

PEAK_FP64_VALU = 78.6e12   # 256 CUs x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
PEAK_HBM = 8.0e12

# Algorithmic work per unique in-cutoff pair and per slice-atom (FMA = 2 flops,
# rsqrt = 1 flop, rounding to integer not counted); derivation in the design doc.
FLOP_FORCE_PAIR = 41
FLOP_HV_PAIR = 59
FLOP_SLICE_ATOM = 39
BYTES_SLICE_ATOM = 48       # read x_n (24 B) + write g_n (24 B)

# HBM bytes per launch of lj_fused_kernel on the default workload and tuning,
# from rocprofv3 FETCH_SIZE / WRITE_SIZE runs scaled by a 512 MiB copy
# (profiles/lj_fused_lj864x4096.md).  Reported only while the kernel sources
# still hash to `sha`; any change to them makes `traffic` null until the
# counters are taken again.
MEASURED_TRAFFIC = {"sha": "65928b4739e1e40d", "read_bytes": 1.6344e9, "write_bytes": 8.9391e8}
TRAFFIC_SOURCES = ["paper_1907_09529_amd/csrc/lj_fused.hip", "paper_1907_09529_amd/csrc/device.hpp",
                   "paper_1907_09529_amd/csrc/internal.hpp"]


def kernel_sources_sha() -> str:
    import hashlib
    h = hashlib.sha256()
    for rel in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def pairs_per_atom(X: np.ndarray, box: float, rc: float, n_sample: int = 8) -> float:
    """Mean number of unique pairs within r_c per atom over sampled slices (k-d tree count)."""
    from scipy.spatial import cKDTree
    idx = np.linspace(0, X.shape[0] - 1, n_sample).astype(int)
    tot = 0
    for n in idx:
        pts = np.mod(X[n].T, box)
        tree = cKDTree(pts, boxsize=box)
        tot += len(tree.query_pairs(rc, output_type="ndarray"))
    return tot / (len(idx) * X.shape[2])


class HipEvents:
    """hipEvent pair used to time one kernel on the library's stream."""
    hip = None

    def __init__(self):
        if HipEvents.hip is None:
            HipEvents.hip = ctypes.CDLL("libamdhip64.so")
        self.a = ctypes.c_void_p()
        self.b = ctypes.c_void_p()
        assert self.hip.hipEventCreate(ctypes.byref(self.a)) == 0
        assert self.hip.hipEventCreate(ctypes.byref(self.b)) == 0

    def elapsed_ms(self) -> float:
        assert self.hip.hipEventSynchronize(self.b) == 0
        ms = ctypes.c_float(0)
        assert self.hip.hipEventElapsedTime(ctypes.byref(ms), self.a, self.b) == 0
        return float(ms.value)

    def close(self):
        self.hip.hipEventDestroy(self.a)
        self.hip.hipEventDestroy(self.b)


def cpu_baseline(X: np.ndarray, w, target_s: float = 12.0) -> dict:
    """The oracle (as written) on a bounded sample of the same path, all host cores."""
    import multiprocessing as mp
    cores = min(os.cpu_count() or 1, 16)
    t0 = time.perf_counter()
    _oracle_chunk((X[0:3], w))
    t1 = time.perf_counter() - t0           # two slices of oracle work
    per_slice = max(t1 / 2.0, 1e-3)
    per_core = max(1, int(target_s / per_slice))
    n = min(per_core * cores, X.shape[0] - 2)
    bounds = np.linspace(0, n, cores + 1).astype(int)
    chunks = [(X[bounds[c]:bounds[c + 1] + 1], w) for c in range(cores) if bounds[c + 1] > bounds[c]]
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(len(chunks)) as pool:
        done = sum(pool.map(_oracle_chunk, chunks))
    dt = time.perf_counter() - t0
    return {"value": done * w.n_atoms / dt, "unit": "slice_atom_evals/s", "cores": len(chunks),
            "kind": "oracle",
            "sample": f"{done} of {w.n_steps} steps of the benchmark path (action terms + "
                      f"Hessian-vector products + gradient rows), {len(chunks)} processes, "
                      f"{dt:.1f} s wall"}


def _oracle_chunk(args):
    Xc, w = args
    from oracle import forces as OF
    from oracle.potentials import LennardJones
    pot = LennardJones(eps=w.eps, sigma=w.sigma, rc=w.cutoff, box=w.box)
    mu, c = w.dt / w.gamma, 1.0 / (2.0 * w.D * w.dt)
    r_prev = None
    count = 0
    for n in range(Xc.shape[0] - 1):
        d = OF.minimum_image(Xc[n + 1] - Xc[n], w.box)
        r = d - mu * OF.forces(Xc[n], pot)
        _ = np.sum(r * r) / (4.0 * w.D * w.dt)
        q = OF.hessian_vec(Xc[n], r, pot)
        g = c * (-r + mu * q)
        if r_prev is not None:
            g += c * r_prev
        r_prev = r
        count += 1
    return count


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant", choices=["fused", "plain", "fp32_force"], default="fused")
    ap.add_argument("--workload", default="lj864")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--list", choices=["auto", "full", "half"], default="auto")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--skin", type=float, default=0.0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after timing, run one device copy of this many MiB (for counter calibration)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the time-sharded "
              "multi-GPU design is described in DESIGN.md and not built.", file=sys.stderr)
        return 2

    w = W.workload(args.workload)
    print(f"[bench] generating {w.name}: {w.n_steps} steps x {w.n_atoms} atoms", file=sys.stderr,
          flush=True)
    X = W.tethered_path(w)
    baseline = None
    if not args.no_cpu_baseline:
        # before any GPU initialisation: the worker processes are forked from here
        print("[bench] timing the CPU oracle baseline", file=sys.stderr, flush=True)
        baseline = cpu_baseline(X, w)

    import torch
    import paper_1907_09529_amd as P

    P.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    precision = "fp32_force" if args.variant == "fp32_force" else "fp64"
    path = P.make_path(w.n_steps, w.n_atoms, 3, w.dt, w.D, w.gamma, precision)
    pot = P.make_potential("lj", eps=w.eps, sigma=w.sigma, rc=w.cutoff, box=w.box)
    if args.variant == "plain":
        tuning = P.make_tuning("plain")
    elif args.list != "auto" or args.tile or args.skin or args.block:
        tuning = P.make_tuning("fused", block=args.block, tile=args.tile, skin=args.skin,
                               neighbour_list=args.list)
    else:
        tuning = None
    x = torch.from_numpy(X).to(dev)
    grad = torch.empty_like(x)
    act = torch.empty(1, dtype=torch.float64, device=dev)
    per_step = torch.empty(w.n_steps, dtype=torch.float64, device=dev)
    ws = P.workspace(P.pamd_workspace_size(path, pot, tuning))
    if args.autotune and args.variant != "plain":
        big = P.workspace(max(P.pamd_workspace_size(path, pot, P.make_tuning("fused", tile=2, block=b, skin=0.45))
                              for b in (64, 256, 512, 1024)))
        best = P.pamd_autotune(path, pot, x, grad, big)
        print(f"[bench] autotuned: block {best.block} tile {best.tile} skin {best.skin}",
              file=sys.stderr, flush=True)
        ws = P.workspace(P.pamd_workspace_size(path, pot, tuning))
    stream = torch.cuda.current_stream()

    def step():
        P.pamd_action_grad(path, pot, x, grad, action=act, per_step=per_step, ws=ws,
                           tuning=tuning, stream=stream)

    print(f"[bench] warmup {args.warmup} steps, variant {args.variant}", file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    events = [HipEvents() for _ in range(args.steps)]
    lib = P.load()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        lib.pamd_profile_events(events[k].a, events[k].b)
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernel_ms = [e.elapsed_ms() for e in events]
    if args.copy_probe_mb:
        n = args.copy_probe_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
    for e in events:
        e.close()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    units = w.n_steps * w.n_atoms
    value = units / (ms_per_step * 1e-3)
    k_ms = float(np.mean(kernel_ms))
    ppa = pairs_per_atom(X, w.box, w.cutoff)
    flop_unit = ppa * (FLOP_FORCE_PAIR + FLOP_HV_PAIR) + FLOP_SLICE_ATOM
    achieved = flop_unit * units / (k_ms * 1e-3)
    traffic = None
    default_run = (args.variant == "fused" and args.workload == "lj864" and tuning is None
                   and not args.autotune)
    if default_run and MEASURED_TRAFFIC["sha"] and MEASURED_TRAFFIC["sha"] == kernel_sources_sha():
        traffic = MEASURED_TRAFFIC["read_bytes"] + MEASURED_TRAFFIC["write_bytes"]
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU, "traffic": traffic,
            "traffic_unit": "bytes per launch (HBM read + write)",
            "kernel": "lj_fused_kernel" if args.variant != "plain" else "plain pipeline",
            "kernel_ms": k_ms, "flop_per_slice_atom": flop_unit, "pairs_per_atom": ppa,
            "hbm_algorithmic_GBps": BYTES_SLICE_ATOM * units / (k_ms * 1e-3) / 1e9}
    out = {
        "metric": "slice_atom_action_grad_evals_per_s",
        "value": value,
        "unit": "slice_atom_evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precision == "fp64" else "f32_pair/f64_accum",
        "data": "synthetic",
        "config": {"workload": f"LJ {w.n_atoms} atoms x {w.n_steps} steps, rho 0.8442, T 1, "
                               f"rc 2.5, dt 1e-4, {args.variant}",
                   "neighbour_list": args.list,
                   "n_atoms": w.n_atoms, "n_steps": w.n_steps, "variant": args.variant,
                   "parallelism": "single GPU"},
        "roofline": roof,
    }
    if baseline is not None:
        out["cpu_baseline"] = baseline
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
