"""Benchmark: slice-atom action+gradient evaluations per second on one MI355X.

Workload (default): Lennard-Jones path, 864 atoms at reduced density 0.8442,
T = 1, r_c = 2.5 sigma, cubic periodic box, dt = 1e-4, D = gamma = 1, 4096
time steps.  The input is a seeded Euler-Maruyama path (Eq. 2) integrated on
the GPU from the FCC lattice with the workload's own normal draws, slices
1..N then perturbed by N(0, 0.01^2); it is resident in device memory before
timing (``--input tethered`` selects the force-free stand-in instead).  One
benchmark step = one pamd_action_grad call (FP64): action, per-step terms and
the gradient of every slice.

Prints one JSON line with the metric, the roofline of the dominant kernel
(measured with HIP events around that kernel inside the timed region), the
unfused (plain) form timed on the same input, and a CPU baseline: the oracle,
timed on a bounded sample of the same path on this host's cores, in a child
process that never touches the GPU.
"""
from __future__ import annotations

import argparse
import ctypes
import dataclasses
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

# Algorithmic work, fixed before any kernel tuning (FMA = 2 flops, rsqrt = 1):
# per unique in-cutoff pair, the force (difference, minimum image, r^2, the
# pair scalar of Eq. 16, both atoms' sums) and the Hessian-vector product
# (the scalars U'/r and (U'' - U'/r)/r^2, K w for w = rho_i - rho_j, both
# atoms' sums); per slice-atom the residual, |r|^2 and the gradient row.
# The roofline fraction uses these.
FLOP_FORCE_PAIR = 34
FLOP_HV_PAIR = 56
FLOP_SLICE_ATOM = 25
# A recount of every operation the fused kernel's source performs per unique
# pair (the Hessian-vector pass recomputes the geometry: 29 of its 59), reported
# beside the fraction, never in it.
RECOUNT_FORCE_PAIR = 41
RECOUNT_HV_PAIR = 59
RECOUNT_SLICE_ATOM = 39
BYTES_SLICE_ATOM = 48       # read x_n (24 B) + write g_n (24 B)

# HBM bytes per launch of the default fused kernel (lj_fused_exl_kernel) on
# the default workload, input and tuning, from rocprofv3 FETCH_SIZE /
# WRITE_SIZE runs scaled by a 2 GiB elementwise kernel that reads and writes
# known amounts (profiles/lj_fused_exl_lj864x4096.md).  Reported only while
# the kernel sources still hash to `sha`; any change to them makes `traffic`
# null until the counters are taken again.
MEASURED_TRAFFIC = {"sha": "a9b21d8431193886", "input": "em", "read_bytes": 1.02048e9,
                    "write_bytes": 2.75417e8}
# VALU instruction counters of the same kernel, input and tuning (per launch;
# rocprofv3 --pmc, wave-level counts): the FP64 operations it issued, to set
# beside the algorithmic fraction (they include candidates beyond the cutoff
# and each pair's second evaluation from the partner's list).
MEASURED_VALU = {"sha": "a9b21d8431193886", "input": "em", "valu": 4.34554e8,
                 "fma_f64": 9.80155e7, "mul_f64": 6.87759e7, "add_f64": 5.86676e7,
                 "trans_f64": 7.54478e6}
# the kernel's sources and the planner that picks its launch
TRAFFIC_SOURCES = ["paper_1907_09529_amd/csrc/lj_fused.hip", "paper_1907_09529_amd/csrc/device.hpp",
                   "paper_1907_09529_amd/csrc/internal.hpp", "paper_1907_09529_amd/csrc/lj_pair.hpp",
                   "paper_1907_09529_amd/csrc/api.cpp", "include/pamd.h"]


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


def em_path_device(w, P, torch, dev):
    """Seeded Euler-Maruyama path of workload w (Eq. 2): the GPU integrator
    steps the lattice with the workload's normal draws xi, then slices 1..N get
    the workload's perturbation eta.  Same draws as the oracle-built test
    inputs; the integrator is deterministic, so the path is too."""
    x0 = W.initial_lattice(w.n_atoms, w.box)
    xi, eta = W.draw_noise(w)
    path = P.make_path(w.n_steps, w.n_atoms, 3, w.dt, w.D, w.gamma, "fp64")
    pot = P.make_potential("lj", eps=w.eps, sigma=w.sigma, rc=w.cutoff, box=w.box)
    x = torch.empty((w.n_steps + 1, 3, w.n_atoms), dtype=torch.float64, device=dev)
    P.pamd_em_integrate(path, pot, torch.from_numpy(x0).to(dev), torch.from_numpy(xi).to(dev), x)
    del xi
    x[1:].add_(torch.from_numpy(eta).to(dev), alpha=w.perturb_sd)
    torch.cuda.synchronize()
    return x


def input_path(args, w, P, torch, dev):
    """The benchmark input on the device, and a name for it."""
    if getattr(args, "input", "em") == "tethered":
        return (torch.from_numpy(W.tethered_path(w)).to(dev),
                "force-free tethered stand-in around the FCC lattice")
    t0 = time.perf_counter()
    x = em_path_device(w, P, torch, dev)
    print(f"[bench] EM input path on the GPU: {time.perf_counter() - t0:.1f} s", file=sys.stderr,
          flush=True)
    return x, (f"seeded Euler-Maruyama path (Eq. 2) from the FCC lattice, seed {w.seed}, "
               f"+ N(0, {w.perturb_sd:g}^2)")


def cpu_baseline_child(X: np.ndarray, target_s: float = 12.0, method: str = "brute",
                       workload: str = "lj864", member: int = -1) -> dict:
    """Runs cpu_baseline on the host array X in a child Python process that
    never initialises the GPU, so its worker pool can fork safely."""
    import subprocess
    import tempfile
    fd, fn = tempfile.mkstemp(suffix=".npy", dir="/tmp")
    os.close(fd)
    try:
        np.save(fn, np.ascontiguousarray(X))
        cmd = [sys.executable, os.path.abspath(__file__), "--oracle-baseline", fn,
               "--workload", workload, "--baseline-member", str(member),
               "--baseline-target", str(target_s), "--baseline-method", method]
        print(f"[bench] timing the CPU oracle baseline ({X.shape[0] - 1} steps available)",
              file=sys.stderr, flush=True)
        res = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        if res.returncode != 0:
            raise RuntimeError(f"oracle baseline failed: {res.stderr[-2000:]}")
        return json.loads(res.stdout.strip().splitlines()[-1])
    finally:
        os.remove(fn)


def oracle_baseline_main(args) -> int:
    """Child-process side of cpu_baseline_child (no GPU)."""
    X = np.load(args.oracle_baseline, mmap_mode="r")
    if args.baseline_member >= 0:
        w = W.batch_members()[args.baseline_member]
    else:
        w = W.workload(args.workload)
    print(json.dumps(cpu_baseline(np.asarray(X), w, args.baseline_target, args.baseline_method)),
          flush=True)
    return 0


def cpu_baseline(X: np.ndarray, w, target_s: float = 12.0, method: str = "brute") -> dict:
    """The oracle (as written) on a bounded sample of the same path, all host cores."""
    import multiprocessing as mp
    cores = min(os.cpu_count() or 1, 16)
    t0 = time.perf_counter()
    _oracle_chunk((X[0:3], w, method))
    t1 = time.perf_counter() - t0           # two slices of oracle work
    per_slice = max(t1 / 2.0, 1e-3)
    per_core = max(1, int(target_s / per_slice))
    n = min(per_core * cores, X.shape[0] - 2)
    bounds = np.linspace(0, n, cores + 1).astype(int)
    chunks = [(X[bounds[c]:bounds[c + 1] + 1], w, method) for c in range(cores)
              if bounds[c + 1] > bounds[c]]
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
    Xc, w, method = args
    from oracle import forces as OF
    from oracle.potentials import LennardJones
    pot = LennardJones(eps=w.eps, sigma=w.sigma, rc=w.cutoff, box=w.box)
    mu, c = w.dt / w.gamma, 1.0 / (2.0 * w.D * w.dt)
    r_prev = None
    count = 0
    for n in range(Xc.shape[0] - 1):
        d = OF.minimum_image(Xc[n + 1] - Xc[n], w.box)
        r = d - mu * OF.forces(Xc[n], pot, method)
        _ = np.sum(r * r) / (4.0 * w.D * w.dt)
        q = OF.hessian_vec(Xc[n], r, pot, method)
        g = c * (-r + mu * q)
        if r_prev is not None:
            g += c * r_prev
        r_prev = r
        count += 1
    return count


def _parser():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--variant", choices=["fused", "plain", "fp32_force"], default="fused")
    ap.add_argument("--workload", default="lj864",
                    help="lj864 (default), lj108, lj27, ho1d, batch64, sweep4000, "
                         "em864 or em27 (sequential Euler-Maruyama integration), "
                         "pamd864 or pamd27 (the path-based integration loop), "
                         "langevin864 (gradient-informed path move), "
                         "ho_table2 (the harmonic integration schedules: accuracy and rate)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--list", choices=["auto", "full", "half"], default="auto")
    ap.add_argument("--tile", type=int, default=0)
    ap.add_argument("--skin", type=float, default=0.0)
    ap.add_argument("--block", type=int, default=0)
    ap.add_argument("--slots", type=int, default=0, help="LDS slot arrays (0 = library choice)")
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="after timing, run one device copy of this many MiB (for counter calibration)")
    ap.add_argument("--input", choices=["em", "tethered"], default="em",
                    help="LJ input path: seeded Euler-Maruyama run (default) or the tethered stand-in")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip timing the unfused form beside the fused one")
    # internal: the CPU baseline's child process
    ap.add_argument("--oracle-baseline", default="", help=argparse.SUPPRESS)
    ap.add_argument("--baseline-member", type=int, default=-1, help=argparse.SUPPRESS)
    ap.add_argument("--baseline-target", type=float, default=12.0, help=argparse.SUPPRESS)
    ap.add_argument("--baseline-method", default="brute", help=argparse.SUPPRESS)
    return ap


def _line(metric_value, ms, args, dtype, config, roof, baseline,
          metric="slice_atom_action_grad_evals_per_s", unit="slice_atom_evals/s", extra=None):
    out = {
        "metric": metric,
        "value": metric_value,
        "unit": unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": config,
        "roofline": roof,
    }
    if baseline is not None:
        out["cpu_baseline"] = baseline
    if extra:
        out.update(extra)
    print(json.dumps(out), flush=True)


def main(argv=None) -> int:
    args = _parser().parse_args(argv)
    if args.oracle_baseline:
        return oracle_baseline_main(args)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); sharding the "
              "path along time across GPUs is a design that is not built.", file=sys.stderr)
        return 2
    if args.workload == "batch64":
        return bench_batch(args)
    if args.workload == "sweep4000":
        return bench_sweep(args)
    if args.workload in ("em864", "em27"):
        return bench_em(args, W.workload("lj" + args.workload[2:]))
    if args.workload in ("pamd864", "pamd27"):
        return bench_pamd(args, W.workload("lj" + args.workload[4:]))
    if args.workload == "langevin864":
        return bench_langevin(args, W.workload("lj864"))
    if args.workload == "ho_table2":
        return bench_ho_table2(args)
    w = W.workload(args.workload)
    if w.potential == "harmonic":
        return bench_harmonic(args, w)
    return bench_path(args, w)


def _time_calls(step, n_warm, n_timed, lib, torch):
    """Runs step() n_warm + n_timed times; returns (wall ms per call, the main
    kernel's HIP-event ms per call) over the timed calls."""
    for _ in range(n_warm):
        step()
    torch.cuda.synchronize()
    events = [HipEvents() for _ in range(n_timed)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(n_timed):
        lib.pamd_profile_events(events[k].a, events[k].b)
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kernel_ms = [e.elapsed_ms() for e in events]
    for e in events:
        e.close()
    return (t1 - t0) * 1e3 / n_timed, float(np.mean(kernel_ms))


def bench_path(args, w) -> int:
    """One Lennard-Jones path: one step = one pamd_action_grad call."""
    import torch
    import paper_1907_09529_amd as P

    lib = P.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print(f"[bench] input {w.name}: {w.n_steps} steps x {w.n_atoms} atoms ({args.input})",
          file=sys.stderr, flush=True)
    x, input_name = input_path(args, w, P, torch, dev)
    precision = "fp32_force" if args.variant == "fp32_force" else "fp64"
    path = P.make_path(w.n_steps, w.n_atoms, 3, w.dt, w.D, w.gamma, precision)
    pot = P.make_potential("lj", eps=w.eps, sigma=w.sigma, rc=w.cutoff, box=w.box)
    if args.variant == "plain":
        tuning = P.make_tuning("plain")
    elif args.list != "auto" or args.tile or args.skin or args.block or args.slots:
        tuning = P.make_tuning("fused", block=args.block, tile=args.tile, skin=args.skin,
                               neighbour_list=args.list, slot_arrays=args.slots)
    else:
        tuning = None
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
    launch = P.pamd_launch_info(path, pot, tuning)
    stream = torch.cuda.current_stream()

    def step():
        P.pamd_action_grad(path, pot, x, grad, action=act, per_step=per_step, ws=ws,
                           tuning=tuning, stream=stream)

    default_run = (args.variant == "fused" and args.workload == "lj864" and tuning is None
                   and not args.autotune)
    plain_run = None
    if default_run and not args.no_plain:
        # The unfused form on the same input, timed first.  Its untimed calls
        # (about 90 ms of load) also bring the shader clock to its sustained
        # level, which the first ~50 ms of load do not reach, so both legs of
        # the fused/plain ratio run at it.
        tplain = P.make_tuning("plain")
        wsp = P.workspace(P.pamd_workspace_size(path, pot, tplain))
        gp = torch.empty_like(x)
        actp = torch.empty(1, dtype=torch.float64, device=dev)

        def step_plain():
            P.pamd_action_grad(path, pot, x, gp, action=actp, ws=wsp, tuning=tplain, stream=stream)

        n_plain = max(1, min(args.steps, 5))
        print(f"[bench] plain form: 30 untimed and {n_plain} timed calls", file=sys.stderr, flush=True)
        p_ms, p_kms = _time_calls(step_plain, 30, n_plain, lib, torch)
        del wsp
        plain_run = (p_ms, gp, actp)
    print(f"[bench] warmup {args.warmup} steps, variant {args.variant}", file=sys.stderr, flush=True)
    ms_per_step, k_ms = _time_calls(step, args.warmup, args.steps, lib, torch)
    if args.copy_probe_mb:
        # counter calibration: an elementwise kernel over the whole device
        # that reads and writes copy_probe_mb MiB each (dst = src + 1)
        n = args.copy_probe_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.add(src, 1.0, out=dst)
        torch.cuda.synchronize()
        del src, dst
    units = w.n_steps * w.n_atoms
    value = units / (ms_per_step * 1e-3)
    idx = np.linspace(0, w.n_steps, 8).astype(int)
    ppa = pairs_per_atom(x[torch.from_numpy(idx).to(dev)].cpu().numpy(), w.box, w.cutoff)
    flop_unit = ppa * (FLOP_FORCE_PAIR + FLOP_HV_PAIR) + FLOP_SLICE_ATOM
    recount_unit = ppa * (RECOUNT_FORCE_PAIR + RECOUNT_HV_PAIR) + RECOUNT_SLICE_ATOM
    achieved = flop_unit * units / (k_ms * 1e-3)
    sha = kernel_sources_sha()
    traffic = None
    if (default_run and MEASURED_TRAFFIC["sha"] == sha
            and MEASURED_TRAFFIC.get("input", "tethered") == args.input):
        traffic = MEASURED_TRAFFIC["read_bytes"] + MEASURED_TRAFFIC["write_bytes"]
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU, "traffic": traffic,
            "traffic_unit": "bytes per launch (HBM read + write)",
            "kernel": ("plain pipeline" if args.variant == "plain" else
                       "lj_fused_exl_kernel" if launch.exact_lists else "lj_fused_kernel"),
            "kernel_ms": k_ms, "flop_per_slice_atom": flop_unit,
            "flop_constants": [FLOP_FORCE_PAIR, FLOP_HV_PAIR, FLOP_SLICE_ATOM],
            "pairs_per_atom": ppa,
            "frac_recount": recount_unit * units / (k_ms * 1e-3) / PEAK_FP64_VALU,
            "hbm_algorithmic_GBps": BYTES_SLICE_ATOM * units / (k_ms * 1e-3) / 1e9}
    if default_run and MEASURED_VALU["sha"] == sha and MEASURED_VALU["input"] == args.input:
        # FP64 operations the kernel issued (wave-level counts x 64 lanes), per
        # second of the live kernel time, against the FP64 vector peak
        ops = 64 * (2 * MEASURED_VALU["fma_f64"] + MEASURED_VALU["mul_f64"]
                    + MEASURED_VALU["add_f64"] + MEASURED_VALU["trans_f64"])
        roof["counter_fp64_frac"] = ops / (k_ms * 1e-3) / PEAK_FP64_VALU
        roof["counter_valu_insts"] = MEASURED_VALU["valu"]
    if args.variant == "fp32_force":
        roof["note"] = ("float32 only in the Hessian-vector pass's pair products (a w + b (d.w) d); "
                        "the pair functions, the force pass and all sums stay float64, so the "
                        "float64 peak applies")
    plain = None
    if plain_run is not None:
        # its agreement with the fused result of the last timed call
        p_ms, gp, actp = plain_run
        torch.cuda.synchronize()
        plain = {"ms_per_call": p_ms, "fused_over_plain": p_ms / ms_per_step,
                 "action_rel_diff": abs(float(actp.item()) - float(act.item())) / abs(float(act.item())),
                 "grad_rel_diff": float((gp - grad).abs().max() / grad.abs().max())}
        del gp
    config = {"workload": f"LJ {w.n_atoms} atoms x {w.n_steps} steps, rho {w.density}, T 1, "
                          f"rc {w.cutoff:.4g}, dt {w.dt:g}, {args.variant}; input: {input_name}",
              "neighbour_list": args.list, "input": args.input,
              "n_atoms": w.n_atoms, "n_steps": w.n_steps, "variant": args.variant,
              "tile": launch.tile, "block": launch.block, "slot_arrays": launch.slot_arrays,
              "exact_lists": launch.exact_lists, "parallelism": "single GPU"}
    baseline = None
    if not args.no_cpu_baseline:
        host = x[:min(w.n_steps + 1, 4097)].cpu().numpy()
        baseline = cpu_baseline_child(host, workload=args.workload)
    extra = {"plain": plain} if plain is not None else {}
    _line(value, ms_per_step, args, "f64" if precision == "fp64" else "f32_pair/f64_accum",
          config, roof, baseline, extra=extra)
    return 0


def bench_harmonic(args, w) -> int:
    """The 1-D harmonic path: one step = one pamd_action_grad call (a single
    streaming kernel; at this size its time is launch latency)."""
    X = W.free_walk_path(w)
    baseline = None
    if not args.no_cpu_baseline:
        from oracle import action as OA
        from oracle.potentials import Harmonic
        pot_o = Harmonic(k=w.k)
        reps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < 2.0:
            OA.per_step_action(X, pot_o, w.dt, w.D, w.gamma)
            OA.path_gradient(X, pot_o, w.dt, w.D, w.gamma)
            reps += 1
        dt = time.perf_counter() - t0
        baseline = {"value": reps * w.n_steps * w.n_atoms / dt, "unit": "slice_atom_evals/s",
                    "cores": 1, "kind": "oracle",
                    "sample": f"whole path x {reps} repetitions (per-step terms + gradient), "
                              f"1 process, {dt:.1f} s wall"}
    import torch
    import paper_1907_09529_amd as P
    P.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    path = P.make_path(w.n_steps, w.n_atoms, w.n_dim, w.dt, w.D, w.gamma, "fp64")
    pot = P.make_potential("harmonic", k=w.k)
    x = torch.from_numpy(X).to(dev)
    grad = torch.empty_like(x)
    act = torch.empty(1, dtype=torch.float64, device=dev)
    per_step = torch.empty(w.n_steps, dtype=torch.float64, device=dev)
    ws = P.workspace(P.pamd_workspace_size(path, pot))
    stream = torch.cuda.current_stream()
    lib = P.load()
    for _ in range(args.warmup):
        P.pamd_action_grad(path, pot, x, grad, action=act, per_step=per_step, ws=ws, stream=stream)
    torch.cuda.synchronize()
    events = [HipEvents() for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        lib.pamd_profile_events(events[k].a, events[k].b)
        P.pamd_action_grad(path, pot, x, grad, action=act, per_step=per_step, ws=ws, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms = float(np.mean([e.elapsed_ms() for e in events]))
    for e in events:
        e.close()
    ms = (t1 - t0) * 1e3 / args.steps
    units = w.n_steps * w.n_atoms
    dof = w.n_atoms * w.n_dim
    # streaming kernel: reads x (N+1 slices), writes g (N+1 slices) and s_n (N)
    nbytes = 8 * (2 * (w.n_steps + 1) * dof + w.n_steps)
    roof = {"bound": "hbm", "achieved": nbytes / (k_ms * 1e-3) / 1e9, "peak": PEAK_HBM / 1e9,
            "unit": "GB/s", "frac": nbytes / (k_ms * 1e-3) / PEAK_HBM, "traffic": None,
            "kernel": "ho_kernel", "kernel_ms": k_ms, "bytes_per_launch": nbytes,
            "note": "launch-latency bound at this size"}
    config = {"workload": f"1-D harmonic path, k {w.k:g}, dt {w.dt:g}, {w.n_steps} steps",
              "n_atoms": w.n_atoms, "n_steps": w.n_steps, "parallelism": "single GPU"}
    _line(units / (ms * 1e-3), ms, args, "f64", config, roof, baseline)
    return 0


def _member_flops(Xs, w) -> float:
    """Algorithmic flops per slice-atom of one LJ path (pairs counted on the given slices)."""
    ppa = pairs_per_atom(Xs, w.box, w.cutoff, n_sample=Xs.shape[0])
    return ppa * (FLOP_FORCE_PAIR + FLOP_HV_PAIR) + FLOP_SLICE_ATOM


def bench_batch(args) -> int:
    """The 64-path batch: one step = one replay of a captured graph holding one
    persistent pamd_batch_run launch over every member."""
    import torch
    import paper_1907_09529_amd as P
    P.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    members = W.batch_members()
    units = sum(m.n_steps * m.n_atoms for m in members)
    t0 = time.perf_counter()
    arrays = [input_path(args, m, P, torch, dev)[0] for m in members]
    print(f"[bench] {len(members)} member inputs on the GPU: {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    flops = sum(_member_flops(X[[0, X.shape[0] - 1]].cpu().numpy(), m) * m.n_steps * m.n_atoms
                for X, m in zip(arrays, members))
    big = max(range(len(members)), key=lambda p: members[p].n_atoms * members[p].n_steps)
    host_big = arrays[big][:min(members[big].n_steps + 1, 4097)].cpu().numpy()
    paths, pots = [], []
    for m in members:
        paths.append(P.make_path(m.n_steps, m.n_atoms, 3, m.dt, m.D, m.gamma, "fp64"))
        pots.append(P.make_potential("lj", eps=m.eps, sigma=m.sigma, rc=m.cutoff, box=m.box))
    b0 = P.PamdBatch(paths, pots)
    x = torch.zeros(b0.x_offsets[-1], dtype=torch.float64, device=dev)
    for p, X in enumerate(arrays):
        x[b0.x_offsets[p]:b0.x_offsets[p] + X.numel()] = X.reshape(-1)
    del arrays
    grad = torch.zeros_like(x)
    act = torch.empty(len(members), dtype=torch.float64, device=dev)

    def time_batch(b):
        """One persistent launch per replay of a captured graph: (ms per step, graph ms)."""
        b.prepare()
        s = torch.cuda.Stream()
        g = P.PamdGraph()
        torch.cuda.synchronize()
        with torch.cuda.stream(s):
            g.begin(s)
            b.pamd_batch_run(x, act, grad_all=grad, stream=s)
            g.end(s)
            for _ in range(args.warmup):
                g.launch(s)
        s.synchronize()
        ev = HipEvents()
        hip = HipEvents.hip
        t0 = time.perf_counter()
        hip.hipEventRecord(ev.a, ctypes.c_void_p(s.cuda_stream))
        for _ in range(args.steps):
            g.launch(s)
        hip.hipEventRecord(ev.b, ctypes.c_void_p(s.cuda_stream))
        s.synchronize()
        t1 = time.perf_counter()
        out = ((t1 - t0) * 1e3 / args.steps, ev.elapsed_ms() / args.steps)
        ev.close()
        g.close()
        return out

    # the built-in tile rule, then the batch autotuner's choice (it times the
    # persistent launch itself for each member-tile policy)
    ms_h, g_ms_h = time_batch(b0)
    print(f"[bench] built-in tiles: {g_ms_h:.3f} ms per launch", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    budget, skin = b0.autotune(x, grad)
    print(f"[bench] batch autotune: tile budget {budget:g} atom-steps, skin {skin:g} sigma "
          f"({time.perf_counter() - t0:.1f} s)", file=sys.stderr, flush=True)
    ms, g_ms = time_batch(b0)
    b0.close()
    roof = {"bound": "alu", "achieved": flops / (g_ms * 1e-3) / 1e12, "peak": PEAK_FP64_VALU / 1e12,
            "unit": "TFLOP/s", "frac": flops / (g_ms * 1e-3) / PEAK_FP64_VALU, "traffic": None,
            "kernel": "graph replay (lj_batch_kernel + batch_finalize_kernel)", "kernel_ms": g_ms,
            "flop_per_launch": flops, "builtin_tiles_ms": g_ms_h,
            "autotune_gain": g_ms_h / g_ms, "tile_budget": budget, "skin_sigma": skin}
    config = {"workload": f"batch of {len(members)} LJ paths, atoms in {{108..2048}}, "
                          f"steps {min(m.n_steps for m in members)}..{max(m.n_steps for m in members)}, "
                          f"one persistent launch, graph-captured; input: {args.input}",
              "n_paths": len(members), "slice_atoms": units, "input": args.input,
              "parallelism": "single GPU"}
    baseline = None
    if not args.no_cpu_baseline:
        # the oracle on the largest member (same per-slice work as the GPU's)
        baseline = cpu_baseline_child(host_big, workload="batch64", member=big)
        baseline["sample"] = f"member {big} ({members[big].n_atoms} atoms): " + baseline["sample"]
    _line(units / (ms * 1e-3), ms, args, "f64", config, roof, baseline)
    return 0


def bench_sweep(args) -> int:
    """The path-sampling sweep (4000 atoms x 16384 steps): one step = one sweep,
    a fragment-wise Metropolis-Hastings move (trial bridges, excess action of
    the trial path, accept/commit) followed by action + gradient of the
    committed path, replayed from a captured graph."""
    w = W.workload("sweep4000")
    import torch
    import paper_1907_09529_amd as P
    P.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print(f"[bench] input {w.name}: {w.n_steps} steps x {w.n_atoms} atoms ({args.input})",
          file=sys.stderr, flush=True)
    x, input_name = input_path(args, w, P, torch, dev)
    flop_unit = _member_flops(x[[0, w.n_steps // 2, w.n_steps]].cpu().numpy(), w)
    host_sample = x[:1025].cpu().numpy()
    path = P.make_path(w.n_steps, w.n_atoms, 3, w.dt, w.D, w.gamma, "fp64")
    pot = P.make_potential("lj", eps=w.eps, sigma=w.sigma, rc=w.cutoff, box=w.box)
    trial = torch.empty_like(x)
    grad = torch.empty_like(x)
    ex = torch.empty(w.n_steps, dtype=torch.float64, device=dev)
    act = torch.empty(1, dtype=torch.float64, device=dev)
    counter = torch.zeros(1, dtype=torch.int64, device=dev)
    info = torch.empty(4, dtype=torch.int32, device=dev)
    ws_mh = P.workspace(P.pamd_mh_workspace_size(path, pot))
    ws = P.workspace(P.pamd_workspace_size(path, pot))
    P.pamd_excess_action(path, pot, x, ex)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    seed = 0x5EED1907

    def sweep(stream):
        P.pamd_mh_step(path, pot, seed, w.l_min, w.l_max, counter, x, ex, trial,
                       step_info=info, ws=ws_mh, stream=stream)
        P.pamd_action_grad(path, pot, x, grad, action=act, ws=ws, stream=stream)

    g = P.PamdGraph()
    with torch.cuda.stream(s):
        g.begin(s)
        sweep(s)
        g.end(s)
        for _ in range(args.warmup):
            g.launch(s)
    s.synchronize()
    ev = HipEvents()
    hip = HipEvents.hip
    t0 = time.perf_counter()
    hip.hipEventRecord(ev.a, ctypes.c_void_p(s.cuda_stream))
    for _ in range(args.steps):
        g.launch(s)
    hip.hipEventRecord(ev.b, ctypes.c_void_p(s.cuda_stream))
    s.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    g_ms = ev.elapsed_ms() / args.steps
    ev.close()
    g.close()
    # the action+gradient kernel alone, timed eagerly after the sweeps
    lib = P.load()
    kev = [HipEvents() for _ in range(3)]
    for e in kev:
        lib.pamd_profile_events(e.a, e.b)
        P.pamd_action_grad(path, pot, x, grad, action=act, ws=ws, stream=torch.cuda.current_stream())
    k_ms = float(np.mean([e.elapsed_ms() for e in kev]))
    for e in kev:
        e.close()
    sweeps = int(counter.item())
    units = w.n_steps * w.n_atoms
    roof = {"bound": "alu", "achieved": flop_unit * units / (k_ms * 1e-3) / 1e12,
            "peak": PEAK_FP64_VALU / 1e12, "unit": "TFLOP/s",
            "frac": flop_unit * units / (k_ms * 1e-3) / PEAK_FP64_VALU, "traffic": None,
            "kernel": "lj_fused_kernel (action + gradient, residuals in global scratch)",
            "kernel_ms": k_ms, "flop_per_slice_atom": flop_unit, "sweep_ms": g_ms}
    config = {"workload": f"path-sampling sweep, LJ {w.n_atoms} atoms x {w.n_steps} steps, "
                          f"levels {w.l_min}..{w.l_max}, MH move + action + gradient per sweep, "
                          f"graph-captured; input: {input_name}",
              "n_atoms": w.n_atoms, "n_steps": w.n_steps, "sweeps_run": sweeps,
              "input": args.input, "parallelism": "single GPU"}
    baseline = None
    if not args.no_cpu_baseline:
        baseline = cpu_baseline_child(host_sample, target_s=12.0, method="cells",
                                      workload="sweep4000")
    _line(units / (ms * 1e-3), ms, args, "f64", config, roof, baseline)
    return 0


# The paper's Lennard-Jones PAMD schedule with the largest speedup (Sec. IV B,
# Simulation 2): N_path = 4096, levels 4..7, N_sample = 1 sweep per shift of
# N_shift = 64 steps, dt = 2 dt_E.
SIM2 = {"n_path": 4096, "l_min": 4, "l_max": 7, "n_sample": 1, "n_shift": 64, "dt_ratio": 2}
EM_STEPS = 4096


def _em_oracle_chunk(args):
    x0, xi, w = args
    from oracle import em as OE
    from oracle.potentials import LennardJones
    pot = LennardJones(eps=w.eps, sigma=w.sigma, rc=w.cutoff, box=w.box)
    OE.em_path(x0, xi, pot, w.dt, w.D, w.gamma)
    return xi.shape[0]


def bench_em(args, w) -> int:
    """Sequential Euler-Maruyama integration (Eq. 2) of one Lennard-Jones
    system at dt_E = dt / 2: one step = one pamd_em_integrate call over 4096
    time steps.  Also times one path-sampling sweep of the paper's Simulation 2
    schedule on the same system and reports the measured counterpart of the
    speedup chi (Eq. 11): the wall time of the N_shift dt / dt_E Euler steps
    that one shifting event advances, over the N_sample sweeps it costs (the
    shift itself is a ring-buffer offset and is not timed)."""
    w_e = dataclasses.replace(w, dt=w.dt / SIM2["dt_ratio"], n_steps=EM_STEPS)
    print(f"[bench] {w.name}: {EM_STEPS} Euler steps of {w.n_atoms} atoms at dt_E {w_e.dt:g}",
          file=sys.stderr, flush=True)
    x0 = W.initial_lattice(w.n_atoms, w.box)
    xi, _ = W.draw_noise(w_e)
    baseline = None
    if not args.no_cpu_baseline:
        import multiprocessing as mp
        t0 = time.perf_counter()
        _em_oracle_chunk((x0, xi[:2], w_e))
        per_step = max((time.perf_counter() - t0) / 2.0, 1e-4)
        cores = min(os.cpu_count() or 1, 16)
        n = max(1, min(int(12.0 / per_step), EM_STEPS))
        # a sequential chain cannot be split over cores: each process runs the
        # same n steps and the rate is that of one chain
        t0 = time.perf_counter()
        with mp.get_context("fork").Pool(1) as pool:
            done = pool.map(_em_oracle_chunk, [(x0, xi[:n], w_e)])[0]
        dt = time.perf_counter() - t0
        baseline = {"value": done * w.n_atoms / dt, "unit": "slice_atom_steps/s", "cores": 1,
                    "kind": "oracle",
                    "sample": f"{done} of {EM_STEPS} sequential Euler steps (brute-force pair "
                              f"forces), one process ({cores} cores idle: the chain is serial), "
                              f"{dt:.1f} s wall"}

    import torch
    import paper_1907_09529_amd as P
    P.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pot = P.make_potential("lj", eps=w.eps, sigma=w.sigma, rc=w.cutoff, box=w.box)
    path_e = P.make_path(EM_STEPS, w.n_atoms, 3, w_e.dt, w.D, w.gamma, "fp64")
    x0_d = torch.from_numpy(x0).to(dev)
    xi_d = torch.from_numpy(xi).to(dev)
    del xi
    out = torch.empty((EM_STEPS + 1, 3, w.n_atoms), dtype=torch.float64, device=dev)
    ws = P.workspace(P.pamd_em_workspace_size(path_e, pot))
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        P.pamd_em_integrate(path_e, pot, x0_d, xi_d, out, ws=ws, stream=stream)
    torch.cuda.synchronize()
    lib = P.load()
    events = [HipEvents() for _ in range(args.steps)]
    t0 = time.perf_counter()
    for k in range(args.steps):
        lib.pamd_profile_events(events[k].a, events[k].b)
        P.pamd_em_integrate(path_e, pot, x0_d, xi_d, out, ws=ws, stream=stream)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms = float(np.mean([e.elapsed_ms() for e in events]))
    for e in events:
        e.close()
    ms = (t1 - t0) * 1e3 / args.steps
    X_e = out.cpu().numpy()
    ppa = pairs_per_atom(X_e, w.box, w.cutoff, n_sample=4)
    flop_unit = ppa * 2 * FLOP_FORCE_PAIR + 12     # full lists: each pair evaluated twice
    units = EM_STEPS * w.n_atoms
    achieved = flop_unit * units / (k_ms * 1e-3)
    peak_cu = PEAK_FP64_VALU / 256                 # one workgroup runs on one CU

    # one sweep of the Simulation 2 schedule on a path of the same system,
    # integrated at the PAMD step dt by the same integrator
    sweep_ms = None
    path_p = P.make_path(SIM2["n_path"], w.n_atoms, 3, w.dt, w.D, w.gamma, "fp64")
    xi_p = torch.from_numpy(W.draw_noise(w.with_steps(SIM2["n_path"]))[0]).to(dev)
    x = torch.empty((SIM2["n_path"] + 1, 3, w.n_atoms), dtype=torch.float64, device=dev)
    P.pamd_em_integrate(path_p, pot, x0_d, xi_p, x,
                        ws=P.workspace(P.pamd_em_workspace_size(path_p, pot)))
    del xi_p
    trial = torch.empty_like(x)
    ex = torch.empty(SIM2["n_path"], dtype=torch.float64, device=dev)
    counter = torch.zeros(1, dtype=torch.int64, device=dev)
    ws_mh = P.workspace(P.pamd_mh_workspace_size(path_p, pot))
    P.pamd_excess_action(path_p, pot, x, ex)
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = P.PamdGraph()
    with torch.cuda.stream(s):
        g.begin(s)
        P.pamd_mh_step(path_p, pot, 0x5EED1907, SIM2["l_min"], SIM2["l_max"], counter, x, ex,
                       trial, ws=ws_mh, stream=s)
        g.end(s)
        for _ in range(args.warmup):
            g.launch(s)
    s.synchronize()
    ev = HipEvents()
    n_sw = max(args.steps, 20)
    HipEvents.hip.hipEventRecord(ev.a, ctypes.c_void_p(s.cuda_stream))
    for _ in range(n_sw):
        g.launch(s)
    HipEvents.hip.hipEventRecord(ev.b, ctypes.c_void_p(s.cuda_stream))
    s.synchronize()
    sweep_ms = ev.elapsed_ms() / n_sw
    ev.close()
    g.close()
    em_step_ms = k_ms / EM_STEPS
    chi_paper = SIM2["n_shift"] * SIM2["dt_ratio"] / SIM2["n_sample"]
    chi = SIM2["n_shift"] * SIM2["dt_ratio"] * em_step_ms / (SIM2["n_sample"] * sweep_ms)

    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": peak_cu / 1e12,
            "unit": "TFLOP/s", "frac": achieved / peak_cu, "traffic": None,
            "kernel": "lj_em_kernel (one workgroup; peak = one CU's FP64 VALU rate)",
            "kernel_ms": k_ms, "flop_per_slice_atom": flop_unit, "pairs_per_atom": ppa}
    config = {"workload": f"sequential Euler-Maruyama, LJ {w.n_atoms} atoms, rho {w.density}, "
                          f"rc {w.cutoff:.4g}, {EM_STEPS} steps at dt_E {w_e.dt:g}",
              "n_atoms": w.n_atoms, "n_steps": EM_STEPS, "em_step_us": em_step_ms * 1e3,
              "sim2_sweep_ms": sweep_ms, "chi_paper": chi_paper, "chi_measured": chi,
              "chi_note": "N_shift dt/dt_E Euler steps (wall) / N_sample graph-replayed sweeps "
                          f"(N_path {SIM2['n_path']}, levels {SIM2['l_min']}..{SIM2['l_max']}) "
                          "on this GPU",
              "parallelism": "single GPU, one workgroup"}
    _line(units / (ms * 1e-3), ms, args, "f64", config, roof, baseline,
          metric="em_slice_atom_steps_per_s", unit="slice_atom_steps/s")
    return 0


def bench_pamd(args, w) -> int:
    """The path-based integration loop with the paper's Simulation 2 schedule
    on one Lennard-Jones system: one step = one shifting event (N_sample MC
    sweeps of the 4096-step path, shift, regrowth, excess of the regrown
    steps), replayed from a captured graph of two events.  Reports the
    simulated time advanced per wall-clock second, the same for sequential
    Euler at dt_E = dt / 2, and their ratio (the measured speedup chi)."""
    n_path, n_shift = SIM2["n_path"], SIM2["n_shift"]
    print(f"[bench] {w.name}: path-based integration, {n_path}-step path, shift {n_shift}",
          file=sys.stderr, flush=True)
    x0 = W.initial_lattice(w.n_atoms, w.box)
    baseline = None
    if not args.no_cpu_baseline:
        from oracle import action as OA
        from oracle.potentials import LennardJones
        pot_o = LennardJones(eps=w.eps, sigma=w.sigma, rc=w.cutoff, box=w.box)
        xi_o, _ = W.draw_noise(w.with_steps(16))
        from oracle import em as OE
        Xo = OE.em_path(x0, xi_o, pot_o, w.dt, w.D, w.gamma)
        t0 = time.perf_counter()
        reps = 0
        while time.perf_counter() - t0 < 10.0:
            OA.per_step_action(Xo, pot_o, w.dt, w.D, w.gamma)
            reps += 1
        per_slice = (time.perf_counter() - t0) / (reps * 16)
        # one event = N_sample sweeps, each evaluating the trial path's n_path steps
        ev_s = SIM2["n_sample"] * n_path * per_slice
        baseline = {"value": n_shift * w.dt / ev_s, "unit": "md_time/s", "cores": 1,
                    "kind": "oracle",
                    "sample": f"{reps} evaluations of the oracle's per-step action on a 16-step "
                              f"path of this system ({per_slice * 1e3:.3f} ms per slice), scaled "
                              f"to one event's {SIM2['n_sample']} x {n_path} slices; the "
                              "trial generation and accept step are not counted"}

    import torch
    import paper_1907_09529_amd as P
    P.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pot = P.make_potential("lj", eps=w.eps, sigma=w.sigma, rc=w.cutoff, box=w.box)
    path = P.make_path(n_path, w.n_atoms, 3, w.dt, w.D, w.gamma, "fp64")
    x0_d = torch.from_numpy(x0).to(dev)
    xi = torch.from_numpy(W.draw_noise(w.with_steps(n_path))[0]).to(dev)
    x = torch.empty((n_path + 1, 3, w.n_atoms), dtype=torch.float64, device=dev)
    P.pamd_em_integrate(path, pot, x0_d, xi, x, ws=P.workspace(P.pamd_em_workspace_size(path, pot)))
    del xi
    x_alt, trial = torch.empty_like(x), torch.empty_like(x)
    ex = torch.empty(n_path, dtype=torch.float64, device=dev)
    ex_alt = torch.empty_like(ex)
    P.pamd_excess_action(path, pot, x, ex)
    counters = torch.zeros(2, dtype=torch.int64, device=dev)
    stats = torch.zeros(62, dtype=torch.int64, device=dev)
    traj = torch.empty((2 * n_shift, 3, w.n_atoms), dtype=torch.float64, device=dev)
    ws = P.workspace(P.pamd_run_workspace_size(path, pot, n_shift))
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    g = P.PamdGraph()
    with torch.cuda.stream(s):
        g.begin(s)
        P.pamd_run(path, pot, 0x5EED1907, SIM2["l_min"], SIM2["l_max"], SIM2["n_sample"], n_shift,
                   2, counters, x, x_alt, trial, ex, ex_alt, traj, level_stats=stats, ws=ws,
                   stream=s)
        g.end(s)
        for _ in range(args.warmup):
            g.launch(s)
    s.synchronize()
    reps = max(1, args.steps // 2)
    ev = HipEvents()
    t0 = time.perf_counter()
    HipEvents.hip.hipEventRecord(ev.a, ctypes.c_void_p(s.cuda_stream))
    for _ in range(reps):
        g.launch(s)
    HipEvents.hip.hipEventRecord(ev.b, ctypes.c_void_p(s.cuda_stream))
    s.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / (2 * reps)
    ev_ms = ev.elapsed_ms() / (2 * reps)
    ev.close()
    g.close()
    assert bool(torch.isfinite(x).all())
    # the excess-mode fused kernel alone on the current path
    lib = P.load()
    kev = [HipEvents() for _ in range(3)]
    for e in kev:
        lib.pamd_profile_events(e.a, e.b)
        P.pamd_excess_action(path, pot, x, ex_alt)
    k_ms = float(np.mean([e.elapsed_ms() for e in kev]))
    for e in kev:
        e.close()
    Xh = x.cpu().numpy()
    ppa = pairs_per_atom(Xh, w.box, w.cutoff, n_sample=4)
    flop_unit = ppa * FLOP_FORCE_PAIR + 24       # force pass, residual, excess terms
    achieved = flop_unit * n_path * w.n_atoms / (k_ms * 1e-3)
    # sequential Euler on the same system at dt_E = dt / 2
    w_e = dataclasses.replace(w, dt=w.dt / SIM2["dt_ratio"], n_steps=EM_STEPS)
    path_e = P.make_path(EM_STEPS, w.n_atoms, 3, w_e.dt, w.D, w.gamma, "fp64")
    xi_e = torch.from_numpy(W.draw_noise(w_e)[0]).to(dev)
    out = torch.empty((EM_STEPS + 1, 3, w.n_atoms), dtype=torch.float64, device=dev)
    ws_e = P.workspace(P.pamd_em_workspace_size(path_e, pot))
    P.pamd_em_integrate(path_e, pot, x0_d, xi_e, out, ws=ws_e)
    eev = HipEvents()
    lib.pamd_profile_events(eev.a, eev.b)
    P.pamd_em_integrate(path_e, pot, x0_d, xi_e, out, ws=ws_e)
    em_step_ms = eev.elapsed_ms() / EM_STEPS
    eev.close()
    md_rate = n_shift * w.dt / (ms * 1e-3)
    em_rate = w_e.dt / (em_step_ms * 1e-3)
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU, "traffic": None,
            "kernel": ("lj_action_exl_kernel" if P.pamd_launch_info(path, pot).exact_lists
                       else "lj_action_kernel") + " (excess action of the trial path)",
            "kernel_ms": k_ms,
            "flop_per_slice_atom": flop_unit, "pairs_per_atom": ppa}
    config = {"workload": f"path-based integration, LJ {w.n_atoms} atoms, rho {w.density}, "
                          f"rc {w.cutoff:.4g}, N_path {n_path}, levels {SIM2['l_min']}.."
                          f"{SIM2['l_max']}, N_sample {SIM2['n_sample']}, N_shift {n_shift}, "
                          f"dt {w.dt:g}, graph-replayed events",
              "n_atoms": w.n_atoms, "n_path": n_path, "event_ms": ms, "event_gpu_ms": ev_ms,
              "md_time_per_s": md_rate, "euler_md_time_per_s": em_rate,
              "euler_step_us": em_step_ms * 1e3, "chi_paper": SIM2["n_shift"] * SIM2["dt_ratio"],
              "chi_measured": md_rate / em_rate, "parallelism": "single GPU"}
    st = stats.cpu().numpy().reshape(31, 2)
    config["acceptance_by_level"] = {str(l): round(float(st[l, 1]) / float(st[l, 0]), 4)
                                     for l in range(31) if st[l, 0] > 0}
    _line(md_rate, ms, args, "f64", config, roof, baseline, metric="md_time_per_wall_s",
          unit="md_time/s")
    return 0


def bench_langevin(args, w, tau: float = 1e-7) -> int:
    """The gradient-informed path move on the benchmark path (864 atoms x
    4096 steps): one step = one pamd_langevin_step (proposal, action and
    gradient of the proposal, fixed-order Metropolis-Hastings test, commit),
    replayed from a captured graph."""
    import torch
    import paper_1907_09529_amd as P
    P.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    print(f"[bench] input {w.name}: {w.n_steps} steps x {w.n_atoms} atoms ({args.input})",
          file=sys.stderr, flush=True)
    x, input_name = input_path(args, w, P, torch, dev)
    path = P.make_path(w.n_steps, w.n_atoms, 3, w.dt, w.D, w.gamma, "fp64")
    pot = P.make_potential("lj", eps=w.eps, sigma=w.sigma, rc=w.cutoff, box=w.box)
    g, y, gy = torch.empty_like(x), torch.empty_like(x), torch.empty_like(x)
    S = torch.empty(1, dtype=torch.float64, device=dev)
    P.pamd_action_grad(path, pot, x, g, action=S)
    counter = torch.zeros(1, dtype=torch.int64, device=dev)
    acc = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = P.workspace(P.pamd_langevin_workspace_size(path, pot))
    s = torch.cuda.Stream()
    torch.cuda.synchronize()
    gr = P.PamdGraph()
    with torch.cuda.stream(s):
        gr.begin(s)
        P.pamd_langevin_step(path, pot, 0x5EED1907, tau, counter, x, g, S, y, gy, acc, ws=ws,
                             stream=s)
        gr.end(s)
        for _ in range(args.warmup):
            gr.launch(s)
    s.synchronize()
    ev = HipEvents()
    t0 = time.perf_counter()
    HipEvents.hip.hipEventRecord(ev.a, ctypes.c_void_p(s.cuda_stream))
    for _ in range(args.steps):
        gr.launch(s)
    HipEvents.hip.hipEventRecord(ev.b, ctypes.c_void_p(s.cuda_stream))
    s.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    ev.close()
    # acceptance over as many further moves, read back one by one (untimed)
    n_acc = 0
    for _ in range(args.steps):
        gr.launch(s)
        s.synchronize()
        n_acc += int(acc.item())
    gr.close()
    lib = P.load()
    kev = [HipEvents() for _ in range(3)]
    for e in kev:
        lib.pamd_profile_events(e.a, e.b)
        P.pamd_action_grad(path, pot, y, gy)
    k_ms = float(np.mean([e.elapsed_ms() for e in kev]))
    for e in kev:
        e.close()
    idx = torch.from_numpy(np.linspace(0, w.n_steps, 8).astype(int)).to(dev)
    ppa = pairs_per_atom(y[idx].cpu().numpy(), w.box, w.cutoff)
    flop_unit = ppa * (FLOP_FORCE_PAIR + FLOP_HV_PAIR) + FLOP_SLICE_ATOM
    units = w.n_steps * w.n_atoms
    achieved = flop_unit * units / (k_ms * 1e-3)
    kname = ("lj_fused_exl_kernel" if P.pamd_launch_info(path, pot).exact_lists
             else "lj_fused_kernel")
    roof = {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_FP64_VALU / 1e12,
            "unit": "TFLOP/s", "frac": achieved / PEAK_FP64_VALU, "traffic": None,
            "kernel": f"{kname} (action + gradient of the proposal)", "kernel_ms": k_ms,
            "flop_per_slice_atom": flop_unit, "pairs_per_atom": ppa}
    config = {"workload": f"gradient-informed path move, LJ {w.n_atoms} atoms x {w.n_steps} steps, "
                          f"tau {tau:g}, graph-replayed moves; start path: {input_name}",
              "n_atoms": w.n_atoms, "n_steps": w.n_steps, "tau": tau,
              "acceptance": n_acc / args.steps, "parallelism": "single GPU"}
    _line(units / (ms * 1e-3), ms, args, "f64", config, roof, None,
          metric="langevin_move_slice_atoms_per_s", unit="slice_atoms/s")
    return 0


# The paper's harmonic-oscillator schedules (Sec. IV A, Table II): k = beta =
# D = gamma = 1, PAMD at dt = 0.4, Euler at dt_E = 0.025.
HO_SIMS = [
    {"name": "Simulation 1", "n_path": 16, "n_sample": 2, "n_shift": 2, "l_min": 3, "l_max": 3,
     "paper": {"chi": 16, "E_eq": 0.003, "E_dyn": 0.003}},
    {"name": "Simulation 2", "n_path": 256, "n_sample": 1, "n_shift": 8, "l_min": 4, "l_max": 5,
     "paper": {"chi": 128, "E_eq": 0.003, "E_dyn": 0.011}},
    {"name": "Simulation 3", "n_path": 4096, "n_sample": 1, "n_shift": 64, "l_min": 4, "l_max": 8,
     "paper": {"chi": 1024, "E_eq": 0.005, "E_dyn": 0.029}},
]


def _ho_errors(x: np.ndarray, dt: float) -> dict:
    """E_eq (Eq. 12) and E_dyn (Eqs. 13-15) of harmonic trajectories sampled
    every dt (x: time x independent trajectories).

    E_eq: L2 distance between the sampled and the exact (unit normal) position
    densities, both normalised; from a histogram (bins 0.25 wide on [-5, 5],
    noisy at these trajectory lengths) and from the normal density with the
    sampled variance.  E_dyn: |kappa - kappa_s| / k with kappa_s the slope of
    the log autocovariance fitted on t in [0, 4]."""
    grid = np.linspace(-12.0, 12.0, 24001)
    dg = grid[1] - grid[0]
    p = np.exp(-0.5 * grid ** 2) / math.sqrt(2 * math.pi)
    var = float(np.mean(x * x))
    q = np.exp(-0.5 * grid ** 2 / var) / math.sqrt(2 * math.pi * var)
    e_fit = math.sqrt(float(np.sum((p - q) ** 2)) * dg)
    edges = np.linspace(-5.0, 5.0, 41)
    h, _ = np.histogram(x, bins=edges, density=True)
    mid = 0.5 * (edges[1:] + edges[:-1])
    ph = np.exp(-0.5 * mid ** 2) / math.sqrt(2 * math.pi)
    e_hist = math.sqrt(float(np.sum((ph - h) ** 2)) * (edges[1] - edges[0]))
    x = x.reshape(x.shape[0], -1)
    lags = np.arange(0, int(round(4.0 / dt)) + 1)
    c = np.array([np.mean(x[:x.shape[0] - k] * x[k:]) for k in lags])
    slope = np.polyfit(lags * dt, np.log(c), 1)[0]
    return {"E_eq_fit": e_fit, "E_eq_hist": e_hist, "E_dyn": abs(1.0 + slope), "variance": var}


def bench_ho_table2(args, t_total: float = 100000.0, euler_dofs: int = 64) -> int:
    """The three harmonic schedules of Table II run by the integration loop on
    the GPU (one degree of freedom, x_0 drawn from the dt = 0.4 Euler chain's
    stationary law), each over t_total time units, beside the GPU Euler
    integrator at dt_E = 0.025 (euler_dofs independent oscillators over
    t_total / 4 each); reports E_eq and E_dyn next to the paper's.  The JSON value is Simulation 1's
    simulated time per wall-clock second."""
    import torch
    import paper_1907_09529_amd as P
    P.load()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    pot = P.make_potential("harmonic", k=1.0)
    dt, dt_e = 0.4, 0.025
    rng = np.random.default_rng(W.SEED_BASE + 40)
    results, sim1_rate, sim1_ms = [], None, None
    for sim in HO_SIMS:
        n_path, n_shift = sim["n_path"], sim["n_shift"]
        n_events = int(round(t_total / (dt * n_shift)))
        X = np.zeros((n_path + 1, 1, 1))
        X[0] = rng.standard_normal() * math.sqrt(1.25)
        for n in range(n_path):
            X[n + 1] = 0.6 * X[n] + math.sqrt(0.8) * rng.standard_normal()
        path = P.make_path(n_path, 1, 1, dt, 1.0, 1.0)
        x = torch.from_numpy(X).to(dev)
        ex = torch.empty(n_path, dtype=torch.float64, device=dev)
        P.pamd_excess_action(path, pot, x, ex)
        counters = torch.zeros(2, dtype=torch.int64, device=dev)
        traj = torch.empty((n_events * n_shift, 1, 1), dtype=torch.float64, device=dev)
        ws = P.workspace(P.pamd_run_workspace_size(path, pot, n_shift))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P.pamd_run(path, pot, 0x5EED + n_path, sim["l_min"], sim["l_max"], sim["n_sample"],
                   n_shift, n_events, counters, x, torch.empty_like(x), torch.empty_like(x), ex,
                   torch.empty_like(ex), traj, ws=ws)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        err = _ho_errors(traj.cpu().numpy().ravel()[n_path:], dt)
        rate = n_events * n_shift * dt / wall
        if sim1_rate is None:
            sim1_rate, sim1_ms = rate, wall * 1e3 / n_events
        results.append({"name": sim["name"], "events": n_events, "event_ms": wall * 1e3 / n_events,
                        "md_time_per_s": rate, **{k: round(v, 4) for k, v in err.items()},
                        "paper": sim["paper"]})
    # Euler at dt_E: independent oscillators from the stationary law
    n_e = int(round(t_total / 4 / dt_e))
    path_e = P.make_path(n_e, euler_dofs, 1, dt_e, 1.0, 1.0)
    xi = torch.randn((n_e, 1, euler_dofs), dtype=torch.float64, device=dev,
                     generator=torch.Generator(device=dev).manual_seed(W.SEED_BASE + 41))
    x0 = torch.from_numpy(rng.standard_normal((1, euler_dofs))).to(dev)
    out = torch.empty((n_e + 1, 1, euler_dofs), dtype=torch.float64, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    P.pamd_em_integrate(path_e, pot, x0, xi, out)
    torch.cuda.synchronize()
    wall_e = time.perf_counter() - t0
    err_e = _ho_errors(out.cpu().numpy()[1:, 0, :], dt_e)
    euler = {"dt_E": dt_e, "steps": n_e, "oscillators": euler_dofs,
             "md_time_per_s": n_e * dt_e / wall_e,
             **{k: round(v, 4) for k, v in err_e.items()},
             "paper": {"E_eq": 0.003, "E_dyn": 0.010}}
    roof = {"bound": "hbm", "achieved": None, "peak": PEAK_HBM / 1e9, "unit": "GB/s",
            "frac": None, "traffic": None,
            "note": "launch-bound: one degree of freedom; the loop's kernels move bytes, not "
                    "bandwidth"}
    config = {"workload": f"harmonic oscillator integration, Table II schedules at dt {dt}, "
                          f"{t_total:g} time units each, Euler at dt_E {dt_e}",
              "simulations": results, "euler": euler,
              "exact_euler_law_dt0.4": {"variance": 1.25, "E_eq": 0.0498, "E_dyn": 0.2771},
              "parallelism": "single GPU"}
    _line(sim1_rate, sim1_ms, args, "f64", config, roof, None, metric="md_time_per_wall_s",
          unit="md_time/s")
    return 0


if __name__ == "__main__":
    sys.exit(main())
