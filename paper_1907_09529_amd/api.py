"""Python binding of libpamd with the C entry points' names.

Every function marshals torch tensors (device pointers, the current HIP
stream) into the C ABI and raises ``PamdError`` on failure; all arithmetic
runs in the library's HIP kernels.  Paths are float64 tensors of shape
(n_steps + 1, n_dim, n_atoms), contiguous, on the current HIP device.
"""
from __future__ import annotations

import ctypes
import dataclasses
from typing import Optional, Sequence

import torch

from . import _lib
from ._lib import (PamdPath, PamdPotential, PamdTuning, PamdLaunch, PamdError, PAMD_HARMONIC, PAMD_LJ,
                   PAMD_FP64, PAMD_FP32_FORCE, PAMD_ALGO_AUTO, PAMD_ALGO_FUSED,
                   PAMD_ALGO_PLAIN)

__all__ = [
    "PamdPath", "PamdPotential", "PamdTuning", "PamdLaunch", "PamdError", "make_path",
    "make_potential", "make_tuning", "pamd_workspace_size", "pamd_launch_info", "pamd_action", "pamd_action_grad",
    "pamd_action_grad_noalloc",
    "pamd_excess_action", "pamd_log_norm", "pamd_mh_workspace_size", "pamd_mh_step",
    "pamd_em_workspace_size", "pamd_em_integrate", "pamd_shift", "pamd_run_workspace_size",
    "pamd_run", "pamd_langevin_workspace_size", "pamd_langevin_step", "pamd_autotune",
    "pamd_batch_workspace_size", "pamd_batch_action_grad", "PamdBatch", "PamdGraph", "workspace",
]


# ---------------------------------------------------------------------------
# descriptors
# ---------------------------------------------------------------------------
def make_path(n_steps: int, n_atoms: int, n_dim: int, dt: float, D: float, gamma: float,
              precision: str = "fp64") -> PamdPath:
    prec = {"fp64": PAMD_FP64, "fp32_force": PAMD_FP32_FORCE}[precision]
    return PamdPath(int(n_steps), int(n_atoms), int(n_dim), float(dt), float(D), float(gamma),
                    prec, 0)


def make_potential(kind: str, k: float = 1.0, eps: float = 1.0, sigma: float = 1.0,
                   rc: float = 2.5, box: float = 0.0) -> PamdPotential:
    if kind == "harmonic":
        return PamdPotential(PAMD_HARMONIC, 0, float(k), 0.0, 0.0, 0.0, 0.0)
    if kind == "lj":
        return PamdPotential(PAMD_LJ, 0, 0.0, float(eps), float(sigma), float(rc), float(box))
    raise ValueError(kind)


def make_tuning(algo: str = "auto", block: int = 0, tile: int = 0, max_neighbours: int = 0,
                skin: float = 0.0, neighbour_list: str = "auto", slot_arrays: int = 0) -> PamdTuning:
    a = {"auto": PAMD_ALGO_AUTO, "fused": PAMD_ALGO_FUSED, "plain": PAMD_ALGO_PLAIN}[algo]
    nl = {"auto": 0, "full": 1, "half": 2}[neighbour_list]
    return PamdTuning(a, int(block), int(tile), int(max_neighbours), float(skin), nl,
                      int(slot_arrays))


def _ref(s):
    return ctypes.byref(s) if s is not None else None


class _Dev:
    """A tensor argument whose size, type and layout have been checked; its
    device is checked in _call, after every argument's size (so that a
    wrongly sized buffer is reported as such wherever it stands)."""
    __slots__ = ("t", "name")

    def __init__(self, t, name):
        self.t, self.name = t, name


def _ptr(t: Optional[torch.Tensor], dtype=torch.float64, name: str = "tensor",
         numel: Optional[int] = None):
    """Checks what the C ABI cannot: element type, contiguity and size (the
    library reads or writes exactly ``numel`` elements, so a smaller tensor is
    refused); _call then checks the device (the current HIP device)."""
    if t is None:
        return None
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, {numel} needed")
    return _Dev(t, name)


def _call(fn: str, *args):
    out = []
    for a in args:
        if isinstance(a, _Dev):
            if not a.t.is_cuda:
                raise ValueError(f"{a.name} must be a device tensor")
            if a.t.device.index != torch.cuda.current_device():
                raise ValueError(f"{a.name} is on {a.t.device}, not the current device "
                                 f"cuda:{torch.cuda.current_device()}")
            a = ctypes.c_void_p(a.t.data_ptr())
        elif isinstance(a, _Stream):
            a = a.handle()
        out.append(a)
    return _lib.call(fn, *out)


def _path_elems(path: PamdPath) -> int:
    """Elements of a path (or gradient) buffer: (N + 1) n_dim n_atoms."""
    return (int(path.n_steps) + 1) * int(path.n_dim) * int(path.n_atoms)


def _dof(path: PamdPath) -> int:
    return int(path.n_dim) * int(path.n_atoms)


class _Stream:
    """The HIP stream argument, resolved in _call after the tensor checks
    (None means torch's current stream)."""
    __slots__ = ("s",)

    def __init__(self, s):
        self.s = s

    def handle(self) -> ctypes.c_void_p:
        s = torch.cuda.current_stream() if self.s is None else self.s
        return ctypes.c_void_p(s.cuda_stream if hasattr(s, "cuda_stream") else int(s))


def _stream(stream) -> _Stream:
    return _Stream(stream)


def workspace(nbytes: int, device=None) -> torch.Tensor:
    """Device buffer for a workspace (allocated by torch, never by the library)."""
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8,
                       device=device if device is not None else torch.cuda.current_device())


# ---------------------------------------------------------------------------
# single paths
# ---------------------------------------------------------------------------
def pamd_workspace_size(path: PamdPath, pot: PamdPotential,
                        tuning: Optional[PamdTuning] = None) -> int:
    n = ctypes.c_size_t(0)
    _call("pamd_workspace_size", ctypes.byref(path), ctypes.byref(pot), _ref(tuning),
              ctypes.byref(n))
    return int(n.value)


def pamd_launch_info(path: PamdPath, pot: PamdPotential,
                     tuning: Optional[PamdTuning] = None) -> PamdLaunch:
    out = PamdLaunch()
    _call("pamd_launch_info", ctypes.byref(path), ctypes.byref(pot), _ref(tuning),
          ctypes.byref(out))
    return out


def _ws(path, pot, tuning, ws, sizer=pamd_workspace_size):
    need = sizer(path, pot, tuning)
    if ws is None:
        ws = workspace(need)
    return ws, need


def pamd_action(path, pot, x, action, per_step=None, ws=None, tuning=None, stream=None):
    args = (_ptr(x, name="x", numel=_path_elems(path)), _ptr(action, name="action", numel=1),
            _ptr(per_step, name="per_step", numel=path.n_steps))
    ws, _ = _ws(path, pot, tuning, ws)
    _call("pamd_action", ctypes.byref(path), ctypes.byref(pot), _ref(tuning), *args,
              _ptr(ws, None, "ws"), ctypes.c_size_t(ws.numel()), _stream(stream))


def pamd_action_grad(path, pot, x, grad, action=None, per_step=None, step_weights=None,
                     ws=None, tuning=None, stream=None):
    args = (_ptr(x, name="x", numel=_path_elems(path)),
            _ptr(step_weights, name="step_weights", numel=path.n_steps),
            _ptr(action, name="action", numel=1),
            _ptr(per_step, name="per_step", numel=path.n_steps),
            _ptr(grad, name="grad", numel=_path_elems(path)))
    ws, _ = _ws(path, pot, tuning, ws)
    _call("pamd_action_grad", ctypes.byref(path), ctypes.byref(pot), _ref(tuning), *args,
              _ptr(ws, None, "ws"), ctypes.c_size_t(ws.numel()), _stream(stream))


def pamd_action_grad_noalloc(path, pot, x, grad, action=None, per_step=None,
                             step_weights=None, tuning=None, stream=None):
    """pamd_action_grad without a workspace (the library's static scratch)."""
    _call("pamd_action_grad_noalloc", ctypes.byref(path), ctypes.byref(pot), _ref(tuning),
          _ptr(x, name="x", numel=_path_elems(path)),
          _ptr(step_weights, name="step_weights", numel=path.n_steps),
          _ptr(action, name="action", numel=1),
          _ptr(per_step, name="per_step", numel=path.n_steps),
          _ptr(grad, name="grad", numel=_path_elems(path)), _stream(stream))


def pamd_excess_action(path, pot, x, excess, per_step=None, ws=None, tuning=None, stream=None):
    args = (_ptr(x, name="x", numel=_path_elems(path)),
            _ptr(excess, name="excess", numel=path.n_steps),
            _ptr(per_step, name="per_step", numel=path.n_steps))
    ws, _ = _ws(path, pot, tuning, ws)
    _call("pamd_excess_action", ctypes.byref(path), ctypes.byref(pot), _ref(tuning), *args,
              _ptr(ws, None, "ws"), ctypes.c_size_t(ws.numel()), _stream(stream))


def pamd_log_norm(path: PamdPath) -> float:
    return float(_lib.load().pamd_log_norm(ctypes.byref(path)))


# ---------------------------------------------------------------------------
# path sampling
# ---------------------------------------------------------------------------
def pamd_mh_workspace_size(path, pot, tuning=None) -> int:
    n = ctypes.c_size_t(0)
    _call("pamd_mh_workspace_size", ctypes.byref(path), ctypes.byref(pot), _ref(tuning),
              ctypes.byref(n))
    return int(n.value)


def pamd_mh_step(path, pot, seed: int, l_min: int, l_max: int, sweep_counter: torch.Tensor,
                 x: torch.Tensor, excess: torch.Tensor, trial: torch.Tensor,
                 frag_delta=None, frag_accept=None, step_info=None, ws=None, tuning=None,
                 stream=None):
    ws, _ = _ws(path, pot, tuning, ws, pamd_mh_workspace_size)
    _call("pamd_mh_step", ctypes.byref(path), ctypes.byref(pot), _ref(tuning),
              ctypes.c_uint64(seed), ctypes.c_int32(l_min), ctypes.c_int32(l_max),
              _ptr(sweep_counter, torch.int64, "sweep_counter", 1),
              _ptr(x, name="x", numel=_path_elems(path)),
              _ptr(excess, name="excess", numel=path.n_steps),
              _ptr(trial, name="trial", numel=_path_elems(path)),
              _ptr(frag_delta, name="frag_delta", numel=path.n_steps + 2),
              _ptr(frag_accept, torch.int32, "frag_accept", path.n_steps + 2),
              _ptr(step_info, torch.int32, "step_info", 4), _ptr(ws, None, "ws"),
              ctypes.c_size_t(ws.numel()), _stream(stream))


# ---------------------------------------------------------------------------
# path-based integration: shifting events and the loop
# ---------------------------------------------------------------------------
def pamd_shift(path, seed: int, n_shift: int, event_counter: torch.Tensor, x_in, x_out,
               excess_in=None, excess_out=None, traj_out=None, stream=None):
    _call("pamd_shift", ctypes.byref(path), ctypes.c_uint64(seed), ctypes.c_int32(n_shift),
              _ptr(event_counter, torch.int64, "event_counter", 1),
              _ptr(x_in, name="x_in", numel=_path_elems(path)),
              _ptr(x_out, name="x_out", numel=_path_elems(path)),
              _ptr(excess_in, name="excess_in", numel=path.n_steps),
              _ptr(excess_out, name="excess_out", numel=path.n_steps),
              _ptr(traj_out, name="traj_out", numel=int(n_shift) * _dof(path)),
              _stream(stream))


def pamd_run_workspace_size(path, pot, n_shift: int, tuning=None) -> int:
    n = ctypes.c_size_t(0)
    _call("pamd_run_workspace_size", ctypes.byref(path), ctypes.byref(pot), _ref(tuning),
              ctypes.c_int32(n_shift), ctypes.byref(n))
    return int(n.value)


def pamd_run(path, pot, seed: int, l_min: int, l_max: int, n_sample: int, n_shift: int,
             n_events: int, counters: torch.Tensor, x, x_alt, trial, excess, excess_alt,
             traj_out=None, level_stats=None, ws=None, tuning=None, stream=None):
    if ws is None:
        ws = workspace(pamd_run_workspace_size(path, pot, n_shift, tuning))
    _call("pamd_run", ctypes.byref(path), ctypes.byref(pot), _ref(tuning),
              ctypes.c_uint64(seed), ctypes.c_int32(l_min), ctypes.c_int32(l_max),
              ctypes.c_int32(n_sample), ctypes.c_int32(n_shift), ctypes.c_int32(n_events),
              _ptr(counters, torch.int64, "counters", 2),
              _ptr(x, name="x", numel=_path_elems(path)),
              _ptr(x_alt, name="x_alt", numel=_path_elems(path)),
              _ptr(trial, name="trial", numel=_path_elems(path)),
              _ptr(excess, name="excess", numel=path.n_steps),
              _ptr(excess_alt, name="excess_alt", numel=path.n_steps),
              _ptr(traj_out, name="traj_out", numel=int(n_events) * int(n_shift) * _dof(path)),
              _ptr(level_stats, torch.int64, "level_stats", 62), _ptr(ws, None, "ws"),
              ctypes.c_size_t(ws.numel()), _stream(stream))


# ---------------------------------------------------------------------------
# gradient-informed (Langevin) path move
# ---------------------------------------------------------------------------
def pamd_langevin_workspace_size(path, pot, tuning=None) -> int:
    n = ctypes.c_size_t(0)
    _call("pamd_langevin_workspace_size", ctypes.byref(path), ctypes.byref(pot),
              _ref(tuning), ctypes.byref(n))
    return int(n.value)


def pamd_langevin_step(path, pot, seed: int, tau: float, move_counter: torch.Tensor, x, grad,
                       action, y, grad_y, accepted=None, log_alpha=None, ws=None, tuning=None,
                       stream=None):
    ws, _ = _ws(path, pot, tuning, ws, pamd_langevin_workspace_size)
    _call("pamd_langevin_step", ctypes.byref(path), ctypes.byref(pot), _ref(tuning),
              ctypes.c_uint64(seed), ctypes.c_double(tau),
              _ptr(move_counter, torch.int64, "move_counter", 1),
              _ptr(x, name="x", numel=_path_elems(path)),
              _ptr(grad, name="grad", numel=_path_elems(path)),
              _ptr(action, name="action", numel=1), _ptr(y, name="y", numel=_path_elems(path)),
              _ptr(grad_y, name="grad_y", numel=_path_elems(path)),
              _ptr(accepted, torch.int32, "accepted", 1),
              _ptr(log_alpha, name="log_alpha", numel=1), _ptr(ws, None, "ws"),
              ctypes.c_size_t(ws.numel()), _stream(stream))


# ---------------------------------------------------------------------------
# sequential Euler-Maruyama integration
# ---------------------------------------------------------------------------
def pamd_em_workspace_size(path, pot, tuning=None) -> int:
    n = ctypes.c_size_t(0)
    _call("pamd_em_workspace_size", ctypes.byref(path), ctypes.byref(pot), _ref(tuning),
              ctypes.byref(n))
    return int(n.value)


def pamd_em_integrate(path, pot, x0, noise, x_out, ws=None, tuning=None, stream=None):
    ws, _ = _ws(path, pot, tuning, ws, pamd_em_workspace_size)
    _call("pamd_em_integrate", ctypes.byref(path), ctypes.byref(pot), _ref(tuning),
              _ptr(x0, name="x0", numel=_dof(path)),
              _ptr(noise, name="noise", numel=int(path.n_steps) * _dof(path)),
              _ptr(x_out, name="x_out", numel=_path_elems(path)),
              _ptr(ws, None, "ws"), ctypes.c_size_t(ws.numel()), _stream(stream))


def pamd_autotune(path, pot, x, grad_scratch, ws, stream=None) -> PamdTuning:
    best = PamdTuning()
    _call("pamd_autotune", ctypes.byref(path), ctypes.byref(pot),
              _ptr(x, name="x", numel=_path_elems(path)),
              _ptr(grad_scratch, name="grad_scratch", numel=_path_elems(path)),
              _ptr(ws, None, "ws"),
              ctypes.c_size_t(ws.numel()), _stream(stream), ctypes.byref(best))
    return best


# ---------------------------------------------------------------------------
# batches and graphs
# ---------------------------------------------------------------------------
class PamdBatch:
    """A batch of independent paths packed into single device buffers."""

    def __init__(self, paths: Sequence[PamdPath], pots: Sequence[PamdPotential],
                 tuning: Optional[PamdTuning] = None):
        n = len(paths)
        self.n_paths = n
        self._paths = (PamdPath * n)(*paths)
        self._pots = (PamdPotential * n)(*pots)
        handle = ctypes.c_void_p()
        _call("pamd_batch_create", ctypes.c_int32(n), self._paths, self._pots, _ref(tuning),
                  ctypes.byref(handle))
        self._h = handle
        xo = (ctypes.c_int64 * (n + 1))()
        so = (ctypes.c_int64 * (n + 1))()
        nb = ctypes.c_size_t(0)
        _call("pamd_batch_layout", self._h, xo, so, ctypes.byref(nb))
        self.x_offsets = list(xo)
        self.step_offsets = list(so)
        self.ws_bytes = int(nb.value)
        self.ws = None

    def prepare(self, ws: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        if ws is None:
            ws = workspace(self.ws_bytes)
        _call("pamd_batch_prepare", self._h, _ptr(ws, None, "ws"), ctypes.c_size_t(ws.numel()),
                  _stream(stream))
        self.ws = ws
        return ws

    def autotune(self, x_all, grad_all=None, stream=None):
        """Times the member-tile policies on x_all, keeps the fastest and
        prepares the batch for it; returns (tile budget, skin in sigma)."""
        nb = ctypes.c_size_t(0)
        _call("pamd_batch_autotune_workspace_size", self._h, ctypes.byref(nb))
        ws = workspace(int(nb.value))
        budget, skin = ctypes.c_double(0.0), ctypes.c_double(0.0)
        nx = self.x_offsets[-1]
        _call("pamd_batch_autotune", self._h, _ptr(x_all, name="x_all", numel=nx),
              _ptr(grad_all, name="grad_all", numel=nx), _ptr(ws, None, "ws"),
              ctypes.c_size_t(ws.numel()), _stream(stream), ctypes.byref(budget),
              ctypes.byref(skin))
        n = ctypes.c_size_t(0)
        _call("pamd_batch_layout", self._h, None, None, ctypes.byref(n))
        self.ws_bytes = int(n.value)
        self.ws = ws
        return budget.value, skin.value

    def pamd_batch_run(self, x_all, actions, grad_all=None, per_step_all=None,
                       weights_all=None, stream=None):
        if self.ws is None:
            self.prepare(stream=stream)
        nx, ns = self.x_offsets[-1], self.step_offsets[-1]
        _call("pamd_batch_run", self._h, _ptr(x_all, name="x_all", numel=nx),
                  _ptr(weights_all, name="weights_all", numel=ns),
                  _ptr(actions, name="actions", numel=self.n_paths),
                  _ptr(per_step_all, name="per_step_all", numel=ns),
                  _ptr(grad_all, name="grad_all", numel=nx),
                  _ptr(self.ws, None, "ws"), ctypes.c_size_t(self.ws.numel()), _stream(stream))

    def view(self, packed: torch.Tensor, p: int) -> torch.Tensor:
        """Member p's path (or gradient) inside a packed buffer, shaped (N+1, n_dim, n_atoms)."""
        pp = self._paths[p]
        n = (pp.n_steps + 1) * pp.n_dim * pp.n_atoms
        o = self.x_offsets[p]
        return packed[o:o + n].view(pp.n_steps + 1, pp.n_dim, pp.n_atoms)

    def steps_view(self, packed: torch.Tensor, p: int) -> torch.Tensor:
        o = self.step_offsets[p]
        return packed[o:o + self._paths[p].n_steps]

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.load().pamd_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pamd_batch_workspace_size(paths: Sequence[PamdPath], pots: Sequence[PamdPotential]) -> int:
    n = len(paths)
    nb = ctypes.c_size_t(0)
    _call("pamd_batch_workspace_size", ctypes.c_int32(n), (PamdPath * n)(*paths),
          (PamdPotential * n)(*pots), ctypes.byref(nb))
    return int(nb.value)


def pamd_batch_action_grad(paths: Sequence[PamdPath], pots: Sequence[PamdPotential],
                           xs: Sequence[torch.Tensor], actions: torch.Tensor,
                           grads: Optional[Sequence[Optional[torch.Tensor]]] = None,
                           ws: Optional[torch.Tensor] = None, stream=None):
    """Actions (and gradients) of independent paths given as separate tensors."""
    n = len(paths)
    if len(pots) != n or len(xs) != n or (grads is not None and len(grads) != n):
        raise ValueError("paths, pots, xs (and grads) must have the same length")
    xa = [_ptr(x, name=f"xs[{p}]", numel=_path_elems(paths[p])) for p, x in enumerate(xs)]
    ga = None if grads is None else [
        _ptr(g, name=f"grads[{p}]", numel=_path_elems(paths[p])) for p, g in enumerate(grads)]
    act = _ptr(actions, name="actions", numel=n)
    if ws is None:
        ws = workspace(pamd_batch_workspace_size(paths, pots))
    # device checks (as in _call) for the pointer arrays
    def addr(a):
        if a is None:
            return None
        if not a.t.is_cuda or a.t.device.index != torch.cuda.current_device():
            raise ValueError(f"{a.name} must be a tensor on the current device")
        return a.t.data_ptr()
    x_arr = (ctypes.c_void_p * n)(*[addr(a) for a in xa])
    g_arr = None if ga is None else (ctypes.c_void_p * n)(*[addr(a) for a in ga])
    _call("pamd_batch_action_grad", ctypes.c_int32(n), (PamdPath * n)(*paths),
          (PamdPotential * n)(*pots), x_arr, act, g_arr, _ptr(ws, None, "ws"),
          ctypes.c_size_t(ws.numel()), _stream(stream))


class PamdGraph:
    """Captures the pamd_* calls enqueued on a stream between begin() and end()."""

    def __init__(self):
        self._h = ctypes.c_void_p()

    def begin(self, stream):
        _call("pamd_graph_begin", _stream(stream))

    def end(self, stream):
        _call("pamd_graph_end", _stream(stream), ctypes.byref(self._h))

    def launch(self, stream):
        _call("pamd_graph_launch", self._h, _stream(stream))

    def close(self):
        if self._h.value:
            _lib.load().pamd_graph_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
