"""Energy, force and Hessian-vector product of one configuration (one time slice).

A configuration is an array of shape (n_dim, n_atoms) (coordinates by
component).  Forces are F = -dV/dx, the quantity -V'(x) of Eqs. 1-3.

Pair interactions (Sec. IV B, Eq. 16) under periodic boundaries in a cubic
box use the minimum-image displacement d_ij = x_i - x_j - L rint((x_i - x_j)/L)
(round half to even) and include a pair when r_ij^2 <= r_c^2.  With r = |d|:

    F_i   = sum_j  -U'(r)/r * d_ij
    (H v)_i = sum_j  K_ij (v_i - v_j),
    K_ij  = (U'(r)/r) I + (U''(r) - U'(r)/r) d_ij d_ij^T / r^2,

the second being the product of the Hessian of E = sum_{i<j} U(r_ij) with a
vector v, written out without forming H (H_ii = sum_j K_ij, H_ij = -K_ij).
"""
from __future__ import annotations

import itertools

import numpy as np

from .potentials import Harmonic, LennardJones


def minimum_image(d, box: float):
    """Nearest periodic image of a displacement in a cubic box of edge ``box``."""
    if box <= 0:
        return d
    shift = np.rint(np.real(d) / box)
    return d - box * shift


def pairs_brute(x, pot: LennardJones):
    """All pairs i < j within the cutoff: O(N^2) reference enumeration.

    Returns (i, j, d) with d of shape (3, P), d[:, p] = min-image(x_i - x_j).
    """
    n = x.shape[1]
    i, j = np.triu_indices(n, k=1)
    d = minimum_image(x[:, i] - x[:, j], pot.box)
    r2 = np.real(np.sum(d * d, axis=0))
    keep = r2 <= pot.rc * pot.rc
    return i[keep], j[keep], d[:, keep]


def pairs_cells(x, pot: LennardJones):
    """The same pair set found with a cell list (cells of edge >= r_c).

    The box is split into n_c = floor(L / r_c) cells per axis; a pair within
    the cutoff always lies in the same or adjacent cells.  Requires n_c >= 3
    so that the 27 neighbouring cells are distinct.
    """
    box = pot.box
    nc = int(np.floor(box / pot.rc))
    if nc < 3:
        raise ValueError("cell list needs at least 3 cells per axis")
    xr = np.real(x)
    wrapped = xr - box * np.floor(xr / box)
    cell = np.minimum((wrapped / box * nc).astype(np.int64), nc - 1)
    members = {}
    for a in range(x.shape[1]):
        members.setdefault(tuple(cell[:, a]), []).append(a)
    out_i, out_j = [], []
    offsets = list(itertools.product((-1, 0, 1), repeat=3))
    for a in range(x.shape[1]):
        ca = cell[:, a]
        cand = []
        for off in offsets:
            key = tuple((ca + np.array(off)) % nc)
            cand.extend(members.get(key, []))
        cand = np.array(sorted(b for b in cand if b > a), dtype=np.int64)
        if cand.size == 0:
            continue
        d = minimum_image(xr[:, [a]] - xr[:, cand], box)
        r2 = np.sum(d * d, axis=0)
        sel = cand[r2 <= pot.rc * pot.rc]
        out_i.extend([a] * sel.size)
        out_j.extend(sel.tolist())
    i = np.array(out_i, dtype=np.int64)
    j = np.array(out_j, dtype=np.int64)
    d = minimum_image(x[:, i] - x[:, j], box)
    return i, j, d


def _pairs(x, pot, method):
    if method == "brute":
        return pairs_brute(x, pot)
    if method == "cells":
        return pairs_cells(x, pot)
    raise ValueError(method)


def energy(x, pot, method: str = "brute"):
    """Potential energy of one configuration."""
    if isinstance(pot, Harmonic):
        return 0.5 * pot.k * np.sum(x * x)
    i, j, d = _pairs(x, pot, method)
    r = np.sqrt(np.sum(d * d, axis=0))
    return np.sum(pot.U(r))


def forces(x, pot, method: str = "brute"):
    """F = -grad V for one configuration, shape (n_dim, n_atoms)."""
    if isinstance(pot, Harmonic):
        return -pot.k * x
    i, j, d = _pairs(x, pot, method)
    r = np.sqrt(np.sum(d * d, axis=0))
    fpair = -pot.dU(r) / r * d                  # force on i from j; j receives the opposite
    f = np.zeros(x.shape, dtype=np.result_type(x, fpair))
    for c in range(x.shape[0]):
        np.add.at(f[c], i, fpair[c])
        np.add.at(f[c], j, -fpair[c])
    return f


def hessian_vec(x, v, pot, method: str = "brute"):
    """H(x) v for the potential energy Hessian H, shape (n_dim, n_atoms)."""
    if isinstance(pot, Harmonic):
        return pot.k * v
    i, j, d = _pairs(x, pot, method)
    r = np.sqrt(np.sum(d * d, axis=0))
    a = pot.dU(r) / r
    b = (pot.d2U(r) - a) / (r * r)
    w = v[:, i] - v[:, j]
    dw = np.sum(d * w, axis=0)
    kw = a * w + b * dw * d                     # K_ij (v_i - v_j); pair j gets K_ji (v_j - v_i) = -kw
    q = np.zeros(x.shape, dtype=np.result_type(x, v, kw))
    for c in range(x.shape[0]):
        np.add.at(q[c], i, kw[c])
        np.add.at(q[c], j, -kw[c])
    return q


def neighbour_counts(x, pot, method: str = "brute"):
    """Number of partners within the cutoff for every atom."""
    i, j, _ = _pairs(x, pot, method)
    cnt = np.zeros(x.shape[1], dtype=np.int64)
    np.add.at(cnt, i, 1)
    np.add.at(cnt, j, 1)
    return cnt
