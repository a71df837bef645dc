"""Plain NumPy reference of the chaining-mesh binning.

Test infrastructure only.  The chaining mesh is the cell list of the
particle-particle part of a P^3M code (Habib et al. 2012, Sec. II): N =
floor(|box| / r_cut) cells per axis of side L = |box| / N >= r_cut, so every
pair closer than r_cut lies in adjacent cells.  Periodic boxes wrap
coordinates into [0, box) (a coordinate equal to box after the wrap maps to
0); open domains [0, |box|) clamp outside particles into the edge cells.
Particles are ordered by cell index (cx * N + cy) * N + cz, then inside a
cell by the Morton code of their sub-cell (the cell split into S^3 equal
sub-cells, S = 4 while the cell index and the code fit in 31 bits, else 2 or
1), then by input index; they are stored as float32 coordinates relative to
their cell's lower corner plus the mass.
"""
from __future__ import annotations

import math

import numpy as np


def grid(box: float, r_cut: float):
    b = abs(float(box))
    rc = float(np.float32(r_cut))
    N = max(1, int(math.floor(b / rc)))
    while N > 1 and b / N < rc:
        N -= 1
    return N, b / N


def _bits(ncell: int) -> int:
    b = 0
    while (1 << b) < ncell:
        b += 1
    return b


def sub_levels(N: int) -> int:
    cb = _bits(N ** 3)
    return 2 if cb + 6 <= 31 else (1 if cb + 3 <= 31 else 0)


def chaining_mesh(pos, mass, box: float, r_cut: float):
    """Returns (keys (n,), perm (n,), cell_start (N^3+1,), rec (n,4) float32)."""
    pos = np.asarray(pos, dtype=np.float64)
    N, L = grid(box, r_cut)
    b = abs(float(box))
    v = pos.copy()
    if box > 0:
        v = pos - b * np.floor(pos / b)
        v = np.where(v >= b, v - b, v)
    with np.errstate(invalid="ignore"):
        k = np.floor(v / L)
    c = np.where(np.isnan(k), 0, np.clip(np.nan_to_num(k, nan=0.0), 0, N - 1)).astype(np.int64)
    keys = (c[:, 0] * N + c[:, 1]) * N + c[:, 2]
    lev = sub_levels(N)
    code = np.zeros(keys.shape, dtype=np.int64)
    if lev:
        S = 1 << lev
        with np.errstate(invalid="ignore"):
            t = np.floor((v - c * L) / L * S)
        sub = np.where(np.isnan(t), 0, np.clip(np.nan_to_num(t, nan=0.0), 0, S - 1)).astype(np.int64)
        for b in range(lev):
            code |= (((sub[:, 0] >> b) & 1) << (3 * b + 2)) | (((sub[:, 1] >> b) & 1) << (3 * b + 1)) \
                | (((sub[:, 2] >> b) & 1) << (3 * b))
    perm = np.lexsort((np.arange(keys.size), code, keys))
    sk = keys[perm]
    cell_start = np.searchsorted(sk, np.arange(N ** 3 + 1), side="left")
    rel = (v[perm] - c[perm] * L).astype(np.float32)
    rec = np.concatenate([rel, np.asarray(mass, np.float32)[perm, None]], axis=1)
    return keys, perm, cell_start, rec
