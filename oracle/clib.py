"""ctypes wrapper around the C oracle (``sr_oracle.c``).

Test infrastructure only (see the package docstring)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sr_oracle.c")
_LIB = os.path.join(_HERE, "libsr_oracle.so")
_lib = None


def library_path() -> str:
    return _LIB


def build(force_rebuild: bool = True) -> str:
    """Compile the oracle with gcc (float64, OpenMP, no fast-math)."""
    if force_rebuild or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared",
                               "-fno-fast-math", "-ffp-contract=off",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force_rebuild=False)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I64 = ctypes.c_int64
        lib.oracle_force.argtypes = [P, P, I64, ctypes.c_double, ctypes.c_float,
                                     ctypes.c_float, P, P, I64, P, P, P]
        lib.oracle_force.restype = ctypes.c_int
        lib.oracle_force_vjp.argtypes = [P, P, I64, ctypes.c_double,
                                         ctypes.c_float, ctypes.c_float, P, P,
                                         P, I64, P, P, P, ctypes.c_double, P]
        lib.oracle_force_vjp.restype = ctypes.c_int
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def num_threads() -> int:
    return int(_load().oracle_num_threads())


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _prep(pos, mass, poly, targets):
    pos = np.ascontiguousarray(pos, dtype=np.float64)
    mass = np.ascontiguousarray(mass, dtype=np.float32)
    poly = np.ascontiguousarray(poly, dtype=np.float32)
    assert pos.ndim == 2 and pos.shape[1] == 3 and mass.shape == (pos.shape[0],)
    assert poly.shape == (6,)
    if targets is not None:
        targets = np.ascontiguousarray(targets, dtype=np.int64)
        assert targets.ndim == 1
        if targets.size and (targets.min() < 0 or targets.max() >= pos.shape[0]):
            raise IndexError("target index out of range")
    return pos, mass, poly, targets


def force(pos, mass, box, r_cut, eps, poly, targets=None):
    """Accelerations (nt,3), summed Newtonian magnitudes (nt,) and in-cut-off
    neighbour counts (nt,) for the targets (all particles by default)."""
    pos, mass, poly, targets = _prep(pos, mass, poly, targets)
    nt = pos.shape[0] if targets is None else targets.size
    acc = np.zeros((nt, 3))
    an = np.zeros(nt)
    cnt = np.zeros(nt, dtype=np.int64)
    rc = _load().oracle_force(_ptr(pos), _ptr(mass), pos.shape[0], float(box),
                              float(r_cut), float(eps), _ptr(poly),
                              _ptr(targets), nt, _ptr(acc), _ptr(an), _ptr(cnt))
    if rc != 0:
        raise MemoryError("oracle_force failed")
    return acc, an, cnt


def force_vjp(pos, mass, box, r_cut, eps, poly, g, targets=None, cut_band=None,
              pair_floor=False):
    """dL/dx (nt,3) for L = sum g . a, and the error floor B (nt,): the summed
    magnitudes of the Newtonian and grid-polynomial parts of f and f' times
    |w| over the particle's pairs.

    With ``cut_band`` also returns the summed pair-term magnitude of pairs
    within a relative band |s - r_cut^2| <= cut_band r_cut^2 (nt,): the
    result is discontinuous there, since f' jumps at the cut-off.

    With ``pair_floor`` also returns (last) the tighter floor
    sum_j (|f| + 2 |f'| s) |w_kj| over the in-cut-off pairs (nt,)."""
    pos, mass, poly, targets = _prep(pos, mass, poly, targets)
    g = np.ascontiguousarray(g, dtype=np.float64)
    assert g.shape == pos.shape
    nt = pos.shape[0] if targets is None else targets.size
    out = np.zeros((nt, 3))
    bn = np.zeros(nt)
    pm = np.zeros(nt)
    amb = np.zeros(nt)
    rc = _load().oracle_force_vjp(_ptr(pos), _ptr(mass), pos.shape[0],
                                  float(box), float(r_cut), float(eps),
                                  _ptr(poly), _ptr(g), _ptr(targets), nt,
                                  _ptr(out), _ptr(bn), _ptr(pm),
                                  float(cut_band or 0.0), _ptr(amb))
    if rc != 0:
        raise MemoryError("oracle_force_vjp failed")
    res = [out, bn]
    if cut_band is not None:
        res.append(amb)
    if pair_floor:
        res.append(pm)
    return tuple(res)


def rel_err_floored(approx, exact, floor_mag, floor_frac=0.1):
    """Per-particle error |a - a*| / max(|a*|, floor_frac * A), where A is the
    summed pair magnitude of that particle.  Plain relative error whenever the
    sum is not dominated by cancelling pair terms."""
    approx = np.asarray(approx, dtype=np.float64)
    exact = np.asarray(exact, dtype=np.float64)
    num = np.linalg.norm(approx - exact, axis=1)
    den = np.maximum(np.linalg.norm(exact, axis=1), floor_frac * np.asarray(floor_mag))
    out = np.zeros_like(num)
    nz = den > 0
    out[nz] = num[nz] / den[nz]
    out[~nz] = np.where(num[~nz] > 0, np.inf, 0.0)
    return out
