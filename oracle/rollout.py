"""Float64 stream-kick-stream subcycles and their adjoint.

Test infrastructure only.  The short-range part of the split-operator time
step (Habib et al. 2012, Sec. II, Eq. 6): within a long-range step the
short-range map M_sr(t/n_c) is applied n_c times, each a symmetric
composition of a half stream, a kick with the short-range force and a
second half stream.  Newtonian coefficients are used (x += h v, v += h a),
with the step h given by the caller; the paper does not print the
cosmological factors.
"""
from __future__ import annotations

import numpy as np

from . import clib


def _wrap(x, box):
    if box > 0:
        x = x - box * np.floor(x / box)
        x[x >= box] = 0.0
    return x


def sks(x0, v0, mass, box, r_cut, eps, poly, h, n_c, force_fn=None):
    """Run n_c subcycles; returns (x, v, checkpoints) where checkpoints[k] is
    the position at which the k-th force was evaluated."""
    if force_fn is None:
        def force_fn(x):
            return clib.force(x, mass, box, r_cut, eps, poly)[0]
    x = np.array(x0, dtype=np.float64, copy=True)
    v = np.array(v0, dtype=np.float64, copy=True)
    cps = []
    for _ in range(n_c):
        x = _wrap(x + 0.5 * h * v, box)
        cps.append(x.copy())
        v = v + h * force_fn(x)
        x = _wrap(x + 0.5 * h * v, box)
    return x, v, cps


def sks_vjp(cps, mass, box, r_cut, eps, poly, h, gx, gv, vjp_fn=None):
    """Reverse pass through the subcycles given the cotangents (gx, gv) of the
    final state; returns the cotangents of the initial (x, v).  Each subcycle
    (x1 = x + h/2 v; v' = v + h a(x1); x' = x1 + h/2 v') is reversed by
    gv += h/2 gx; gx += J^T (h gv) at x1; gv += h/2 gx."""
    if vjp_fn is None:
        def vjp_fn(x, g):
            return clib.force_vjp(x, mass, box, r_cut, eps, poly, g)[0]
    gx = np.array(gx, dtype=np.float64, copy=True)
    gv = np.array(gv, dtype=np.float64, copy=True)
    for x1 in reversed(cps):
        gv = gv + 0.5 * h * gx
        gx = gx + vjp_fn(x1, h * gv)
        gv = gv + 0.5 * h * gx
    return gx, gv


def full_step(x0, v0, mass, box, ng, r_cut, eps, poly, dt, n_c, sigma=0.8, n_s=3):
    """One full step of the split-operator scheme (Sec. II, Eq. 6):
    M_full(t) = M_lr(t/2) (M_sr(t/n_c))^n_c M_lr(t/2).  M_lr is a kick with
    the long-range PM acceleration (positions frozen); M_sr is the
    stream-kick-stream subcycle with the short-range force.  Newtonian
    coefficients (v += t a, x += t v), float64.  Returns (x, v)."""
    from . import pm
    x = np.array(x0, dtype=np.float64, copy=True)
    v = np.array(v0, dtype=np.float64, copy=True)
    v = v + 0.5 * dt * pm.accel(x, mass, box, ng, sigma, n_s)
    x, v, _ = sks(x, v, mass, box, r_cut, eps, poly, dt / n_c, n_c)
    v = v + 0.5 * dt * pm.accel(x, mass, box, ng, sigma, n_s)
    return x, v
