"""All-pairs NumPy float64 oracle for tiny inputs.

Test infrastructure only.  Independent of the C cell-list oracle: no cells,
every (i, j) pair is formed explicitly, the polynomial goes through
``numpy.polynomial.polynomial.polyval``.  It computes the same definition
(Habib et al. 2012, Sec. III, Eq. 7 with the short-range condition applied
per pair): a_i = sum_{j != i, s < r_cut^2} m_j f(s_ij) d_ij,
f(s) = (s + eps)^(-3/2) - poly5(s), d_ij = x_j - x_i (minimum image when
periodic).
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial import polynomial as P


def _pairs(pos, box, idx):
    d = pos[None, :, :] - pos[idx][:, None, :]
    if box > 0:
        d -= box * np.rint(d / box)
    return d


def force(pos, mass, box, r_cut, eps, poly, targets=None, chunk=256):
    pos = np.asarray(pos, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float32).astype(np.float64)
    c = np.asarray(poly, dtype=np.float32).astype(np.float64)
    rc2 = float(np.float32(r_cut)) ** 2
    e = float(np.float32(eps))
    n = pos.shape[0]
    idx_all = np.arange(n) if targets is None else np.asarray(targets)
    out = np.zeros((idx_all.size, 3))
    for s0 in range(0, idx_all.size, chunk):
        idx = idx_all[s0:s0 + chunk]
        d = _pairs(pos, box, idx)
        s = np.einsum("ijk,ijk->ij", d, d)
        keep = (s < rc2) & (np.arange(n)[None, :] != idx[:, None])
        f = np.where(keep, (s + e) ** -1.5 - P.polyval(s, c), 0.0)
        out[s0:s0 + idx.size] = np.einsum("ij,ijk->ik", f * mass[None, :], d)
    return out


def force_vjp(pos, mass, box, r_cut, eps, poly, g, targets=None, chunk=256):
    """dL/dx_k for L = sum_i g_i . a_i, by the chain rule over every pair:
    dL/dx_k = sum_j [f w + 2 f' (d.w) d], w = m_k g_j - m_j g_k."""
    pos = np.asarray(pos, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float32).astype(np.float64)
    g = np.asarray(g, dtype=np.float64)
    c = np.asarray(poly, dtype=np.float32).astype(np.float64)
    dc = P.polyder(c)
    rc2 = float(np.float32(r_cut)) ** 2
    e = float(np.float32(eps))
    n = pos.shape[0]
    idx_all = np.arange(n) if targets is None else np.asarray(targets)
    out = np.zeros((idx_all.size, 3))
    for s0 in range(0, idx_all.size, chunk):
        idx = idx_all[s0:s0 + chunk]
        d = _pairs(pos, box, idx)
        s = np.einsum("ijk,ijk->ij", d, d)
        keep = (s < rc2) & (np.arange(n)[None, :] != idx[:, None])
        f = np.where(keep, (s + e) ** -1.5 - P.polyval(s, c), 0.0)
        fp = np.where(keep, -1.5 * (s + e) ** -2.5 - P.polyval(s, dc), 0.0)
        w = mass[idx][:, None, None] * g[None, :, :] - mass[None, :, None] * g[idx][:, None, :]
        dw = np.einsum("ijk,ijk->ij", d, w)
        out[s0:s0 + idx.size] = (np.einsum("ij,ijk->ik", f, w)
                                 + np.einsum("ij,ijk->ik", 2.0 * fp * dw, d))
    return out


def potential(pos, mass, box, r_cut, eps, poly):
    """Total pair potential energy whose negative gradient, divided by the
    particle's mass, is the acceleration: psi(s) = -(s+eps)^(-1/2)
    - sum_k c_k s^(k+1) / (2(k+1)) + const, with const chosen so that
    psi(r_cut^2) = 0 (only pairs inside the cut-off contribute; the constant
    makes the energy continuous at the cut-off but leaves forces unchanged).

    W = sum_{i<j} m_i m_j psi(s_ij).  Since d psi/ds = f(s)/2,
    -dW/dx_i = sum_j m_i m_j f(s) d_ij = m_i a_i.
    """
    pos = np.asarray(pos, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float32).astype(np.float64)
    c = np.asarray(poly, dtype=np.float32).astype(np.float64)
    ic = np.concatenate([[0.0], c / (2.0 * np.arange(1, 7))])   # integral / 2
    rc2 = float(np.float32(r_cut)) ** 2
    e = float(np.float32(eps))

    def psi(s):
        return -(s + e) ** -0.5 - P.polyval(s, ic)

    n = pos.shape[0]
    d = _pairs(pos, box, np.arange(n))
    s = np.einsum("ijk,ijk->ij", d, d)
    iu = np.triu_indices(n, 1)
    s = s[iu]
    mm = mass[iu[0]] * mass[iu[1]]
    keep = s < rc2
    return float(np.sum(mm[keep] * (psi(s[keep]) - psi(rc2))))


def newton_magnitude(pos, mass, box, r_cut, eps, targets=None, chunk=256):
    """A_i = sum_{j != i, s < r_cut^2} m_j (s + eps)^(-3/2) |d_ij|: the summed
    magnitude of the Newtonian parts of the pair forces of Eq. 7 on particle
    i, before the grid polynomial cancels any of it (the scale that floors
    relative force errors)."""
    pos = np.asarray(pos, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float32).astype(np.float64)
    rc2 = float(np.float32(r_cut)) ** 2
    e = float(np.float32(eps))
    n = pos.shape[0]
    idx_all = np.arange(n) if targets is None else np.asarray(targets)
    out = np.zeros(idx_all.size)
    for s0 in range(0, idx_all.size, chunk):
        idx = idx_all[s0:s0 + chunk]
        d = _pairs(pos, box, idx)
        s = np.einsum("ijk,ijk->ij", d, d)
        keep = (s < rc2) & (np.arange(n)[None, :] != idx[:, None])
        r = np.sqrt(s)
        out[s0:s0 + idx.size] = np.where(keep, mass[None, :] * r * (s + e) ** -1.5,
                                         0.0).sum(axis=1)
    return out


def vjp_floors(pos, mass, box, r_cut, eps, poly, g, targets=None, chunk=256):
    """The two magnitudes that floor relative VJP errors, per target k, over
    its in-cut-off pairs (w = m_k g_j - m_j g_k, N = (s + eps)^(-3/2),
    p the grid polynomial):

    B_k = sum_j (N + |p| + 2 s (1.5 N / (s + eps) + |p'|)) |w|, the parts of
          f and f' before the polynomial cancels the Newtonian term;
    P_k = sum_j (|f| + 2 |f'| s) |w|, the parts f w and 2 f' (d.w) d of the
          pair term with |d.w| bounded by |d||w|.
    """
    pos = np.asarray(pos, dtype=np.float64)
    mass = np.asarray(mass, dtype=np.float32).astype(np.float64)
    g = np.asarray(g, dtype=np.float64)
    c = np.asarray(poly, dtype=np.float32).astype(np.float64)
    dc = P.polyder(c)
    rc2 = float(np.float32(r_cut)) ** 2
    e = float(np.float32(eps))
    n = pos.shape[0]
    idx_all = np.arange(n) if targets is None else np.asarray(targets)
    b_out = np.zeros(idx_all.size)
    p_out = np.zeros(idx_all.size)
    for s0 in range(0, idx_all.size, chunk):
        idx = idx_all[s0:s0 + chunk]
        d = _pairs(pos, box, idx)
        s = np.einsum("ijk,ijk->ij", d, d)
        keep = (s < rc2) & (np.arange(n)[None, :] != idx[:, None])
        newt = (s + e) ** -1.5
        pv = P.polyval(s, c)
        dpv = P.polyval(s, dc)
        f = newt - pv
        fp = -1.5 * newt / (s + e) - dpv
        w = mass[idx][:, None, None] * g[None, :, :] - mass[None, :, None] * g[idx][:, None, :]
        wn = np.sqrt(np.einsum("ijk,ijk->ij", w, w))
        bterm = (newt + np.abs(pv) + 2.0 * s * (1.5 * newt / (s + e) + np.abs(dpv))) * wn
        pterm = (np.abs(f) + 2.0 * np.abs(fp) * s) * wn
        b_out[s0:s0 + idx.size] = np.where(keep, bterm, 0.0).sum(axis=1)
        p_out[s0:s0 + idx.size] = np.where(keep, pterm, 0.0).sum(axis=1)
    return b_out, p_out
