"""Coefficients of the grid-force polynomial f_grid(s) = poly5(s).

The paper obtains the filtered grid force by sampling particle pairs through
its spectral particle-mesh solver, fits a form with the right asymptotics and
replaces it over the short compact range by a fifth-order polynomial in
s = r.r (Habib et al. 2012, Sec. II, the paragraph after the particle-mesh
description; Sec. III, Eq. 7).  The particle-mesh solver is not part of this
library and the paper prints no coefficients, so this module states a
stand-in that produces polynomials of the same shape:

* the grid force of a unit mass is taken as the force of a Gaussian cloud,
  g(s) = M_G(r) / r^3 with M_G the mass of a 3-D Gaussian of standard
  deviation sigma_eff inside radius r;
* sigma_eff^2 = sigma^2/2 + n_s/12 + 2/12 grid cells^2 is the variance of the
  spectral filter of Sec. II, Eq. 5 (exp(-k^2 sigma^2/4) with sigma = 0.8 and a
  sinc^n_s smoothing with n_s = 3) plus the cloud-in-cell smoothing;
* least squares of degree 5 in s on 4097 uniform nodes over [0, r_cut^2],
  in float64, subject to the equality poly(r_cut^2) = (r_cut^2 + eps)^(-3/2)
  so that f_SR(r_cut^2) = 0 and the cut-off is continuous;
* the float64 coefficients are rounded to float32; those float32 values are
  the parameters every implementation receives.

This is input generation: it evaluates no force sum.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np
from scipy.special import gammainc

SIGMA_FILTER = 0.8      # Sec. II, Eq. 5, nominal filter width (grid cells)
N_S = 3                 # Sec. II, Eq. 5, sinc power
N_NODES = 4097


def sigma_eff_cells(sigma: float = SIGMA_FILTER, n_s: int = N_S) -> float:
    """Gaussian-equivalent width, in grid cells, of filter + CIC smoothing."""
    return math.sqrt(sigma * sigma / 2.0 + n_s / 12.0 + 2.0 / 12.0)


def gaussian_grid_force(s: np.ndarray, sigma: float) -> np.ndarray:
    """g(s) = M_G(sqrt(s)) / s^(3/2) for a unit-mass Gaussian of width sigma.

    M_G(r) is the chi-distribution CDF with 3 degrees of freedom,
    P(3/2, r^2 / (2 sigma^2)); at s -> 0 the limit sqrt(2/pi)/(3 sigma^3) is
    used through its series so that the node s = 0 is finite.
    """
    s = np.asarray(s, dtype=np.float64)
    z = s / (2.0 * sigma * sigma)
    out = np.empty_like(s)
    small = z < 1e-4
    big = ~small
    out[big] = gammainc(1.5, z[big]) / s[big] ** 1.5
    # P(3/2, z) = z^(3/2)/Gamma(5/2) * (1 - 3z/5 + 3z^2/14 - ...)
    zs = z[small]
    lim = 1.0 / ((2.0 * sigma * sigma) ** 1.5 * math.gamma(2.5))
    out[small] = lim * (1.0 - 0.6 * zs + (3.0 / 14.0) * zs * zs)
    return out


@dataclasses.dataclass
class FGridFit:
    coeffs: np.ndarray          # float32[6], c_0..c_5 of f_grid in s
    coeffs64: np.ndarray        # the float64 fit before rounding
    r_cut: float                # float32 value (as a Python float)
    eps: float                  # float32 value (as a Python float)
    cell: float                 # grid cell size in box units
    sigma: float                # sigma_eff in box units
    max_fit_err: float          # max |poly - g| / (s + eps)^(-3/2) on the nodes
    constraint_resid: float     # |poly32(r_cut^2) - (r_cut^2+eps)^(-3/2)| / same


def fit_fgrid(cell: float, r_cut_cells: float = 3.0,
              eps_cells2: float = 1e-5 * 128.0 ** 2,
              sigma_cells: float | None = None) -> FGridFit:
    """Constrained degree-5 least-squares fit of the grid force (see module doc).

    ``cell`` is the particle-mesh grid spacing in box units, ``r_cut_cells``
    the matching scale in cells (3 in Sec. II), ``eps_cells2`` the softening
    in cells^2 (0.164 cell^2 reproduces eps = 1e-5 box^2 on a 128^3 grid).
    """
    r_cut = float(np.float32(r_cut_cells * cell))
    eps = float(np.float32(eps_cells2 * cell * cell))
    sig = (sigma_cells if sigma_cells is not None else sigma_eff_cells()) * cell
    rc2 = r_cut * r_cut
    u = np.linspace(0.0, 1.0, N_NODES)
    s = u * rc2
    g = gaussian_grid_force(s, sig)
    target = (rc2 + eps) ** -1.5
    # p(u) = target + (u - 1) q(u), q of degree 4: the constraint holds exactly
    A = np.stack([(u - 1.0) * u ** m for m in range(5)], axis=1)
    qc, *_ = np.linalg.lstsq(A, g - target, rcond=None)
    a = np.zeros(6)
    a[0] = target
    for m in range(5):
        a[m + 1] += qc[m]
        a[m] -= qc[m]
    c64 = np.array([a[k] / rc2 ** k for k in range(6)])
    c32 = c64.astype(np.float32)
    newt = (s + eps) ** -1.5
    p64 = np.polyval(c64[::-1], s)
    max_err = float(np.max(np.abs(p64 - g) / newt))
    p32_at_rc = sum(float(c32[k]) * rc2 ** k for k in range(6))
    cres = abs(p32_at_rc - target) / target
    return FGridFit(coeffs=c32, coeffs64=c64, r_cut=r_cut, eps=eps, cell=cell,
                    sigma=sig, max_fit_err=max_err, constraint_resid=cres)
