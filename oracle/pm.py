"""Float64 oracle for the long-range spectral particle-mesh (PM) force.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg call it; the GPU library never does, and this module never
imports the GPU library.

Habib et al. 2012, Sec. II (the long/medium-range solver):

1. the particles' masses are deposited on a periodic grid of ng^3 cells of
   side D = box / ng with Cloud-In-Cell (CIC) weights, giving the density
   rho = mass / D^3 at the grid points;
2. in Fourier space the density is smoothed by the isotropising filter of
   Eq. 5, S(k) = exp(-k^2 sigma^2 / 4) [sin(k D / 2) / (k D / 2)]^n_s with
   sigma in grid cells (read as the smoothing sinc: the printed factor
   (2k/D) sin(kD/2) is not dimensionless), nominally sigma = 0.8, n_s = 3;
3. the potential is the sixth-order periodic influence function applied to
   the filtered density: phi = -4 pi S rho / K6(k), where K6 is the Fourier
   symbol of minus the sixth-order central-difference Laplacian,
   K6 = sum_axes [49/18 - 3 cos(k_a D) + (3/10) cos(2 k_a D)
   - (1/45) cos(3 k_a D)] / D^2 (about k^2 for small k), and phi(0) = 0;
4. each component of the acceleration a = -grad phi is taken by fourth-order
   spectral differencing, the Fourier symbol i (4/3 sin(k_a D)
   - 1/6 sin(2 k_a D)) / D of the fourth-order central difference, and
   transformed back;
5. the three acceleration grids are interpolated to the particles with the
   same CIC weights.

The paper names the influence function and the differencing operator only
by order and origin; the two symbols above are the central-difference
readings of "sixth-order" and "fourth-order".  The gravitational constant
is 1.  The FFT is numpy's (a library primitive); everything is float64.
"""
from __future__ import annotations

import numpy as np


def _cic(pos, box, ng):
    """Lower grid index (n, 3) and the CIC weights (n, 3, 2) of each particle
    on the periodic grid; grid point g sits at g D."""
    D = box / ng
    u = np.asarray(pos, dtype=np.float64) / D
    u = u - ng * np.floor(u / ng)
    i0 = np.floor(u).astype(np.int64)
    f = u - i0
    i0 %= ng
    w = np.stack([1.0 - f, f], axis=-1)
    return i0, w


def cic_deposit(pos, mass, box, ng):
    """Mass on the grid points (ng, ng, ng), CIC weights, periodic."""
    i0, w = _cic(pos, box, ng)
    m = np.asarray(mass, dtype=np.float64)
    grid = np.zeros((ng, ng, ng))
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                wt = m * w[:, 0, a] * w[:, 1, b] * w[:, 2, c]
                np.add.at(grid, ((i0[:, 0] + a) % ng, (i0[:, 1] + b) % ng,
                                 (i0[:, 2] + c) % ng), wt)
    return grid


def cic_interpolate(grid, pos, box):
    """Values of a periodic grid at the particles, CIC weights."""
    ng = grid.shape[0]
    i0, w = _cic(pos, box, ng)
    out = np.zeros(i0.shape[0])
    for a in (0, 1):
        for b in (0, 1):
            for c in (0, 1):
                out += (w[:, 0, a] * w[:, 1, b] * w[:, 2, c] *
                        grid[(i0[:, 0] + a) % ng, (i0[:, 1] + b) % ng,
                             (i0[:, 2] + c) % ng])
    return out


def wavenumbers(box, ng):
    """Angular wavenumbers of numpy's FFT order, one axis."""
    return 2.0 * np.pi * np.fft.fftfreq(ng, d=box / ng)


def filter_symbol(kmag, D, sigma=0.8, n_s=3):
    """Eq. 5 with sigma in grid cells: exp(-k^2 (sigma D)^2 / 4) times
    [sin(k D / 2) / (k D / 2)]^n_s (1 at k = 0)."""
    x = 0.5 * kmag * D
    sinc = np.where(x == 0.0, 1.0, np.sin(x) / np.where(x == 0.0, 1.0, x))
    return np.exp(-0.25 * (kmag * sigma * D) ** 2) * sinc ** n_s


def laplacian6_symbol(k, D):
    """Minus the Fourier symbol of the sixth-order central-difference second
    derivative along one axis."""
    kd = k * D
    return (49.0 / 18.0 - 3.0 * np.cos(kd) + 0.3 * np.cos(2 * kd)
            - np.cos(3 * kd) / 45.0) / (D * D)


def gradient4_symbol(k, D):
    """Fourier symbol (divided by i) of the fourth-order central difference."""
    kd = k * D
    return (4.0 / 3.0 * np.sin(kd) - np.sin(2 * kd) / 6.0) / D


def potential_hat(rho_hat, box, sigma=0.8, n_s=3):
    """phi(k) = -4 pi S(k) rho(k) / K6(k), phi(0) = 0."""
    ng = rho_hat.shape[0]
    D = box / ng
    k1 = wavenumbers(box, ng)
    kx, ky, kz = np.meshgrid(k1, k1, k1, indexing="ij")
    kmag = np.sqrt(kx * kx + ky * ky + kz * kz)
    K6 = laplacian6_symbol(kx, D) + laplacian6_symbol(ky, D) + laplacian6_symbol(kz, D)
    S = filter_symbol(kmag, D, sigma, n_s)
    with np.errstate(divide="ignore", invalid="ignore"):
        phi = np.where(K6 > 0, -4.0 * np.pi * S * rho_hat / np.where(K6 > 0, K6, 1.0), 0.0)
    phi[0, 0, 0] = 0.0
    return phi


def accel_grids(pos, mass, box, ng, sigma=0.8, n_s=3):
    """The three acceleration grids a = -grad phi (ng, ng, ng) each."""
    D = box / ng
    rho = cic_deposit(pos, mass, box, ng) / D ** 3
    phi = potential_hat(np.fft.fftn(rho), box, sigma, n_s)
    k1 = wavenumbers(box, ng)
    out = []
    for axis in range(3):
        shape = [1, 1, 1]
        shape[axis] = ng
        g = gradient4_symbol(k1, D).reshape(shape)
        out.append(np.real(np.fft.ifftn(-1j * g * phi)))
    return out


def accel(pos, mass, box, ng, sigma=0.8, n_s=3):
    """Long-range accelerations (n, 3) of the particles."""
    grids = accel_grids(pos, mass, box, ng, sigma, n_s)
    return np.stack([cic_interpolate(g, pos, box) for g in grids], axis=1)


def pair_force_samples(box, ng, r_max, n_sources=8, per_source=2000, seed=0,
                       sigma=0.8, n_s=3):
    """The PM force between pairs, sampled as the paper samples it (Sec. II,
    the paragraph on matching the short-range force): one unit mass at a
    random position and massless test particles at random directions and
    separations r <= r_max (uniform in r^2), one solve per source.  Returns
    (s = r^2, radial force over r, attractive positive)."""
    rng = np.random.default_rng(seed)
    ss, gs = [], []
    for _ in range(n_sources):
        x0 = rng.random(3) * box
        u = rng.standard_normal((per_source, 3))
        u /= np.linalg.norm(u, axis=1)[:, None]
        r = r_max * np.sqrt(rng.random(per_source))
        r = np.maximum(r, 1e-3 * r_max)
        tp = x0 + r[:, None] * u
        pos = np.concatenate([x0[None], tp])
        mass = np.zeros(len(pos))
        mass[0] = 1.0
        a = accel(pos, mass, box, ng, sigma, n_s)[1:]
        radial = -(a * u).sum(axis=1)
        ss.append(r * r)
        gs.append(radial / r)
    return np.concatenate(ss), np.concatenate(gs)


def fit_grid_force(box, ng, r_cut, eps, n_sources=8, per_source=2000, seed=0,
                   sigma=0.8, n_s=3):
    """The grid-force polynomial f_grid(s) fitted to sampled PM pair forces:
    degree 5 in s by least squares over the samples with s <= r_cut^2,
    constrained to f_grid(r_cut^2) = (r_cut^2 + eps)^(-3/2) so that the
    short-range kernel f(s) = (s + eps)^(-3/2) - f_grid(s) vanishes at the
    cut-off (Sec. II: the fitted filtered grid force, replaced over the
    compact short range by a fifth-order polynomial).  r_cut and eps as the
    float32 values the kernels use.  Returns float32 coefficients c_0..c_5
    of f_grid in s."""
    rc2 = float(np.float32(r_cut)) ** 2
    e = float(np.float32(eps))
    s, g = pair_force_samples(box, ng, float(np.float32(r_cut)), n_sources,
                              per_source, seed, sigma, n_s)
    u = s / rc2
    target = (rc2 + e) ** -1.5
    # p(u) = target + (u - 1) q(u), q of degree 4, satisfies the constraint
    A = np.stack([(u - 1.0) * u ** m for m in range(5)], axis=1)
    qc, *_ = np.linalg.lstsq(A, g - target, rcond=None)
    a = np.zeros(6)
    a[0] = target
    for m in range(5):
        a[m + 1] += qc[m]
        a[m] -= qc[m]
    return np.array([a[k] / rc2 ** k for k in range(6)]).astype(np.float32)
