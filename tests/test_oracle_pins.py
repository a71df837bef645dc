"""Pins for the float64 oracle against facts that do not come from the
oracle itself: a second independent implementation, the potential the force
derives from, the textbook softened inverse-square law, symmetry and
conservation laws, and exact special cases.  All run on the CPU.

The definition pinned is Habib et al. 2012, Sec. III, Eq. 7 (f_SR) with the
short-range condition applied per pair.
"""
import json
import math
import os

import numpy as np
import pytest
from scipy.spatial.distance import cdist

import oracle
from oracle import brute
from workloads import make_config, plummer_clustered, fit_fgrid

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _small_case(n=600, seed=11, grid=16, box=1.0):
    """A clustered set on a coarse grid so that neighbour counts are large."""
    pos, _ = plummer_clustered(n, seed, 6, 0.6, 1.0 / grid)
    fit = fit_fgrid(1.0 / grid)
    rng = np.random.default_rng(seed)
    mass = (rng.random(n) * 0.5 + 0.75).astype(np.float32) / n
    return pos * box, mass, box, fit


def test_cell_list_matches_all_pairs_cfg1_subset(oracle_lib):
    w = make_config("cfg1")
    idx = np.random.default_rng(1).choice(w.n, 1000, replace=False)
    a, an, _ = oracle.force(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly)
    b = brute.force(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly, targets=idx)
    assert oracle.rel_err_floored(b, a[idx], an[idx]).max() <= 1e-12


@pytest.mark.parametrize("box", [1.0, -1.0])
def test_cell_list_matches_all_pairs_clustered(oracle_lib, box):
    pos, mass, _, fit = _small_case()
    a, an, _ = oracle.force(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs)
    b = brute.force(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs)
    assert oracle.rel_err_floored(b, a, an).max() <= 1e-12


@pytest.mark.parametrize("box", [1.0, -1.0])
def test_acceleration_is_minus_potential_gradient(oracle_lib, box):
    """m_i a_i = -dW/dx_i with W the pair potential whose s-derivative is f/2
    (integrated term by term, independently of the force formula)."""
    rng = np.random.default_rng(5)
    n = 24
    fit = fit_fgrid(1.0 / 8.0)          # r_cut = 3/8 of the box
    pos = 0.3 + 0.4 * rng.random((n, 3)) if box < 0 else rng.random((n, 3))
    mass = (0.5 + rng.random(n)).astype(np.float32)
    a, _, _ = oracle.force(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs)
    h = 1e-6
    rc2 = float(np.float32(fit.r_cut)) ** 2
    checked = 0
    for i in range(n):
        for ax in range(3):
            # skip probes whose step moves a pair across the cut-off
            d = pos - pos[i]
            if box > 0:
                d -= np.rint(d)
            r = np.sqrt((d * d).sum(1))
            r[i] = 0.0
            if np.any(np.abs(r - math.sqrt(rc2)) < 4 * h):
                continue
            vals = []
            for step in (h, -h, 2 * h, -2 * h):
                p = pos.copy()
                p[i, ax] += step
                vals.append(brute.potential(p, mass, box, fit.r_cut, fit.eps, fit.coeffs))
            # fourth-order central difference
            grad = (8 * (vals[0] - vals[1]) - (vals[2] - vals[3])) / (12 * h)
            scale = max(abs(float(mass[i]) * a[i, ax]), 1e-3 * np.abs(mass[i] * a[i]).max())
            assert abs(-grad - float(mass[i]) * a[i, ax]) <= 1e-5 * scale + 1e-9
            checked += 1
    assert checked > 3 * n // 2


def test_plummer_softened_direct_sum(oracle_lib):
    """poly = 0, open boundaries, r_cut beyond the system: the textbook
    Plummer-softened direct sum a_i = sum_j m_j (x_j - x_i)/(r^2+eps)^(3/2)."""
    rng = np.random.default_rng(3)
    n = 300
    pos = rng.normal(0.0, 1.0, (n, 3))
    mass = rng.random(n).astype(np.float32)
    eps = float(np.float32(0.01))
    poly = np.zeros(6, np.float32)
    a, _, cnt = oracle.force(pos, mass, -1.0, 1e3, eps, poly)
    r2 = cdist(pos, pos, "sqeuclidean")
    w = mass.astype(np.float64)[None, :] / (r2 + eps) ** 1.5
    np.fill_diagonal(w, 0.0)
    ref = w @ pos - w.sum(1)[:, None] * pos
    assert np.all(cnt == n - 1)
    assert np.allclose(a, ref, rtol=1e-11, atol=1e-11 * np.abs(ref).max())


def test_inverse_square_law_and_direction(oracle_lib):
    """Two bodies, poly = 0, eps tiny: |a_1| = m_2 / r^2 pointing to body 2,
    and the same pair straddling the periodic boundary gives the same force."""
    poly = np.zeros(6, np.float32)
    eps = float(np.float32(1e-30))
    r = 0.013
    m2 = np.float32(3.0)
    pos = np.array([[0.5, 0.5, 0.5], [0.5 + r, 0.5, 0.5]])
    mass = np.array([1.0, m2], np.float32)
    a, _, _ = oracle.force(pos, mass, 1.0, 0.05, eps, poly)
    assert a[0, 0] > 0 and a[1, 0] < 0
    assert math.isclose(a[0, 0], float(m2) / r ** 2, rel_tol=1e-12)
    assert abs(a[0, 1]) == 0.0 and abs(a[0, 2]) == 0.0
    wrap = np.array([[0.995, 0.2, 0.7], [0.995 + r - 1.0, 0.2, 0.7]])
    b, _, _ = oracle.force(wrap, mass, 1.0, 0.05, eps, poly)
    assert np.allclose(b, a, rtol=1e-9, atol=0)


def test_newton_third_law(oracle_lib):
    pos, mass, box, fit = _small_case(n=2000, seed=21)
    a, an, cnt = oracle.force(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs)
    m = mass.astype(np.float64)
    mom = np.abs((m[:, None] * a).sum(0))
    assert cnt.sum() > 10000
    assert np.all(mom <= 1e-14 * (m * an).sum())


def test_translation_invariance(oracle_lib):
    pos, mass, box, fit = _small_case(n=1500, seed=22)
    a, an, _ = oracle.force(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs)
    shift = np.array([0.3141, 0.7183, 0.5772])
    p2 = (pos + shift) % 1.0
    b, _, _ = oracle.force(p2, mass, box, fit.r_cut, fit.eps, fit.coeffs)
    assert oracle.rel_err_floored(b, a, an).max() <= 1e-12


@pytest.mark.parametrize("perm,flip", [((1, 2, 0), (False, False, False)),
                                       ((0, 1, 2), (True, False, False)),
                                       ((2, 0, 1), (False, True, True))])
def test_cubic_symmetry_equivariance(oracle_lib, perm, flip):
    pos, mass, box, fit = _small_case(n=1500, seed=23)
    a, an, _ = oracle.force(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs)
    p2 = pos[:, perm].copy()
    expect = a[:, perm].copy()
    for ax in range(3):
        if flip[ax]:
            p2[:, ax] = (1.0 - p2[:, ax]) % 1.0
            expect[:, ax] = -expect[:, ax]
    b, _, _ = oracle.force(p2, mass, box, fit.r_cut, fit.eps, fit.coeffs)
    assert oracle.rel_err_floored(b, expect, an).max() <= 1e-12


def test_permutation_equivariance(oracle_lib):
    pos, mass, box, fit = _small_case(n=1500, seed=24)
    a, an, _ = oracle.force(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs)
    p = np.random.default_rng(0).permutation(pos.shape[0])
    b, _, _ = oracle.force(pos[p], mass[p], box, fit.r_cut, fit.eps, fit.coeffs)
    assert oracle.rel_err_floored(b, a[p], an[p]).max() <= 1e-12


def test_linear_in_masses(oracle_lib):
    pos, mass, box, fit = _small_case(n=1200, seed=25)
    rng = np.random.default_rng(1)
    m1 = (rng.random(pos.shape[0]) / 100).astype(np.float32)
    m2 = (rng.random(pos.shape[0]) / 100).astype(np.float32)
    # pick masses whose float32 sum is exact so the comparison is clean
    m1 = np.float32(2.0 ** -7) * np.round(m1 * 2 ** 20) / np.float32(2 ** 13)
    m2 = np.float32(2.0 ** -7) * np.round(m2 * 2 ** 20) / np.float32(2 ** 13)
    a1, an1, _ = oracle.force(pos, m1, box, fit.r_cut, fit.eps, fit.coeffs)
    a2, an2, _ = oracle.force(pos, m2, box, fit.r_cut, fit.eps, fit.coeffs)
    a3, _, _ = oracle.force(pos, (m1 + m2).astype(np.float32), box, fit.r_cut,
                            fit.eps, fit.coeffs)
    assert oracle.rel_err_floored(a3, a1 + a2, an1 + an2).max() <= 1e-12


def test_symmetric_stencil_cancels(oracle_lib):
    """A particle at the centre of 8 equal masses on cube corners, and of 6 on
    octahedron vertices, feels no force (by symmetry)."""
    fit = fit_fgrid(1.0 / 64.0)
    h = 0.25 * fit.r_cut
    c = np.array([0.5, 0.5, 0.5])
    corners = np.array([[sx, sy, sz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)]) * h
    octa = np.concatenate([np.eye(3), -np.eye(3)]) * 1.7 * h
    pos = np.concatenate([c[None], c + corners, c + octa])
    mass = np.full(pos.shape[0], np.float32(0.25))
    a, an, _ = oracle.force(pos, mass, 1.0, fit.r_cut, fit.eps, fit.coeffs)
    assert np.abs(a[0]).max() <= 1e-14 * an[0]
    assert np.abs(a[1]).max() > 1e-3 * an[1]


def test_periodic_lattice_cancels(oracle_lib):
    """Every particle of a perfect periodic cubic lattice feels no force; a
    wrong minimum image or a missing neighbour cell breaks the symmetry."""
    g = 12
    ax = (np.arange(g) + 0.5) / g
    pos = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    fit = fit_fgrid(1.0 / 24.0)       # r_cut = 1/8: the 6 + 12 nearest lattice sites inside
    mass = np.full(pos.shape[0], np.float32(1.0 / pos.shape[0]))
    a, an, cnt = oracle.force(pos, mass, 1.0, fit.r_cut, fit.eps, fit.coeffs)
    assert np.all(cnt == 18)
    assert np.abs(a).max() <= 1e-13 * an.max()


def test_isolated_particle_is_exactly_zero(oracle_lib):
    fit = fit_fgrid(1.0 / 128.0)
    pos = np.array([[0.1, 0.1, 0.1], [0.5, 0.5, 0.5], [0.5 + 0.5 * fit.r_cut, 0.5, 0.5]])
    mass = np.ones(3, np.float32)
    a, an, cnt = oracle.force(pos, mass, 1.0, fit.r_cut, fit.eps, fit.coeffs)
    assert np.all(a[0] == 0.0) and an[0] == 0.0 and cnt[0] == 0
    assert cnt[1] == 1 and cnt[2] == 1


def test_cutoff_is_strict(oracle_lib):
    fit = fit_fgrid(1.0 / 128.0)
    rc = float(np.float32(fit.r_cut))
    inside = np.nextafter(rc, 0.0)
    for sep, expect in ((inside * (1 - 1e-12), 1), (rc * (1 + 1e-12), 0)):
        pos = np.array([[0.5, 0.5, 0.5], [0.5 + sep, 0.5, 0.5]])
        _, _, cnt = oracle.force(pos, np.ones(2, np.float32), 1.0, fit.r_cut,
                                 fit.eps, fit.coeffs)
        assert cnt[0] == expect


def test_fit_shape_and_paper_constants():
    consts = json.load(open(os.path.join(GOLDEN, "paper_constants.json")))
    assert consts["match_cells"]["value"] == 3
    fit = fit_fgrid(1.0 / 128.0, consts["match_cells"]["value"])
    assert fit.coeffs.shape == (consts["poly_degree"]["value"] + 1,)
    assert fit.coeffs.size == consts["poly_coeff_registers"]["value"]
    # the equality constraint makes f_SR vanish at the cut-off (float32 coefficients)
    assert fit.constraint_resid < 1e-5
    # the stand-in grid force is matched to a few percent of Newtonian
    assert fit.max_fit_err < 0.025
    # the paper's instruction accounting: 16 FMA x 4 lanes x 2 + 10 x 4 = 168
    q = consts["qpx_width"]["value"]
    fma = consts["kernel_fma_instructions"]["value"]
    tot = consts["kernel_instructions"]["value"]
    assert fma * q * 2 + (tot - fma) * q == consts["kernel_flops"]["value"]
    assert tot * q * 2 == consts["kernel_flops_if_all_fma"]["value"]
    assert round(168 / 208, 2) == consts["kernel_theoretical_fraction"]["value"]


def test_gaussian_grid_force_against_quadrature():
    """The stand-in grid force M_G(r)/r^3 against direct numerical
    integration of a Gaussian density, and its Newtonian far field."""
    from scipy.integrate import quad
    from workloads.fgrid import gaussian_grid_force
    sig = 0.7
    for r in (1e-3, 0.3, 1.0, 2.5):
        m, _ = quad(lambda t: 4 * math.pi * t * t * math.exp(-t * t / (2 * sig * sig))
                    / (2 * math.pi * sig * sig) ** 1.5, 0, r, epsabs=0, epsrel=1e-13)
        assert math.isclose(gaussian_grid_force(np.array([r * r]), sig)[0], m / r ** 3,
                            rel_tol=1e-9)
    far = gaussian_grid_force(np.array([100.0]), sig)[0]
    assert math.isclose(far, 100.0 ** -1.5, rel_tol=1e-12)


@pytest.mark.parametrize("box", [1.0, -1.0])
def test_binning_reference_properties(box):
    """The NumPy chaining mesh: pairs inside r_cut sit in adjacent cells,
    records rebuild the positions, order is by cell then input index."""
    from oracle import binning
    pos, mass, _, fit = _small_case(n=3000, seed=26)
    keys, perm, cs, rec = binning.chaining_mesh(pos, mass, box, fit.r_cut)
    N, L = binning.grid(box, fit.r_cut)
    assert L >= float(np.float32(fit.r_cut))
    sk = keys[perm]
    assert np.all(np.diff(sk) >= 0)
    # inside a cell: sub-cells in Morton order, input order inside a sub-cell
    lev = binning.sub_levels(N)
    rel = rec[:, :3].astype(np.float64) / L * (1 << lev)
    s3 = np.clip(np.floor(rel), 0, (1 << lev) - 1).astype(np.int64)
    same_cell = np.diff(sk) == 0
    sub_id = s3[:, 0] * 100 + s3[:, 1] * 10 + s3[:, 2]
    same_sub = same_cell & (np.diff(sub_id) == 0)
    assert np.all(np.diff(perm)[same_sub] > 0)
    assert lev == 2
    assert np.array_equal(np.diff(cs), np.bincount(keys, minlength=N ** 3))
    c = np.stack([sk // (N * N), (sk // N) % N, sk % N], 1)
    back = c * L + rec[:, :3].astype(np.float64)
    assert np.abs(back - pos[perm]).max() <= 2 * L * 2.0 ** -24
    assert np.array_equal(rec[:, 3], mass[perm])
    # every pair inside the cut-off lies in adjacent cells (with wrap)
    d = pos[:, None, :] - pos[None, :, :]
    if box > 0:
        d -= np.rint(d)
    close = np.argwhere((d * d).sum(-1) < float(np.float32(fit.r_cut)) ** 2)
    ci = np.stack([keys // (N * N), (keys // N) % N, keys % N], 1)
    dc = np.abs(ci[close[:, 0]] - ci[close[:, 1]])
    if box > 0:
        dc = np.minimum(dc, N - dc)
    assert close.shape[0] > 3000 and dc.max() <= 1
