"""Pins for the oracle's vector-jacobian product and its subcycle rollout:
central finite differences of the oracle's own forward sum (a different
route to the same derivative), the dot-product test, translation invariance
of the loss, linearity in the cotangent, an independent all-pairs VJP, and
time reversibility and momentum conservation of the float64 stream-kick-
stream map (Habib et al. 2012, Sec. II, Eq. 6)."""
import numpy as np
import pytest

import oracle
from oracle import brute, rollout
from workloads import plummer_clustered, fit_fgrid


def _case(n=500, seed=31, grid=16, box=1.0):
    pos, _ = plummer_clustered(n, seed, 5, 0.6, 1.0 / grid)
    fit = fit_fgrid(1.0 / grid)
    rng = np.random.default_rng(seed)
    mass = ((rng.random(n) * 0.5 + 0.75) / n).astype(np.float32)
    g = rng.standard_normal((n, 3))
    return pos, mass, box, fit, g


def _loss(pos, mass, box, fit, g):
    a, _, _ = oracle.force(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs)
    return float(np.sum(g * a))


def _near_cutoff(pos, k, box, rc, h):
    d = pos - pos[k]
    if box > 0:
        d -= np.rint(d)
    r = np.sqrt((d * d).sum(1))
    r[k] = -1.0
    return np.any(np.abs(r - rc) < 3 * h)


@pytest.mark.parametrize("box", [1.0, -1.0])
def test_vjp_matches_central_differences(oracle_lib, box):
    pos, mass, _, fit, g = _case()
    vjp, bn = oracle.force_vjp(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs, g)
    h = 1e-4 * fit.cell
    rc = float(np.float32(fit.r_cut))
    rng = np.random.default_rng(0)
    ks = rng.choice(pos.shape[0], 40, replace=False)
    checked = 0
    for k in ks:
        if _near_cutoff(pos, k, box, rc, h):
            continue
        for ax in range(3):
            p1, p2 = pos.copy(), pos.copy()
            p1[k, ax] += h
            p2[k, ax] -= h
            fd = (_loss(p1, mass, box, fit, g) - _loss(p2, mass, box, fit, g)) / (2 * h)
            assert abs(fd - vjp[k, ax]) <= 1e-5 * max(abs(vjp[k, ax]), 0.1 * bn[k]) + 1e-12
            checked += 1
    assert checked >= 60


def test_vjp_dot_product_test(oracle_lib):
    """<g, J v> from a directional finite difference equals <J^T g, v>."""
    pos, mass, box, fit, g = _case(seed=32)
    rng = np.random.default_rng(2)
    v = rng.standard_normal(pos.shape)
    vjp, _ = oracle.force_vjp(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs, g)
    h = 1e-7 * fit.cell
    fd = (_loss(pos + h * v, mass, box, fit, g) - _loss(pos - h * v, mass, box, fit, g)) / (2 * h)
    rhs = float(np.sum(vjp * v))
    assert abs(fd - rhs) <= 1e-5 * np.abs(vjp * v).sum()


def test_vjp_sums_to_zero_and_is_linear(oracle_lib):
    pos, mass, box, fit, g = _case(seed=33)
    v1, b1 = oracle.force_vjp(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs, g)
    # translating every particle leaves L unchanged: sum_k dL/dx_k = 0
    assert np.all(np.abs(v1.sum(0)) <= 1e-13 * b1.sum())
    g2 = np.random.default_rng(9).standard_normal(g.shape)
    v2, b2 = oracle.force_vjp(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs, g2)
    v3, _ = oracle.force_vjp(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs, 2.0 * g - 3.0 * g2)
    assert oracle.rel_err_floored(v3, 2 * v1 - 3 * v2, 2 * b1 + 3 * b2).max() <= 1e-12


@pytest.mark.parametrize("box", [1.0, -1.0])
def test_vjp_cell_list_matches_all_pairs(oracle_lib, box):
    pos, mass, _, fit, g = _case(seed=34)
    v1, b1 = oracle.force_vjp(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs, g)
    v2 = brute.force_vjp(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs, g)
    assert oracle.rel_err_floored(v2, v1, b1).max() <= 1e-12


def _rollout_case():
    pos, mass, box, fit, _ = _case(n=300, seed=35)
    rng = np.random.default_rng(3)
    a, _, _ = oracle.force(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs)
    h = float(np.sqrt(0.01 * fit.cell / np.sqrt((a * a).sum(1).mean())))
    v = rng.standard_normal(pos.shape) * fit.cell / h * 0.01
    return pos, v, mass, box, fit, h


def test_sks_time_reversible_and_conserves_momentum(oracle_lib):
    pos, v, mass, box, fit, h = _rollout_case()
    x1, v1, _ = rollout.sks(pos, v, mass, box, fit.r_cut, fit.eps, fit.coeffs, h, 5)
    assert np.abs(x1 - pos).max() > 1e-3 * fit.cell
    x0, v0, _ = rollout.sks(x1, v1, mass, box, fit.r_cut, fit.eps, fit.coeffs, -h, 5)
    dx = x0 - pos
    dx -= np.rint(dx)
    assert np.abs(dx).max() <= 1e-12
    assert np.abs(v0 - v).max() <= 1e-10 * np.abs(v).max()
    m = mass.astype(np.float64)[:, None]
    p0, p1 = (m * v).sum(0), (m * v1).sum(0)
    assert np.all(np.abs(p1 - p0) <= 1e-13 * (m * np.abs(v1)).sum())


def test_sks_adjoint_matches_finite_differences(oracle_lib):
    pos, v, mass, box, fit, h = _rollout_case()
    rng = np.random.default_rng(4)
    gx = rng.standard_normal(pos.shape)
    x1, v1, cps = rollout.sks(pos, v, mass, box, fit.r_cut, fit.eps, fit.coeffs, h, 5)
    gx0, gv0 = rollout.sks_vjp(cps, mass, box, fit.r_cut, fit.eps, fit.coeffs, h,
                               gx, np.zeros_like(gx))

    def L(p, vv):
        xf, _, _ = rollout.sks(p, vv, mass, box, fit.r_cut, fit.eps, fit.coeffs, h, 5)
        return float(np.sum(gx * xf))

    dirx = rng.standard_normal(pos.shape)
    dirv = rng.standard_normal(pos.shape)
    eps_fd = 1e-7 * fit.cell
    fdx = (L(pos + eps_fd * dirx, v) - L(pos - eps_fd * dirx, v)) / (2 * eps_fd)
    fdv = (L(pos, v + eps_fd * dirv) - L(pos, v - eps_fd * dirv)) / (2 * eps_fd)
    assert abs(fdx - np.sum(gx0 * dirx)) <= 1e-6 * np.abs(gx0 * dirx).sum()
    assert abs(fdv - np.sum(gv0 * dirv)) <= 1e-6 * np.abs(gv0 * dirv).sum()


def test_vjp_cutoff_band_bounds_the_jump(oracle_lib):
    """A pair moved across r_cut changes the VJP by at most the band
    magnitude the oracle reports (f' jumps at the cut-off, f does not)."""
    fit = fit_fgrid(1.0 / 64.0)
    rc = float(np.float32(fit.r_cut))
    mass = np.array([0.3, 0.7], np.float32)
    g = np.array([[0.2, -1.0, 0.5], [1.0, 0.3, -0.4]])
    vals = []
    for sep in (rc * (1 - 1e-9), rc * (1 + 1e-9)):
        pos = np.array([[0.5, 0.5, 0.5], [0.5 + sep, 0.5, 0.5]])
        out, bn, amb = oracle.force_vjp(pos, mass, 1.0, fit.r_cut, fit.eps, fit.coeffs,
                                        g, cut_band=1e-6)
        _, _, amb0 = oracle.force_vjp(pos, mass, 1.0, fit.r_cut, fit.eps, fit.coeffs,
                                      g, cut_band=0.0)
        assert np.all(amb0 == 0.0) and np.all(amb > 0.0)
        vals.append((out, amb))
    jump = np.linalg.norm(vals[0][0] - vals[1][0], axis=1)
    assert np.all(jump > 0.1 * vals[0][1])       # the jump is a full pair term
    assert np.all(jump <= vals[0][1] * (1 + 1e-6))
