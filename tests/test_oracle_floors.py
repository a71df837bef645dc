"""Pins for the magnitudes that floor the relative errors of every parity
test: A_i (forces), and B_k and P_k (VJP).  Each is checked against an
independent NumPy implementation and against identities that tie it to the
oracle's own force and VJP values on single pairs, which are pinned
elsewhere (brute force, finite differences, the potential, the dot-product
test).

Definitions (Habib et al. 2012, Sec. III, Eq. 7, f(s) = N(s) - p(s) with
N = (s + eps)^(-3/2) and p the grid polynomial; w = m_k g_j - m_j g_k):
  A_i = sum_j m_j N |d_ij|
  B_k = sum_j (N + |p| + 2 s (1.5 N / (s + eps) + |p'|)) |w|
  P_k = sum_j (|f| + 2 |f'| s) |w|
"""
import math

import numpy as np
import pytest

import oracle
from oracle import brute
from workloads import fit_fgrid, plummer_clustered


def _case(n=500, seed=21, grid=16):
    pos, _ = plummer_clustered(n, seed, 5, 0.6, 1.0 / grid)
    fit = fit_fgrid(1.0 / grid)
    rng = np.random.default_rng(seed)
    mass = (rng.random(n) * 0.5 + 0.75).astype(np.float32) / n
    g = rng.standard_normal((n, 3))
    return pos, mass, fit, g


@pytest.mark.parametrize("box", [1.0, -1.0])
def test_newton_magnitude_matches_numpy(oracle_lib, box):
    pos, mass, fit, _ = _case()
    _, an, cnt = oracle.force(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs)
    ref = brute.newton_magnitude(pos, mass, box, fit.r_cut, fit.eps)
    assert np.mean(cnt > 0) > 0.9
    np.testing.assert_allclose(an, ref, rtol=1e-12, atol=0.0)


@pytest.mark.parametrize("box", [1.0, -1.0])
def test_vjp_floors_match_numpy(oracle_lib, box):
    pos, mass, fit, g = _case()
    _, bn, pm = oracle.force_vjp(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs, g,
                                 pair_floor=True)
    bref, pref = brute.vjp_floors(pos, mass, box, fit.r_cut, fit.eps, fit.coeffs, g)
    np.testing.assert_allclose(bn, bref, rtol=1e-12, atol=0.0)
    np.testing.assert_allclose(pm, pref, rtol=1e-12, atol=0.0)
    # the tighter floor never exceeds the other
    assert np.all(pm <= bn * (1 + 1e-12))


def _two_body(r, axis=np.array([0.6, 0.0, 0.8])):
    x0 = np.array([0.4, 0.45, 0.5])
    pos = np.stack([x0, x0 + r * axis])
    return pos


def test_newton_magnitude_two_body_closed_form(oracle_lib):
    """Two bodies at separation r: A_0 = m_1 r / (r^2 + eps)^(3/2), and with
    the polynomial switched off the force has exactly that magnitude."""
    fit = fit_fgrid(1.0 / 16)
    mass = np.array([0.7, 1.3], dtype=np.float32)
    zero = np.zeros(6, dtype=np.float32)
    e = float(np.float32(fit.eps))
    for frac in (0.05, 0.3, 0.7, 0.95):
        r = frac * float(np.float32(fit.r_cut))
        pos = _two_body(r)
        a0, an0, _ = oracle.force(pos, mass, -1.0, fit.r_cut, fit.eps, zero)
        _, an, _ = oracle.force(pos, mass, -1.0, fit.r_cut, fit.eps, fit.coeffs)
        d = pos[1] - pos[0]
        s = float(d @ d)
        closed = float(mass[1]) * math.sqrt(s) / (s + e) ** 1.5
        assert an[0] == pytest.approx(closed, rel=1e-13)
        assert an0[0] == pytest.approx(closed, rel=1e-13)      # independent of poly
        assert np.linalg.norm(a0[0]) == pytest.approx(an[0], rel=1e-13)


def test_newton_magnitude_equals_force_for_collinear_neighbours(oracle_lib):
    """With the polynomial off, pair forces on a particle whose neighbours all
    lie on one ray point the same way, so |a| equals their summed magnitude;
    for neighbours on both sides the magnitude is strictly larger."""
    fit = fit_fgrid(1.0 / 16)
    rc = float(np.float32(fit.r_cut))
    zero = np.zeros(6, dtype=np.float32)
    u = np.array([2.0, -1.0, 2.0]) / 3.0
    x0 = np.array([0.5, 0.5, 0.5])
    ts = np.array([0.1, 0.25, 0.5, 0.8, 0.97]) * rc
    pos = np.vstack([x0, x0 + ts[:, None] * u])
    mass = np.array([1.0, 0.5, 2.0, 1.5, 0.25, 3.0], dtype=np.float32)
    a, an, _ = oracle.force(pos, mass, -1.0, fit.r_cut, fit.eps, zero)
    assert np.linalg.norm(a[0]) == pytest.approx(an[0], rel=1e-13)
    pos2 = pos.copy()
    pos2[2] = x0 - ts[1] * u                                   # one neighbour flipped
    a2, an2, _ = oracle.force(pos2, mass, -1.0, fit.r_cut, fit.eps, zero)
    assert an2[0] == pytest.approx(an[0], rel=1e-13)
    assert np.linalg.norm(a2[0]) < 0.9 * an2[0]


def _single_pair_vjp(pos, mass, fit, poly, gj):
    """VJP on particle 0 of a two-body set with g_0 = 0 and g_1 = gj."""
    g = np.zeros((2, 3))
    g[1] = gj
    out, bn, pm = oracle.force_vjp(pos, mass, -1.0, fit.r_cut, fit.eps, poly, g,
                                   pair_floor=True)
    return out[0], bn[0], pm[0]


@pytest.mark.parametrize("frac", [0.02, 0.2, 0.5, 0.72, 0.85, 0.97])
def test_vjp_floors_from_single_pair_vjps(oracle_lib, frac):
    """For one pair, with g_0 = 0 so that w = m_0 g_1, the VJP on particle 0
    is f w + 2 f' (d.w) d.  With w perpendicular to d it is f w; with w along
    d it is (f + 2 f' s) w.  Running it with the polynomial on and off gives
    N, p, f' and p' times |w| as differences of VJP values, from which both
    floors follow:
      P = |a| + |b - a|
      B = a0 + |a0 - a| + (a0 - b0) + |(b0 - a0) - (b - a)|
    where a, b are the VJP components along w for w perpendicular and
    parallel to d, and a0, b0 the same with the polynomial off."""
    fit = fit_fgrid(1.0 / 16)
    rc = float(np.float32(fit.r_cut))
    zero = np.zeros(6, dtype=np.float32)
    axis = np.array([0.6, 0.0, 0.8])
    perp = np.array([0.0, 1.0, 0.0])
    pos = _two_body(frac * rc, axis)
    mass = np.array([0.7, 1.3], dtype=np.float32)
    wn = float(mass[0])                                       # |w| for a unit g_1
    o_perp, bn, pm = _single_pair_vjp(pos, mass, fit, fit.coeffs, perp)
    o_par, bn2, pm2 = _single_pair_vjp(pos, mass, fit, fit.coeffs, axis)
    o_perp0, _, _ = _single_pair_vjp(pos, mass, fit, zero, perp)
    o_par0, _, _ = _single_pair_vjp(pos, mass, fit, zero, axis)
    # the outputs lie along w
    for o, dirn in ((o_perp, perp), (o_par, axis), (o_perp0, perp), (o_par0, axis)):
        assert np.linalg.norm(o - (o @ dirn) * dirn) <= 1e-12 * np.linalg.norm(o) + 1e-300
    a, b = o_perp @ perp, o_par @ axis
    a0, b0 = o_perp0 @ perp, o_par0 @ axis
    p_expect = abs(a) + abs(b - a)
    b_expect = a0 + abs(a0 - a) + (a0 - b0) + abs((b0 - a0) - (b - a))
    assert bn == pytest.approx(bn2, rel=1e-14)                # |w| is the same
    assert pm == pytest.approx(p_expect, rel=1e-9)
    assert pm2 == pytest.approx(p_expect, rel=1e-9)
    assert bn == pytest.approx(b_expect, rel=1e-9)
    # with the polynomial off the two floors coincide: N (1 + 3 s/(s+eps)) |w|
    _, bz, pz = _single_pair_vjp(pos, mass, fit, zero, perp)
    assert bz == pytest.approx(pz, rel=1e-13)
    assert bz == pytest.approx(2 * a0 - b0, rel=1e-9)
    assert bz == pytest.approx(a0 / wn * wn * (1 + 3 * (frac * rc) ** 2
                                               / ((frac * rc) ** 2 + float(np.float32(fit.eps)))),
                               rel=1e-6)
