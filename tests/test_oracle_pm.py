"""Pins for the float64 PM oracle (the long-range force of Habib et al. 2012,
Sec. II) against facts that do not come from its own pipeline: mass
conservation and the transpose relation of CIC deposit and interpolation,
momentum conservation, a uniform lattice, a single Fourier mode in closed
form, the Newtonian limit of a pair far apart, and the split itself: the
short-range kernel of Eq. 7 plus the PM pair force give the Newtonian force
across the matching scale."""
import numpy as np
import pytest

from oracle import pm
from workloads import fit_fgrid


def test_cic_conserves_mass_and_is_the_transpose_of_interpolation():
    rng = np.random.default_rng(1)
    box, ng = 2.0, 16
    pos = rng.random((500, 3)) * box * 3 - box       # outside the box too
    mass = rng.random(500) + 0.5
    grid = pm.cic_deposit(pos, mass, box, ng)
    assert grid.sum() == pytest.approx(mass.sum(), rel=1e-14)
    # on a grid point: all of the mass there
    D = box / ng
    g1 = pm.cic_deposit(np.array([[3 * D, 5 * D, 15 * D]]), np.array([2.0]), box, ng)
    assert g1[3, 5, 15] == 2.0 and g1.sum() == 2.0
    # <deposit(p, m), G> = m interp(G, p) for any grid G
    G = rng.standard_normal((ng, ng, ng))
    lhs = np.array([(pm.cic_deposit(p[None], np.array([1.0]), box, ng) * G).sum()
                    for p in pos[:20]])
    assert np.allclose(lhs, pm.cic_interpolate(G, pos[:20], box), rtol=1e-12, atol=1e-12)
    assert np.allclose(pm.cic_interpolate(np.full((ng,) * 3, 7.0), pos, box), 7.0)


def test_momentum_is_conserved():
    rng = np.random.default_rng(2)
    box, ng = 1.0, 32
    pos = rng.random((2000, 3))
    pos[:1000] = 0.5 + 0.05 * rng.standard_normal((1000, 3))
    mass = rng.random(2000) + 0.1
    a = pm.accel(pos, mass, box, ng)
    p = (mass[:, None] * a).sum(0)
    assert np.abs(p).max() <= 1e-12 * (mass[:, None] * np.abs(a)).sum()


def test_uniform_lattice_has_no_force():
    box, ng = 1.0, 16
    g = (np.arange(ng) + 0.5) / ng
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    a = pm.accel(pos, np.ones(len(pos)), box, ng)
    assert np.abs(a).max() <= 1e-10


@pytest.mark.parametrize("m0", [1, 3, 7])
def test_single_fourier_mode_in_closed_form(m0):
    """Particles on the grid points with masses 1 + A cos(k0 x): every
    operator of the pipeline is diagonal in Fourier space, so the
    acceleration is Phi D(k0) sin(k0 x) with Phi = -4 pi rho0 A S(k0) /
    K6(k0), rho0 the mean density."""
    box, ng, A = 1.0, 32, 0.3
    D = box / ng
    g = np.arange(ng) * D
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    k0 = 2 * np.pi * m0 / box
    mass = 1.0 + A * np.cos(k0 * pos[:, 0])
    a = pm.accel(pos, mass, box, ng)
    rho0 = 1.0 / D ** 3
    kd = k0 * D
    S = np.exp(-0.25 * (k0 * 0.8 * D) ** 2) * (np.sin(kd / 2) / (kd / 2)) ** 3
    K6 = (49 / 18 - 3 * np.cos(kd) + 0.3 * np.cos(2 * kd) - np.cos(3 * kd) / 45) / D ** 2
    Dk = (4 / 3 * np.sin(kd) - np.sin(2 * kd) / 6) / D
    phi = -4 * np.pi * rho0 * A * S / K6
    expect = phi * Dk * np.sin(k0 * pos[:, 0])
    scale = np.abs(expect).max()
    assert np.abs(a[:, 0] - expect).max() <= 1e-10 * scale
    assert np.abs(a[:, 1:]).max() <= 1e-10 * scale


def test_pair_far_apart_is_newtonian():
    """Two unit masses 6 grid cells apart in a 128-cell periodic box: the
    filtered PM force is the Newtonian one up to the smoothing (negligible at
    6 cells), the periodic images and the grid's anisotropy (a few tenths
    of a percent), and points along the separation."""
    box, ng = 1.0, 128
    D = box / ng
    rng = np.random.default_rng(3)
    for _ in range(4):
        x0 = rng.random(3)
        u = rng.standard_normal(3)
        u /= np.linalg.norm(u)
        r = 6.0 * D
        pos = np.stack([x0, x0 + r * u])
        a = pm.accel(pos, np.array([1.0, 0.0]), box, ng)
        # a massless test particle: the force on it from the unit mass
        got = a[1]
        newton = -u / r ** 2
        assert np.linalg.norm(got - newton) <= 0.02 * np.linalg.norm(newton)


def test_split_recovers_newtonian_force():
    """The short-range kernel is the Newtonian force minus the fitted grid
    force (Eq. 7).  With f_grid fitted to sampled PM pair forces, as the
    paper fits it, the PM pair force plus m f_SR(s) d is the (softened)
    Newtonian force again inside the matching scale, up to the grid's
    anisotropy (a few percent per pair, averaged here over orientations and
    offsets); at and beyond 3 cells the PM force alone is Newtonian."""
    box, ng = 1.0, 64
    D = box / ng
    r_cut = float(np.float32(3.0 * D))
    eps = float(np.float32(0.164 * D * D))
    c = pm.fit_grid_force(box, ng, r_cut, eps, seed=7).astype(np.float64)
    rng = np.random.default_rng(4)
    for rc in (0.75, 1.5, 2.0, 2.5, 3.5):
        r = rc * D
        tot = []
        for _ in range(16):
            x0 = rng.random(3)
            u = rng.standard_normal(3)
            u /= np.linalg.norm(u)
            pos = np.stack([x0, x0 + r * u])
            a_pm = pm.accel(pos, np.array([1.0, 0.0]), box, ng)[1]
            s = r * r
            fsr = ((s + eps) ** -1.5 - np.polynomial.polynomial.polyval(s, c)
                   if s < r_cut ** 2 else 0.0)
            a_sr = -fsr * r * u           # d = x_0 - x_1 = -r u, m_0 = 1
            tot.append(np.dot(a_pm + a_sr, -u) * r * r)
        mean = float(np.mean(tot))
        newton = r ** 3 / (r * r + eps) ** 1.5 if r < r_cut else 1.0
        assert mean == pytest.approx(newton, rel=0.03), (rc, mean, newton)


def test_gaussian_stand_in_differs_from_the_pm_fit():
    """The Gaussian-cloud stand-in for f_grid (workloads/fgrid.py) is weaker
    smoothing than this PM: inside 2 cells it overestimates the grid force
    by more than 10%; at the matching scale both equal the softened
    Newtonian term by construction."""
    box, ng = 1.0, 64
    D = box / ng
    fit = fit_fgrid(D)
    c_pm = pm.fit_grid_force(box, ng, fit.r_cut, fit.eps, seed=7).astype(np.float64)
    c_st = fit.coeffs.astype(np.float64)
    s = (np.array([1.0, 1.5]) * D) ** 2
    pv = np.polynomial.polynomial.polyval
    assert np.all(pv(s, c_st) > 1.1 * pv(s, c_pm))
    rc2 = float(np.float32(fit.r_cut)) ** 2
    assert pv(rc2, c_st) == pytest.approx(pv(rc2, c_pm), rel=1e-6)


def _full_case():
    from workloads import plummer_clustered
    box, ng = 1.0, 16
    D = box / ng
    pos, _ = plummer_clustered(3000, 61, 6, 0.6, D)
    rng = np.random.default_rng(62)
    # float32 masses, as the short-range force receives them, so that both
    # forces act on the same masses
    mass = ((rng.random(3000) + 0.5) / 3000).astype(np.float32).astype(np.float64)
    v = 0.3 * rng.standard_normal((3000, 3))
    r_cut = float(np.float32(3.0 * D))
    eps = float(np.float32(0.164 * D * D))
    poly = pm.fit_grid_force(box, ng, r_cut, eps, n_sources=4, per_source=1000, seed=3)
    return box, ng, pos, mass, v, r_cut, eps, poly


def test_full_step_is_time_reversible_and_conserves_momentum():
    """M_full is a symmetric composition of kicks and streams, so a step of
    dt followed by a step of -dt returns to the start; both forces conserve
    momentum, so the total momentum is unchanged."""
    from oracle import rollout
    box, ng, pos, mass, v, r_cut, eps, poly = _full_case()
    dt = 2e-3
    x1, v1 = rollout.full_step(pos, v, mass, box, ng, r_cut, eps, poly, dt, 3)
    x2, v2 = rollout.full_step(x1, v1, mass, box, ng, r_cut, eps, poly, -dt, 3)
    d = x2 - pos
    d -= np.rint(d / box) * box
    assert np.abs(d).max() <= 1e-12 and np.abs(v2 - v).max() <= 1e-10 * np.abs(v).max()
    # the momentum change is dt times the summed forces, zero up to their
    # rounding: bounded against dt times the summed force magnitudes
    from oracle import clib
    a_lr = pm.accel(pos, mass, box, ng)
    a_sr = clib.force(pos, mass.astype(np.float32), box, r_cut, eps, poly)[0]
    scale = dt * (mass[:, None] * (np.abs(a_lr) + np.abs(a_sr))).sum()
    p0 = (mass[:, None] * v).sum(0)
    p1 = (mass[:, None] * v1).sum(0)
    assert np.abs(p1 - p0).max() <= 1e-12 * scale + 1e-15 * (mass[:, None] * np.abs(v)).sum()


def test_full_step_reduces_to_its_parts():
    """With n_c = 1 the full step is kick(dt/2, PM) stream(dt/2)
    kick(dt, SR) stream(dt/2) kick(dt/2, PM), composed here by hand from
    the oracle's maps."""
    from oracle import rollout, clib
    box, ng, pos, mass, v, r_cut, eps, poly = _full_case()
    dt = 1e-3
    x1, v1 = rollout.full_step(pos, v, mass, box, ng, r_cut, eps, poly, dt, 1)
    vv = v + 0.5 * dt * pm.accel(pos, mass, box, ng)
    xx = pos + 0.5 * dt * vv
    xx -= np.floor(xx / box) * box
    vv = vv + dt * clib.force(xx, mass.astype(np.float32), box, r_cut, eps, poly)[0]
    xx = xx + 0.5 * dt * vv
    xx -= np.floor(xx / box) * box
    vv = vv + 0.5 * dt * pm.accel(xx, mass, box, ng)
    assert np.abs(x1 - xx).max() <= 1e-13 and np.abs(v1 - vv).max() <= 1e-12
