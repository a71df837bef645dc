"""Parity of the HIP adjoint (VJP) kernel and the autograd wrapper with the
float64 oracle's VJP, and with central finite differences of the oracle's
forward sum.  Tolerance: |g - g*| <= 1e-4 max(|g*|, 0.1 B) + J, B the summed
magnitude of the Newtonian and grid-polynomial parts of that particle's pair
terms (the VJP's analogue of the force's Newtonian floor) and J the magnitude
of its pair terms within 1e-6 r_cut^2 of the cut-off.  f' jumps at r_cut, so a pair on the cut
contributes fully or not at all depending on the precision of the cut-off
test (float32 in the kernel, as the paper's single-precision short-range
force; float64 in the oracle).  J is zero for almost every particle."""
import numpy as np
import pytest
import torch

import oracle
import paper_1211_4864_amd as hsr
from workloads import make_config, plummer_clustered, cotangent
from workloads.configs import _finish
from conftest import to_dev, sample_targets
from oracle import binning

pytestmark = pytest.mark.gpu
TOL = 1e-4


def _clustered(n, grid, n_halo, seed, box=1.0):
    pos, meta = plummer_clustered(n, seed, n_halo, 0.6, 1.0 / grid)
    return _finish(f"plummer{n}_g{grid}", pos, seed, grid, meta, box=box)


def _gpu_vjp(w, g, device):
    pos, mass = to_dev(w, device)
    gt = torch.from_numpy(g).to(device)
    out = hsr.force_vjp(pos, mass, w.box, w.r_cut, w.eps, w.poly, gt)
    torch.cuda.synchronize()
    return out.cpu().numpy()


BAND = 1e-6


def _check(w, g, got, targets=None, pair_floor_tol=None):
    """Asserts the VJP error under the floor B (Newtonian and polynomial parts
    before they cancel) and reports it under the tighter floor P (the pair
    terms' own magnitudes (|f| + 2|f'| s)|w|); with pair_floor_tol, also
    asserts the error under P.  Returns the max errors under B and P."""
    ref, bn, amb, pm = oracle.force_vjp(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly,
                                        g.astype(np.float64), targets=targets,
                                        cut_band=BAND, pair_floor=True)
    sub = got if targets is None else got[targets]
    dev = np.linalg.norm(sub - ref, axis=1)
    lim = TOL * np.maximum(np.linalg.norm(ref, axis=1), 0.1 * bn) + amb
    clean = amb == 0.0
    err = oracle.rel_err_floored(sub[clean], ref[clean], bn[clean])
    perr = oracle.rel_err_floored(sub[clean], ref[clean], pm[clean])
    worst = int(np.argmax(perr)) if perr.size else 0
    print(f"{w.name}: vjp checked={sub.shape[0]} (on the cut: {(~clean).sum()}) "
          f"max err off the cut={err.max():.3e}; under the pair-term floor "
          f"max {perr.max():.3e}, {(perr > TOL).sum()} above {TOL:g} "
          f"(worst: B/P = {bn[clean][worst] / max(pm[clean][worst], 1e-300):.1f})",
          flush=True)
    assert np.all(np.isfinite(sub))
    assert np.all(dev <= lim)
    assert err.max() <= TOL
    if pair_floor_tol is not None:
        assert perr.max() <= pair_floor_tol
    return float(err.max()), float(perr.max())


@pytest.mark.parametrize("box", [1.0, -1.0])
def test_vjp_clustered_full(cuda, box):
    w = _clustered(1 << 16, 32, 40, 21, box=box)
    g = cotangent(w.n, 4)
    _check(w, g, _gpu_vjp(w, g, cuda))


def test_vjp_stress_block_sampled(cuda):
    """VJP on the 256^3 workload with ten massive halos in one 2x2x2-cell
    block (one cell of ~26000 particles), on sampled targets, a quarter of
    them from the most populated cells."""
    w = make_config("cfg3s")
    keys = binning.chaining_mesh(w.pos, w.mass, w.box, w.r_cut)[0]
    g = cotangent(w.n, 4)
    _check(w, g, _gpu_vjp(w, g, cuda), sample_targets(w.n, keys, 1000, seed=32))


@pytest.mark.parametrize("frac", [1.0, 0.01])
def test_vjp_unequal_masses(cuda, frac):
    """General (unequal-mass) path of the VJP kernel, alone and mixed with
    equal-mass rounds."""
    w = _clustered(1 << 16, 32, 40, 22)
    rng = np.random.default_rng(23)
    m = np.full(w.n, np.float32(1.0 / w.n))
    pick = rng.random(w.n) < frac
    m[pick] = (10.0 ** rng.uniform(-1.0, 1.0, int(pick.sum())) / w.n).astype(np.float32)
    w.mass = m
    g = cotangent(w.n, 4)
    _check(w, g, _gpu_vjp(w, g, cuda))


def test_vjp_coincident_unequal_masses_small_eps(cuda):
    """Unequal masses with a small softening (1e-3 cell^2) and pairs of
    distinct particles at exactly the same position.  A coincident pair has
    d = 0, so its VJP term is f(0) w with f(0) = eps^(-3/2) - c_0 large; the
    self pair must contribute exactly nothing (w = 0), which with this eps
    would otherwise show even as a rounding residual of m_k g_k."""
    base = _clustered(1 << 14, 32, 12, 24)
    rng = np.random.default_rng(25)
    dup = rng.choice(base.n, 400, replace=False)
    pos = np.concatenate([base.pos, base.pos[dup]], axis=0)
    w = _finish("coincident", pos, 24, 32, base.meta, eps_cells2=1e-3)
    m = (10.0 ** rng.uniform(-1.0, 1.0, w.n) / w.n).astype(np.float32)
    w.mass = m
    g = cotangent(w.n, 26)
    _check(w, g, _gpu_vjp(w, g, cuda))
    # The forward on the same set: coincident pairs contribute d = 0.  With a
    # softening this small the float32 frame coordinates (absolute error up
    # to 2^-24 of two cell sides) are coarse against the softening length:
    # a pair at s ~ eps has a relative separation error up to 2^-23 Lc /
    # sqrt(eps), 1.2e-5 here (9.4e-7 at the workloads' 0.164 cell^2), so the
    # bound is the larger of that and 1e-5.
    ref, an, _ = oracle.force(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly)
    pos_t, mass_t = to_dev(w, cuda)
    acc = hsr.force(pos_t, mass_t, w.box, w.r_cut, w.eps, w.poly).cpu().numpy()
    lc = abs(w.box) / hsr.grid_dim(w.box, w.r_cut)
    bound = max(1e-5, 2.0 ** -23 * lc / np.sqrt(float(np.float32(w.eps))))
    err = oracle.rel_err_floored(acc, ref, an).max()
    print(f"coincident forward: max err {err:.3e} (bound {bound:.3e})", flush=True)
    assert err <= bound


def test_vjp_cfg4_full_and_finite_differences(cuda):
    """128^3 clustered particles, g ~ N(0,1): VJP vs the oracle VJP on every
    particle (about a minute of oracle time on 16 host cores) and vs central
    differences (h = 1e-4 cell, float64 on the oracle) on 64 random
    particles."""
    w = make_config("cfg4")
    g = w.meta["g"]
    got = _gpu_vjp(w, g, cuda)
    _check(w, g, got)
    assert np.abs(got.sum(0)).max() <= 1e-5 * np.abs(got).sum()
    rng = np.random.default_rng(64)
    ks = rng.choice(w.n, 64, replace=False)
    h = 1e-4 * w.cell
    rc = float(np.float32(w.r_cut))
    gd = g.astype(np.float64)
    _, bn = oracle.force_vjp(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly, gd, targets=ks)
    checked = 0
    for t, k in enumerate(ks):
        d = w.pos - w.pos[k]
        d -= np.rint(d)
        r = np.sqrt((d * d).sum(1))
        r[k] = -1
        if np.any(np.abs(r - rc) < 3 * h):
            continue                      # a pair crosses the cut-off within the probe
        # L changes only through a_k and the accelerations of k's neighbours
        idx = np.unique(np.concatenate([[k], np.nonzero(r < rc + 3 * h)[0]]))
        for ax in range(3):
            vals = []
            for s in (h, -h):
                p = w.pos.copy()
                p[k, ax] += s
                a, _, _ = oracle.force(p, w.mass, w.box, w.r_cut, w.eps, w.poly, targets=idx)
                vals.append(float(np.sum(gd[idx] * a)))
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(got[k, ax] - fd) <= TOL * max(abs(fd), 0.1 * bn[t]) + 1e-9 * bn[t]
            checked += 1
    assert checked >= 120


def test_autograd_matches_vjp_and_dot_product(cuda):
    w = _clustered(1 << 15, 32, 30, 22)
    pos, mass = to_dev(w, cuda)
    pos.requires_grad_(True)
    acc = hsr.sr_force(pos, mass, w.box, w.r_cut, w.eps, w.poly)
    g = torch.from_numpy(cotangent(w.n, 5)).to(cuda)
    (grad,) = torch.autograd.grad((acc * g).sum(), pos)
    direct = hsr.force_vjp(pos.detach(), mass, w.box, w.r_cut, w.eps, w.poly, g)
    assert torch.equal(grad, direct)
    # <g, J v> by a float64 directional difference of the oracle equals <J^T g, v>
    v = np.random.default_rng(6).standard_normal(w.pos.shape)
    h = 1e-6 * w.cell
    gd = g.cpu().numpy().astype(np.float64)
    ap, _, _ = oracle.force(w.pos + h * v, w.mass, w.box, w.r_cut, w.eps, w.poly)
    am, _, _ = oracle.force(w.pos - h * v, w.mass, w.box, w.r_cut, w.eps, w.poly)
    lhs = float(np.sum(gd * (ap - am))) / (2 * h)
    rhs = float(np.sum(grad.cpu().numpy() * v))
    assert abs(lhs - rhs) <= 1e-4 * np.abs(grad.cpu().numpy() * v).sum()


def test_vjp_linear_in_cotangent_and_reproducible(cuda):
    w = _clustered(1 << 15, 32, 30, 23)
    g1 = cotangent(w.n, 7)
    a = _gpu_vjp(w, g1, cuda)
    b = _gpu_vjp(w, g1, cuda)
    assert np.array_equal(a, b)
    c = _gpu_vjp(w, (2.0 * g1).astype(np.float32), cuda)
    assert np.array_equal(c, 2.0 * a)            # scaling by 2 is exact in float32
