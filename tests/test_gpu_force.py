"""Parity of the HIP forward path (binning, work list, pair kernel) with the
float64 oracle.  Tolerance: per particle |a - a*| <= 1e-5 max(|a*|, 0.1 A),
A the particle's summed Newtonian pair magnitude (the relative error,
floored where pair terms cancel)."""
import numpy as np
import pytest
import torch

import oracle
from oracle import binning
import paper_1211_4864_amd as hsr
from workloads import make_config, plummer_clustered, nfw_clustered, fit_fgrid
from workloads.configs import Workload, _finish
from conftest import to_dev, sample_targets

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _gpu_acc(w, device):
    pos, mass = to_dev(w, device)
    acc = hsr.force(pos, mass, w.box, w.r_cut, w.eps, w.poly)
    torch.cuda.synchronize()
    return acc.cpu().numpy().astype(np.float64)


def _check(w, acc, targets=None):
    ref, an, _ = oracle.force(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly, targets=targets)
    got = acc if targets is None else acc[targets]
    err = oracle.rel_err_floored(got, ref, an)
    raw = np.linalg.norm(got - ref, axis=1) / np.maximum(np.linalg.norm(ref, axis=1), 1e-300)
    print(f"{w.name}: n={w.n} checked={got.shape[0]} max err={err.max():.3e} "
          f"median raw rel={np.median(raw):.3e} p99 raw={np.quantile(raw, 0.99):.3e}",
          flush=True)
    assert np.all(np.isfinite(got))
    assert err.max() <= TOL
    return err


def _clustered(n, grid, n_halo, seed, box=1.0):
    pos, meta = plummer_clustered(n, seed, n_halo, 0.6, 1.0 / grid)
    return _finish(f"plummer{n}_g{grid}", pos, seed, grid, meta, box=box)


@pytest.mark.parametrize("box", [1.0, -1.0])
def test_binning_matches_reference_order(cuda, box):
    w = _clustered(1 << 16, 32, 40, 7, box=box)
    pos, mass = to_dev(w, cuda)
    cs, perm, rec = hsr.bin(pos, mass, w.box, w.r_cut)
    torch.cuda.synchronize()
    keys, p_ref, cs_ref, rec_ref = binning.chaining_mesh(w.pos, w.mass, w.box, w.r_cut)
    assert np.array_equal(cs.cpu().numpy(), cs_ref)
    assert np.array_equal(perm.cpu().numpy(), p_ref)
    assert np.array_equal(rec.cpu().numpy().view(np.uint32), rec_ref.view(np.uint32))


def test_force_cfg1_full(cuda):
    w = make_config("cfg1")
    _check(w, _gpu_acc(w, cuda))


@pytest.mark.parametrize("grid,n_halo,seed", [(32, 40, 8), (16, 6, 9), (48, 300, 10)])
def test_force_clustered_full(cuda, grid, n_halo, seed):
    """Dense cells (several LDS tiles per item, ragged tails) on sets the
    oracle finishes in seconds."""
    w = _clustered(1 << 16, grid, n_halo, seed)
    _check(w, _gpu_acc(w, cuda))


def test_force_nfw_open_full(cuda):
    pos, meta = nfw_clustered(1 << 16, 12, 80, 0.7, 1.0 / 32)
    w = _finish("nfw_open", pos * 0.98 + 0.01, 12, 32, meta, box=-1.0)
    _check(w, _gpu_acc(w, cuda))


def _keys(w):
    return binning.chaining_mesh(w.pos, w.mass, w.box, w.r_cut)[0]


def test_force_cfg2_full(cuda):
    """The 128^3 Plummer-clustered workload, every particle against the
    oracle (1.35e9 in-cut-off pairs; about half a minute of oracle time on
    16 host cores)."""
    w = make_config("cfg2")
    _check(w, _gpu_acc(w, cuda))


def test_force_cfg3_sampled(cuda):
    """The 256^3 NFW-clustered workload at the benchmark's launch shape."""
    w = make_config("cfg3")
    acc = _gpu_acc(w, cuda)
    _check(w, acc, sample_targets(w.n, _keys(w), 2000, seed=3))
    # properties that hold at any size: every particle finite, third law
    m = w.mass.astype(np.float64)[:, None]
    mom = np.abs((m * acc).sum(0))
    assert np.all(np.isfinite(acc))
    assert np.all(mom <= 1e-6 * (m * np.abs(acc)).sum(0))


def test_force_stress_block_sampled(cuda):
    """The 256^3 workload with its ten most massive halos moved into one
    2x2x2-cell block: one chaining cell holds ~26000 particles.  A quarter of
    the checked targets come from the most populated cells."""
    w = make_config("cfg3s")
    keys = _keys(w)
    assert np.bincount(keys).max() > 10_000
    acc = _gpu_acc(w, cuda)
    _check(w, acc, sample_targets(w.n, keys, 2000, seed=31))
    m = w.mass.astype(np.float64)[:, None]
    assert np.all(np.isfinite(acc))
    assert np.all(np.abs((m * acc).sum(0)) <= 1e-6 * (m * np.abs(acc)).sum(0))


def test_ghost_shell_interior_matches_periodic(cuda):
    """Open domain with a periodic-image ghost shell gives the periodic
    forces on the active particles (particle overloading)."""
    w5 = make_config("cfg5_32")
    n_act = w5.meta["n_active"]
    a_open = _gpu_acc(w5, cuda)[:n_act]
    per = Workload("per", w5.pos[:n_act] - w5.meta["shell"], w5.mass[:n_act], 1.0,
                   w5.r_cut, w5.eps, w5.poly, w5.cell, w5.seed, w5.fit, {})
    per.pos = per.pos - np.floor(per.pos)
    a_per = _gpu_acc(per, cuda)
    ref, an, _ = oracle.force(per.pos, per.mass, 1.0, per.r_cut, per.eps, per.poly)
    assert oracle.rel_err_floored(a_open, ref, an).max() <= TOL
    assert oracle.rel_err_floored(a_per, ref, an).max() <= TOL


def test_runs_on_the_callers_stream(cuda):
    """The library launches on torch's current stream: results on a side
    stream equal those on the default stream, and the side stream's work
    is ordered after the inputs it waits for."""
    w = _clustered(1 << 15, 64, 30, 17)
    a_default = _gpu_acc(w, cuda)
    side = torch.cuda.Stream(device=cuda)          # default priority
    pos, mass = to_dev(w, cuda)
    side.wait_stream(torch.cuda.current_stream(cuda))
    with torch.cuda.stream(side):
        acc = hsr.force(pos, mass, w.box, w.r_cut, w.eps, w.poly)
        g = torch.ones((w.n, 3), dtype=torch.float32, device=cuda)
        gpos = hsr.force_vjp(pos, mass, w.box, w.r_cut, w.eps, w.poly, g)
    side.synchronize()
    assert np.array_equal(acc.cpu().numpy().astype(np.float64), a_default)
    g0 = torch.ones((w.n, 3), dtype=torch.float32, device=cuda)
    gpos0 = hsr.force_vjp(pos, mass, w.box, w.r_cut, w.eps, w.poly, g0)
    torch.cuda.synchronize()
    assert np.array_equal(gpos.cpu().numpy(), gpos0.cpu().numpy())


def test_reproducible_and_integer_cell_translation(cuda):
    # r_cut = 3/192 = 1/64 gives 64 chaining cells of exact side 2^-6: an
    # integer-cell shift in x and y leaves every cell-relative coordinate and
    # the whole work decomposition unchanged
    w = _clustered(1 << 15, 192, 30, 13)
    assert hsr.grid_dim(1.0, w.r_cut) == 64
    a1 = _gpu_acc(w, cuda)
    a2 = _gpu_acc(w, cuda)
    assert np.array_equal(a1, a2)
    shifted = Workload("shift", (w.pos + np.array([5 / 64, 17 / 64, 0.0])) % 1.0, w.mass,
                       w.box, w.r_cut, w.eps, w.poly, w.cell, w.seed, w.fit, {})
    a3 = _gpu_acc(shifted, cuda)
    assert np.array_equal(a1, a3)
    shifted.pos = (w.pos + np.array([0.0, 0.0, 0.3141])) % 1.0
    a4 = _gpu_acc(shifted, cuda)
    ref, an, _ = oracle.force(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly)
    assert oracle.rel_err_floored(a4, ref, an).max() <= TOL


def test_edge_cases(cuda):
    fit = fit_fgrid(1.0 / 128)
    mass1 = np.ones(1, np.float32)
    # one particle, isolated particles: exactly zero
    one = Workload("one", np.array([[0.3, 0.4, 0.5]]), mass1, 1.0, fit.r_cut, fit.eps,
                   fit.coeffs, fit.cell, 0, fit, {})
    assert np.all(_gpu_acc(one, cuda) == 0.0)
    iso = np.array([[0.1, 0.1, 0.1], [0.5, 0.5, 0.5], [0.5 + 0.5 * fit.r_cut, 0.5, 0.5],
                    [0.9, 0.2, 0.6]])
    w = Workload("iso", iso, np.ones(4, np.float32), 1.0, fit.r_cut, fit.eps, fit.coeffs,
                 fit.cell, 0, fit, {})
    a = _gpu_acc(w, cuda)
    assert np.all(a[0] == 0.0) and np.all(a[3] == 0.0)
    _check(w, a)
    # every particle in one cell (one item per 64 targets, thousands of sources)
    rng = np.random.default_rng(4)
    dense = 0.5 + rng.random((3000, 3)) * fit.r_cut * 0.9
    w = Workload("dense", dense, np.full(3000, np.float32(1 / 3000)), 1.0, fit.r_cut,
                 fit.eps, fit.coeffs, fit.cell, 0, fit, {})
    _check(w, _gpu_acc(w, cuda))
    # the smallest periodic box (3 cells per axis) and open boxes of 1 and 2 cells
    for box, scale in ((3.1 * fit.r_cut, 3.1), (-1.5 * fit.r_cut, 1.5), (-2.5 * fit.r_cut, 2.5)):
        p = rng.random((500, 3)) * scale * fit.r_cut
        w = Workload("small", p, np.full(500, np.float32(1 / 500)), box, fit.r_cut, fit.eps,
                     fit.coeffs, fit.cell, 0, fit, {})
        _check(w, _gpu_acc(w, cuda))
    # positions outside the periodic box are wrapped; a coordinate equal to the box is 0
    p = rng.random((2000, 3))
    w = Workload("wrap", p, np.full(2000, np.float32(1 / 2000)), 1.0, fit.r_cut, fit.eps,
                 fit.coeffs, fit.cell, 0, fit, {})
    base = _gpu_acc(w, cuda)
    w.pos = p + rng.integers(-3, 4, p.shape)
    w.pos[0] = [1.0, 0.5, 0.5]
    moved = _gpu_acc(w, cuda)
    w.pos = p.copy()
    w.pos[0] = [0.0, 0.5, 0.5]
    ref_moved = _gpu_acc(w, cuda)
    assert np.allclose(moved[1:], base[1:], rtol=1e-5, atol=1e-5 * np.abs(base).max())
    assert np.allclose(moved[0], ref_moved[0], rtol=1e-5, atol=1e-5 * np.abs(base).max())


def _mixed_masses(w, seed, frac=1.0):
    """Masses 10^U(-1, 1) / n on a fraction of the particles (the rest keep
    1/n): every pair kernel round with an unequal mass takes the general
    path, the others the equal-mass one."""
    rng = np.random.default_rng(seed)
    m = np.full(w.n, np.float32(1.0 / w.n))
    pick = rng.random(w.n) < frac
    m[pick] = (10.0 ** rng.uniform(-1.0, 1.0, int(pick.sum())) / w.n).astype(np.float32)
    w.mass = m
    return w


@pytest.mark.parametrize("frac,box", [(1.0, 1.0), (0.01, 1.0), (1.0, -1.0)])
def test_force_unequal_masses(cuda, frac, box):
    """General (unequal-mass) path of the pair kernel, alone and mixed with
    equal-mass rounds."""
    w = _mixed_masses(_clustered(1 << 16, 32, 40, 15, box=box), 16, frac)
    _check(w, _gpu_acc(w, cuda))


@pytest.mark.parametrize("cells", [4, 5, 6])
def test_small_periodic_boxes_with_runs(cuda, cells):
    """Boxes of 4 to 6 chaining cells per axis, sparse enough that pairs of
    cells along z merge into runs, with runs that wrap around the periodic
    boundary in their windows; unequal masses."""
    fit = fit_fgrid(0.999 / (3 * cells))      # r_cut just below 1 / cells
    assert hsr.grid_dim(1.0, fit.r_cut) == cells
    rng = np.random.default_rng(20 + cells)
    n = 3 * cells ** 3
    w = Workload("runs", rng.random((n, 3)), np.full(n, np.float32(1.0 / n)), 1.0,
                 fit.r_cut, fit.eps, fit.coeffs, fit.cell, 0, fit, {})
    w = _mixed_masses(w, 30 + cells)
    _check(w, _gpu_acc(w, cuda))


def test_pair_counts(cuda):
    w = _clustered(1 << 16, 32, 40, 14)
    pos, _ = to_dev(w, cuda)
    cand, inside = hsr.count_pairs(pos, w.box, w.r_cut, w.eps)
    _, _, cnt = oracle.force(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly)
    # the in-cut-off decision is taken in float32 on the GPU: only pairs within
    # rounding of r_cut may differ
    assert abs(inside - int(cnt.sum())) <= 4
    keys, perm, cs, _ = binning.chaining_mesh(w.pos, w.mass, w.box, w.r_cut)
    N, _ = binning.grid(w.box, w.r_cut)
    occ = np.diff(cs).reshape(N, N, N)
    # the kernel evaluates each item's source window (the 3 x 3 x (zlen + 2)
    # cells around its run of cells) minus the sources the staging cull
    # proves to be out of range
    assert inside <= cand <= window_pairs(occ, periodic=True)


def window_pairs(occ, periodic, zrun=4, item=64):
    """Sum over targets of their item's window size minus one, for the run
    rule of the work list: an aligned block of `zrun` cells along z (at most
    N - 2 of them in a periodic box) holding at most `item` targets is one
    run, every other cell is a run of its own."""
    N = occ.shape[0]

    def window(x, y, z0, n):
        win = 0
        for a in (-1, 0, 1):
            for b in (-1, 0, 1):
                for c in range(-1, n + 1):
                    xx, yy, zz = x + a, y + b, z0 + c
                    if periodic:
                        win += occ[xx % N, yy % N, zz % N]
                    elif 0 <= xx < N and 0 <= yy < N and 0 <= zz < N:
                        win += occ[xx, yy, zz]
        return int(win)

    total = 0
    for x in range(N):
        for y in range(N):
            col = occ[x, y]
            for z0 in range(0, N, zrun):
                block = min(zrun, N - z0)
                zl = min(block, N - 2) if periodic else block
                runs = []
                if zl >= 2 and col[z0:z0 + zl].sum() <= item:
                    runs.append((z0, zl))
                    runs += [(z, 1) for z in range(z0 + zl, z0 + block)]
                else:
                    runs = [(z, 1) for z in range(z0, z0 + block)]
                for z, n in runs:
                    t = int(col[z:z + n].sum())
                    if t:
                        total += t * (window(x, y, z, n) - 1)
    return total
