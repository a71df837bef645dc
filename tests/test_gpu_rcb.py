"""RCB fat leaves (Habib et al. 2012, Sec. III: recursive coordinate
bisection at the centre of mass along the longest side, leaves sharing one
interaction list) inside the chaining cells: the tree the GPU builds is
checked node by node against its definition, and the forces and VJP computed
with its leaves as work items against the float64 oracle, at the same
tolerances as the chaining-mesh path."""
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


def _clustered(n, grid, n_halo, seed, box=1.0):
    pos, meta = plummer_clustered(n, seed, n_halo, 0.6, 1.0 / grid)
    return _finish(f"plummer{n}_g{grid}", pos, seed, grid, meta, box=box)


def _check_tree(w, device, leaf_max):
    pos, mass = to_dev(w, device)
    cs_b, perm_b, rec_b = hsr.bin(pos, mass, w.box, w.r_cut)
    cs, perm, rec, ls, nodes, split = hsr.rcb_bin(pos, mass, w.box, w.r_cut, leaf_max,
                                                  with_nodes=True)
    torch.cuda.synchronize()
    cs_b, perm_b, rec_b = cs_b.cpu().numpy(), perm_b.cpu().numpy(), rec_b.cpu().numpy()
    cs, perm, rec = cs.cpu().numpy(), perm.cpu().numpy(), rec.cpu().numpy()
    ls, nodes, split = ls.cpu().numpy(), nodes.cpu().numpy(), split.cpu().numpy()
    n = w.n
    # same cells, same particles per cell, records travel with their particle
    assert np.array_equal(cs, cs_b)
    assert np.array_equal(np.sort(perm), np.arange(n))
    inv_b = np.empty(n, dtype=np.int64)
    inv_b[perm_b] = np.arange(n)
    assert np.array_equal(rec, rec_b[inv_b[perm]])
    cell_of = np.repeat(np.arange(cs.size - 1), np.diff(cs))
    assert np.array_equal(cell_of, np.repeat(np.arange(cs.size - 1), np.diff(cs_b)))
    assert np.array_equal(cell_of[inv_b[perm]], cell_of)
    # leaves tile every cell, at most leaf_max each
    assert ls[0] == 0 and ls[-1] == n and np.all(np.diff(ls) > 0)
    assert np.diff(ls).max() <= leaf_max
    occupied = cs[:-1][np.diff(cs) > 0]
    assert np.all(np.isin(occupied, ls))
    assert np.all(cell_of[ls[:-1]] == cell_of[ls[1:] - 1])
    # every internal node: split at the centre of mass along the longest side
    leaf_set = set(zip(ls[:-1].tolist(), np.diff(ls).tolist()))
    node_set = set(zip(nodes[:, 0].tolist(), nodes[:, 1].tolist()))
    assert len(node_set) == nodes.shape[0]
    index_cuts = 0
    for (b, c, left, axis), sp in zip(nodes, split):
        assert c > leaf_max and 0 < left < c
        r = rec[b:b + c, :3].astype(np.float64)
        m = rec[b:b + c, 3].astype(np.float64)
        ext = r.max(0) - r.min(0)
        com = (m[:, None] * r).sum(0) / m.sum()
        if axis == 3:
            index_cuts += 1
            assert left == c // 2
            rr = rec[b:b + c, int(np.argmax(ext))]
            assert np.all(rr < sp) or np.all(rr >= sp)
        else:
            assert ext[axis] >= ext.max() * (1 - 1e-6)
            # float32 sums: per-thread runs of c / 256 terms, then a tree
            tol = (c / 256 + 16) * 2.0 ** -23 * np.abs(r[:, axis]).max() + 1e-6 * ext[axis]
            assert abs(sp - com[axis]) <= tol
            assert np.all(rec[b:b + left, axis] < sp)
            assert np.all(rec[b + left:b + c, axis] >= sp)
        for cb, cc in ((b, left), (b + left, c - left)):
            assert ((cb, cc) in leaf_set) if cc <= leaf_max else ((cb, cc) in node_set)
    roots = [(int(cs[k]), int(cs[k + 1] - cs[k])) for k in range(cs.size - 1)
             if cs[k + 1] - cs[k] > leaf_max]
    assert all(rt in node_set for rt in roots)
    print(f"{w.name}: leaf_max {leaf_max}: {ls.size - 1} leaves, {nodes.shape[0]} nodes, "
          f"{index_cuts} index cuts, mean leaf {n / (ls.size - 1):.1f}", flush=True)
    return ls


@pytest.mark.parametrize("box", [1.0, -1.0])
@pytest.mark.parametrize("leaf_max", [64, 128])
def test_rcb_tree_structure(cuda, box, leaf_max):
    w = _clustered(1 << 16, 32, 40, 31, box=box)
    _check_tree(w, cuda, leaf_max)


def test_rcb_coincident_particles_and_tiny_leaves(cuda):
    """Coincident particles force index cuts; leaf_max 1 makes every particle
    a leaf of its own."""
    base = _clustered(1 << 12, 16, 4, 33)
    pos = np.concatenate([base.pos, np.repeat(base.pos[:3], 300, axis=0)], axis=0)
    w = _finish("coincident", pos, 33, 16, base.meta)
    ls = _check_tree(w, cuda, 16)
    assert ls.size > 1
    ls1 = _check_tree(_clustered(1 << 11, 16, 3, 34), cuda, 1)
    assert np.all(np.diff(ls1) == 1)


def _force_err(w, device, leaf_max, targets=None):
    pos, mass = to_dev(w, device)
    acc = hsr.force_rcb(pos, mass, w.box, w.r_cut, w.eps, w.poly, leaf_max)
    torch.cuda.synchronize()
    acc = acc.cpu().numpy().astype(np.float64)
    ref, an, _ = oracle.force(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly, targets=targets)
    sub = acc if targets is None else acc[targets]
    return oracle.rel_err_floored(sub, ref, an)


def _vjp_err(w, device, leaf_max, targets=None):
    pos, mass = to_dev(w, device)
    g = cotangent(w.n, 4)
    out = hsr.force_vjp_rcb(pos, mass, w.box, w.r_cut, w.eps, w.poly,
                            torch.from_numpy(g).to(device), leaf_max)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    ref, bn, amb = oracle.force_vjp(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly,
                                    g.astype(np.float64), targets=targets, cut_band=1e-6)
    sub = out if targets is None else out[targets]
    dev = np.linalg.norm(sub - ref, axis=1)
    assert np.all(dev <= 1e-4 * np.maximum(np.linalg.norm(ref, axis=1), 0.1 * bn) + amb)
    clean = amb == 0.0
    return oracle.rel_err_floored(sub[clean], ref[clean], bn[clean])


@pytest.mark.parametrize("leaf_max", [64, 128])
def test_rcb_force_vjp_cfg1_full(cuda, leaf_max):
    w = make_config("cfg1")
    fe = _force_err(w, cuda, leaf_max)
    ve = _vjp_err(w, cuda, leaf_max)
    print(f"cfg1 rcb {leaf_max}: force {fe.max():.3e} vjp {ve.max():.3e}", flush=True)
    assert fe.max() <= 1e-5 and ve.max() <= 1e-4


@pytest.mark.parametrize("box", [1.0, -1.0])
def test_rcb_force_vjp_clustered_full(cuda, box):
    w = _clustered(1 << 16, 32, 40, 35, box=box)
    fe = _force_err(w, cuda, 64)
    ve = _vjp_err(w, cuda, 64)
    print(f"{w.name} box {box}: force {fe.max():.3e} vjp {ve.max():.3e}", flush=True)
    assert fe.max() <= 1e-5 and ve.max() <= 1e-4


@pytest.mark.parametrize("name", ["cfg2", "cfg3s"])
def test_rcb_force_vjp_sampled(cuda, name):
    """cfg2 (128^3 Plummer-clustered) and the cfg3s stress block (a
    26000-particle cell), sampled targets, a quarter from the most
    populated cells."""
    w = make_config(name)
    keys = binning.chaining_mesh(w.pos, w.mass, w.box, w.r_cut)[0]
    tg = sample_targets(w.n, keys, 2000, seed=36)
    fe = _force_err(w, cuda, 64, tg)
    ve = _vjp_err(w, cuda, 64, tg)
    print(f"{name} rcb: force {fe.max():.3e} vjp {ve.max():.3e} on {tg.size} targets",
          flush=True)
    assert fe.max() <= 1e-5 and ve.max() <= 1e-4


def test_rcb_empty_and_validation(cuda):
    pos = torch.zeros((0, 3), dtype=torch.float64, device=cuda)
    mass = torch.zeros(0, dtype=torch.float32, device=cuda)
    out = hsr.force_rcb(pos, mass, 1.0, 0.1, 1e-5, [0] * 6)
    assert out.shape == (0, 3)
    cs, perm, rec, ls = hsr.rcb_bin(pos, mass, 1.0, 0.1)
    assert ls.cpu().tolist() == [0]
    w = _clustered(1 << 10, 16, 2, 37)
    p, m = to_dev(w, cuda)
    with pytest.raises(hsr.HaccSrError) as e:
        hsr.force_rcb(p, m, w.box, w.r_cut, w.eps, w.poly, leaf_max=0)
    assert e.value.code == -1
