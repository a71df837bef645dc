"""Parity of the plain comparison kernels (one thread per target, global-memory
sources, branch cut-off, float64 sums) with the float64 oracle.

They are not the product path; these tests show that they compute the same
operation at the same accuracy as the tiled kernels, so that the speed of the
two can be compared at equal accuracy.  The per-pair arithmetic is the tiled
kernels' float32 formula and the sums are float64 (more accurate than the
tiled kernels' compensated float32 sums), so the tolerances are the tiled
kernels': forces 1e-5 and the VJP 1e-4 of the floored relative error, plus
the cut-off band for the VJP."""
import numpy as np
import pytest
import torch

import oracle
import paper_1211_4864_amd as hsr
from workloads import make_config, plummer_clustered, cotangent
from workloads.configs import _finish
from conftest import to_dev

pytestmark = pytest.mark.gpu
TOL_FORCE = 1e-5
TOL_VJP = 1e-4


def _clustered(n, grid, n_halo, seed, box=1.0):
    pos, meta = plummer_clustered(n, seed, n_halo, 0.6, 1.0 / grid)
    return _finish(f"plummer{n}_g{grid}", pos, seed, grid, meta, box=box)


CASES = [("cfg1", None), ("plummer", (1 << 16, 32, 40, 8, 1.0)),
         ("plummer_open", (1 << 15, 16, 6, 9, -1.0))]


def _workload(args):
    return make_config("cfg1") if args is None else _clustered(*args)


@pytest.mark.parametrize("name,args", CASES)
def test_force_plain_matches_oracle(cuda, name, args):
    w = _workload(args)
    pos, mass = to_dev(w, cuda)
    acc = hsr.force_plain(pos, mass, w.box, w.r_cut, w.eps, w.poly)
    torch.cuda.synchronize()
    got = acc.cpu().numpy().astype(np.float64)
    ref, an, _ = oracle.force(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly)
    err = oracle.rel_err_floored(got, ref, an)
    print(f"{w.name}: plain force max err {err.max():.3e}", flush=True)
    assert np.all(np.isfinite(got))
    assert err.max() <= TOL_FORCE


@pytest.mark.parametrize("name,args", CASES)
def test_vjp_plain_matches_oracle(cuda, name, args):
    w = _workload(args)
    g = cotangent(w.n, 4)
    pos, mass = to_dev(w, cuda)
    out = hsr.force_vjp_plain(pos, mass, w.box, w.r_cut, w.eps, w.poly,
                              torch.from_numpy(g).to(cuda))
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref, bn, amb = oracle.force_vjp(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly,
                                    g.astype(np.float64), cut_band=1e-6)
    dev = np.linalg.norm(got - ref, axis=1)
    lim = TOL_VJP * np.maximum(np.linalg.norm(ref, axis=1), 0.1 * bn) + amb
    clean = amb == 0.0
    err = oracle.rel_err_floored(got[clean], ref[clean], bn[clean])
    print(f"{w.name}: plain vjp max err off the cut {err.max():.3e} "
          f"(on the cut: {(~clean).sum()})", flush=True)
    assert np.all(np.isfinite(got))
    assert np.all(dev <= lim)
    assert err.max() <= TOL_VJP


def test_plain_agrees_with_tiled(cuda):
    """Same binning, same pair formula: the two forward kernels differ only
    in summation order, far inside the accuracy target."""
    w = _clustered(1 << 16, 32, 40, 8, 1.0)
    pos, mass = to_dev(w, cuda)
    a = hsr.force(pos, mass, w.box, w.r_cut, w.eps, w.poly).double()
    b = hsr.force_plain(pos, mass, w.box, w.r_cut, w.eps, w.poly).double()
    torch.cuda.synchronize()
    _, an, _ = oracle.force(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly)
    d = oracle.rel_err_floored(a.cpu().numpy(), b.cpu().numpy(), an)
    print(f"tiled vs plain: max floored difference {d.max():.3e}", flush=True)
    assert d.max() <= 2 * TOL_FORCE


def test_plain_empty_and_validation(cuda):
    w = make_config("cfg1")
    z = torch.empty((0, 3), dtype=torch.float64, device=cuda)
    zm = torch.empty((0,), dtype=torch.float32, device=cuda)
    assert hsr.force_plain(z, zm, w.box, w.r_cut, w.eps, w.poly).shape == (0, 3)
    pos, mass = to_dev(w, cuda)
    with pytest.raises(hsr.HaccSrError):
        hsr.force_plain(pos, mass, w.box, -w.r_cut, w.eps, w.poly)
