"""The allocation-free force entry point (hacc_sr_force_noalloc), called
through the C ABI: its output equals hacc_sr_force's on two calls in a row,
the second with a smaller input (its scratch array keeps the first call's
contents), and both meet the oracle's tolerance; sizes beyond its scratch
array are refused before any GPU work."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_1211_4864_amd as hsr
from paper_1211_4864_amd import _lib
from workloads import plummer_clustered
from workloads.configs import _finish

pytestmark = pytest.mark.gpu


def _noalloc(lib, pos, mass, w, out):
    stream = torch.cuda.current_stream(pos.device)
    _lib.check(lib.hacc_sr_set_stream(ctypes.c_void_p(stream.cuda_stream)))
    return lib.hacc_sr_force_noalloc(
        ctypes.c_void_p(pos.data_ptr()), ctypes.c_void_p(mass.data_ptr()), pos.shape[0],
        float(w.box), float(w.r_cut), float(w.eps), _lib.poly_array(w.poly),
        ctypes.c_void_p(out.data_ptr()))


def test_noalloc_matches_force_twice(cuda):
    lib = hsr.load()
    results = []
    for n, seed in ((1 << 17, 41), (40000, 42)):
        pos_np, meta = plummer_clustered(n, seed, 30, 0.6, 1.0 / 32)
        w = _finish(f"noalloc{n}", pos_np, seed, 32, meta)
        pos = torch.from_numpy(w.pos).to(cuda)
        mass = torch.from_numpy(w.mass).to(cuda)
        ref = hsr.force(pos, mass, w.box, w.r_cut, w.eps, w.poly)
        out = torch.full((n, 3), float("nan"), dtype=torch.float32, device=cuda)
        assert _noalloc(lib, pos, mass, w, out) == 0
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        assert np.array_equal(got, ref.cpu().numpy())
        a, an, _ = oracle.force(w.pos, w.mass, w.box, w.r_cut, w.eps, w.poly)
        err = oracle.rel_err_floored(got.astype(np.float64), a, an).max()
        print(f"noalloc n={n}: bitwise equal to hacc_sr_force, oracle err {err:.3e}",
              flush=True)
        assert err <= 1e-5
        results.append(got)


def test_noalloc_refuses_oversize(cuda):
    lib = hsr.load()
    n = 1 << 24
    pos = torch.zeros((1, 3), dtype=torch.float64, device=cuda)
    mass = torch.zeros(1, dtype=torch.float32, device=cuda)
    out = torch.zeros((1, 3), dtype=torch.float32, device=cuda)

    class W:
        box, r_cut, eps, poly = 1.0, 3.0 / 256, 2.5e-6, [0.0] * 6

    # the size check runs on the host before any launch (n is only compared)
    rc = lib.hacc_sr_force_noalloc(ctypes.c_void_p(pos.data_ptr()),
                                   ctypes.c_void_p(mass.data_ptr()), n, W.box,
                                   W.r_cut, W.eps, _lib.poly_array(W.poly),
                                   ctypes.c_void_p(out.data_ptr()))
    assert rc == _lib.ENOSPACE
