"""The VJP on a kept binning (hacc_sr_force_vjp_binned): the reverse pass of a
stream-kick-stream subcycle (Habib et al. 2012, Sec. II, Eq. 6) takes the
force derivative at the position where the forward pass evaluated the force
(Sec. III, Eq. 7), so it may reuse that call's binning.  The result must be
bitwise the VJP that bins again, the token must be refused once anything
else has written the workspace, and the VJP must be taken at the binned
positions, whatever happened to the position array since."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1211_4864_amd as hsr
from paper_1211_4864_amd import _lib
from workloads import plummer_clustered, cotangent
from workloads.configs import _finish
from conftest import to_dev

pytestmark = pytest.mark.gpu


def _workload(n=1 << 15, seed=31, box=1.0):
    pos, meta = plummer_clustered(n, seed, 25, 0.6, 1.0 / 32)
    return _finish(f"plummer{n}_g32", pos, seed, 32, meta, box=box)


def _binned_rc(token, w, g, out):
    return _lib.load().hacc_sr_force_vjp_binned(
        int(token), w.n, float(w.box), float(w.r_cut), float(w.eps),
        _lib.poly_array(w.poly), ctypes.c_void_p(g.data_ptr()),
        ctypes.c_void_p(out.data_ptr()))


@pytest.mark.parametrize("box", [1.0, -1.0])
def test_binned_vjp_bitwise_and_skips_binning(cuda, box):
    w = _workload(box=box)
    pos, mass = to_dev(w, cuda)
    g = torch.from_numpy(cotangent(w.n, 32)).to(cuda)
    ref = hsr.force_vjp(pos, mass, w.box, w.r_cut, w.eps, w.poly, g)
    hsr.force(pos, mass, w.box, w.r_cut, w.eps, w.poly)
    token = hsr.binning_token()
    assert token > 0
    torch.cuda.synchronize()
    hsr.timing_enable(True)
    got = hsr.force_vjp(pos, mass, w.box, w.r_cut, w.eps, w.poly, g, binned=token)
    torch.cuda.synchronize()
    n_w, _ = hsr.timing_read(hsr.TIMER_WORKLIST)
    n_v, _ = hsr.timing_read(hsr.TIMER_VJP)
    hsr.timing_enable(False)
    assert n_v == 1 and n_w == 0            # the pair kernel ran, no new work list
    assert torch.equal(got, ref)
    # the token stays valid after the binned VJP: a second one is the same
    again = hsr.force_vjp(pos, mass, w.box, w.r_cut, w.eps, w.poly, g, binned=token)
    assert torch.equal(again, ref)
    print(f"binned vjp box {box}: bitwise equal, token {token}", flush=True)


def test_binned_vjp_uses_the_binned_positions(cuda):
    """After the force call the position array moves (a stream); the binned
    VJP is still the VJP at the positions of the force call."""
    w = _workload(seed=33)
    pos, mass = to_dev(w, cuda)
    g = torch.from_numpy(cotangent(w.n, 34)).to(cuda)
    x = pos.clone()
    hsr.force(x, mass, w.box, w.r_cut, w.eps, w.poly)
    token = hsr.binning_token()
    v = torch.full_like(x, 0.3)
    hsr.stream(x, v, 0.01, w.box)           # x changes; the binning does not
    got = hsr.force_vjp(x, mass, w.box, w.r_cut, w.eps, w.poly, g, binned=token)
    ref = hsr.force_vjp(pos, mass, w.box, w.r_cut, w.eps, w.poly, g)
    assert torch.equal(got, ref)


def test_binned_vjp_refused_when_stale(cuda):
    w = _workload(seed=35)
    pos, mass = to_dev(w, cuda)
    g = torch.from_numpy(cotangent(w.n, 36)).to(cuda)
    out = torch.empty((w.n, 3), dtype=torch.float64, device=cuda)
    ref = hsr.force_vjp(pos, mass, w.box, w.r_cut, w.eps, w.poly, g)
    hsr.force(pos, mass, w.box, w.r_cut, w.eps, w.poly)
    token = hsr.binning_token()
    # another size or geometry, or no token: refused before any GPU work
    assert _binned_rc(0, w, g, out) == _lib.ESTALE
    assert _binned_rc(token + 1, w, g, out) == _lib.ESTALE
    other = _finish(w.name, w.pos[: w.n // 2], 35, 32, {}, box=w.box)
    assert _binned_rc(token, other, g, out) == _lib.ESTALE
    # each of these writes the workspace and retires the binning
    retire = [
        lambda: hsr.force_plain(pos, mass, w.box, w.r_cut, w.eps, w.poly),
        lambda: hsr.pm_accel(pos, mass, w.box, 32),
        lambda: hsr.bin(pos, mass, w.box, w.r_cut),
        lambda: hsr.count_pairs(pos, w.box, w.r_cut, w.eps),
        lambda: hsr.force_rcb(pos, mass, w.box, w.r_cut, w.eps, w.poly),
    ]
    for k, call in enumerate(retire):
        hsr.force(pos, mass, w.box, w.r_cut, w.eps, w.poly)
        token = hsr.binning_token()
        call()
        torch.cuda.synchronize()
        assert hsr.binning_token() == 0, k
        _lib._bind(pos.device, w.n, w.box, w.r_cut)
        assert _binned_rc(token, w, g, out) == _lib.ESTALE, k
        # the binding falls back to binning again, with the same result
        got = hsr.force_vjp(pos, mass, w.box, w.r_cut, w.eps, w.poly, g, binned=token)
        assert torch.equal(got, ref), k
    # kicks and streams leave it in place
    hsr.force(pos, mass, w.box, w.r_cut, w.eps, w.poly)
    token = hsr.binning_token()
    vel = torch.zeros_like(pos)
    acc = torch.zeros((w.n, 3), dtype=torch.float32, device=cuda)
    hsr.kick(vel, acc, 0.1)
    hsr.stream(pos.clone(), vel, 0.1, w.box)
    assert hsr.binning_token() == token
    _lib._bind(pos.device, w.n, w.box, w.r_cut)
    assert _binned_rc(token, w, g, out) == 0
    torch.cuda.synchronize()
    assert torch.equal(out, ref)


def test_rollout_reuses_the_last_binning(cuda):
    """A 3-subcycle differentiable rollout: its backward pass bins 2 times,
    not 3, and its gradient is bitwise the one with every VJP binning again."""
    w = _workload(n=1 << 14, seed=37)
    pos, mass = to_dev(w, cuda)
    h, n_c = 1e-3, 3
    gx = torch.from_numpy(np.random.default_rng(38).standard_normal((w.n, 3))).to(cuda)

    def run(reuse):
        x0 = pos.clone().requires_grad_(True)
        v0 = torch.zeros_like(pos).requires_grad_(True)
        xf, vf = hsr.rollout_sks(x0, v0, mass, w.box, w.r_cut, w.eps, w.poly, h, n_c)
        torch.cuda.synchronize()
        if not reuse:
            hsr.count_pairs(pos, w.box, w.r_cut, w.eps)    # retires the kept binning
        hsr.timing_enable(True)
        (gx * xf).sum().backward()
        torch.cuda.synchronize()
        n_w, _ = hsr.timing_read(hsr.TIMER_WORKLIST)
        hsr.timing_enable(False)
        return x0.grad.clone(), v0.grad.clone(), n_w

    gx1, gv1, nw1 = run(True)
    gx2, gv2, nw2 = run(False)
    assert (nw1, nw2) == (n_c - 1, n_c)
    assert torch.equal(gx1, gx2) and torch.equal(gv1, gv2)
