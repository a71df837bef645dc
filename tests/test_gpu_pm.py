"""The long-range spectral PM solver on the GPU (Habib et al. 2012, Sec. II)
against the float64 oracle (oracle/pm.py).  Float32 grids and FFTs spread
their rounding over the whole field, so the bound is absolute, relative to
the rms acceleration: max_i |a_i - a*_i| <= 1e-5 rms|a*| (a float32
emulation of the same pipeline with library FFTs reads 4e-7; the margin
covers the float32 twiddles and the order of the FFT's sums)."""
import numpy as np
import pytest
import torch

from oracle import pm
import paper_1211_4864_amd as hsr
from workloads import make_config, plummer_clustered

pytestmark = pytest.mark.gpu
TOL = 1e-5


def _gpu(pos, mass, box, ng, device, sigma=0.8, n_s=3):
    p = torch.from_numpy(np.ascontiguousarray(pos, dtype=np.float64)).to(device)
    m = torch.from_numpy(np.ascontiguousarray(mass, dtype=np.float32)).to(device)
    out = hsr.pm_accel(p, m, box, ng, sigma, n_s)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64)


def _check(got, ref, name):
    err = np.linalg.norm(got - ref, axis=1)
    rms = np.sqrt((np.linalg.norm(ref, axis=1) ** 2).mean())
    print(f"{name}: max |da| / rms|a| = {err.max() / rms:.3e}", flush=True)
    assert np.all(np.isfinite(got))
    assert err.max() <= TOL * rms


@pytest.mark.parametrize("ng", [8, 32, 64])
def test_pm_clustered_matches_oracle(cuda, ng):
    n = 50000
    pos, _ = plummer_clustered(n, 51, 20, 0.6, 1.0 / max(ng, 32))
    mass = np.full(n, np.float32(1.0 / n))
    _check(_gpu(pos, mass, 1.0, ng, cuda), pm.accel(pos, mass, 1.0, ng), f"plummer ng={ng}")


@pytest.mark.parametrize("ng,n", [(16, 60000), (256, 200000), (512, 100000)])
def test_pm_grid_shapes_match_oracle(cuda, ng, n):
    """Every transform shape of the kernels (16 = 4 x 4 with 16-line tiles,
    256 = 16 x 16, 512 = 32 x 16 with 8-line tiles); at 512 most cells hold
    one particle, at 16 most waves share cells."""
    pos, _ = plummer_clustered(n, 54 + ng, 30, 0.5, 1.0 / max(ng, 32))
    rng = np.random.default_rng(55)
    mass = ((rng.random(n) + 0.5) / n).astype(np.float32)
    ref = pm.accel(pos, mass.astype(np.float64), 1.0, ng)
    _check(_gpu(pos, mass, 1.0, ng, cuda), ref, f"plummer ng={ng} n={n}")


def test_pm_permuted_input_bitwise(cuda):
    """The deposit sums in fixed point after a sort by cell, so the solve
    does not depend on the input order: a permuted input gives the
    permuted output, bitwise."""
    n, ng = 70000, 64
    pos, _ = plummer_clustered(n, 56, 10, 0.7, 1.0 / ng)
    rng = np.random.default_rng(57)
    mass = ((rng.random(n) + 0.5) / n).astype(np.float32)
    perm = rng.permutation(n)
    a = _gpu(pos, mass, 1.0, ng, cuda)
    b = _gpu(pos[perm], mass[perm], 1.0, ng, cuda)
    assert np.array_equal(a[perm], b)


def test_pm_shared_cells(cuda):
    """Runs of particles in one grid cell longer than a wave (and a run of
    exactly coincident particles), beside a uniform background."""
    rng = np.random.default_rng(58)
    ng, D = 32, 1.0 / 32
    lump = np.array([0.3, 0.6, 0.1]) + rng.random((5000, 3)) * 0.9 * D
    same = np.tile([[0.71, 0.22, 0.93]], (3000, 1))
    back = rng.random((20000, 3))
    pos = np.concatenate([lump, same, back])
    mass = np.concatenate([np.full(5000, 2e-5), np.full(3000, 1e-5),
                           np.full(20000, 3e-5)]).astype(np.float32)
    ref = pm.accel(pos, mass.astype(np.float64), 1.0, ng)
    _check(_gpu(pos, mass, 1.0, ng, cuda), ref, "shared cells")


def test_pm_box_units_unequal_masses_and_filter(cuda):
    """Box of side 3, unequal masses, positions outside the box (wrapped),
    and a different filter (sigma 1.2, n_s 2)."""
    rng = np.random.default_rng(52)
    n = 30000
    pos = rng.random((n, 3)) * 3.6 - 0.3
    mass = (rng.random(n) + 0.2).astype(np.float32)
    ref = pm.accel(pos, mass.astype(np.float64), 3.0, 32, 1.2, 2)
    _check(_gpu(pos, mass, 3.0, 32, cuda, 1.2, 2), ref, "box 3 unequal")


def test_pm_cfg2_matches_oracle(cuda):
    """The 128^3 Plummer-clustered workload on its own 128^3 PM grid."""
    w = make_config("cfg2")
    ref = pm.accel(w.pos, w.mass.astype(np.float64), w.box, 128)
    _check(_gpu(w.pos, w.mass, w.box, 128, cuda), ref, "cfg2 ng=128")


def test_pm_single_mode_momentum_and_reproducibility(cuda):
    """A single Fourier mode in closed form on the grid points; total
    momentum zero; two calls bitwise equal."""
    box, ng, A, m0 = 1.0, 32, 0.3, 3
    D = box / ng
    g = np.arange(ng) * D
    pos = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    k0 = 2 * np.pi * m0 / box
    mass = (1.0 + A * np.cos(k0 * pos[:, 0])).astype(np.float32)
    got = _gpu(pos, mass, box, ng, cuda)
    kd = k0 * D
    S = np.exp(-0.25 * (k0 * 0.8 * D) ** 2) * (np.sin(kd / 2) / (kd / 2)) ** 3
    K6 = (49 / 18 - 3 * np.cos(kd) + 0.3 * np.cos(2 * kd) - np.cos(3 * kd) / 45) / D ** 2
    Dk = (4 / 3 * np.sin(kd) - np.sin(2 * kd) / 6) / D
    expect = -4 * np.pi * A / D ** 3 * S / K6 * Dk * np.sin(k0 * pos[:, 0])
    scale = np.abs(expect).max()
    assert np.abs(got[:, 0] - expect).max() <= 1e-5 * scale
    assert np.abs(got[:, 1:]).max() <= 1e-5 * scale
    rng = np.random.default_rng(53)
    n = 40000
    p2 = rng.random((n, 3))
    m2 = (rng.random(n) + 0.5).astype(np.float32)
    a1 = _gpu(p2, m2, 1.0, 32, cuda)
    a2 = _gpu(p2, m2, 1.0, 32, cuda)
    assert np.array_equal(a1, a2)
    mom = (m2[:, None].astype(np.float64) * a1).sum(0)
    assert np.abs(mom).max() <= 1e-5 * (m2[:, None] * np.abs(a1)).sum()


def test_pm_empty_and_validation(cuda):
    pos = torch.zeros((0, 3), dtype=torch.float64, device=cuda)
    mass = torch.zeros(0, dtype=torch.float32, device=cuda)
    assert hsr.pm_accel(pos, mass, 1.0, 16).shape == (0, 3)
    with pytest.raises(hsr.HaccSrError):
        hsr.pm_accel(pos, mass, 1.0, 24)
