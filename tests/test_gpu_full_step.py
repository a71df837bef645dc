"""One full split-operator step on the GPU (Habib et al. 2012, Sec. II,
Eq. 6: a half kick with the long-range PM force, n_c stream-kick-stream
subcycles with the short-range force, a half kick) against the float64
oracle's composition of the same maps, with the grid-force polynomial
fitted to this PM's sampled pair forces.

Each short-range force is within 1e-5 max(|a|, 0.1 A) of the float64 one
and each PM force within 1e-5 of the rms PM acceleration.  Over one step of
length dt the velocity error is at most dt times those, and the position
error dt^2 times them; a factor 3 covers the forces' drift inside the
step."""
import numpy as np
import pytest
import torch

import oracle
from oracle import pm, rollout
import paper_1211_4864_amd as hsr
from workloads import plummer_clustered

pytestmark = pytest.mark.gpu


def test_full_step_matches_oracle(cuda):
    box, ng, n = 1.0, 32, 40000
    D = box / ng
    pos, _ = plummer_clustered(n, 71, 12, 0.6, D)
    rng = np.random.default_rng(72)
    mass = (rng.random(n) * 0.5 + 0.75).astype(np.float32) / n
    r_cut = float(np.float32(3.0 * D))
    eps = float(np.float32(0.164 * D * D))
    poly = pm.fit_grid_force(box, ng, r_cut, eps, n_sources=4, per_source=2000, seed=73)
    a_lr = pm.accel(pos, mass.astype(np.float64), box, ng)
    a_sr, an, _ = oracle.force(pos, mass, box, r_cut, eps, poly)
    amax = float(np.sqrt((np.linalg.norm(a_lr + a_sr, axis=1) ** 2).mean()))
    v0 = 0.05 * rng.standard_normal((n, 3)) * amax * 1e-2
    dt = 0.2 * np.sqrt(D / amax)
    n_c = 3
    xr, vr = rollout.full_step(pos, v0, mass.astype(np.float64), box, ng, r_cut, eps, poly,
                               dt, n_c)
    x = torch.from_numpy(pos.copy()).to(cuda)
    v = torch.from_numpy(v0.copy()).to(cuda)
    m = torch.from_numpy(mass).to(cuda)
    hsr.full_step(x, v, m, box, ng, r_cut, eps, poly, dt, n_c)
    torch.cuda.synchronize()
    x, v = x.cpu().numpy(), v.cpu().numpy()
    rms_lr = float(np.sqrt((np.linalg.norm(a_lr, axis=1) ** 2).mean()))
    da = 1e-5 * rms_lr + 1e-5 * np.maximum(np.linalg.norm(a_sr, axis=1), 0.1 * an)
    dv = np.linalg.norm(v - vr, axis=1)
    dx = x - xr
    dx -= np.rint(dx / box) * box
    dx = np.linalg.norm(dx, axis=1)
    print(f"full step: dt {dt:.3e}, max |dv| / bound {np.max(dv / (3 * dt * da)):.3e}, "
          f"max |dx| / bound {np.max(dx / (3 * dt * dt * da + 1e-15)):.3e}", flush=True)
    assert np.all(dv <= 3 * dt * da)
    assert np.all(dx <= 3 * dt * dt * da + 1e-15)
    assert np.all((x >= 0) & (x < box))
