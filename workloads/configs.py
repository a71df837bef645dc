"""Seeded particle sets that stand in for the paper's cosmological workloads.

The paper runs on cosmological initial conditions evolved to a clustered
state (Sec. V); none of those particle sets are available, so these
generators draw particles with the same qualitative structure: a uniform
background plus dense halos whose masses span several decades, so that
chaining-cell occupancy ranges from empty to thousands of particles.

All draws come from ``numpy.random.default_rng(seed)``; positions are float64
in the periodic unit box [0, 1)^3 and masses are float32 equal to 1/N.  The
input order of the particles is a random permutation, as it would be after a
domain exchange.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Callable

import numpy as np
from scipy.special import lambertw

from .fgrid import fit_fgrid, FGridFit


@dataclasses.dataclass
class Workload:
    name: str
    pos: np.ndarray          # (n, 3) float64
    mass: np.ndarray         # (n,) float32
    box: float               # > 0 periodic cube [0, box); < 0 open domain [0, -box)
    r_cut: float             # float32 value
    eps: float               # float32 value
    poly: np.ndarray         # float32[6]
    cell: float              # particle-mesh grid cell (r_cut = 3 cells)
    seed: int
    fit: FGridFit
    meta: dict

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def _wrap_unit(x: np.ndarray) -> np.ndarray:
    x = x - np.floor(x)
    x[x >= 1.0] = 0.0
    return x


def _isotropic(rng: np.random.Generator, n: int) -> np.ndarray:
    mu = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    st = np.sqrt(1.0 - mu * mu)
    return np.stack([st * np.cos(phi), st * np.sin(phi), mu], axis=1)


def uniform_gauss(n: int, seed: int, sigma: float) -> np.ndarray:
    """U[0,1)^3 plus Gaussian displacements of width ``sigma``, wrapped."""
    rng = np.random.default_rng(seed)
    x = rng.random((n, 3)) + rng.normal(0.0, sigma, (n, 3))
    return _wrap_unit(x)


def plummer_clustered(n: int, seed: int, n_halo: int, frac: float,
                      cell: float, a_cells=(0.5, 3.0), logm=(0.0, 3.0)):
    """Plummer spheres (truncated at 10 scale radii) + uniform background.

    Halo masses are 10^U(logm); particles per halo are multinomial over the
    masses; scale radii are U(a_cells) grid cells.  Radii invert the Plummer
    enclosed-mass fraction X = r^3 / (r^2 + a^2)^(3/2).
    """
    rng = np.random.default_rng(seed)
    m = 10.0 ** rng.uniform(logm[0], logm[1], n_halo)
    counts = rng.multinomial(int(frac * n), m / m.sum())
    centres = rng.random((n_halo, 3))
    a = rng.uniform(a_cells[0], a_cells[1], n_halo) * cell
    hid = np.repeat(np.arange(n_halo), counts)
    nh = hid.size
    xmax = (100.0 / 101.0) ** 1.5
    X = np.maximum(rng.uniform(0.0, xmax, nh), 1e-300)
    r = a[hid] / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    halo = centres[hid] + r[:, None] * _isotropic(rng, nh)
    bg = rng.random((n - nh, 3))
    x = _wrap_unit(np.concatenate([halo, bg], axis=0))
    perm = rng.permutation(n)
    meta = dict(n_halo=n_halo, halo_particles=int(nh),
                largest_halo=int(counts.max()) if n_halo else 0)
    return x[perm], meta


def _nfw_mu(x):
    return np.log1p(x) - x / (1.0 + x)


def nfw_clustered(n: int, seed: int, n_halo: int, frac: float, cell: float,
                  rvir_cells: float = 4.0, logm=(0.0, 4.0), conc=(4.0, 15.0),
                  stress_block: bool = False, chunk: int = 1 << 22):
    """NFW halos (truncated at r_vir) + uniform background.

    Masses 10^U(logm); concentration U(conc); r_vir = rvir_cells cells times
    (M / M_max)^(1/3).  Radii invert the NFW enclosed-mass fraction
    mu(x)/mu(c) = U with the principal Lambert-W branch:
    x = -1 / W0(-exp(-1 - U mu(c))) - 1, r = (r_vir / c) x.
    ``stress_block`` moves the ten most massive halo centres into one
    2x2x2-cell block (an occupancy stress variant).
    """
    rng = np.random.default_rng(seed)
    m = 10.0 ** rng.uniform(logm[0], logm[1], n_halo)
    counts = rng.multinomial(int(frac * n), m / m.sum())
    centres = rng.random((n_halo, 3))
    c = rng.uniform(conc[0], conc[1], n_halo)
    rvir = rvir_cells * cell * (m / m.max()) ** (1.0 / 3.0)
    if stress_block:
        top = np.argsort(-m)[:10]
        base = np.floor(rng.random(3) / cell) * cell
        centres[top] = base + rng.random((10, 3)) * 2.0 * cell
    hid = np.repeat(np.arange(n_halo), counts)
    nh = hid.size
    halo = np.empty((nh, 3))
    for s in range(0, nh, chunk):
        h = hid[s:s + chunk]
        u = rng.random(h.size)
        arg = -np.exp(-1.0 - u * _nfw_mu(c[h]))
        w = lambertw(arg, 0).real
        x = -1.0 / w - 1.0
        r = rvir[h] / c[h] * x
        halo[s:s + h.size] = centres[h] + r[:, None] * _isotropic(rng, h.size)
    bg = rng.random((n - nh, 3))
    xall = _wrap_unit(np.concatenate([halo, bg], axis=0))
    del halo, bg
    perm = rng.permutation(n)
    meta = dict(n_halo=n_halo, halo_particles=int(nh),
                largest_halo=int(counts.max()) if n_halo else 0)
    return xall[perm], meta


def add_ghost_shell(pos: np.ndarray, width: float):
    """Periodic images of the unit box that fall within ``width`` of a face.

    Returns the active particles followed by the ghosts, translated by
    +width so that the open domain [-width, 1+width)^3 becomes
    [0, 1 + 2 width)^3, and the index array of each ghost's source particle.
    This is the overloaded domain of Sec. II (particle overloading): the
    ghosts are passive copies that let every active particle see all of its
    neighbours without communication.
    """
    near = np.any((pos < width) | (pos >= 1.0 - width), axis=1)
    idx = np.nonzero(near)[0]
    sub = pos[idx]
    ghosts, src = [], []
    for ox in (-1, 0, 1):
        for oy in (-1, 0, 1):
            for oz in (-1, 0, 1):
                if ox == 0 and oy == 0 and oz == 0:
                    continue
                im = sub + np.array([ox, oy, oz], dtype=np.float64)
                ok = np.all((im >= -width) & (im < 1.0 + width), axis=1)
                ghosts.append(im[ok])
                src.append(idx[ok])
    g = np.concatenate(ghosts, axis=0) if ghosts else np.zeros((0, 3))
    s = np.concatenate(src) if src else np.zeros(0, dtype=np.int64)
    allpos = np.concatenate([pos, g], axis=0) + width
    return allpos, s


def cotangent(n: int, seed: int) -> np.ndarray:
    """Loss weights g_i ~ N(0, 1) in float32, shape (n, 3)."""
    return np.random.default_rng(seed).standard_normal((n, 3)).astype(np.float32)


def _finish(name, pos, seed, grid, meta, box=1.0, eps_cells2=1e-5 * 128.0 ** 2):
    cell = 1.0 / grid
    fit = fit_fgrid(cell, 3.0, eps_cells2)
    n = pos.shape[0]
    mass = np.full(n, np.float32(1.0 / n), dtype=np.float32)
    meta = dict(meta)
    meta["grid"] = grid
    return Workload(name=name, pos=np.ascontiguousarray(pos, dtype=np.float64),
                    mass=mass, box=box, r_cut=fit.r_cut, eps=fit.eps,
                    poly=fit.coeffs.copy(), cell=cell, seed=seed, fit=fit,
                    meta=meta)


def _cfg1(**kw):
    n = kw.get("n", 32768)
    pos = uniform_gauss(n, kw.get("seed", 1), 0.3 / 128.0)
    return _finish("cfg1", pos, kw.get("seed", 1), 128, {})


def _cfg2(**kw):
    n = kw.get("n", 128 ** 3)
    n_halo = kw.get("n_halo", 2000)
    pos, meta = plummer_clustered(n, kw.get("seed", 2), n_halo, 0.6, 1.0 / 128.0)
    return _finish("cfg2", pos, kw.get("seed", 2), 128, meta)


def _cfg3(stress=False, **kw):
    grid = kw.get("grid", 256)
    n = kw.get("n", grid ** 3)
    n_halo = kw.get("n_halo", 20000)
    pos, meta = nfw_clustered(n, kw.get("seed", 3), n_halo, 0.7, 1.0 / grid,
                              stress_block=stress)
    return _finish("cfg3s" if stress else "cfg3", pos, kw.get("seed", 3), grid,
                   meta)


def _cfg5(**kw):
    """One GPU's share: a periodic 512^3 parent plus a 3-cell ghost shell."""
    grid = kw.get("grid", 512)
    n = kw.get("n", grid ** 3)
    n_halo = kw.get("n_halo", max(1, int(round(160000 * (grid / 512.0) ** 3))))
    seed = kw.get("seed", 5)
    pos, meta = nfw_clustered(n, seed, n_halo, 0.7, 1.0 / grid)
    cell = 1.0 / grid
    width = 3.0 * cell
    allpos, src = add_ghost_shell(pos, width)
    meta = dict(meta, n_active=n, n_ghost=int(src.size), ghost_src=src,
                shell=width)
    w = _finish("cfg5" if grid == 512 else f"cfg5_{grid}", allpos, seed, grid,
                meta, box=-(1.0 + 2.0 * width))
    # masses of the overloaded copies equal their sources' (all 1/n_active)
    w.mass[:] = np.float32(1.0 / n)
    return w


_CONFIGS: dict[str, Callable[..., Workload]] = {
    "cfg1": _cfg1,
    "cfg2": _cfg2,
    "cfg3": _cfg3,
    "cfg3s": lambda **kw: _cfg3(stress=True, **kw),
    "cfg5": _cfg5,
}


def config_names():
    return list(_CONFIGS)


def make_config(name: str, **kw) -> Workload:
    """Build a named workload; keyword overrides (n, n_halo, grid, seed) give
    reduced instances of the same generator."""
    if name == "cfg4":
        w = _cfg2(**kw)
        w.name = "cfg4"
        w.meta["g"] = cotangent(w.n, kw.get("g_seed", 4))
        return w
    if name.startswith("cfg5_"):
        return _cfg5(grid=int(name.split("_")[1]), **kw)
    return _CONFIGS[name](**kw)
