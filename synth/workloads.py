"""Synthetic voxel scatterers, plane-wave directions and serving request streams.

Everything here is drawn from ``numpy.random.default_rng(seed)``.  For a named
workload the draw order is fixed: permittivity field (array of shape (nz, ny, nx),
raveled so that x runs fastest), then directions, then polarisations, then the
sampled output rows used by accuracy checks.

Units: the free-space wavelength is 1, so the wavenumber is 2*pi.  A lossy medium has
a negative imaginary permittivity part (time factor exp(+j w t), matching the
exp(-j k R) Green's function of Section II).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

TWO_PI = 2.0 * math.pi


@dataclasses.dataclass
class Grid:
    """A box of nx*ny*nz cubic voxels of edge h; user index i = ix + nx*(iy + ny*iz)."""
    nx: int
    ny: int
    nz: int
    h: float
    k0: float
    eps: np.ndarray  # complex128, length N, user order

    @property
    def n(self) -> int:
        return self.nx * self.ny * self.nz


def make_grid(nx: int, ny: int, nz: int, h: float, eps, k0: float = TWO_PI) -> Grid:
    n = nx * ny * nz
    e = np.asarray(eps, dtype=np.complex128)
    if e.ndim == 0:
        e = np.full(n, complex(e), dtype=np.complex128)
    e = np.ascontiguousarray(e.reshape(-1))
    if e.size != n:
        raise ValueError(f"eps has {e.size} entries, grid has {n}")
    return Grid(nx, ny, nz, float(h), float(k0), e)


def random_directions(rng: np.random.Generator, count: int) -> np.ndarray:
    """Unit propagation directions: normalised standard-normal 3-vectors, shape (count, 3)."""
    d = rng.standard_normal((count, 3))
    return d / np.linalg.norm(d, axis=1, keepdims=True)


def random_polarisations(rng: np.random.Generator, dirs: np.ndarray) -> np.ndarray:
    """Unit vectors perpendicular to each direction (recorded; the scalar model ignores them)."""
    p = rng.standard_normal(dirs.shape)
    p -= np.sum(p * dirs, axis=1, keepdims=True) * dirs
    return p / np.linalg.norm(p, axis=1, keepdims=True)


def _centred_coords(nx, ny, nz, h):
    ix = (np.arange(nx) + 0.5) * h - 0.5 * nx * h
    iy = (np.arange(ny) + 0.5) * h - 0.5 * ny * h
    iz = (np.arange(nz) + 0.5) * h - 0.5 * nz * h
    z, y, x = np.meshgrid(iz, iy, ix, indexing="ij")
    return x, y, z


# name -> (sides, box edge in wavelengths, rhs count, compression tolerance, seed)
_SPECS = {
    # 16^3 voxels in a 1-wavelength cube, uniform eps_r = 4, one plane wave
    "c1_plain_16": ((16, 16, 16), 1.0, 1, 1e-4, 1),
    # 32^3 voxels in a 4-wavelength cube, eps_r i.i.d. U[2, 10], 64 plane waves
    "c2_batched_32": ((32, 32, 32), 4.0, 64, 1e-4, 2),
    # 64^3 voxels over [-4, 4]^3 wavelengths: sphere of radius 4 with a negative shell
    "c3_sphere_64": ((64, 64, 64), 8.0, 32, 1e-4, 3),
    # 128^3 voxels in a 12-wavelength cube of 8 lossy slabs
    "c5_slabs_128": ((128, 128, 128), 12.0, 16, 1e-3, 5),
}
CONFIG_NAMES = tuple(_SPECS)


def config(name: str, sample_rows: int | None = None) -> dict:
    """Build one named workload.

    Returns a dict with the grid, the directions ``dirs`` (R x 3), polarisations,
    ``nrhs``, ``tol`` and ``rows`` (sorted user indices drawn without replacement
    for row-sampled accuracy checks).
    """
    sides, box, nrhs, tol, seed = _SPECS[name]
    nx, ny, nz = sides
    h = box / nx
    n = nx * ny * nz
    rng = np.random.default_rng(seed)
    if name.startswith("c1"):
        eps = np.full(n, 4.0 + 0j)
    elif name.startswith("c2"):
        eps = rng.uniform(2.0, 10.0, size=(nz, ny, nx)).reshape(-1).astype(np.complex128)
    elif name.startswith("c3"):
        x, y, z = _centred_coords(nx, ny, nz, h)
        r = np.sqrt(x * x + y * y + z * z).reshape(-1)
        eps = np.ones(n, dtype=np.complex128)
        eps[r <= 4.0] = 20.0
        eps[(r >= 2.0) & (r <= 2.5)] = -2.0 - 0.1j
    elif name.startswith("c5"):
        re = rng.uniform(1.0, 80.0, size=8)
        im = rng.uniform(0.0, 5.0, size=8)
        slab = np.repeat(np.arange(8), nz // 8)  # slab index of each z layer
        per_z = (re - 1j * im)[slab]
        eps = np.broadcast_to(per_z[:, None, None], (nz, ny, nx)).reshape(-1).astype(np.complex128)
    else:  # pragma: no cover
        raise KeyError(name)
    dirs = random_directions(rng, nrhs)
    pols = random_polarisations(rng, dirs)
    if sample_rows is None:
        sample_rows = {"c1": 256, "c2": 256, "c3": 256, "c5": 512}[name[:2]]
    rows = np.sort(rng.choice(n, size=min(sample_rows, n), replace=False))
    return dict(name=name, grid=make_grid(nx, ny, nz, h, eps), dirs=dirs, pols=pols,
                nrhs=nrhs, tol=tol, rows=rows, seed=seed)


def small_case(seed: int, sides=(12, 10, 9), h: float = 1.0 / 10, eps_range=(1.0, 6.0),
               loss: float = 0.0, nrhs: int = 3) -> dict:
    """A seeded non-cubic grid (ragged leaves) with i.i.d. permittivity, for parity tests."""
    nx, ny, nz = sides
    rng = np.random.default_rng(seed)
    n = nx * ny * nz
    re = rng.uniform(eps_range[0], eps_range[1], size=n)
    im = rng.uniform(0.0, loss, size=n) if loss > 0 else np.zeros(n)
    eps = (re - 1j * im).astype(np.complex128)
    dirs = random_directions(rng, nrhs)
    x = (rng.standard_normal((n, nrhs)) + 1j * rng.standard_normal((n, nrhs)))
    return dict(grid=make_grid(nx, ny, nz, h, eps), dirs=dirs, x=x, nrhs=nrhs)


def serving_requests(seed: int = 4, count: int = 200, rate: float = 1.0, sizes=None,
                     scatterers_per_size: int = 3) -> list:
    """Poisson stream of solve requests over cube sizes (default: 16^3 in 1 wavelength,
    32^3 in 4, 64^3 in 8).

    Each request: arrival time (exponential gaps at ``rate`` per second), a size, a
    scatterer drawn from a pool of ``scatterers_per_size`` seeded permittivity fields of
    that size (eps_r ~ U[1, 12] per voxel, so operators can stay resident across
    requests), and a right-hand-side count ~ U{1..16}.
    """
    rng = np.random.default_rng(seed)
    if sizes is None:
        sizes = [((16, 16, 16), 1.0), ((32, 32, 32), 4.0), ((64, 64, 64), 8.0)]
    pool = rng.integers(0, 2**31 - 1, size=(len(sizes), scatterers_per_size))
    t = 0.0
    out = []
    for i in range(count):
        t += rng.exponential(1.0 / rate)
        which = int(rng.integers(0, len(sizes)))
        nrhs = int(rng.integers(1, 17))
        k = int(rng.integers(0, scatterers_per_size))
        out.append(dict(id=i, arrival=t, sides=sizes[which][0], box=sizes[which][1],
                        nrhs=nrhs, eps_seed=int(pool[which, k]), dir_seed=int(rng.integers(0, 2**31 - 1))))
    return out


def request_inputs(req: dict) -> dict:
    """Materialise one serving request's grid and plane-wave directions."""
    nx, ny, nz = req["sides"]
    rng = np.random.default_rng(req["eps_seed"])
    eps = rng.uniform(1.0, 12.0, size=(nz, ny, nx)).reshape(-1).astype(np.complex128)
    dirs = random_directions(np.random.default_rng(req["dir_seed"]), req["nrhs"])
    return dict(grid=make_grid(nx, ny, nz, req["box"] / nx, eps), dirs=dirs)
