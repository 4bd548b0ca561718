"""Oracle: scalar voxel VIE system matrix and exact products (test infrastructure only).

Formulation (Section II, eqs. (1)-(2), (4)-(5)), reduced to the scalar Helmholtz
kernel and point collocation on cubic voxels:

* Green's function g(r, r') = exp(-j k R) / (4 pi R), R = |r - r'| (Section II).
* Contrast kappa = (eps - 1) / eps (Section II, with eps relative to free space).
* Expanding -j w eta0 L[.] with L's prefactor -j k0 gives -k0^2 times the volume
  integral of g (grad-div term dropped), so collocating at voxel centres with a pulse
  basis gives
      Z(m, n) = delta_mn / eps_m - k^2 * kappa_n * G_mn,
  G_mn = h^3 g(r_m, r_n) for m != n (one-point rule) and G_mm = integral of g over
  the sphere of the voxel's volume, radius a = h (3 / (4 pi))^(1/3), which is
  S(a) = (1/k^2) [(1 + j k a) exp(-j k a) - 1].
  In voxel-offset units (d integer, rho = |d|):
      K(d) = (k h)^2 / (4 pi rho) * exp(-j k h rho)     (d != 0)
      K(0) = (1 + j k a) exp(-j k a) - 1
      Z(m, n) = delta_mn / eps_m - K(d_mn) * kappa_n.
* Excitation (Section IV): a plane wave, b_q(m) = exp(-j k dhat_q . (r_m - r_c)).
"""
from __future__ import annotations

import math

import numpy as np

FOUR_PI = 4.0 * math.pi


def equal_volume_radius(h: float) -> float:
    """Radius of the sphere whose volume equals the voxel's, h^3 = (4/3) pi a^3."""
    return h * (3.0 / FOUR_PI) ** (1.0 / 3.0)


def self_term_k2S(k: float, a: float) -> complex:
    """k^2 times the integral of g over a ball of radius a centred on the source point.

    The ball integral is  int_0^a 4 pi r^2 exp(-j k r) / (4 pi r) dr = int_0^a r e^{-jkr} dr,
    whose antiderivative gives (1/k^2)[(1 + j k a) e^{-j k a} - 1].
    """
    x = k * a
    return (1.0 + 1j * x) * np.exp(-1j * x) - 1.0


def contrast(eps: np.ndarray) -> np.ndarray:
    """kappa = (eps - eps0) / eps with eps relative to eps0 (Section II)."""
    return (eps - 1.0) / eps


def voxel_index(grid, idx: np.ndarray) -> np.ndarray:
    """Integer voxel coordinates (ix, iy, iz) of user indices, shape (len, 3)."""
    idx = np.asarray(idx, dtype=np.int64)
    ix = idx % grid.nx
    iy = (idx // grid.nx) % grid.ny
    iz = idx // (grid.nx * grid.ny)
    return np.stack([ix, iy, iz], axis=1)


def voxel_centres(grid, idx=None) -> np.ndarray:
    """Voxel centres h * (i + 1/2) in wavelengths, shape (len, 3)."""
    if idx is None:
        idx = np.arange(grid.n)
    return (voxel_index(grid, idx) + 0.5) * grid.h


def kernel_K(d2: np.ndarray, kh: float, k2S: complex) -> np.ndarray:
    """K(d) from the squared integer offset |d|^2 (exact integer), see module docstring."""
    d2 = np.asarray(d2, dtype=np.float64)
    rho = np.sqrt(d2)
    out = np.empty(d2.shape, dtype=np.complex128)
    nz = d2 > 0
    out[nz] = (kh * kh) / (FOUR_PI * rho[nz]) * np.exp(-1j * kh * rho[nz])
    out[~nz] = k2S
    return out


def entries(grid, rows, cols) -> np.ndarray:
    """Z(rows, cols) for user-index lists, complex128 of shape (len(rows), len(cols))."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    kh = grid.k0 * grid.h
    k2S = self_term_k2S(grid.k0, equal_volume_radius(grid.h))
    pr = voxel_index(grid, rows)
    pc = voxel_index(grid, cols)
    d = pr[:, None, :] - pc[None, :, :]
    d2 = np.sum(d * d, axis=2)
    kap = contrast(grid.eps[cols])
    z = -kernel_K(d2, kh, k2S) * kap[None, :]
    same = rows[:, None] == cols[None, :]
    if np.any(same):
        inv_eps = 1.0 / grid.eps[rows]
        z = z + same * inv_eps[:, None]
    return z


def dense(grid) -> np.ndarray:
    """The full N x N system matrix in user order (small grids only)."""
    idx = np.arange(grid.n)
    return entries(grid, idx, idx)


def direct_rows(grid, x: np.ndarray, rows) -> np.ndarray:
    """(Z x)[rows] by direct O(N) summation per row; x is (N,) or (N, R)."""
    x2 = x.reshape(grid.n, -1)
    cols = np.arange(grid.n)
    out = np.empty((len(rows), x2.shape[1]), dtype=np.complex128)
    for i, m in enumerate(np.asarray(rows)):
        out[i] = entries(grid, [m], cols)[0] @ x2
    return out.reshape((len(rows),) + x.shape[1:])


def fft_matvec(grid, x: np.ndarray) -> np.ndarray:
    """Exact y = Z x for every row, via the discrete-convolution identity.

    On a uniform grid the kernel part sum_n K(d_mn) u_n is a 3-D linear convolution;
    embedding K(d), |d_i| < n_i, in a (2nx, 2ny, 2nz) periodic array turns it into a
    circular convolution computed with FFTs.  y = x / eps - conv(K, kappa * x).
    """
    nx, ny, nz = grid.nx, grid.ny, grid.nz
    kh = grid.k0 * grid.h
    k2S = self_term_k2S(grid.k0, equal_volume_radius(grid.h))
    ax = [np.concatenate([np.arange(n), [0], np.arange(-n + 1, 0)]) for n in (nz, ny, nx)]
    dz, dy, dx = np.meshgrid(*ax, indexing="ij")
    kc = kernel_K(dx * dx + dy * dy + dz * dz, kh, k2S)
    # the index n of each axis is the unused wrap slot (offset +-n never occurs)
    kc[nz, :, :] = 0
    kc[:, ny, :] = 0
    kc[:, :, nx] = 0
    fk = np.fft.fftn(kc)
    x2 = x.reshape(grid.n, -1)
    kap = contrast(grid.eps)
    y = np.empty_like(x2, dtype=np.complex128)
    for q in range(x2.shape[1]):
        u = np.zeros((2 * nz, 2 * ny, 2 * nx), dtype=np.complex128)
        u[:nz, :ny, :nx] = (kap * x2[:, q]).reshape(nz, ny, nx)
        conv = np.fft.ifftn(fk * np.fft.fftn(u))[:nz, :ny, :nx].reshape(-1)
        y[:, q] = x2[:, q] / grid.eps - conv
    return y.reshape(x.shape)


def plane_wave(grid, dirs: np.ndarray) -> np.ndarray:
    """b_q(m) = exp(-j k dhat_q . (r_m - r_c)), r_c the box centre; shape (N, R)."""
    r = voxel_centres(grid)
    rc = 0.5 * grid.h * np.array([grid.nx, grid.ny, grid.nz], dtype=np.float64)
    phase = (r - rc) @ np.asarray(dirs, dtype=np.float64).T
    return np.exp(-1j * grid.k0 * phase)
