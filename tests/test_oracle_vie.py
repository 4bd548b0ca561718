"""Pins for the oracle's system matrix and exact products (Section II formulation)."""
import math

import numpy as np
import pytest

from oracle import vie
from synth.workloads import make_grid, small_case


def test_self_term_matches_quadrature_of_greens_function():
    # k^2 * integral of exp(-jkR)/(4 pi R) over a ball of radius a, by 64-point Gauss-Legendre
    # in the radial variable (the angular integral is 4 pi), independent of the closed form.
    for k, a in [(2 * math.pi, 0.62035 / 16), (2 * math.pi, 0.62035 / 8), (7.3, 0.9), (0.1, 0.2)]:
        xg, wg = np.polynomial.legendre.leggauss(64)
        r = 0.5 * a * (xg + 1.0)
        integral = 0.5 * a * np.sum(wg * 4 * math.pi * r * r * np.exp(-1j * k * r) / (4 * math.pi * r))
        assert abs(vie.self_term_k2S(k, a) - k * k * integral) <= 1e-14 * max(1.0, abs(k * k * integral))


def test_self_term_series_and_static_limit():
    # (1 + jx) e^{-jx} - 1 = x^2/2 - j x^3/3 - x^4/8 + j x^5/30 + O(x^6)
    for x in [1e-3, 1e-2, 0.05]:
        series = x**2 / 2 - 1j * x**3 / 3 - x**4 / 8 + 1j * x**5 / 30
        assert abs(vie.self_term_k2S(x, 1.0) - series) <= 2 * x**6 + 1e-15
    # static limit: S(a) -> a^2 / 2 as k -> 0
    a = 0.37
    for k in [1e-2, 1e-3]:
        assert abs(vie.self_term_k2S(k, a) / k**2 - a * a / 2) < k * a**3 / 2 + 1e-15 / k**2


def test_equal_volume_radius():
    h = 0.125
    a = vie.equal_volume_radius(h)
    assert abs(4.0 / 3.0 * math.pi * a**3 - h**3) < 1e-16


def test_entry_values_16_cube_eps4():
    # 16^3 voxels in one wavelength, eps = 4: values worked by hand from the formulas
    # of Section II (kappa = 3/4, kh = pi/8, ka = kh (3/(4 pi))^(1/3)).
    g = make_grid(16, 16, 16, 1 / 16, 4.0)
    kh = math.pi / 8
    ka = kh * (3 / (4 * math.pi)) ** (1 / 3)
    k2S = ka**2 / 2 - 1j * ka**3 / 3 - ka**4 / 8 + 1j * ka**5 / 30 + ka**6 / 144 - 1j * ka**7 / 840
    z = vie.entries(g, [0, 0, 0], [0, 1, 16 * 16 + 16 + 1])
    assert abs(z[0, 0] - (0.25 - 0.75 * k2S)) < 1e-8
    assert abs(z[0, 0] - (0.228074 + 0.003593j)) < 2e-6
    nn = -0.75 * kh * kh / (4 * math.pi) * complex(math.cos(kh), -math.sin(kh))
    assert abs(z[0, 1] - nn) < 1e-15
    assert abs(z[0, 1] - (-0.0085033 + 0.0035222j)) < 1e-7
    rho = math.sqrt(3.0)
    diag = -0.75 * kh * kh / (4 * math.pi * rho) * complex(math.cos(kh * rho), -math.sin(kh * rho))
    assert abs(z[0, 2] - diag) < 1e-15


def test_structure_symmetry_and_identity_limit():
    c = small_case(3, sides=(5, 4, 3))
    g = c["grid"]
    Z = vie.dense(g)
    kap = vie.contrast(g.eps)
    G = (np.diag(1 / g.eps) - Z) / kap[None, :]  # the kernel matrix K(d_mn)
    assert np.allclose(G, G.T, rtol=0, atol=1e-15)
    # free space everywhere: kappa = 0 so Z is the identity exactly
    g1 = make_grid(5, 4, 3, 0.1, 1.0)
    assert np.array_equal(vie.dense(g1), np.eye(g1.n))


def test_dense_direct_and_fft_products_agree():
    c = small_case(4, sides=(7, 6, 5), eps_range=(1.0, 9.0), loss=2.0)
    g = c["grid"]
    x = c["x"]
    y = vie.dense(g) @ x
    assert np.linalg.norm(vie.fft_matvec(g, x) - y) <= 1e-13 * np.linalg.norm(y)
    rows = [0, 17, g.n - 1]
    assert np.linalg.norm(vie.direct_rows(g, x, rows) - y[rows]) <= 1e-13 * np.linalg.norm(y[rows])


def test_fft_product_brute_force_tiny():
    g = make_grid(2, 3, 2, 0.2, np.linspace(1.5, 3.0, 12) - 0.3j)
    rng = np.random.default_rng(0)
    x = rng.standard_normal(g.n) + 1j * rng.standard_normal(g.n)
    kh = g.k0 * g.h
    a = vie.equal_volume_radius(g.h)
    y = np.zeros(g.n, dtype=complex)
    for m in range(g.n):  # pure-Python double loop over the definition
        im = (m % 2, (m // 2) % 3, m // 6)
        for n in range(g.n):
            jn = (n % 2, (n // 2) % 3, n // 6)
            kap = (g.eps[n] - 1) / g.eps[n]
            if m == n:
                zmn = 1 / g.eps[m] - ((1 + 1j * g.k0 * a) * np.exp(-1j * g.k0 * a) - 1) * kap
            else:
                rho = math.sqrt(sum((p - q) ** 2 for p, q in zip(im, jn)))
                zmn = -kh * kh / (4 * math.pi * rho) * np.exp(-1j * kh * rho) * kap
            y[m] += zmn * x[n]
    assert np.allclose(vie.fft_matvec(g, x), y, rtol=0, atol=1e-13)


def test_plane_wave():
    g = make_grid(5, 5, 5, 0.1, 2.0)
    d = np.array([[0.0, 0.0, -1.0], [0.6, 0.0, 0.8]])
    b = vie.plane_wave(g, d)
    assert np.allclose(np.abs(b), 1.0)
    centre = 2 + 5 * (2 + 5 * 2)  # odd sides: this voxel centre is the box centre
    assert np.allclose(b[centre], 1.0)
    # travelling along -z: one voxel step in +z adds phase +k h
    assert np.isclose(b[centre + 25, 0] / b[centre, 0], np.exp(1j * g.k0 * g.h))


@pytest.mark.parametrize("bad", [0.0])
def test_zero_permittivity_is_singular(bad):
    g = make_grid(2, 2, 2, 0.1, 2.0)
    g.eps[3] = bad
    with np.errstate(divide="ignore", invalid="ignore"):
        z = vie.dense(g)
    assert not np.all(np.isfinite(z))
