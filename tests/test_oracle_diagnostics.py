"""Pins of the oracle's diagnostics (Sec. 5.2, 5.5) to closed forms, the plain
definition of rho_num and the exact mean-mode dynamics."""

import math

import numpy as np

from oracle import diagnostics as D
from oracle import sipf


def _nodes(H, L, idx):
    g = np.arange(H)
    g = np.where(g < H // 2, g, g - H) * (L / H)
    return g[idx]


def test_rho_num_converges_to_the_gaussian_convolution_at_fourth_order():
    """The deposit-filter-inverse route against the plain sum of Gaussians of
    standard deviation L/H0 (periodic images) at fixed H0: the error falls by
    about 2^4 per doubling of H."""
    rng = np.random.default_rng(1)
    X = rng.normal(0.0, 0.2, (300, 3))
    errs = []
    for H in (16, 32, 64):
        prm = sipf.Params(L=2.0, H=H, H0=6.0, M0=5.0)
        rho = D.rho_num(X, prm)
        idx = rng.integers(0, H, (200, 3))
        direct = D.rho_num_direct(X, prm, _nodes(H, 2.0, idx), images=2)
        errs.append(np.abs(rho[idx[:, 0], idx[:, 1], idx[:, 2]] - direct).max() / np.abs(direct).max())
    assert errs[0] / errs[1] > 10 and errs[1] / errs[2] > 10, errs
    assert errs[2] < 2e-5


def test_rho_num_mass_and_positivity_of_a_smooth_cloud():
    rng = np.random.default_rng(2)
    X = rng.uniform(-1.0, 1.0, (5000, 3))
    prm = sipf.Params(L=2.0, H=16, M0=7.5)
    assert abs(D.grid_mass(D.rho_num(X, prm), 2.0) - 7.5) < 1e-12
    # a uniform cloud smoothed at standard deviation L/H0 = 0.5: rho_num is
    # M0 / L^3 up to sampling noise (about 1200 particles per kernel volume)
    rho = D.rho_num(X, sipf.Params(L=2.0, H=16, M0=7.5, H0=4.0))
    assert abs(D.grid_mass(rho, 2.0) - 7.5) < 1e-12
    assert np.abs(rho / (7.5 / 8.0) - 1.0).max() < 0.15


def test_hf_share_of_single_modes():
    H, L = 16, 2.0
    x = np.arange(H) * (L / H)
    X, Y, Z = np.meshgrid(x, x, x, indexing="ij")

    def share(c):
        return D.hf_share(np.fft.fftn(c) / H ** 3)

    # 1 + cos(2 pi 5 x / L): energies 1 (q = 0) and 1/4 + 1/4 (q = +-5)
    assert abs(share(1.0 + np.cos(2 * np.pi * 5 * X / L)) - 1.0 / 3.0) < 1e-13
    # |q| = 3 and |q| = sqrt(12) < 4: no high-frequency energy
    assert share(1.0 + np.cos(2 * np.pi * 3 * Y / L)) < 1e-25
    assert share(np.cos(2 * np.pi * (2 * X + 2 * Y + 2 * Z) / L)) < 1e-25
    # |q| = sqrt(18) >= 4 and exactly |q| = 4: all of it
    assert abs(share(np.sin(2 * np.pi * (3 * X + 3 * Z) / L)) - 1.0) < 1e-13
    assert abs(share(np.cos(2 * np.pi * 4 * Z / L)) - 1.0) < 1e-13
    # two modes with amplitudes 2 and 1: shares 4/5 and 1/5 by Parseval
    assert abs(share(2 * np.cos(2 * np.pi * 6 * X / L) + np.cos(2 * np.pi * 1 * Y / L)) - 0.8) < 1e-13


def test_particle_moments_of_the_uniform_ball():
    """Uniform ball of radius 1: E|X|^2 = 3/5 and E sqrt(x1^2 + x2^2) = 3 pi / 16."""
    rng = np.random.default_rng(3)
    v = rng.normal(size=(400_000, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    X = v * np.cbrt(rng.random(400_000))[:, None]
    assert abs(D.second_moment(X) - 0.6) < 2.5e-3
    assert abs(D.r_num(X) - 3.0 * math.pi / 16.0) < 2.5e-3
    # a ring of radius R in the x1-x2 plane: R_num = R exactly
    th = rng.uniform(0, 2 * np.pi, 1000)
    ring = np.stack([0.7 * np.cos(th), 0.7 * np.sin(th), rng.normal(0, 0.1, 1000)], axis=1)
    assert abs(D.r_num(ring) - 0.7) < 1e-14


def test_c_integral_follows_the_mean_mode_recursion():
    """alpha_0^(n) = A_0 alpha_0^(n-1) + B_0 M0 / L^3 from alpha_0 = 0 gives
    int c_hat = (M0 / k^2) (1 - A_0^n), A_0 = 1 / (1 + tau k^2 / eps)."""
    rng = np.random.default_rng(4)
    prm = sipf.Params(L=2.0, H=8, M0=30.0, k=0.7, eps=0.3, dt=1e-2, chi=1.0, mu=1.0)
    X0 = rng.normal(0.0, 0.2, (200, 3))
    _, alpha = sipf.run(X0, prm, 9)
    A0 = 1.0 / (1.0 + prm.dt * prm.k ** 2 / prm.eps)
    want = prm.M0 / prm.k ** 2 * (1.0 - A0 ** 9)
    assert abs(D.c_integral(alpha, prm.L) - want) < 1e-12 * want


def test_rho_num_2d_converges_to_the_gaussian_convolution():
    """Two dimensions: deposit-filter-inverse against the plain sum of 2-D
    Gaussians of standard deviation L/H0 (periodic images)."""
    rng = np.random.default_rng(11)
    X = rng.normal(0.0, 0.2, (400, 2))
    errs = []
    for H in (16, 32, 64):
        prm = sipf.Params(L=2.0, H=H, H0=6.0, M0=3.0)
        rho = D.rho_num(X, prm)
        assert abs(D.grid_mass(rho, 2.0) - 3.0) < 1e-12
        idx = rng.integers(0, H, (150, 2))
        g = np.arange(H)
        g = np.where(g < H // 2, g, g - H) * (2.0 / H)
        nodes = g[idx]
        s = 2.0 / 6.0
        direct = np.zeros(len(nodes))
        for mx in (-1, 0, 1):
            for my in (-1, 0, 1):
                d = nodes[:, None, :] - X[None, :, :] - 2.0 * np.array([mx, my])
                direct += (3.0 / 400) / (2 * np.pi * s * s) * np.exp(-np.sum(d * d, axis=2) / (2 * s * s)).sum(axis=1)
        errs.append(np.abs(rho[idx[:, 0], idx[:, 1]] - direct).max() / np.abs(direct).max())
    assert errs[0] / errs[1] > 10 and errs[1] / errs[2] > 10, errs


def test_hf_share_2d_and_c_integral_2d():
    H, L = 16, 2.0
    x = np.arange(H) * (L / H)
    X, Y = np.meshgrid(x, x, indexing="ij")
    a = np.fft.fft2(1.0 + np.cos(2 * np.pi * (3 * X + 3 * Y) / L)) / H ** 2
    assert abs(D.hf_share(a) - 1.0 / 3.0) < 1e-13          # |q| = sqrt(18) >= 4
    a = np.fft.fft2(2.0 + np.cos(2 * np.pi * (2 * X + 3 * Y) / L)) / H ** 2
    assert D.hf_share(a) < 1e-25                             # |q| = sqrt(13) < 4
    assert abs(D.c_integral(a, L) - 2.0 * L ** 2) < 1e-12
