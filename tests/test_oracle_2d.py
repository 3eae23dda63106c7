"""Pins of the 2-D step and of the elliptic field update (oracle side): the
2-D stencil, mass, the transform, single-mode elliptic solutions, Brownian
variance, and the pair identity behind the second-moment law of Sec. 2.1
(eq. ``second_moment``)."""

import math

import numpy as np

from oracle import sipf, sipf2d, stencil
from oracle.sipf import Params


def test_stencil_2d_sums_to_one_and_reproduces_cubics():
    rng = np.random.default_rng(0)
    lam = rng.random((200, 2))
    for order, deg in ((2, 1), (4, 3)):
        W = stencil.weights2d(lam, order)
        off = stencil.offsets2d(order)
        assert W.shape == (200, 4 if order == 2 else 12)
        for a in range(deg + 1):
            for b in range(deg + 1 - a):
                got = (W * off[None, :, 0] ** a * off[None, :, 1] ** b).sum(-1)
                assert np.abs(got - lam[:, 0] ** a * lam[:, 1] ** b).max() < 1e-13, (order, a, b)
    W = stencil.weights2d(lam, 4)
    off = stencil.offsets2d(4)
    # degree 4 is not reproduced (fourth-order, not fifth)
    assert np.abs((W * off[None, :, 0] ** 4).sum(-1) - lam[:, 0] ** 4).max() > 0.1
    assert np.abs((W * (off[None, :, 0] * off[None, :, 1]) ** 2).sum(-1) - (lam[:, 0] * lam[:, 1]) ** 2).max() > 0.01


def test_stencil_2d_is_the_3d_stencil_on_a_plane():
    """The 3-D weights at lambda_3 = 0 put all weight on the nodes with
    gamma_3 = 0, and those weights are the 2-D ones."""
    rng = np.random.default_rng(1)
    lam2 = rng.random((50, 2))
    lam3 = np.concatenate([lam2, np.zeros((50, 1))], axis=1)
    W3 = stencil.weights(lam3, 4)
    off3 = stencil.offsets(4)
    W2 = stencil.weights2d(lam2, 4)
    off2 = stencil.offsets2d(4)
    for j, o in enumerate(off2):
        k = [i for i, o3 in enumerate(off3) if tuple(o3) == (o[0], o[1], 0)][0]
        assert np.abs(W3[:, k] - W2[:, j]).max() < 1e-15
    rest = [i for i, o3 in enumerate(off3) if o3[2] != 0]
    assert np.abs(W3[:, rest]).max() < 1e-15


def test_deposit_2d_mass_and_translation():
    rng = np.random.default_rng(2)
    X = rng.uniform(-1, 1, (500, 2))
    phi = sipf2d.deposit(X, 0.37, 16, 2.0)
    assert abs(phi.sum() - 0.37 * 500) < 1e-11
    shifted = sipf2d.deposit(X + np.array([2.0 / 16, 0.0]), 0.37, 16, 2.0)
    assert np.abs(shifted - np.roll(phi, 1, axis=0)).max() < 1e-12


def test_transform_2d_is_the_naive_dft():
    rng = np.random.default_rng(3)
    H, L = 8, 3.0
    phi = rng.normal(size=(H, H))
    beta = sipf2d.forward_transform(phi, L)
    j = np.arange(H)
    q = sipf.freqs(H)
    E = np.exp(-2j * np.pi * np.outer(q, j) / H)
    naive = np.einsum("aj,bk,jk->ab", E, E, phi) / L ** 2
    assert np.abs(beta[q % H][:, q % H] - naive).max() < 1e-12
    back = sipf2d.inverse_transform(beta).real * L ** 2 / H ** 2
    assert np.abs(back - phi).max() < 1e-12


def test_elliptic_single_mode_gradient_2d_and_3d():
    """eps = 0, k = 0: for rho = 1 + cos(2 pi 3 x / L) the periodic solution of
    -Lap c = rho - mean is c = cos(2 pi 3 x / L) / (2 pi 3 / L)^2, so
    dc/dx = -sin(2 pi 3 x / L) / (2 pi 3 / L); the mean mode is dropped."""
    L, H, m = 2.0, 16, 3
    kx = 2 * np.pi * m / L
    x = np.arange(H) * (L / H)
    prm = Params(L=L, H=H, eps=0.0, k=0.0, H0=-1.0, dt=1e-3)
    rho = 1.0 + np.cos(kx * x)[:, None] * np.ones((1, H))
    beta = np.fft.fft2(rho) / H ** 2        # Fourier coefficients of rho
    A, B = sipf2d.mode_factors(prm)
    assert np.all(A == 0) and B[0, 0] == 0.0
    G = sipf2d.gradient_grid(A * 0 + B * beta, prm)
    assert np.abs(G[0] - (-np.sin(kx * x) / kx)[:, None]).max() < 1e-12
    assert np.abs(G[1]).max() < 1e-12
    rho3 = 1.0 + np.cos(kx * x)[None, :, None] * np.ones((H, 1, H))
    beta3 = np.fft.fftn(rho3) / H ** 3
    A3, B3 = sipf.mode_factors(prm)
    assert np.all(A3 == 0) and B3[0, 0, 0] == 0.0
    G3 = sipf.gradient_grid(B3 * beta3, prm)
    assert np.abs(G3[1] - (-np.sin(kx * x) / kx)[None, :, None]).max() < 1e-12
    assert np.abs(G3[0]).max() < 1e-12 and np.abs(G3[2]).max() < 1e-12
    # with k > 0 the screened solution: factor 1 / (kx^2 + k^2)
    prm_k = Params(L=L, H=H, eps=0.0, k=0.7, H0=-1.0, dt=1e-3)
    Gk = sipf2d.gradient_grid(sipf2d.mode_factors(prm_k)[1] * beta, prm_k)
    assert np.abs(Gk[0] - (-kx * np.sin(kx * x) / (kx ** 2 + 0.49))[:, None]).max() < 1e-12


def test_brownian_variance_2d():
    P = 20000
    for scheme in ("strang", "em"):
        prm = Params(L=50.0, H=8, chi=0.0, mu=0.7, dt=1e-2, M0=1.0, scheme=scheme, seed=9)
        X, _ = sipf2d.run(np.zeros((P, 2)), prm, 5)
        var = X.var(axis=0)
        want = 2 * 0.7 * 5 * 1e-2
        assert np.abs(var / want - 1).max() < 0.05, (scheme, var)


def test_first_step_has_no_drift_2d():
    rng = np.random.default_rng(5)
    X0 = rng.normal(0, 0.2, (300, 2))
    prm = Params(L=2.0, H=16, chi=5.0, mu=1.0, dt=1e-3, M0=50.0, eps=0.0, k=0.0, seed=4)
    X1, alpha = sipf2d.step(X0, np.zeros((16, 16), complex), 1, prm)
    from oracle import philox
    Z = philox.normals6(np.arange(300, dtype=np.uint64), 1, 4, 0)
    s = math.sqrt(1e-3)
    assert np.abs(X1 - sipf.wrap(X0 + s * Z[:, 0:2] + s * Z[:, 2:4], 2.0)).max() < 1e-14
    assert alpha[0, 0] == 0.0 and np.abs(alpha).max() > 0


def test_pair_identity_of_the_second_moment_law():
    """Sec. 2.1: d/dt m2 = 4 mu - chi M0 / (2 pi) per unit mass comes from
    E[X . grad c(X)] = -M0 / (4 pi) for the Newtonian potential.  On the
    periodic square the zero-mean Green's function adds |x|^2 / (4 L^2), which
    adds (M0 / (2 L^2)) (m2 - |xbar|^2) to E[X . grad c(X)]; the oracle's
    elliptic gradient at the particles of a uniform disk reproduces the sum to
    1 % (0.25 % measured)."""
    rng = np.random.default_rng(6)
    P = 40000
    th = rng.uniform(0, 2 * np.pi, P)
    r = np.sqrt(rng.random(P))
    X = np.stack([r * np.cos(th), r * np.sin(th)], axis=1)
    M0, L, H = 25.0, 8.0, 128
    prm = Params(L=L, H=H, M0=M0, eps=0.0, k=0.0, chi=1.0, mu=1.0, dt=1e-3)
    beta = sipf2d.forward_transform(sipf2d.deposit(X, M0 / P, H, L), L)
    v = sipf2d.interp(sipf2d.gradient_grid(sipf2d.mode_factors(prm)[1] * beta, prm), X, H, L, 2)
    D = np.mean(np.sum(X * v, axis=1))
    xb = X.mean(axis=0)
    m2 = np.mean(np.sum(X * X, axis=1))
    want = -M0 / (4 * math.pi) + (M0 / L ** 2) * (m2 - xb @ xb) / 2
    assert abs(D - want) < 0.01 * abs(want), (D, want)
    # the background term is resolved: without it the mismatch is 5 %
    assert abs(D + M0 / (4 * math.pi)) > 0.03 * M0 / (4 * math.pi)


def test_half_spectrum_round_trip_2d():
    rng = np.random.default_rng(7)
    a = np.fft.fft2(rng.normal(size=(8, 8)))
    assert np.abs(sipf2d.full_spectrum(sipf2d.half_spectrum(a)) - a).max() < 1e-12


def test_exponential_propagator_is_exact_for_free_modes():
    """Sec. 3.4: kappa = exp(-tau s / eps) makes the homogeneous update exact:
    after n steps a free mode has decayed by exp(-n tau s / eps), and with
    k = 0 the mean of c grows exactly as M0 t / eps (eps C' = M0)."""
    for mod, H in ((sipf, 8), (sipf2d, 16)):
        prm = Params(L=2.0, H=H, eps=0.4, k=0.3, dt=0.01, propagator="exp")
        A, B = mod.mode_factors(prm)
        xi = mod.wavevectors(H, 2.0)
        s = (xi ** 2).sum(axis=0) + 0.09
        assert np.abs(A ** 25 - np.exp(-25 * 0.01 * s / 0.4)).max() < 1e-14
        assert np.abs(B - A * 0.01 / 0.4).max() < 1e-16
    prm = Params(L=2.0, H=8, eps=0.5, k=0.0, dt=0.02, propagator="exp", M0=3.0)
    X = np.random.default_rng(1).normal(0, 0.2, (50, 3))
    _, alpha = sipf.run(X, prm, 7)
    assert abs(alpha[0, 0, 0].real * 8.0 - 3.0 * 7 * 0.02 / 0.5) < 1e-12


def test_exponential_and_implicit_propagators_agree_to_first_order():
    """The two updates differ at O((tau s / eps)^2) per step (Sec. 3.4 remark)."""
    prm_i = Params(L=2.0, H=8, eps=1.0, k=1.0, dt=1e-4)
    prm_e = Params(L=2.0, H=8, eps=1.0, k=1.0, dt=1e-4, propagator="exp")
    Ai, Bi = sipf.mode_factors(prm_i)
    Ae, Be = sipf.mode_factors(prm_e)
    s = (sipf.wavevectors(8, 2.0) ** 2).sum(axis=0) + 1.0
    r = 1e-4 * s
    assert np.abs(Ai - Ae).max() <= (r ** 2).max()
    assert np.abs(Bi - Be).max() <= 1e-4 * (r ** 2).max()
