"""SIPF-PIC step in two dimensions, and the elliptic (eps = 0) field update
(oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 5.2 runs the method on the 2-D parabolic-elliptic system
(k, eps, mu, chi) = (0, 0, 1, 1) on the periodic square [-L/2, L/2)^2.  The
paper gives the 3-D algorithm; the 2-D step here is Algorithm 4 with d = 2.
Readings taken (the paper does not spell out the 2-D or elliptic forms):

* Grid H x H, node g (position g h) stored at g mod H, F_H with L^-2:
  beta_q = L^-2 sum_j phi_j exp(-2 pi i q.j / H), q in {-H/2 .. H/2-1}^2.
* Stencils: ``stencil.weights2d`` (12-node fourth-order deposit, bilinear
  gather).
* Field update: eq. ``alpha_hat_update`` as in 3-D.  With eps = 0 the second
  equation is elliptic, -Lap c + k^2 c = rho: A_q = 0, B_q = 1/(|xi|^2 + k^2),
  and alpha_0 := 0 when k = 0 (on the periodic box the Poisson problem only
  fixes c up to a constant and only sees rho minus its mean).
* Gaussian filter exp(-2 pi^2 |q|^2 / H0^2) on the gradient coefficients,
  H0 = ceil(8 H^(8/13) L^(5/13)) (Sec. 5.2 quotes the same rule).
* Noise: the Philox block of particle id at step n (``philox.normals6``).
  Split step: W^- = sqrt(mu tau) (z0, z1), W^+ = sqrt(mu tau) (z2, z3);
  Euler-Maruyama: W = sqrt(2 mu tau) (z0, z1).
* Mass units: phi is the deposit of weights M0/P, so sum(phi) = M0.
"""

import math

import numpy as np

from . import philox, stencil
from .sipf import Params, cell_and_frac, freqs, mode_factors_s, wrap  # noqa: F401  (Params re-exported)


def deposit(X, w, H, L, order=4):
    """Operator I in 2-D: phi[(g_p + gamma) mod H] += w_p F_gamma(lambda_p)."""
    X = np.asarray(X, dtype=np.float64)
    g, lam = cell_and_frac(X, H, L)
    w = np.broadcast_to(np.asarray(w, dtype=np.float64), (X.shape[0],))
    phi = np.zeros(H * H, dtype=np.float64)
    F = stencil.weights2d(lam, order)
    for j, gam in enumerate(stencil.offsets2d(order)):
        idx = (g + gam) % H
        phi += np.bincount(idx[:, 0] * H + idx[:, 1], weights=w * F[:, j], minlength=H * H)
    return phi.reshape(H, H)


def interp(f, X, H, L, order=2):
    """Operator I* in 2-D; f (..., H, H) -> values (P, ...)."""
    X = np.asarray(X, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    lead = f.shape[:-2]
    g, lam = cell_and_frac(X, H, L)
    F = stencil.weights2d(lam, order)
    ff = f.reshape(lead + (H * H,))
    out = np.zeros((X.shape[0],) + lead)
    for j, gam in enumerate(stencil.offsets2d(order)):
        idx = (g + gam) % H
        vals = np.moveaxis(ff[..., idx[:, 0] * H + idx[:, 1]], -1, 0)
        out += F[:, j].reshape((-1,) + (1,) * len(lead)) * vals
    return out


def wavevectors(H, L):
    q = freqs(H).astype(np.float64) * (2.0 * np.pi / L)
    return np.stack(np.meshgrid(q, q, indexing="ij"))


def forward_transform(phi, L):
    """beta_q = L^-2 sum_j phi_j exp(-2 pi i q.j / H)."""
    return np.fft.fft2(phi) / L ** 2


def inverse_transform(alpha):
    """sum_q alpha_q exp(+2 pi i q.j / H) on the grid."""
    H = alpha.shape[-1]
    return np.fft.ifft2(alpha, axes=(-2, -1)) * H ** 2


def mode_factors(prm):
    """A_q, B_q of eq. ``alpha_hat_update`` (or the exponential propagator of
    Sec. 3.4); the elliptic limit for eps = 0 (see ``sipf.mode_factors_s``)."""
    xi = wavevectors(prm.H, prm.L)
    return mode_factors_s((xi ** 2).sum(axis=0) + prm.k ** 2, prm)


def filter_factors(prm):
    H = prm.H
    if prm.H0 < 0:
        return np.ones((H, H))
    q = freqs(H).astype(np.float64)
    q2 = q[:, None] ** 2 + q[None, :] ** 2
    return np.exp(-2.0 * np.pi ** 2 * q2 / prm.h0() ** 2)


def gradient_grid(alpha, prm):
    """Re F_H^{-1}(i xi Phi alpha), shape (2, H, H)."""
    xi = wavevectors(prm.H, prm.L)
    return inverse_transform(1j * xi * (filter_factors(prm) * alpha)[None]).real


def push(X, G, n, prm, ids):
    H, L, tau = prm.H, prm.L, prm.dt
    Z = philox.normals6(ids, n, prm.seed, prm.instance)
    if prm.scheme == "strang":
        s = math.sqrt(prm.mu * tau)
        Y = X + s * Z[:, 0:2]
        v = interp(G, Y, H, L, prm.g2p_order)
        return wrap(Y + prm.chi * tau * v + s * Z[:, 2:4], L), Y, v
    if prm.scheme == "em":
        s = math.sqrt(2.0 * prm.mu * tau)
        v = interp(G, X, H, L, prm.g2p_order)
        return wrap(X + prm.chi * tau * v + s * Z[:, 0:2], L), X, v
    raise ValueError("scheme must be 'strang' or 'em'")


def step(X, alpha, n, prm, ids=None, record=None):
    """Step n of Algorithm 4 in 2-D: deposit of X^(n-1) updates alpha; the push
    gathers the gradient of alpha^(n-1)."""
    X = np.asarray(X, dtype=np.float64)
    if ids is None:
        ids = np.arange(X.shape[0], dtype=np.uint64)
    phi = deposit(X, prm.M0 / X.shape[0], prm.H, prm.L, prm.p2g_order)
    beta = forward_transform(phi, prm.L)
    A, B = mode_factors(prm)
    alpha_new = A * alpha + B * beta
    G = gradient_grid(alpha, prm)
    Xn, Y, v = push(X, G, n, prm, ids)
    if record is not None:
        record.update(phi=phi, beta=beta, G=G, Y=Y, v=v)
    return Xn, alpha_new


def run(X0, prm, nsteps, alpha0=None, ids=None, first_step=1):
    X = np.asarray(X0, dtype=np.float64).copy()
    H = prm.H
    alpha = np.zeros((H, H), dtype=np.complex128) if alpha0 is None else np.array(alpha0, dtype=np.complex128)
    for n in range(first_step, first_step + nsteps):
        X, alpha = step(X, alpha, n, prm, ids)
    return X, alpha


def half_spectrum(a):
    """ky = 0 .. H/2 of a full (H, H) spectrum (last axis halved)."""
    H = a.shape[-1]
    return np.ascontiguousarray(a[..., : H // 2 + 1])


def full_spectrum(ah):
    """Full (H, H) spectrum of a real field from its ky = 0 .. H/2 half."""
    H = ah.shape[0]
    full = np.zeros((H, H), dtype=np.complex128)
    full[:, : H // 2 + 1] = ah
    kx = (-np.arange(H)) % H
    for ky in range(H // 2 + 1, H):
        full[:, ky] = np.conj(ah[kx, H - ky])
    return full
