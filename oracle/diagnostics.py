"""Run-time diagnostics of the numerical experiments of Sec. 5 (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

* Regularised density rho_num = rho_hat_P * G0, with rho_hat_P the empirical
  measure (weights M0/P) and G0 the isotropic Gaussian of standard deviation
  L/H0 per axis (Sec. 5.2), evaluated on the physical grid.  Its maximum is
  the blow-up indicator of Sec. 5.2 and 5.3.  Reading: "reconstructed on the
  grid" is taken as the method's own route -- the P2G deposit of the
  particles, F_H, the Gaussian factor Phi_q = exp(-2 pi^2 |q|^2 / H0^2) (the
  Fourier transform of G0) and the inverse transform back to the nodes.  It
  differs from the plain convolution by the interpolation error of the
  deposit (fourth order in h for a smooth G0).
* Share of the energy of c_hat in the high-frequency modes |q| >= 4 (Sec. 5.2):
  sum_{|q|>=4} |alpha_q|^2 / sum_q |alpha_q|^2 over the full spectrum.
* Numerical ring radius R_num = (1/P) sum_p sqrt(X_p1^2 + X_p2^2) (Sec. 5.5).
* Second moment m2 = (1/P) sum_p |X_p|^2 (Sec. 5.2, in three dimensions here).
* Mass of rho_num on the grid, sum_j rho_num(x_j) h^3 (= M0), and the integral
  of c_hat over the box, L^3 Re alpha_0.
"""

import numpy as np

from . import sipf, sipf2d


def rho_num(X, prm):
    """rho_num at the grid nodes, (H, H, H) or (H, H) for 2-D positions:
    Re F_H^{-1}(Phi F_H I(rho_hat_P))."""
    X = np.asarray(X, dtype=np.float64)
    m = sipf2d if X.shape[1] == 2 else sipf
    phi = m.deposit(X, prm.M0 / X.shape[0], prm.H, prm.L, prm.p2g_order)
    beta = m.forward_transform(phi, prm.L)
    return m.inverse_transform(m.filter_factors(prm) * beta).real


def rho_num_direct(X, prm, nodes, images=1):
    """Plain definition: sum_p (M0/P) G0(x - X_p) over periodic images, at the
    given node coordinates (N, 3)."""
    X = np.asarray(X, dtype=np.float64)
    nodes = np.asarray(nodes, dtype=np.float64)
    s = prm.L / prm.h0()
    norm = (2.0 * np.pi * s * s) ** -1.5 * prm.M0 / X.shape[0]
    out = np.zeros(nodes.shape[0])
    r = np.arange(-images, images + 1)
    for mx in r:
        for my in r:
            for mz in r:
                shift = prm.L * np.array([mx, my, mz], dtype=np.float64)
                d = nodes[:, None, :] - X[None, :, :] - shift
                out += norm * np.exp(-np.sum(d * d, axis=2) / (2.0 * s * s)).sum(axis=1)
    return out


def grid_mass(rho, L):
    """sum_j rho(x_j) h^d with h = L / H (d = rho.ndim)."""
    H = rho.shape[-1]
    return float(rho.sum() * (L / H) ** rho.ndim)


def hf_share(alpha, qmin=4.0):
    """sum_{|q| >= qmin} |alpha_q|^2 / sum_q |alpha_q|^2 (full spectrum)."""
    alpha = np.asarray(alpha)
    H = alpha.shape[-1]
    q = sipf.freqs(H).astype(np.float64)
    if alpha.ndim == 2:
        q2 = q[:, None] ** 2 + q[None, :] ** 2
    else:
        q2 = q[:, None, None] ** 2 + q[None, :, None] ** 2 + q[None, None, :] ** 2
    e = np.abs(alpha) ** 2
    tot = e.sum()
    return float(e[q2 >= qmin * qmin].sum() / tot) if tot > 0 else 0.0


def r_num(X):
    X = np.asarray(X, dtype=np.float64)
    return float(np.mean(np.sqrt(X[:, 0] ** 2 + X[:, 1] ** 2)))


def second_moment(X):
    X = np.asarray(X, dtype=np.float64)
    return float(np.mean(np.sum(X * X, axis=1)))


def c_integral(alpha, L):
    """Integral of c_hat over the box: L^d Re alpha_0."""
    alpha = np.asarray(alpha)
    return float(L ** alpha.ndim * np.real(alpha.flat[0]))


def all_diagnostics(X, alpha, prm):
    rho = rho_num(X, prm)
    return dict(mass=grid_mass(rho, prm.L), c_integral=c_integral(alpha, prm.L), rho_max=float(rho.max()),
                hf_share=hf_share(alpha), r_num=r_num(X), m2=second_moment(X))
