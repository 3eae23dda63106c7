"""Pathwise adjoint of the SIPF-PIC step (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Loss: L = sum_j phi_j^2 where phi is the Algorithm 2 deposit (mass units, P2G
order ``p2g_order``) of the final positions X^(N).  The gradient is taken along
one noise path: the Philox normals are held fixed, floor() has derivative 0
and the periodic wrap has derivative I (both almost everywhere).  The
transposes of the particle/grid operators follow the adjoint relation
<I rho, f> = <rho, I* f> of Sec. 3.1.

Complex cotangents use the convention a_bar = dL/dRe(a) + i dL/dIm(a), so that
dL = Re(conj(a_bar) da).  With it:
  * alpha^(n) = A alpha^(n-1) + B beta    ->  alpha_bar^(n-1) += A alpha_bar^(n),
                                             beta_bar = B alpha_bar^(n)
  * beta = L^-3 DFT(phi), phi real         ->  phi_bar = L^-3 Re(IDFT_unnorm(beta_bar))
  * G_d = Re IDFT_unnorm(i xi_d Phi alpha) ->  alpha_bar += sum_d (-i xi_d Phi) DFT(G_bar_d)

Returns dL/dX^(0), dL/dchi, dL/dmu.  All forward states are stored (the
checkpointing of the GPU library is a memory strategy, not a different
gradient).
"""

import math

import numpy as np

from . import sipf, stencil


def deposit_adjoint(X, phi_bar, w, H, L, order):
    """X_bar of phi = I(sum_p w delta_{X_p}): w (H/L) sum_gamma phi_bar[g+gamma] dF/dlambda."""
    g, lam = sipf.cell_and_frac(X, H, L)
    dF = stencil.dweights(lam, order)                  # (P, n, 3)
    flat_phi = phi_bar.reshape(-1)
    out = np.zeros_like(np.asarray(X, dtype=np.float64))
    for j, gam in enumerate(stencil.offsets(order)):
        idx = (g + gam) % H
        flat = (idx[:, 0] * H + idx[:, 1]) * H + idx[:, 2]
        out += flat_phi[flat][:, None] * dF[:, j, :]
    return out * (w * H / L)


def interp_jacobian(G, Y, H, L, order):
    """J[p, d, a] = d (I* G_d)(Y_p) / d Y_a (piecewise-polynomial derivative)."""
    g, lam = sipf.cell_and_frac(Y, H, L)
    dF = stencil.dweights(lam, order)                  # (P, n, 3)
    Gf = G.reshape(3, -1)
    J = np.zeros((Y.shape[0], 3, 3))
    for j, gam in enumerate(stencil.offsets(order)):
        idx = (g + gam) % H
        flat = (idx[:, 0] * H + idx[:, 1]) * H + idx[:, 2]
        J += Gf[:, flat].T[:, :, None] * dF[:, j, None, :]
    return J * (H / L)


def interp_transpose(vbar, Y, H, L, order):
    """Transpose of G -> I*G(Y): G_bar_d = deposit of weights vbar[:, d] (Sec. 3.1 adjoint relation)."""
    return np.stack([sipf.deposit(Y, vbar[:, d], H, L, order) for d in range(3)])


def forward_with_tape(X0, prm, nsteps, ids=None):
    """Run the forward pass storing (X^(n-1), alpha^(n-1)) for n = 1..N."""
    P = X0.shape[0]
    if ids is None:
        ids = np.arange(P, dtype=np.uint64)
    H = prm.H
    X = np.asarray(X0, dtype=np.float64).copy()
    alpha = np.zeros((H, H, H), dtype=np.complex128)
    tape = []
    for n in range(1, nsteps + 1):
        tape.append((X.copy(), alpha.copy()))
        X, alpha = sipf.step(X, alpha, n, prm, ids)
    return X, alpha, tape


def loss_and_grad(X0, prm, nsteps, ids=None, phi_bar=None):
    """(L, dL/dX0, dL/dchi, dL/dmu) along the fixed noise path.

    phi_bar None means L = sum phi^2 (so phi_bar = 2 phi); otherwise L is the
    linear functional sum(phi_bar * phi) and phi_bar is the given cotangent.
    """
    X0 = np.asarray(X0, dtype=np.float64)
    P = X0.shape[0]
    if ids is None:
        ids = np.arange(P, dtype=np.uint64)
    H, L, tau, chi = prm.H, prm.L, prm.dt, prm.chi
    w = prm.M0 / P
    XN, _, tape = forward_with_tape(X0, prm, nsteps, ids)
    phiN = sipf.deposit(XN, w, H, L, prm.p2g_order)
    if phi_bar is None:
        loss = float((phiN ** 2).sum())
        phi_bar = 2.0 * phiN
    else:
        phi_bar = np.asarray(phi_bar, dtype=np.float64)
        loss = float((phi_bar * phiN).sum())
    Xbar = deposit_adjoint(XN, phi_bar, w, H, L, prm.p2g_order)
    alpha_bar = np.zeros((H, H, H), dtype=np.complex128)
    chi_bar = 0.0
    s_bar = 0.0
    A, B = sipf.mode_factors(prm)
    xi = sipf.wavevectors(H, L)
    Phi = sipf.filter_factors(prm)
    for n in range(nsteps, 0, -1):
        Xp, alpha_p = tape[n - 1]
        G = sipf.gradient_grid(alpha_p, prm)
        _, Y, v, Zm, Zp = sipf.push(Xp, G, n, prm, ids)
        # X^(n) = wrap(Y + chi tau v + s Z+)  (Euler-Maruyama: Y = X, no Z+)
        chi_bar += tau * float((Xbar * v).sum())
        vbar = chi * tau * Xbar
        J = interp_jacobian(G, Y, H, L, prm.g2p_order)
        Ybar = Xbar + np.einsum("pd,pda->pa", vbar, J)
        Gbar = interp_transpose(vbar, Y, H, L, prm.g2p_order)
        if prm.scheme == "strang":
            s_bar += float((Xbar * Zp).sum()) + float((Ybar * Zm).sum())
        else:
            s_bar += float((Xbar * Zm).sum())
        # alpha^(n) = A alpha^(n-1) + B beta(phi(X^(n-1)))
        beta_bar = B * alpha_bar
        alpha_bar = A * alpha_bar
        # G = Re IDFT(i xi Phi alpha^(n-1))
        for d in range(3):
            alpha_bar = alpha_bar + (-1j * xi[d] * Phi) * np.fft.fftn(Gbar[d])
        phi_bar_n = (np.fft.ifftn(beta_bar) * H ** 3).real / L ** 3
        Xbar = Ybar + deposit_adjoint(Xp, phi_bar_n, w, H, L, prm.p2g_order)
    if prm.scheme == "strang":
        dsdmu = tau / (2.0 * math.sqrt(prm.mu * tau))
    else:
        dsdmu = tau / math.sqrt(2.0 * prm.mu * tau)
    return loss, Xbar, chi_bar, s_bar * dsdmu


def loss_only(X0, prm, nsteps, ids=None, phi_bar=None):
    """Forward loss for finite-difference checks."""
    XN, _ = sipf.run(X0, prm, nsteps, ids=ids)
    phiN = sipf.deposit(XN, prm.M0 / XN.shape[0], prm.H, prm.L, prm.p2g_order)
    if phi_bar is None:
        return float((phiN ** 2).sum())
    return float((np.asarray(phi_bar) * phiN).sum())

