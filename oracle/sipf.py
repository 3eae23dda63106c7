"""SIPF-PIC time step, literal FP64 reading of the paper (oracle side).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

State after step n: particle positions X^(n) (P x 3, in [-L/2, L/2)^3) and the
Fourier coefficients alpha^(n) of the chemo-attractant c (full H^3 complex
array, index k along an axis standing for the frequency q = k for k < H/2 and
q = k - H otherwise, so q runs over U = {-H/2, ..., H/2 - 1}).

Readings of the paper taken here (the paper is silent or ambiguous):

* Index set.  Sec. 2.2 writes U = {-H/2, ..., H/2}^3, which has H + 1 points
  per axis, while Sec. 3.1 builds the physical grid from U with H points per
  axis (from -L/2 to L/2 - L/H).  U is read as {-H/2, ..., H/2 - 1}.
* Grid node g (integer vector, node position g*h) is stored at g mod H; with
  that map the F_H sums need no phase factor.
* The gradient grid is the real part of F_H^{-1}(i xi Phi alpha) (Algorithm 4).
  For a Hermitian alpha this equals zeroing the derivative factor at the
  Nyquist frequency q_d = -H/2, which the GPU library does.
* Both branches of a step read the state of the previous step (Algorithm 4):
  the mode update uses the deposit of X^(n-1); the push gathers the gradient
  of alpha^(n-1).  Hence alpha^(0) = 0 gives a drift-free first step.
* Positions are wrapped back into [-L/2, L/2) after every push ("periodic
  setting", Algorithm 4).
* The Gaussian filter is applied to the gradient coefficients as written in
  Algorithm 4 (not to the density; Sec. 5.1 describes it on the density, and
  both agree when alpha^(0) = 0 since every spectral operation is diagonal and
  linear).  H0 defaults to ceil(8 H^(8/13) L^(5/13)) (Sec. 5.1); H0 < 0
  switches the filter off.
* The source factor of the mode update follows eq. ``alpha_hat_update``
  (1/(|xi|^2 + k^2 + eps/tau)).  The operator-splitting form of Sec. 3.4 uses
  tau instead; the two coincide for eps = 1.
* Mass units: the deposit phi is the accumulator of Algorithm 2
  (phi[q] += M0 F / P), so sum(phi) = M0.
"""

import dataclasses
import math

import numpy as np

from . import philox, stencil


@dataclasses.dataclass
class Params:
    """Problem and discretisation parameters (eq. ``para_system``, Sec. 2.2, Algorithm 4)."""
    L: float = 2.0          # box side, Omega = [-L/2, L/2)^3, periodic
    chi: float = 1.0        # chemotactic sensitivity
    mu: float = 1.0         # particle diffusivity
    eps: float = 1.0        # relaxation constant of c
    k: float = 1.0          # degradation constant of c
    M0: float = 1.0         # total mass carried by the P particles
    dt: float = 1e-4        # time step tau
    H: int = 16             # grid points (Fourier modes) per axis
    H0: float = 0.0         # filter scale; 0 -> Sec. 5.1 rule; < 0 -> no filter
    p2g_order: int = 4      # order of I  (Remark after Definition grid2particle)
    g2p_order: int = 2      # order of I* (same remark)
    scheme: str = "strang"  # "strang" (Algorithm 4) or "em" (eq. rho_hat_update)
    seed: int = 0           # Philox key
    instance: int = 0       # fourth Philox counter word
    propagator: str = "implicit"  # "implicit" (eq. alpha_hat_update) or "exp" (Sec. 3.4)
    positivity: bool = False  # positivity-preserving deposit (``deposit_positive``)

    def h0(self):
        """Filter scale H0 (Sec. 5.1 rule when H0 == 0)."""
        if self.H0 == 0:
            return float(math.ceil(8.0 * self.H ** (8.0 / 13.0) * self.L ** (5.0 / 13.0)))
        return float(self.H0)


# ---------------------------------------------------------------------------
# Particle <-> grid (Sec. 3.1, Definitions particle2grid / grid2particle,
# Algorithms 2 and 3)
# ---------------------------------------------------------------------------

def cell_and_frac(X, H, L):
    """g = floor(X H / L) and lambda = X H / L - g (Sec. 3.1)."""
    s = np.asarray(X, dtype=np.float64) * (H / L)
    g = np.floor(s)
    return g.astype(np.int64), s - g


def deposit(X, w, H, L, order=4):
    """Operator I of Definition ``particle2grid`` applied to sum_p w_p delta_{X_p}.

    Algorithm 2 loop: phi[(g_p + gamma) mod H] += w_p F_gamma(lambda_p).
    X (P, 3); w scalar or (P,).  Returns phi of shape (H, H, H).
    """
    X = np.asarray(X, dtype=np.float64)
    g, lam = cell_and_frac(X, H, L)
    w = np.broadcast_to(np.asarray(w, dtype=np.float64), (X.shape[0],))
    phi = np.zeros(H * H * H, dtype=np.float64)
    offs = stencil.offsets(order)
    F = stencil.weights(lam, order)                      # (P, n_nodes)
    for j, gam in enumerate(offs):
        idx = (g + gam) % H
        flat = (idx[:, 0] * H + idx[:, 1]) * H + idx[:, 2]
        phi += np.bincount(flat, weights=w * F[:, j], minlength=H ** 3)
    return phi.reshape(H, H, H)


def deposit_positive(X, w, H, L, record=None):
    """Positivity-preserving order-4 deposit (reading of Remark ``smoothness``
    and Sec. 3.4): the order-4 weights are negative on the outer nodes, so the
    deposit can be negative next to the edge of the particle cloud.  Every
    particle starts with the order-4 weights; in each round, every particle
    still on order 4 whose 32 stencil nodes include a node where the current
    deposit is negative switches to the order-2 weights of eq. ``2ord`` (its
    inner nodes only).  Rounds repeat until one switches nobody.

    Both weight sets sum to one, so the mass is that of ``deposit``.  A node
    that is still negative has an order-4 contributor with a negative weight
    (order-2 weights are not negative), which the next round switches; the
    result is therefore >= 0, and in the bulk of the cloud, where no node is
    negative, it equals the order-4 deposit.  ``record`` receives the switched
    mask and the number of rounds that switched someone.
    """
    X = np.asarray(X, dtype=np.float64)
    P = X.shape[0]
    g, lam = cell_and_frac(X, H, L)
    w = np.broadcast_to(np.asarray(w, dtype=np.float64), (P,))
    offs = stencil.offsets(4)
    F4 = stencil.weights(lam, 4)
    F2 = np.zeros_like(F4)
    F2[:, :8] = stencil.weights(lam, 2)     # the first 8 nodes of Gamma_4 are Gamma_2, in the same order
    idx = (g[:, None, :] + offs[None, :, :]) % H
    flat = (idx[..., 0] * H + idx[..., 1]) * H + idx[..., 2]    # (P, 32)
    switched = np.zeros(P, dtype=bool)
    rounds = 0
    while True:
        F = np.where(switched[:, None], F2, F4) * w[:, None]
        phi = np.bincount(flat.ravel(), weights=F.ravel(), minlength=H ** 3)
        new = (phi[flat] < 0).any(axis=1) & ~switched
        if not new.any():
            break
        switched |= new
        rounds += 1
    if record is not None:
        record.update(switched=switched, rounds=rounds)
    return phi.reshape(H, H, H)


def interp(f, X, H, L, order=2):
    """Operator I* of Definition ``grid2particle`` (Algorithm 3).

    f has shape (H, H, H) or (..., H, H, H) (leading component axes); returns
    the interpolated values with shape (P,) or (P, ...).
    """
    X = np.asarray(X, dtype=np.float64)
    f = np.asarray(f, dtype=np.float64)
    lead = f.shape[:-3]
    g, lam = cell_and_frac(X, H, L)
    F = stencil.weights(lam, order)
    out = np.zeros((X.shape[0],) + lead, dtype=np.float64)
    ff = f.reshape(lead + (H ** 3,))
    for j, gam in enumerate(stencil.offsets(order)):
        idx = (g + gam) % H
        flat = (idx[:, 0] * H + idx[:, 1]) * H + idx[:, 2]
        vals = np.moveaxis(ff[..., flat], -1, 0)          # (P, ...)
        out += F[:, j].reshape((-1,) + (1,) * len(lead)) * vals
    return out


# ---------------------------------------------------------------------------
# Spectral side (Sec. 3.1 F_H convention, eq. alpha_hat_update, Algorithm 4)
# ---------------------------------------------------------------------------

def freqs(H):
    """Signed frequency of array index k: k for k < H/2, k - H otherwise."""
    k = np.arange(H)
    return np.where(k < H // 2, k, k - H)


def wavevectors(H, L):
    """xi_q = 2 pi q / L on the full (H, H, H) index grid, shape (3, H, H, H)."""
    q = freqs(H).astype(np.float64) * (2.0 * np.pi / L)
    return np.stack(np.meshgrid(q, q, q, indexing="ij"))


def forward_transform(phi, L):
    """beta_q = F_H I(rho)(xi_q) = L^-3 sum_j phi_j exp(-2 pi i q.j / H).

    Sec. 3.1 F_H convention applied to the sum of grid deltas produced by I;
    the FFT is the library primitive that Algorithm 2 names.
    """
    return np.fft.fftn(phi) / L ** 3


def inverse_transform(alpha):
    """F_H^{-1} alpha on the grid: sum_q alpha_q exp(+2 pi i q.j / H) (Sec. 3.1)."""
    H = alpha.shape[-1]
    return np.fft.ifftn(alpha, axes=(-3, -2, -1)) * H ** 3


def mode_factors(prm):
    """A_q = 1/(1 + tau/eps (|xi|^2 + k^2)), B_q = 1/(|xi|^2 + k^2 + eps/tau).

    Eq. ``alpha_hat_update`` / the mode update of Algorithm 4.  With eps = 0 the
    c-equation of eq. ``system`` is elliptic, -Lap c + k^2 c = rho: A_q = 0,
    B_q = 1/(|xi|^2 + k^2), and alpha_0 := 0 when k = 0 (the periodic Poisson
    problem fixes c only up to a constant and sees rho minus its mean).
    """
    xi = wavevectors(prm.H, prm.L)
    return mode_factors_s((xi ** 2).sum(axis=0) + prm.k ** 2, prm)


def mode_factors_s(s, prm):
    """A, B as functions of s = |xi|^2 + k^2 (any dimension).

    implicit (eq. alpha_hat_update): A = 1/(1 + tau s/eps), B = 1/(s + eps/tau),
    i.e. alpha' = A (alpha + (tau/eps) beta);
    exponential (Sec. 3.4): the attenuation kappa = exp(-tau s/eps) in place of
    A, alpha' = kappa (alpha + (tau/eps) beta).  Sec. 3.4 prints the source
    weight as tau; it equals tau/eps for eps = 1, and tau/eps is the weight of
    the implicit form, so that is the reading taken;
    elliptic (eps = 0): A = 0, B = 1/s, B = 0 where s = 0.
    """
    if prm.eps == 0:
        if prm.propagator != "implicit":
            raise ValueError("the exponential propagator needs eps > 0")
        return np.zeros_like(s), np.where(s > 0, 1.0 / np.where(s > 0, s, 1.0), 0.0)
    r = prm.dt / prm.eps
    if prm.propagator == "exp":
        A = np.exp(-r * s)
        return A, A * r
    if prm.propagator != "implicit":
        raise ValueError("propagator must be 'implicit' or 'exp'")
    A = 1.0 / (1.0 + r * s)
    B = 1.0 / (s + prm.eps / prm.dt)
    return A, B


def filter_factors(prm):
    """Phi_q = exp(-2 pi^2 |q|^2 / H0^2) (Algorithm 4); ones when H0 < 0."""
    H = prm.H
    if prm.H0 < 0:
        return np.ones((H, H, H))
    q = freqs(H).astype(np.float64)
    q2 = q[:, None, None] ** 2 + q[None, :, None] ** 2 + q[None, None, :] ** 2
    return np.exp(-2.0 * np.pi ** 2 * q2 / prm.h0() ** 2)


def mode_update(alpha, beta, prm):
    """alpha^(n) = A alpha^(n-1) + B beta^(n-1) (eq. ``alpha_hat_update``)."""
    A, B = mode_factors(prm)
    return A * alpha + B * beta


def gradient_grid(alpha, prm):
    """grad c on the grid: Re F_H^{-1}(i xi_q alpha_q Phi_q) (Algorithm 4).

    Returns (3, H, H, H); component d is the derivative along axis d.
    """
    xi = wavevectors(prm.H, prm.L)
    Phi = filter_factors(prm)
    return inverse_transform(1j * xi * (Phi * alpha)[None]).real


# ---------------------------------------------------------------------------
# Particle push (Algorithm 4 split step; eq. rho_hat_update Euler-Maruyama)
# ---------------------------------------------------------------------------

def wrap(X, L):
    """Periodic image in [-L/2, L/2): x - L floor((x + L/2) / L)."""
    return X - L * np.floor((X + L / 2.0) / L)


def min_image(D, L):
    """Minimum-image difference of two positions, in [-L/2, L/2)."""
    return wrap(D, L)


def push(X, G, n, prm, ids):
    """Particle branch of step n given the gradient grid G of alpha^(n-1).

    Split form (Algorithm 4):  Y = X + W^-,  X' = wrap(Y + chi tau I*G(Y) + W^+),
    W^-, W^+ ~ N(0, mu tau I_3).  Euler-Maruyama form (eq. ``rho_hat_update``):
    X' = wrap(X + chi tau I*G(X) + W), W ~ N(0, 2 mu tau I_3).
    Returns (X', Y, v, Zm, Zp) with v = I*G(Y); Zp is None for Euler-Maruyama.
    """
    H, L, tau = prm.H, prm.L, prm.dt
    if prm.scheme == "strang":
        s = math.sqrt(prm.mu * tau)
        Z6 = philox.normals6(ids, n, prm.seed, prm.instance)
        Zm, Zp = Z6[:, 0:3], Z6[:, 3:6]
        Y = X + s * Zm
        v = interp(G, Y, H, L, prm.g2p_order)
        return wrap(Y + prm.chi * tau * v + s * Zp, L), Y, v, Zm, Zp
    if prm.scheme == "em":
        s = math.sqrt(2.0 * prm.mu * tau)
        Z = philox.normals6(ids, n, prm.seed, prm.instance)[:, 0:3]
        v = interp(G, X, H, L, prm.g2p_order)
        return wrap(X + prm.chi * tau * v + s * Z, L), X, v, Z, None
    raise ValueError("scheme must be 'strang' or 'em'")


def step(X, alpha, n, prm, ids=None, record=None):
    """One SIPF-PIC step n (Algorithm 4): (X^(n-1), alpha^(n-1)) -> (X^(n), alpha^(n)).

    Field branch: phi = I(rho^(n-1)) (Algorithm 2 loop), beta = F_H phi,
    alpha^(n) = A alpha^(n-1) + B beta.  Particle branch: gradient of
    alpha^(n-1) on the grid, then ``push``.  ``record`` (dict or None) receives
    the intermediate phi, beta, G, v.
    """
    X = np.asarray(X, dtype=np.float64)
    P = X.shape[0]
    if ids is None:
        ids = np.arange(P, dtype=np.uint64)
    if prm.positivity:
        phi = deposit_positive(X, prm.M0 / P, prm.H, prm.L)
    else:
        phi = deposit(X, prm.M0 / P, prm.H, prm.L, prm.p2g_order)
    beta = forward_transform(phi, prm.L)
    alpha_new = mode_update(alpha, beta, prm)
    G = gradient_grid(alpha, prm)
    Xn, Y, v, Zm, Zp = push(X, G, n, prm, ids)
    if record is not None:
        record.update(phi=phi, beta=beta, G=G, Y=Y, v=v, Zm=Zm, Zp=Zp)
    return Xn, alpha_new


def run(X0, prm, nsteps, alpha0=None, ids=None, first_step=1, callback=None):
    """Run ``nsteps`` steps starting at step index ``first_step``.

    alpha0 None means c(x, 0) = 0 (Algorithm 4 initialisation).
    """
    X = np.asarray(X0, dtype=np.float64).copy()
    H = prm.H
    alpha = np.zeros((H, H, H), dtype=np.complex128) if alpha0 is None else np.array(alpha0, dtype=np.complex128)
    for n in range(first_step, first_step + nsteps):
        X, alpha = step(X, alpha, n, prm, ids)
        if callback is not None:
            callback(n, X, alpha)
    return X, alpha


def final_density_loss(X, prm):
    """sum_j phi_j^2 with phi the order-p2g deposit of X in mass units (Algorithm 2)."""
    phi = deposit(X, prm.M0 / X.shape[0], prm.H, prm.L, prm.p2g_order)
    return float((phi ** 2).sum()), phi


# ---------------------------------------------------------------------------
# Direct O(P H^3) SIPF sums (Algorithm 1, eqs. beta_hat_comp and gradc)
# ---------------------------------------------------------------------------

def direct_beta(X, M0, H, L):
    """beta_q = M0/(P L^3) sum_p exp(-2 pi i q.X_p / L) (eq. ``beta_hat_comp``)."""
    X = np.asarray(X, dtype=np.float64)
    q = freqs(H).astype(np.float64) * (2.0 * np.pi / L)
    ex = np.exp(-1j * np.outer(X[:, 0], q))   # (P, H)
    ey = np.exp(-1j * np.outer(X[:, 1], q))
    ez = np.exp(-1j * np.outer(X[:, 2], q))
    return np.einsum("pa,pb,pc->abc", ex, ey, ez) * (M0 / (X.shape[0] * L ** 3))


def direct_gradient(alpha, X, prm, use_filter=True):
    """sum_q i xi_q Phi_q alpha_q exp(i xi_q . X_p), real part (eq. ``gradc``)."""
    X = np.asarray(X, dtype=np.float64)
    H, L = prm.H, prm.L
    q = freqs(H).astype(np.float64) * (2.0 * np.pi / L)
    a = alpha * (filter_factors(prm) if use_filter else 1.0)
    ex = np.exp(1j * np.outer(X[:, 0], q))
    ey = np.exp(1j * np.outer(X[:, 1], q))
    ez = np.exp(1j * np.outer(X[:, 2], q))
    out = np.empty((X.shape[0], 3))
    out[:, 0] = np.einsum("abc,pa,pb,pc->p", 1j * q[:, None, None] * a, ex, ey, ez).real
    out[:, 1] = np.einsum("abc,pa,pb,pc->p", 1j * q[None, :, None] * a, ex, ey, ez).real
    out[:, 2] = np.einsum("abc,pa,pb,pc->p", 1j * q[None, None, :] * a, ex, ey, ez).real
    return out


def sipf_direct_step(X, alpha, n, prm, ids=None, use_filter=True):
    """One step of the direct SIPF method (Algorithm 1): beta from the direct
    sum over the particles (eq. beta_hat_comp), alpha by eq. alpha_hat_update,
    drift from the direct gradient sum at the particles (eq. gradc, real part;
    no grid).  Euler-Maruyama push as Algorithm 1 prints it (scheme "em"), or
    the split push of Algorithm 4 (scheme "strang") for a like-for-like
    comparison with SIPF-PIC.  ``use_filter`` applies Phi_q to the gradient
    sum (Algorithm 1 has none; prm.H0 < 0 also switches it off).
    """
    X = np.asarray(X, dtype=np.float64)
    P = X.shape[0]
    if ids is None:
        ids = np.arange(P, dtype=np.uint64)
    beta = direct_beta(X, prm.M0, prm.H, prm.L)
    alpha_new = mode_update(alpha, beta, prm)
    tau, L = prm.dt, prm.L
    Z6 = philox.normals6(ids, n, prm.seed, prm.instance)
    if prm.scheme == "em":
        v = direct_gradient(alpha, X, prm, use_filter)
        return wrap(X + prm.chi * tau * v + math.sqrt(2.0 * prm.mu * tau) * Z6[:, 0:3], L), alpha_new
    s = math.sqrt(prm.mu * tau)
    Zm, Zp = Z6[:, 0:3], Z6[:, 3:6]
    Y = X + s * Zm
    v = direct_gradient(alpha, Y, prm, use_filter)
    return wrap(Y + prm.chi * tau * v + s * Zp, L), alpha_new


def sipf_direct_run(X0, prm, nsteps, use_filter=True):
    """nsteps of ``sipf_direct_step`` from alpha^(0) = 0."""
    X = np.asarray(X0, dtype=np.float64).copy()
    H = prm.H
    alpha = np.zeros((H, H, H), dtype=np.complex128)
    for n in range(1, nsteps + 1):
        X, alpha = sipf_direct_step(X, alpha, n, prm, use_filter=use_filter)
    return X, alpha


# ---------------------------------------------------------------------------
# Half-spectrum view used by the GPU library (kz = 0 .. H/2)
# ---------------------------------------------------------------------------

def half_spectrum(a):
    """Keep the last-axis indices 0..H/2 of a full (H, H, H) spectrum."""
    H = a.shape[-1]
    return np.ascontiguousarray(a[..., : H // 2 + 1])


def full_spectrum(ah):
    """Rebuild the full spectrum of a real field from its kz = 0..H/2 half."""
    H = ah.shape[0]
    full = np.zeros((H, H, H), dtype=np.complex128)
    full[..., : H // 2 + 1] = ah
    kx = (-np.arange(H)) % H
    for kz in range(H // 2 + 1, H):
        full[:, :, kz] = np.conj(ah[kx][:, kx, H - kz])
    return full
