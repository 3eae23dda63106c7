"""Radially symmetric reference solution and the truncated quantile discrepancy
(oracle side) for the convergence study of Sec. 5.1.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 5.1 reduces the Keller-Segel system for a spherically symmetric density
psi(r, t) to its radial form (eq. ``1D``) and solves it with an implicit finite
volume method on a ball of radius R_ball, chosen so that the ball and the
periodic cube [-L/2, L/2)^3 have the same volume.  The paper gives no further
detail; this module writes the radial equations in conservation form,

    psi_t   = r^-2 d/dr [ r^2 (mu psi_r - chi psi c_r) ],
    eps c_t = r^-2 d/dr [ r^2 c_r ] - k^2 c + psi,

(expanding the derivatives gives eq. ``1D``), with zero flux at r = 0 (the
face has zero area) and at r = R_ball.  Each step is backward Euler: first c
from psi^n, then psi with the drift of c^(n+1) -- diffusion centred, drift
upwinded by the sign of c_r at the face.  Both are tridiagonal solves; the
psi update conserves mass to rounding.

The comparison criterion is the mass fraction m(r) inside radius r and the
truncated quantile discrepancy E = (1/(m+1)) sum_{j<=m} |q_{j/n} - qhat_{j/n}|
with n = 1000 and m = ceil(3n/4) - 1.
"""

import math

import numpy as np
from scipy.linalg import solve_banded


def ball_radius(L):
    """R_ball with (4 pi / 3) R^3 = L^3 (Sec. 5.1)."""
    return (3.0 * L ** 3 / (4.0 * math.pi)) ** (1.0 / 3.0)


class Grid:
    """N finite volumes on [0, R]: faces r_f (N+1), centres r_c, volumes V."""

    def __init__(self, R, N):
        self.R, self.N = float(R), int(N)
        self.rf = np.linspace(0.0, self.R, self.N + 1)
        self.rc = 0.5 * (self.rf[1:] + self.rf[:-1])
        self.V = 4.0 * math.pi / 3.0 * (self.rf[1:] ** 3 - self.rf[:-1] ** 3)
        self.A = 4.0 * math.pi * self.rf ** 2          # face areas
        self.dr = self.R / self.N

    def ball_average(self, radius, value):
        """Cell averages of value * 1{r <= radius} (exact volume fractions)."""
        inner = np.clip(self.rf[:-1], 0.0, radius)
        outer = np.clip(self.rf[1:], 0.0, radius)
        return value * (4.0 * math.pi / 3.0) * (outer ** 3 - inner ** 3) / self.V


def _diffusion_matrix(g, coef):
    """Banded (3 x N) matrix of  -(1/V_i) sum_faces A coef (u_j - u_i)/dr,
    i.e. the negative radial Laplacian times coef with zero-flux ends."""
    N = g.N
    w = g.A[1:-1] * coef / g.dr                 # interior faces 1 .. N-1
    lower = np.zeros(N)
    upper = np.zeros(N)
    diag = np.zeros(N)
    diag[:-1] += w / g.V[:-1]
    diag[1:] += w / g.V[1:]
    upper[1:] = -w / g.V[:-1]                   # row i, column i+1 (banded layout)
    lower[:-1] = -w / g.V[1:]                   # row i+1, column i
    return lower, diag, upper


def step_c(g, c, psi, eps, k, dt):
    """eps (c' - c)/dt = lap c' - k^2 c' + psi  (backward Euler)."""
    lo, d, up = _diffusion_matrix(g, 1.0)
    ab = np.zeros((3, g.N))
    ab[0] = up
    ab[1] = d + k * k + eps / dt
    ab[2] = lo
    return solve_banded((1, 1), ab, psi + (eps / dt) * c)


def step_psi(g, psi, c, mu, chi, dt):
    """(psi' - psi)/dt = div(mu grad psi' - chi psi' grad c)  (backward Euler,
    upwind drift at each face, zero flux at both ends)."""
    N = g.N
    lo, d, up = _diffusion_matrix(g, mu)
    # drift velocity at interior faces: u = chi dc/dr
    u = chi * (c[1:] - c[:-1]) / g.dr
    flux_w = g.A[1:-1] * u                      # outward volume flux through face i+1/2
    # upwind: face between i and i+1 carries psi_i u if u > 0, else psi_{i+1} u
    pos = np.maximum(flux_w, 0.0)
    neg = np.minimum(flux_w, 0.0)
    # d/dt psi_i V_i = -(F_{i+1/2} - F_{i-1/2}) with F = pos psi_i + neg psi_{i+1}
    diag = d.copy()
    diag[:-1] += pos / g.V[:-1]
    diag[1:] -= neg / g.V[1:]
    upper = up.copy()
    lower = lo.copy()
    upper[1:] += neg / g.V[:-1]
    lower[:-1] -= pos / g.V[1:]
    ab = np.zeros((3, N))
    ab[0] = upper
    ab[1] = diag + 1.0 / dt
    ab[2] = lower
    return solve_banded((1, 1), ab, psi / dt)


def solve(M0=80.0, mu=1.0, chi=1.0, eps=1e-4, k=0.1, T=0.02, dt=1e-5, L=8.0, N=400_000,
          ball=1.0, callback=None):
    """Reference psi(r, T) and c(r, T) for psi(r, 0) = M0 / |B_ball| on r <= ball,
    c(r, 0) = 0 (Sec. 5.1).  Returns (grid, psi, c)."""
    g = Grid(ball_radius(L), N)
    psi = g.ball_average(ball, M0 / (4.0 * math.pi / 3.0 * ball ** 3))
    c = np.zeros(g.N)
    nsteps = int(round(T / dt))
    for n in range(1, nsteps + 1):
        c = step_c(g, c, psi, eps, k, dt)
        psi = step_psi(g, psi, c, mu, chi, dt)
        if callback is not None:
            callback(n, g, psi, c)
    return g, psi, c


def mass_fraction(g, psi):
    """m at the faces r_f: cumulative mass fraction (m(0) = 0, m(R) = 1)."""
    cm = np.concatenate([[0.0], np.cumsum(psi * g.V)])
    return cm / cm[-1]


def quantiles_reference(g, psi, probs):
    """r with m(r) = p: the mass fraction is linear in r^3 within a cell (psi
    is constant there), so invert that piecewise."""
    m = mass_fraction(g, psi)
    probs = np.asarray(probs, dtype=np.float64)
    i = np.clip(np.searchsorted(m, probs, side="right") - 1, 0, g.N - 1)
    dm = m[i + 1] - m[i]
    t = np.where(dm > 0, (probs - m[i]) / np.where(dm > 0, dm, 1.0), 0.0)
    r3 = g.rf[i] ** 3 + t * (g.rf[i + 1] ** 3 - g.rf[i] ** 3)
    return np.cbrt(r3)


def quantiles_particles(X, probs):
    """Empirical quantiles of |X_p| (numpy's default linear interpolation)."""
    r = np.sqrt(np.sum(np.asarray(X, dtype=np.float64) ** 2, axis=1))
    return np.quantile(r, probs)


def truncation(n=1000):
    """Probabilities j/n, j = 0 .. m with m = ceil(3n/4) - 1 (Sec. 5.1)."""
    m = math.ceil(3 * n / 4) - 1
    return np.arange(m + 1) / n


def discrepancy(q, qhat):
    """E = mean |q_j - qhat_j| over the truncated quantiles."""
    return float(np.mean(np.abs(np.asarray(q) - np.asarray(qhat))))


def heat_ball(r, t, mu, rho0, ball=1.0):
    """Free-space solution of psi_t = mu lap psi from rho0 1{|x| <= ball}:
    the ball's indicator convolved with the heat kernel, written in r."""
    r = np.asarray(r, dtype=np.float64)
    s = math.sqrt(4.0 * mu * t)
    a = (ball - r) / s
    b = (ball + r) / s
    from scipy.special import erf
    term = 0.5 * (erf(a) + erf(b))
    term -= (s / (2.0 * math.sqrt(math.pi) * r)) * (np.exp(-a * a) - np.exp(-b * b))
    return rho0 * term


def screened_ball(r, k, R, rho0, ball=1.0):
    """Steady c of -lap c + k^2 c = rho0 1{r <= ball} on the ball of radius R with
    c'(R) = 0: c = rho0/k^2 + A sinh(kr)/r inside, B sinh(kr)/r + C cosh(kr)/r
    outside, with c and c' continuous at r = ball."""
    import numpy.linalg as la
    a = ball
    sh, ch = math.sinh, math.cosh

    def f(x):      # sinh(kx)/x and its derivative
        return sh(k * x) / x, (k * ch(k * x) * x - sh(k * x)) / (x * x)

    def gfun(x):   # cosh(kx)/x and its derivative
        return ch(k * x) / x, (k * sh(k * x) * x - ch(k * x)) / (x * x)
    fa, dfa = f(a)
    ga, dga = gfun(a)
    fR, dfR = f(R)
    gR, dgR = gfun(R)
    # unknowns A, B, C:  A fa + rho0/k^2 = B fa + C ga;  A dfa = B dfa + C dga;  B dfR + C dgR = 0
    M = np.array([[fa, -fa, -ga], [dfa, -dfa, -dga], [0.0, dfR, dgR]])
    rhs = np.array([-rho0 / k ** 2, 0.0, 0.0])
    A, B, C = la.solve(M, rhs)
    r = np.asarray(r, dtype=np.float64)
    inside = rho0 / k ** 2 + A * np.sinh(k * r) / r
    outside = B * np.sinh(k * r) / r + C * np.cosh(k * r) / r
    return np.where(r <= a, inside, outside)
