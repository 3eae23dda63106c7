"""Pins of the radial reference solution and of the quantile discrepancy
(Sec. 5.1) against closed forms and exact properties (CPU)."""

import math

import numpy as np
import pytest

from oracle import radial


def test_ball_radius_matches_the_cube_volume():
    R = radial.ball_radius(8.0)
    assert abs(4.0 * math.pi / 3.0 * R ** 3 - 512.0) < 1e-9
    assert abs(R - 4.9628) < 1e-4   # the value quoted in Sec. 5.1


def test_ball_average_is_exact():
    g = radial.Grid(radial.ball_radius(8.0), 1000)
    psi = g.ball_average(1.0, 60.0 / math.pi)
    assert abs(np.sum(psi * g.V) - 80.0) < 1e-10


def test_mass_is_conserved():
    g = radial.Grid(radial.ball_radius(8.0), 2000)
    psi = g.ball_average(1.0, 60.0 / math.pi)
    c = np.zeros(g.N)
    for _ in range(200):
        c = radial.step_c(g, c, psi, 1e-4, 0.1, 1e-5)
        psi = radial.step_psi(g, psi, c, 1.0, 1.0, 1e-5)
    assert abs(np.sum(psi * g.V) - 80.0) < 1e-10 * 80.0
    assert psi.min() > -1e-12           # upwind drift + implicit diffusion keep psi >= 0


def test_pure_diffusion_matches_the_heat_kernel():
    """chi = 0: psi is the uniform ball smoothed by the heat kernel."""
    rho0, mu, T, dt = 60.0 / math.pi, 1.0, 2e-3, 2e-6
    g = radial.Grid(8.0, 8000)
    psi = g.ball_average(1.0, rho0)
    c = np.zeros(g.N)
    for _ in range(int(round(T / dt))):
        psi = radial.step_psi(g, psi, c, mu, 0.0, dt)
    exact = radial.heat_ball(g.rc, T, mu, rho0)
    assert np.abs(psi - exact).max() < 2e-4 * rho0   # O(dt + dr^2): 8e-5 at these sizes


def test_steady_field_matches_the_screened_ball():
    """Frozen uniform-ball source: one backward-Euler c step with eps/dt -> 0 is
    the Neumann solution of -lap c + k^2 c = psi."""
    k, R, rho0 = 0.5, 4.0, 1.0
    g = radial.Grid(R, 4000)
    psi = g.ball_average(1.0, rho0)
    c = radial.step_c(g, np.zeros(g.N), psi, 1e-30, k, 1.0)
    exact = radial.screened_ball(g.rc, k, R, rho0)
    assert np.abs(c - exact).max() < 1e-6 * np.abs(exact).max()   # O(dr^2): 2.4e-7


def test_reference_quantiles_of_the_uniform_ball():
    g = radial.Grid(radial.ball_radius(8.0), 5000)
    psi = g.ball_average(1.0, 60.0 / math.pi)
    p = radial.truncation(1000)
    q = radial.quantiles_reference(g, psi, p)
    assert np.abs(q - np.cbrt(p)).max() < 1e-9
    assert len(p) == 750 and p[-1] == 0.749


def test_discrepancy_of_sampled_balls_falls_like_inverse_sqrt_P():
    g = radial.Grid(radial.ball_radius(8.0), 5000)
    psi = g.ball_average(1.0, 60.0 / math.pi)
    p = radial.truncation(1000)
    q = radial.quantiles_reference(g, psi, p)
    errs = []
    for P in (4000, 64000):
        e = []
        for s in range(8):
            rng = np.random.default_rng([s, P])
            v = rng.normal(size=(P, 3))
            X = v / np.linalg.norm(v, axis=1)[:, None] * np.cbrt(rng.random(P))[:, None]
            e.append(radial.discrepancy(q, radial.quantiles_particles(X, p)))
        errs.append(np.mean(e))
    slope = math.log(errs[1] / errs[0]) / math.log(16.0)
    assert -0.65 < slope < -0.35


def _paper_values():
    import os
    vals = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.txt")) as f:
        for line in f:
            if line.strip() and not line.startswith("#"):
                name, value = line.split()[:2]
                vals[name] = float(value)
    return vals


def test_reference_reproduces_the_printed_quantile():
    """The full problem of Sec. 5.1 on 4e4 volumes: the 0.999 mass quantile at
    T = 0.02 is the one the paper prints (the stored 4e5-volume reference gives
    1.450463)."""
    vals = _paper_values()
    g, psi, c = radial.solve(N=40_000)
    q999 = float(radial.quantiles_reference(g, psi, [0.999])[0])
    assert abs(q999 - vals["q999"]) < 2e-4
    assert abs(g.R - vals["R_ball"]) < 1e-4
    assert abs(np.sum(psi * g.V) - 80.0) < 1e-8


def test_stored_reference_quantiles_are_consistent():
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "radial_e1_quantiles.txt")
    head = [l for l in open(path) if l.startswith("#")]
    q999 = float([l for l in head if l.startswith("# q999")][0].split()[2])
    assert abs(q999 - _paper_values()["q999"]) < 2e-5
    data = np.loadtxt(path)
    assert data.shape == (750, 2)
    assert np.all(np.diff(data[:, 1]) > 0) and data[0, 1] == 0.0
