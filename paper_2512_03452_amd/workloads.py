"""Seeded synthetic workloads (initial particle positions and parameter sets).

This module only draws inputs: it holds none of the method's arithmetic and is
shared by the tests, the bench and the smoke check.  Positions are returned as
float64 numpy arrays of shape (P, 3) inside the box [-L/2, L/2)^3 (L = 2 for
every workload below except the convergence-study ball, which lives in the box
of side 8); callers cast them to the working precision.

The paper runs on synthetic initial densities only (no datasets); the shapes
below follow its experiment types at the sizes of the workloads this library
is measured on:
  * blob        -- i.i.d. N(0, sd^2 I) (single-point collapse initial data)
  * mix         -- half uniform on the box, half N(0, sd^2 I)
  * torus       -- ring of major radius R in the xy-plane with Gaussian tube
                   cross-section sd (shape of the collapsing-ring run)
  * ball        -- uniform in the unit ball (initial data of the convergence
                   study, Sec. 5.1)
  * disk        -- uniform in a disk, positions (P, 2) (the 2-D experiments of
                   Sec. 5.2)
"""

import math

import numpy as np

L_BOX = 2.0


def _wrap(X, L=L_BOX):
    return X - L * np.floor((X + L / 2.0) / L)


def blob(P, sd, seed=0):
    rng = np.random.default_rng([seed, 1])
    return _wrap(rng.normal(0.0, sd, (P, 3)))


def mix(P, sd, seed=0):
    rng = np.random.default_rng([seed, 2])
    half = P // 2
    X = np.empty((P, 3))
    X[:half] = rng.uniform(-L_BOX / 2, L_BOX / 2, (half, 3))
    X[half:] = rng.normal(0.0, sd, (P - half, 3))
    return _wrap(X)


def torus(P, R=0.5, sd=0.05, seed=0):
    rng = np.random.default_rng([seed, 3])
    th = rng.uniform(0.0, 2.0 * math.pi, P)
    a = rng.normal(0.0, sd, P)
    b = rng.normal(0.0, sd, P)
    X = np.stack([(R + a) * np.cos(th), (R + a) * np.sin(th), b], axis=1)
    return _wrap(X)


def ball(P, radius=1.0, seed=0):
    """i.i.d. uniform in the ball |x| <= radius (the initial density of the
    convergence study, Sec. 5.1)."""
    rng = np.random.default_rng([seed, 5])
    v = rng.normal(size=(P, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    return v * (radius * np.cbrt(rng.random(P)))[:, None]


def disk(P, radius=1.0, seed=0):
    """i.i.d. uniform in the disk |x| <= radius, shape (P, 2) (the initial
    density of the 2-D experiments of Sec. 5.2)."""
    rng = np.random.default_rng([seed, 6])
    th = rng.uniform(0.0, 2.0 * math.pi, P)
    r = radius * np.sqrt(rng.random(P))
    return np.stack([r * np.cos(th), r * np.sin(th)], axis=1)


# Convergence study of Sec. 5.1: uniform ball of radius 1, M0 = 80,
# mu = chi = 1, eps = 1e-4, k = 0.1, tau = 1e-5, 2000 steps, L = 8.
E1_PARAMS = dict(L=8.0, chi=1.0, mu=1.0, eps=1e-4, k=0.1, M0=80.0, dt=1e-5)
E1_STEPS = 2000

# name -> (parameters, P, steps, position generator)
CONFIGS = {
    "fp64_blob_h32": dict(
        params=dict(L=2.0, chi=1.0, mu=1.0, eps=1.0, k=1.0, M0=60.0, dt=1e-4, H=32, precision="fp64", seed=0),
        P=10_000, steps=100, init=lambda P, seed=0: blob(P, 0.1, seed)),
    "fp32_mix_h64": dict(
        params=dict(L=2.0, chi=1.0, mu=1.0, eps=1.0, k=1.0, M0=80.0, dt=5e-5, H=64, precision="fp32", seed=0),
        P=1_000_000, steps=200, init=lambda P, seed=0: mix(P, 0.15, seed)),
    "fp32_ring_h128": dict(
        params=dict(L=2.0, chi=1.0, mu=1.0, eps=1.0, k=1.0, M0=200.0, dt=2e-5, H=128, precision="fp32", seed=0),
        P=10_000_000, steps=500, init=lambda P, seed=0: torus(P, 0.5, 0.05, seed)),
    "fp32_adjoint_h64": dict(
        params=dict(L=2.0, chi=1.0, mu=1.0, eps=1.0, k=1.0, M0=80.0, dt=5e-5, H=64, precision="fp32", seed=0),
        P=2_000_000, steps=100, init=lambda P, seed=0: blob(P, 0.1, seed)),
}


def ensemble(n=64, seed=0):
    """Per-instance parameters and positions of the batched-ensemble workload.

    P log-uniform in [1e4, 1e6], H in {32, 64}, chi ~ U[0.5, 2], M0 ~ U[40, 120],
    Gaussian blob sd 0.1, eps = mu = k = 1, dt = 5e-5; instance i uses Philox
    counter word i.
    """
    rng = np.random.default_rng([seed, 4])
    out = []
    for i in range(n):
        P = int(round(10 ** rng.uniform(4.0, 6.0)))
        H = int(rng.choice([32, 64]))
        chi = float(rng.uniform(0.5, 2.0))
        M0 = float(rng.uniform(40.0, 120.0))
        prm = dict(L=2.0, chi=chi, mu=1.0, eps=1.0, k=1.0, M0=M0, dt=5e-5, H=H, precision="fp32",
                   seed=seed, instance=i)
        out.append(dict(params=prm, P=P, X0=blob(P, 0.1, seed * 1000 + i + 17)))
    return out
