"""Pins of the oracle's positivity-preserving deposit (``oracle.sipf.deposit_positive``,
reading of Remark ``smoothness`` and Sec. 3.4), CPU only.

Each test fixes the result by something other than the function itself: the
order-4 and order-2 deposits it must reduce to, exact mass, the sign of every
node, and where in the cloud particles may switch.
"""

import math

import numpy as np
import pytest

from oracle import sipf, stencil


def _ball(P, R, seed):
    rng = np.random.default_rng(seed)
    v = rng.standard_normal((P, 3))
    v /= np.linalg.norm(v, axis=1)[:, None]
    return v * R * rng.random(P)[:, None] ** (1.0 / 3.0)


def _sheet():
    """A thin sheet of 2681 particles whose positive deposit on H = 16 takes two
    rounds (switching the first shell leaves new negative nodes next to it)."""
    rng = np.random.default_rng(28)
    P = int(rng.integers(50, 4000))
    X = rng.uniform(-1, 1, (P, 3))
    X[:, 2] = rng.normal(0, rng.uniform(0.005, 0.1), P)
    return sipf.wrap(X, 2.0)


@pytest.mark.parametrize("H,kind", [(16, "ball"), (32, "ball"), (12, "ball"), (22, "blob"), (16, "sparse"),
                                    (16, "sheet")])
def test_nonnegative_with_the_order4_mass(H, kind):
    L = 2.0
    rng = np.random.default_rng(H)
    if kind == "ball":
        X = _ball(20000, 0.5, H)
    elif kind == "blob":
        X = sipf.wrap(rng.normal(0.2, 0.15, (8000, 3)), L)
    elif kind == "sheet":
        X = _sheet()
    else:
        X = rng.uniform(-1, 1, (40, 3))
    w = 3.0 / X.shape[0]
    rec = {}
    phi = sipf.deposit_positive(X, w, H, L, record=rec)
    p4 = sipf.deposit(X, w, H, L, 4)
    assert p4.min() < -1e-3 * w          # the order-4 deposit has negative nodes here
    assert phi.min() >= 0.0
    assert abs(phi.sum() - 3.0) < 1e-12 * 3.0
    assert rec["rounds"] >= 1 and rec["switched"].any()
    if kind == "sheet":
        assert rec["rounds"] == 2


def test_equals_the_order4_deposit_where_nothing_is_negative():
    """A dense uniform cloud has no negative node: no particle switches."""
    H, L = 8, 2.0
    X = np.random.default_rng(3).uniform(-1, 1, (200000, 3))
    p4 = sipf.deposit(X, 1e-5, H, L, 4)
    assert p4.min() > 0
    rec = {}
    phi = sipf.deposit_positive(X, 1e-5, H, L, record=rec)
    assert rec["rounds"] == 0 and not rec["switched"].any()
    assert np.abs(phi - p4).max() < 1e-13 * p4.max()


def test_isolated_particles_fall_back_to_trilinear_weights():
    """A lone particle off the cell faces has negative outer weights, so every
    particle of a sparse set ends on the order-2 weights of eq. 2ord."""
    H, L = 32, 2.0
    h = L / H
    centers = np.array([(i, j, k) for i in range(4) for j in range(4) for k in range(4)], float) * 8 - 14
    lam = np.random.default_rng(5).uniform(0.1, 0.9, (64, 3))
    X = (centers + lam) * h
    w = np.random.default_rng(6).uniform(0.5, 2.0, 64)
    rec = {}
    phi = sipf.deposit_positive(X, w, H, L, record=rec)
    assert rec["switched"].all() and rec["rounds"] == 1
    assert np.abs(phi - sipf.deposit(X, w, H, L, 2)).max() < 1e-15
    # a particle at a cell centre spreads 1/8 to each of its 8 cell corners
    one = sipf.deposit_positive(np.full((1, 3), 0.5 * h), 1.0, H, L)
    assert np.allclose(one[:2, :2, :2], 1 / 8) and abs(one.sum() - 1) < 1e-15


def test_only_particles_near_the_edge_of_the_cloud_switch():
    """Negative nodes lie within the stencil reach of the ball's edge, so a
    switched particle is within 2 sqrt(3) cells of the surface on the inside,
    and particles deeper than that keep the order-4 weights."""
    H, L, R = 32, 2.0, 0.5
    h = L / H
    X = _ball(30000, R, 9)
    rec = {}
    sipf.deposit_positive(X, 1.0 / 30000, H, L, record=rec)
    r = np.linalg.norm(X, axis=1)
    s = rec["switched"]
    reach = 2 * math.sqrt(3) * h
    assert r[s].min() > R - reach - 0.5 * h
    assert not s[r < R - reach - 0.5 * h].any()
    assert s[r > R - 0.25 * h].mean() > 0.9


def test_step_uses_it_when_asked():
    """Params.positivity routes the step's deposit through deposit_positive:
    beta of the first step is the transform of the positive deposit."""
    X = _ball(3000, 0.4, 2)
    for pos in (False, True):
        prm = sipf.Params(L=2.0, chi=1.0, mu=0.0, eps=1.0, k=1.0, M0=10.0, dt=1e-3, H=16, positivity=pos)
        rec = {}
        sipf.step(X, np.zeros((16, 16, 16), complex), 1, prm, record=rec)
        want = sipf.deposit_positive(X, 10.0 / 3000, 16, 2.0) if pos else sipf.deposit(X, 10.0 / 3000, 16, 2.0, 4)
        assert np.abs(rec["phi"] - want).max() < 1e-15
    assert (rec["phi"] >= 0).all()


def test_trilinear_layout_matches_the_inner_nodes():
    """The order-2 nodes are the first eight of Gamma_4, in the same order (the
    fallback puts eq. 2ord's weights there and zero on the outer nodes)."""
    assert np.array_equal(stencil.offsets(4)[:8], stencil.offsets(2))


def test_positive_deposit_and_exponential_propagator_keep_c_nonnegative():
    """Sec. 3.4: with a non-negative deposit and the exponential propagator, c
    stays non-negative up to rounding once the diffusion length of one step
    reaches the grid spacing (tau >= h^2 here); the order-4 deposit or the
    implicit propagator leave clearly negative values in the same run."""
    X0 = _ball(20000, 0.3, 1)

    def cmin(pos, prop):
        prm = sipf.Params(L=2.0, chi=0.0, mu=0.0, eps=1.0, k=1.0, M0=10.0, dt=4e-3, H=32, positivity=pos,
                          propagator=prop)
        _, a = sipf.run(X0, prm, 3)
        c = sipf.inverse_transform(a).real
        return c.min() / c.max()

    assert cmin(True, "exp") > -1e-15
    assert cmin(False, "exp") < -1e-14
    assert cmin(True, "implicit") < -1e-7
