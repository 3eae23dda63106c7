"""Closed forms of the 2-D second-moment law used by the Sec. 5.2 studies."""

import math

import pytest

pytest.importorskip("torch")

from paper_2512_03452_amd import critical2d  # noqa: E402


@pytest.mark.parametrize("M0", [22.0, 24.6, 25.0, 8 * math.pi, 27.0])
def test_whole_plane_law_gives_the_printed_value_at_t2(M0):
    """eq. second_moment from the unit disk (m2(0) = 1/2): m2(2) = 17/2 - M0/pi."""
    assert abs(critical2d.whole_plane_m2(0.5, M0, 2.0) - (17.0 / 2.0 - M0 / math.pi)) < 1e-12


def test_periodic_law_solves_its_ode_and_tends_to_the_whole_plane():
    M0, L, m0 = 25.0, 10.0, 0.5
    a, b = 4.0 - M0 / (2 * math.pi), M0 / L ** 2
    for t in (0.1, 0.7, 2.0):
        dt = 1e-6
        d = (critical2d.periodic_m2(m0, M0, L, t + dt) - critical2d.periodic_m2(m0, M0, L, t - dt)) / (2 * dt)
        assert abs(d - (a + b * critical2d.periodic_m2(m0, M0, L, t))) < 1e-6
    assert critical2d.periodic_m2(m0, M0, L, 0.0) == pytest.approx(m0)
    far = critical2d.periodic_m2(m0, M0, 1e4, 2.0)
    assert abs(far - critical2d.whole_plane_m2(m0, M0, 2.0)) < 1e-6
