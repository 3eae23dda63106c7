"""Host logic of the convergence study (Sec. 5.1): quantile levels, empirical
quantiles, discrepancy, slopes and the reference table reader."""

import os

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import radial  # noqa: E402
from paper_2512_03452_amd import convergence, workloads  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "radial_e1_quantiles.txt")


def test_levels_match_the_oracle_truncation():
    assert np.array_equal(convergence.probabilities(), radial.truncation(1000))
    assert convergence.M_QUANT == 749


def test_empirical_quantiles_match_numpy():
    rng = np.random.default_rng(3)
    X = rng.normal(size=(12345, 3))
    p = convergence.probabilities()
    got = convergence.empirical_quantiles(torch.as_tensor(X), p).numpy()
    want = radial.quantiles_particles(X, p)
    assert np.abs(got - want).max() < 1e-13


def test_discrepancy_and_slope():
    q = np.linspace(0.0, 1.0, 750)
    assert convergence.discrepancy(q, q + 0.25) == pytest.approx(0.25)
    assert convergence.discrepancy(q, q) == 0.0
    x = 2.0 ** np.arange(11, 21)
    assert convergence.slope(x, 3.0 * x ** -0.5) == pytest.approx(-0.5)


def test_reference_table_reads_and_rejects_bad_tables(tmp_path):
    q = convergence.load_reference(GOLDEN)
    assert q.shape == (750,) and q[0] == 0.0 and np.all(np.diff(q) > 0)
    bad = tmp_path / "bad.txt"
    np.savetxt(bad, np.zeros((10, 2)))
    with pytest.raises(ValueError):
        convergence.load_reference(str(bad))


def test_ball_sampler_is_uniform_in_the_unit_ball():
    X = workloads.ball(200_000, 1.0, seed=4)
    r = np.linalg.norm(X, axis=1)
    assert r.max() <= 1.0
    # |X|^3 is U(0, 1) for the uniform ball
    assert abs(np.mean(r ** 3) - 0.5) < 3e-3
    assert np.abs(X.mean(axis=0)).max() < 5e-3
    assert not np.array_equal(X, workloads.ball(200_000, 1.0, seed=5))


def test_grid_bytes_counts_the_instance_grids():
    """Four H^3 real grids and five half spectra per 3-D instance (the batch
    memory budget of the study)."""
    from paper_2512_03452_amd import convergence
    assert convergence.grid_bytes(256) == 4 * 256 ** 3 * 4 + 5 * 256 * 256 * 129 * 8
    assert convergence.grid_bytes(64, "fp64") == 2 * convergence.grid_bytes(64)
