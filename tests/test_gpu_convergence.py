"""Convergence study of Sec. 5.1 at reduced size on the GPU.

Uniform-ball initial data, the paper's parameters and 2000 steps to T = 0.02;
the truncated quantile discrepancy is taken against the radial reference that
oracle/radial.py wrote (tests/golden/radial_e1_quantiles.txt).  Eight
independent runs per configuration.  The bounds follow from the theory of
Sec. 4 and the full study (30 runs per configuration, P up to 2^20, H up to
128): the particle error falls like P^-1/2 while the grid error is below it,
the grid error falls at least like H^-16/13 while the sampling error is below
it.  The slope bounds leave room for eight runs' scatter (the run-to-run
standard deviation is about half the mean).
"""

import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2512_03452_amd import convergence  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "radial_e1_quantiles.txt")


def test_reduced_convergence_study():
    q_ref = convergence.load_reference(GOLDEN)
    Ps = [2 ** 11, 2 ** 13, 2 ** 15]
    Hs = [8, 16, 32]
    configs = [(P, 64) for P in Ps] + [(2 ** 17, H) for H in Hs]
    print("E1 reduced study", configs, flush=True)
    res, secs = convergence.run_study(configs, 8, q_ref, seed=11,
                                      log=lambda s: (print(s, flush=True), sys.stdout.flush()))
    eP = [res[(P, 64)]["mean"] for P in Ps]
    eH = [res[(2 ** 17, H)]["mean"] for H in Hs]
    print("E vs P", eP, "E vs H", eH, "seconds", secs, flush=True)
    sP = convergence.slope(Ps, eP)
    sH = convergence.slope(Hs, eH)
    assert -0.8 < sP < -0.25, sP
    assert sH < -16.0 / 13.0, sH
    # absolute level: at H = 32 and P = 2^17 the full study's mean is below 0.005
    assert eH[-1] < 0.006
    for v in res.values():
        assert np.all(np.isfinite(v["E"])) and np.all(v["E"] > 0)
