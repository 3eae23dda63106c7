"""The direct SIPF method (Algorithm 1) on the GPU against the FP64 oracle
(oracle.sipf.sipf_direct_step): FP64 to 1e-9 in positions and 1e-11 in alpha;
FP32 to 1e-4 in alpha (phases advanced by up to H complex multiplications
along q_z) and 1e-5 in positions."""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import sipf as osipf  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2512_03452_amd as pkg  # noqa: E402
from paper_2512_03452_amd import workloads  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oparams(**kw):
    kw = dict(kw)
    for k in ("precision", "tile", "resort_every", "chunk", "dim", "method"):
        kw.pop(k, None)
    return osipf.Params(**kw)


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    return np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel())


@pytest.mark.parametrize("H,P,scheme,H0,precision", [
    (8, 500, "em", -1.0, "fp64"),
    (16, 333, "strang", 0.0, "fp64"),
    (8, 1, "em", -1.0, "fp64"),
    (32, 4000, "em", -1.0, "fp32"),
    (64, 2000, "strang", 0.0, "fp32"),
    # mixed-radix grids (q_z runs of 6, 11, 23, 15; ragged pair groups)
    (12, 700, "em", -1.0, "fp64"),
    (22, 999, "strang", 0.0, "fp64"),
    (46, 300, "em", -1.0, "fp32"),
    (90, 64, "em", -1.0, "fp32"),
])
def test_direct_sipf_matches_oracle(H, P, scheme, H0, precision):
    say("direct", H, P, scheme, H0, precision)
    kw = dict(L=2.0, chi=1.5, mu=1.0, eps=1.0, k=1.0, M0=40.0, dt=2e-3, H=H, H0=H0, scheme=scheme,
              precision=precision, seed=8, method="direct")
    X0 = workloads.blob(P, 0.2, seed=H).astype(np.float32 if precision == "fp32" else np.float64)
    sim = pkg.Sim(X0, **kw)
    nsteps = 4
    sim.run(nsteps)
    Xo, ao = osipf.sipf_direct_run(X0.astype(np.float64), oparams(**kw), nsteps, use_filter=H0 >= 0)
    X = sim.positions().cpu().numpy().astype(np.float64)
    A = sim.field("alpha").cpu().numpy()
    assert sim.n == nsteps
    if precision == "fp64":
        assert np.abs(osipf.min_image(X - Xo, 2.0)).max() < 1e-9
        assert rel_l2(A, osipf.half_spectrum(ao)) < 1e-11
    else:
        assert np.abs(osipf.min_image(X - Xo, 2.0)).max() < 1e-5
        err = rel_l2(A, osipf.half_spectrum(ao))
        say(" alpha rel L2", err)
        assert err < 1e-5
    sim.close()


def test_direct_context_rejects_grid_calls():
    sim = pkg.Sim(workloads.blob(100, 0.2, seed=1), L=2.0, H=8, precision="fp64", method="direct")
    for call in (lambda: sim.field("rho"), lambda: sim.field("grad"), sim.diagnostics, lambda: sim.adjoint(2)):
        with pytest.raises(pkg.SipfError):
            call()
    sim.close()
    with pytest.raises(pkg.SipfError):
        pkg.Batch([dict(params=dict(H=8, method="direct"), X0=workloads.blob(10, 0.2).astype(np.float32))] * 2)
