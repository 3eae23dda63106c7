"""Parity of the library's pathwise adjoint (sipf_adjoint, Rollout) with the
FP64 oracle adjoint, which is itself pinned to central finite differences.

Tolerances: FP64 path 1e-9 relative; FP32 path 1e-3 relative (the stated
gradient tolerance of the float path)."""

import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import adjoint as oadj  # noqa: E402
from oracle import sipf as osipf  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2512_03452_amd as pkg  # noqa: E402
from paper_2512_03452_amd import _lib  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return np.linalg.norm((a - b).ravel()) / max(np.linalg.norm(b.ravel()), 1e-300)


@pytest.mark.parametrize("precision,H,P,N,K,scheme", [
    ("fp64", 8, 300, 4, 2, "strang"),  # 40 (ky, kz) columns: a part-filled x-pencil block
    ("fp64", 16, 400, 5, 2, "strang"),
    # segments of 20 and 4 steps, the first one's gradient grids made in
    # batches of 16 and 4 (at 40 steps this collapse amplifies rounding-order
    # differences to about 2e-9 for every checkpoint interval, 1 to 40)
    ("fp64", 16, 400, 24, 20, "strang"),
    ("fp64", 16, 300, 4, 4, "em"),
    ("fp64", 32, 1000, 6, 5, "strang"),
    ("fp32", 32, 3000, 10, 3, "strang"),
    ("fp32", 64, 20000, 8, 4, "em"),
])
def test_adjoint_matches_oracle(precision, H, P, N, K, scheme):
    say("adjoint", precision, H, P, N, K, scheme)
    kw = dict(L=2.0, chi=1.5, mu=0.8, eps=1.0, k=1.0, M0=80.0, dt=2e-3 if H <= 16 else 5e-4, H=H, seed=3,
              scheme=scheme)
    X0 = osipf.wrap(np.random.default_rng(P).normal(0, 0.2, (P, 3)), 2.0)
    X0 = X0.astype(np.float32 if precision == "fp32" else np.float64)
    sim = pkg.Sim(X0, precision=precision, **kw)
    loss, dchi, dmu, dX0 = sim.adjoint(N, K)
    dX0 = dX0.cpu().numpy()
    prm = osipf.Params(**kw)
    ol, odX, ochi, omu = oadj.loss_and_grad(X0.astype(np.float64), prm, N)
    tol = 1e-9 if precision == "fp64" else 1e-3
    assert abs(loss - ol) < tol * abs(ol)
    assert abs(dchi - ochi) < tol * max(abs(ochi), 1e-12)
    assert abs(dmu - omu) < tol * max(abs(omu), 1e-12)
    assert rel(dX0, odX) < tol
    # the context holds X^(N) afterwards
    assert sim.n == N
    Xn, _ = osipf.run(X0.astype(np.float64), prm, N)
    ptol = 1e-9 if precision == "fp64" else 1e-4
    assert np.abs(osipf.min_image(sim.positions().cpu().numpy() - Xn, 2.0)).max() < ptol


def test_adjoint_linear_cotangent_and_rollout():
    """Rollout.backward passes grad_phi as phi_bar: d(sum(w * phi))/dX0 equals the
    oracle adjoint of the same linear functional."""
    H, P, N = 16, 500, 4
    kw = dict(L=2.0, eps=1.0, k=1.0, M0=60.0, dt=2e-3, H=H, seed=5, precision="fp64")
    X0 = osipf.wrap(np.random.default_rng(9).normal(0, 0.25, (P, 3)), 2.0)
    w = np.random.default_rng(10).standard_normal((H, H, H))
    X = torch.tensor(X0, dtype=torch.float64, device="cuda", requires_grad=True)
    chi = torch.tensor(1.2, dtype=torch.float64, requires_grad=True)
    mu = torch.tensor(0.9, dtype=torch.float64, requires_grad=True)
    phi = pkg.Rollout.apply(X, chi, mu, kw, N, 2)
    loss = (phi * torch.tensor(w, device="cuda")).sum()
    loss.backward()
    prm = osipf.Params(chi=1.2, mu=0.9, **{k: v for k, v in kw.items() if k != "precision"})
    ol, odX, ochi, omu = oadj.loss_and_grad(X0, prm, N, phi_bar=w)
    assert abs(loss.item() - ol) < 1e-9 * abs(ol)
    assert rel(X.grad.cpu().numpy(), odX) < 1e-9
    assert abs(chi.grad.item() - ochi) < 1e-9 * abs(ochi)
    assert abs(mu.grad.item() - omu) < 1e-9 * abs(omu)


def test_adjoint_requires_initial_state():
    sim = pkg.Sim(np.zeros((10, 3)), H=8, precision="fp64")
    sim.step()
    with pytest.raises(_lib.SipfError) as e:
        sim.adjoint(2, 1)
    assert e.value.code == _lib.SIPF_ESTATE


# The adjoint workload's shape (H = 64, blob of sd 0.1, M0 = 80, tau = 5e-5,
# N = 100 steps, a checkpoint every K = 10), with 1e5 particles in FP64 and
# 2e4 in FP32 so that the FP64 oracle finishes within a minute.  Over 100
# steps this collapsing run
# amplifies input perturbations about 1e7-fold in dL/dX0 (two FP64 runs from
# X0 and from X0 perturbed by 1e-12 differ by 2e-5 relative; from X0 rounded
# through float32 they differ by O(1)), so FP32 forward rounding alone
# decides its gradient: there the FP32 path is compared only in the two
# conditioned variants below (N = 50; M0 = 20 at N = 100), where FP32 and FP64
# agree to 3e-5.  FP64 against the FP64 oracle: rounding-order differences of
# order 1e-16 amplified 1e7-fold give about 1e-9; 1e-8 bounds them (the
# stated gradient tolerance is 1e-3).
@pytest.mark.parametrize("precision,P,N,M0,tol", [
    ("fp64", 100000, 100, 80.0, 1e-8),
    ("fp32", 20000, 50, 80.0, 1e-3),
    ("fp32", 20000, 100, 20.0, 1e-3),
])
def test_adjoint_at_the_adjoint_workload_shape(precision, P, N, M0, tol):
    from paper_2512_03452_amd import workloads
    cfg = workloads.CONFIGS["fp32_adjoint_h64"]
    K = 10
    kw = dict(cfg["params"], M0=M0)
    kw.pop("precision")
    say("adjoint workload shape", precision, "P", P, "N", N, "K", K, "M0", M0)
    X0 = cfg["init"](P, seed=7).astype(np.float32 if precision == "fp32" else np.float64)
    sim = pkg.Sim(X0, precision=precision, **kw)
    loss, dchi, dmu, dX0 = sim.adjoint(N, K)
    dX0 = dX0.cpu().numpy()
    sim.close()
    say("  gpu", loss, dchi, dmu)
    ol, odX, ochi, omu = oadj.loss_and_grad(X0.astype(np.float64), osipf.Params(**kw), N)
    say("  oracle", ol, ochi, omu, "rel dX0", rel(dX0, odX), "rel dchi", abs(dchi - ochi) / abs(ochi),
        "rel dmu", abs(dmu - omu) / abs(omu))
    assert abs(loss - ol) < tol * abs(ol)
    assert abs(dchi - ochi) < tol * abs(ochi)
    assert abs(dmu - omu) < tol * abs(omu)
    assert rel(dX0, odX) < tol
