"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances (float32 path): Philox integers and cell indices bit-exact; grid
fields (deposit, alpha, gradient) within 1e-5 relative L2 per step; positions
within 1e-4 (minimum image) after 100 steps.  Float64 path: grids within
1e-12 relative L2, positions within 1e-9.
"""

import math
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import philox as ophilox  # noqa: E402
from oracle import sipf as osipf  # noqa: E402

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

import paper_2512_03452_amd as pkg  # noqa: E402
from paper_2512_03452_amd import workloads  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128 if np.iscomplexobj(a) or np.iscomplexobj(b) else np.float64)
    b = np.asarray(b, dtype=a.dtype)
    nb = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0)


def oparams(**kw):
    """Oracle parameters from library keyword arguments."""
    kw = dict(kw)
    kw.pop("precision", None)
    for k in ("tile", "resort_every", "chunk", "particle_pass"):
        kw.pop(k, None)
    sch = kw.pop("scheme", "strang")
    return osipf.Params(scheme=sch if isinstance(sch, str) else ("strang" if sch == 0 else "em"), **kw)


def hermitian_alpha(H, seed, scale, dtype):
    """Half spectrum of a random real field (exactly representable in dtype)."""
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((H, H, H))
    full = np.fft.fftn(f) * scale / H ** 3
    # decay high modes so the gradient stays moderate
    q = osipf.freqs(H).astype(float)
    q2 = q[:, None, None] ** 2 + q[None, :, None] ** 2 + q[None, None, :] ** 2
    full *= np.exp(-q2 / (H / 4) ** 2)
    half = osipf.half_spectrum(full)
    cd = np.complex64 if dtype == "fp32" else np.complex128
    return half.astype(cd)


def to_np(t):
    return t.detach().cpu().numpy()


# ---------------------------------------------------------------------------
# a1: Philox integers (bit-exact) and normals
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_philox_bit_exact(precision):
    say("philox", precision)
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2 ** 32, (5000, 4), dtype=np.uint64).astype(np.uint32)
    ctr[0] = 0
    ctr[1] = 0xFFFFFFFF
    ctr[2:1000, 0] = np.arange(998)
    ctr[2:1000, 1] = 7
    ctr[2:1000, 2] = 1
    ctr[2:1000, 3] = 0
    seed = 0x1234_5678_9ABC_DEF0
    raw, z = pkg.dbg_philox(ctr, seed, precision)
    k0, k1 = ophilox.seed_key(seed)
    ref = np.stack(ophilox.philox4x32_10(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3], k0, k1), axis=1)
    assert np.array_equal(raw.astype(np.uint64), ref)
    # normals: the oracle's Box-Muller on the same counters (float64)
    zr = ophilox.normals6_counter(ctr[:, 0], ctr[:, 1], ctr[:, 2], ctr[:, 3], seed)
    tol = 2e-6 if precision == "fp32" else 1e-13
    assert np.abs(to_np(z) - zr).max() < tol * 6


# ---------------------------------------------------------------------------
# a2: cell indices (bit-exact)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("precision,H", [("fp32", 64), ("fp32", 128), ("fp64", 32)])
def test_cells_bit_exact(precision, H):
    say("cells", precision, H)
    rng = np.random.default_rng(1)
    X = rng.uniform(-1, 1, (20000, 3))
    h = 2.0 / H
    X[:200] = np.round(X[:200] / h) * h          # exactly on cell faces
    X[200:210] = -1.0
    X[210:220] = np.nextafter(1.0, 0.0)
    X = X.astype(np.float32 if precision == "fp32" else np.float64)
    cells = to_np(pkg.dbg_cells(X, H=H, precision=precision))
    g, _ = osipf.cell_and_frac(X.astype(np.float64), H, 2.0)
    assert np.array_equal(cells, g)


def test_cells_non_power_of_two_box_away_from_faces():
    H, L = 64, 3.0
    X = np.random.default_rng(2).uniform(-1.5, 1.5, (20000, 3)).astype(np.float32)
    cells = to_np(pkg.dbg_cells(X, H=H, L=L))
    g, lam = osipf.cell_and_frac(X.astype(np.float64), H, L)
    away = (np.minimum(lam, 1 - lam) > 1e-5).all(axis=1)
    assert away.mean() > 0.99
    assert np.array_equal(cells[away], g[away])


# ---------------------------------------------------------------------------
# a3: deposit through the sort + LDS-window path
# ---------------------------------------------------------------------------

def _positions(kind, P, seed):
    rng = np.random.default_rng(seed)
    if kind == "uniform":
        return rng.uniform(-1, 1, (P, 3))
    if kind == "blob":
        return osipf.wrap(rng.normal(0, 0.05, (P, 3)), 2.0)
    if kind == "faces":
        X = rng.uniform(-1, 1, (P, 3))
        X[: P // 2] = np.round(X[: P // 2] * 8) / 8
        return osipf.wrap(X, 2.0)
    if kind == "corner":
        return osipf.wrap(rng.normal(-1.0, 0.03, (P, 3)), 2.0)
    raise ValueError(kind)


@pytest.mark.parametrize("precision,H,P,kind", [
    ("fp32", 8, 1, "uniform"), ("fp32", 8, 7, "uniform"), ("fp32", 16, 3000, "blob"),
    ("fp32", 32, 54321, "uniform"), ("fp32", 64, 100003, "blob"), ("fp32", 64, 20000, "faces"),
    ("fp32", 128, 200001, "blob"), ("fp32", 128, 50000, "corner"), ("fp32", 32, 4097, "corner"),
    ("fp64", 32, 30001, "blob"), ("fp64", 64, 10000, "uniform"), ("fp64", 8, 5, "corner"),
    ("fp32", 256, 300001, "blob"), ("fp32", 256, 40000, "corner"),
])
def test_deposit_parity(precision, H, P, kind):
    say("deposit", precision, H, P, kind)
    X = _positions(kind, P, seed=H + P)
    X = X.astype(np.float32 if precision == "fp32" else np.float64)
    M0 = 37.5
    phi = to_np(pkg.dbg_deposit(X, H=H, precision=precision, M0=M0))
    ref = osipf.deposit(X.astype(np.float64), M0 / P, H, 2.0, 4)
    tol = 1e-5 if precision == "fp32" else 1e-12
    assert rel_l2(phi, ref) < tol
    assert abs(phi.sum() - M0) < (1e-5 if precision == "fp32" else 1e-12) * M0


# ---------------------------------------------------------------------------
# a4-a9: one full step from a non-trivial state
# ---------------------------------------------------------------------------

def _state_np(sim):
    return to_np(sim.positions()).astype(np.float64), to_np(sim.field("alpha")).astype(np.complex128)


# FP32 3-D steps have two particle passes (sorted items, two-phase): each
# FP32 case runs both.
_STEP_CASES = [
    ("fp32", 8, 333, "strang"), ("fp32", 16, 4099, "strang"), ("fp32", 32, 20001, "em"),
    ("fp32", 64, 65537, "strang"), ("fp32", 128, 100000, "strang"),
    ("fp64", 16, 2001, "strang"), ("fp64", 32, 10000, "em"), ("fp64", 64, 5000, "strang"),
    ("fp32", 256, 200003, "strang"),
]


@pytest.mark.parametrize("precision,H,P,scheme,pp", [
    c + (pp,) for c in _STEP_CASES for pp in (("sorted", "two_phase") if c[0] == "fp32" else ("default",))])
def test_one_step_parity(precision, H, P, scheme, pp):
    say("step", precision, H, P, scheme, pp)
    kw = dict(L=2.0, chi=3.0, mu=0.5, eps=1.0, k=1.0, M0=50.0, dt=1e-3, H=H, seed=11, scheme=scheme,
              particle_pass=pp)
    X0 = osipf.wrap(np.random.default_rng(H).normal(0, 0.3, (P, 3)), 2.0)
    X0 = X0.astype(np.float32 if precision == "fp32" else np.float64)
    a0 = hermitian_alpha(H, seed=H, scale=40.0, dtype=precision)
    sim = pkg.Sim(X0, alpha0=a0, precision=precision, **kw)
    Xs, As = _state_np(sim)
    assert np.array_equal(Xs, X0.astype(np.float64))
    prm = oparams(**kw)
    afull = osipf.full_spectrum(As)
    G0 = osipf.gradient_grid(afull, prm)
    tol = 1e-5 if precision == "fp32" else 1e-12
    assert rel_l2(to_np(sim.field("grad")), G0) < tol
    sim.step()
    X1, A1 = _state_np(sim)
    rec = {}
    Xo, ao = osipf.step(Xs, afull, 1, prm, record=rec)
    assert rel_l2(A1, osipf.half_spectrum(ao)) < tol
    assert rel_l2(to_np(sim.field("grad")), osipf.gradient_grid(osipf.full_spectrum(A1), prm)) < tol
    # position error budget: rounding of O(1) positions plus the relative
    # error of the float gradient times the drift chi tau |v|
    drift = prm.chi * prm.dt * np.abs(rec["v"]).max()
    ptol = (1e-6 + 1e-5 * drift) if precision == "fp32" else (1e-12 + 1e-11 * drift)
    assert np.abs(osipf.min_image(X1 - Xo, 2.0)).max() < ptol
    assert sim.n == 1


# ---------------------------------------------------------------------------
# trajectories (positions after 100 steps)
# ---------------------------------------------------------------------------

def test_trajectory_fp64_h32_blob_100_steps():
    cfg = workloads.CONFIGS["fp64_blob_h32"]
    say("trajectory fp64 H=32 P=1e4")
    X0 = cfg["init"](cfg["P"])
    sim = pkg.Sim(X0, **cfg["params"])
    sim.run(cfg["steps"])
    X, A = _state_np(sim)
    prm = oparams(**cfg["params"])
    Xo, ao = osipf.run(X0, prm, cfg["steps"])
    assert np.abs(osipf.min_image(X - Xo, 2.0)).max() < 1e-9
    assert rel_l2(A, osipf.half_spectrum(ao)) < 1e-12
    assert sim.n == cfg["steps"]
    r = 1 / (1 + prm.dt * prm.k ** 2 / prm.eps)
    a00 = prm.dt * prm.M0 / (prm.eps * prm.L ** 3) * r * (1 - r ** 100) / (1 - r)
    assert abs(A[0, 0, 0].real - a00) < 1e-13 * a00


@pytest.mark.parametrize("scheme,pp", [("strang", "sorted"), ("strang", "two_phase"), ("em", "sorted"),
                                       ("em", "two_phase")])
def test_trajectory_fp32_h64_mix_100_steps(scheme, pp):
    """Parameters of the H=64 mixed workload (M0 = 80, dt = 5e-5) at P = 30000."""
    say("trajectory fp32 H=64", scheme, pp)
    cfg = workloads.CONFIGS["fp32_mix_h64"]
    P = 30000
    X0 = cfg["init"](P).astype(np.float32)
    kw = dict(cfg["params"], scheme=scheme, particle_pass=pp)
    sim = pkg.Sim(X0, **kw)
    sim.run(100)
    X, A = _state_np(sim)
    prm = oparams(**kw)
    Xo, ao = osipf.run(X0.astype(np.float64), prm, 100)
    assert np.abs(osipf.min_image(X - Xo, 2.0)).max() < 1e-4
    assert rel_l2(A, osipf.half_spectrum(ao)) < 1e-5


def _golden_mix_trajectory():
    """ids, positions and low modes of alpha stored by
    tests/golden/make_mix_h64_trajectory.py (FP64 oracle, 100 steps)."""
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "mix_h64_p1e6_100steps.txt")
    ids, X, alpha = [], [], {}
    with open(path) as f:
        for line in f:
            if line.startswith("# alpha"):
                _, _, qx, qy, qz, re_, im_ = line.split()
                alpha[(int(qx), int(qy), int(qz))] = complex(float(re_), float(im_))
            elif not line.startswith("#"):
                i, x, y, z = line.split()
                ids.append(int(i))
                X.append((float(x), float(y), float(z)))
    return np.array(ids), np.array(X), alpha


@pytest.mark.parametrize("pp", ["sorted", "two_phase"])
def test_trajectory_fp32_mix_full_size_100_steps(pp):
    """The mixed workload at its full size (H = 64, P = 1e6, M0 = 80,
    dt = 5e-5, the launch configuration the benchmark uses): after 100 steps
    the 1024 stored particles lie within 1e-4 (minimum image) of the FP64
    oracle's positions, and the modes 0 <= q <= 3 of alpha within 1e-5 of the
    largest of them."""
    cfg = workloads.CONFIGS["fp32_mix_h64"]
    ids, Xg, ag = _golden_mix_trajectory()
    say("trajectory fp32 mix full size", cfg["P"], pp)
    X0 = cfg["init"](cfg["P"]).astype(np.float32)
    sim = pkg.Sim(X0, **dict(cfg["params"], particle_pass=pp))
    sim.run(100)
    X = to_np(sim.positions()).astype(np.float64)
    A = to_np(sim.field("alpha")).astype(np.complex128)
    sim.close()
    err = np.abs(osipf.min_image(X[ids] - Xg, 2.0)).max()
    amax = max(abs(v) for v in ag.values())
    aerr = max(abs(A[q] - v) for q, v in ag.items()) / amax
    say(" max position error", err, "alpha error", aerr)
    assert err < 1e-4
    assert aerr < 1e-5


@pytest.mark.parametrize("scheme", ["strang", "em"])
def test_stepwise_parity_strong_aggregation(scheme):
    """M0 = 400: the dynamics amplifies rounding differences (the oracle itself
    turns a 1e-7 perturbation into ~4e-3 after 100 steps), so parity is checked
    per step along the GPU trajectory: at steps 1, 30, 60, 100 the oracle takes
    the GPU state and advances it one step."""
    say("stepwise fp32 H=64 M0=400", scheme)
    cfg = workloads.CONFIGS["fp32_mix_h64"]
    P = 30000
    X0 = cfg["init"](P).astype(np.float32)
    kw = dict(cfg["params"], scheme=scheme, M0=400.0)
    prm = oparams(**kw)
    sim = pkg.Sim(X0, **kw)
    done = 0
    for n in (1, 30, 60, 100):
        sim.run(n - 1 - done)
        Xk, Ak = _state_np(sim)
        sim.step()
        done = n
        X1, A1 = _state_np(sim)
        rec = {}
        Xo, ao = osipf.step(Xk, osipf.full_spectrum(Ak), n, prm, record=rec)
        assert rel_l2(A1, osipf.half_spectrum(ao)) < 1e-5, n
        drift = prm.chi * prm.dt * np.abs(rec["v"]).max()
        assert np.abs(osipf.min_image(X1 - Xo, 2.0)).max() < 1e-6 + 1e-5 * drift, n
    assert sim.n == 100


# ---------------------------------------------------------------------------
# full-size configurations in the bench launch configuration (sampled checks)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,nsteps,pp", [("fp32_mix_h64", 3, "sorted"), ("fp32_mix_h64", 3, "two_phase"),
                                            ("fp32_ring_h128", 3, "sorted"), ("fp32_ring_h128", 3, "two_phase")])
def test_full_size_sampled(name, nsteps, pp):
    cfg = workloads.CONFIGS[name]
    P = cfg["P"]
    say("full size", name, P, pp)
    X0 = cfg["init"](P).astype(np.float32)
    sim = pkg.Sim(X0, **dict(cfg["params"], particle_pass=pp))
    sim.run(nsteps)
    prm = oparams(**cfg["params"])
    Xk, Ak = _state_np(sim)
    Gk = to_np(sim.field("grad"))
    # closed form of the q = 0 coefficient (exact mass conservation of the deposit)
    r = 1 / (1 + prm.dt * prm.k ** 2 / prm.eps)
    a00 = prm.dt * prm.M0 / (prm.eps * prm.L ** 3) * r * (1 - r ** nsteps) / (1 - r)
    assert abs(Ak[0, 0, 0].real - a00) < 2e-5 * a00
    # gradient grid of the GPU's alpha
    afull = osipf.full_spectrum(Ak)
    assert rel_l2(Gk, osipf.gradient_grid(afull, prm)) < 1e-5
    # deposit of the current positions (all particles, oracle in batches)
    rho = to_np(sim.field("rho")).astype(np.float64)
    ref = np.zeros_like(rho)
    for s in range(0, P, 1_000_000):
        ref += osipf.deposit(Xk[s:s + 1_000_000], prm.M0 / P, prm.H, prm.L, 4)
    assert rel_l2(rho, ref) < 1e-5
    assert abs(rho.sum() - prm.M0) < 1e-5 * prm.M0
    # next step: alpha everywhere, positions of sampled particles one by one
    sim.step()
    X1, A1 = _state_np(sim)
    beta = osipf.forward_transform(ref, prm.L)
    a1 = osipf.mode_update(afull, beta, prm)
    assert rel_l2(A1, osipf.half_spectrum(a1)) < 1e-5
    ids = np.random.default_rng(5).choice(P, 2000, replace=False).astype(np.uint64)
    Gref = osipf.gradient_grid(afull, prm)
    Xs, _, _, _, _ = osipf.push(Xk[ids.astype(np.int64)], Gref, nsteps + 1, prm, ids)
    assert np.abs(osipf.min_image(X1[ids.astype(np.int64)] - Xs, 2.0)).max() < 2e-6
