"""Batched ensembles, graph replay, snapshots and the autotuner on the GPU.

Each instance of a batch must compute what the FP64 oracle computes for its
own parameters (same tolerances as the single-instance parity tests), and what
a standalone context computes (up to summation order).  Graph replay, a
snapshot round trip and tuned tile / chunk / re-sort settings may change only
the summation order of the deposit, never the arithmetic.
"""

import os
import math
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


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.complex128)
    b = np.asarray(b, dtype=np.complex128)
    nb = np.linalg.norm(b.ravel())
    return np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0)


def oparams(**kw):
    kw = dict(kw)
    kw.pop("precision", None)
    for k in ("tile", "resort_every", "chunk", "particle_pass"):
        kw.pop(k, None)
    return osipf.Params(**kw)


def to_np(t):
    return t.detach().cpu().numpy()


def _instances(precision, specs, seed=0, pp="default"):
    """specs: (H, P, chi, M0, mu) per instance; blob initial data, distinct streams."""
    out = []
    for i, (H, P, chi, M0, mu) in enumerate(specs):
        X0 = workloads.blob(P, 0.15, seed=100 + i)
        X0 = X0.astype(np.float32 if precision == "fp32" else np.float64)
        prm = dict(L=2.0, chi=chi, mu=mu, eps=1.0, k=1.0, M0=M0, dt=1e-3 if precision == "fp64" else 5e-5, H=H,
                   precision=precision, seed=seed + 7, instance=i, particle_pass=pp)
        out.append(dict(params=prm, X0=X0))
    return out


# ragged particle counts (one particle, primes, several sort chunks), three grid sizes
SPECS_FP64 = [(16, 1, 1.0, 30.0, 1.0), (8, 333, 2.0, 50.0, 0.5), (32, 4099, 0.5, 60.0, 1.0),
              (16, 2000, 1.5, 40.0, 0.8), (32, 9000, 1.0, 80.0, 1.0)]


def test_batch_fp64_each_instance_matches_oracle():
    say("batch fp64 vs oracle", len(SPECS_FP64), "instances")
    inst = _instances("fp64", SPECS_FP64)
    b = pkg.Batch(inst)
    nsteps = 12  # first steps eager, then one captured graph of two re-sort periods
    b.run(nsteps)
    b.sync()
    for i, it in enumerate(inst):
        say(" instance", i, "H", it["params"]["H"], "P", it["X0"].shape[0])
        prm = oparams(**it["params"])
        Xo, ao = osipf.run(it["X0"].astype(np.float64), prm, nsteps)
        X = to_np(b.positions(i)).astype(np.float64)
        A = to_np(b.field(i, "alpha")).astype(np.complex128)
        assert np.abs(osipf.min_image(X - Xo, 2.0)).max() < 1e-9, i
        assert rel_l2(A, osipf.half_spectrum(ao)) < 1e-12, i
        assert b.step_count(i) == nsteps
    b.close()


@pytest.mark.parametrize("pp", ["sorted", "two_phase"])
def test_batch_fp32_instances_match_standalone_contexts(pp):
    specs = [(32, 50000, 0.5, 40.0, 1.0), (64, 12345, 2.0, 120.0, 1.0), (32, 777, 1.2, 90.0, 1.0),
             (64, 65537, 1.0, 60.0, 1.0), (32, 20000, 1.8, 100.0, 1.0), (64, 3001, 0.7, 70.0, 1.0)]
    say("batch fp32 vs standalone", len(specs), "instances", pp)
    inst = _instances("fp32", specs, pp=pp)
    b = pkg.Batch(inst)
    b.run(20)
    for i, it in enumerate(inst):
        sim = pkg.Sim(it["X0"], **it["params"])
        sim.run(20)
        X1, X2 = to_np(b.positions(i)), to_np(sim.positions())
        A1, A2 = to_np(b.field(i, "alpha")), to_np(sim.field("alpha"))
        G1, G2 = to_np(b.field(i, "grad")), to_np(sim.field("grad"))
        sim.close()
        assert np.abs(osipf.min_image(X1.astype(np.float64) - X2, 2.0)).max() < 1e-5, i
        assert rel_l2(A1, A2) < 1e-5, i
        assert rel_l2(G1, G2) < 1e-5, i
    b.close()


@pytest.mark.parametrize("pp", ["sorted", "two_phase"])
def test_batch_fp32_against_oracle_stepwise(pp):
    """Two instances of different H in one batch; the oracle advances the GPU
    state of each by one step at steps 1 and 10."""
    specs = [(32, 20001, 1.5, 100.0, 1.0), (64, 30000, 0.8, 60.0, 1.0)]
    inst = _instances("fp32", specs, pp=pp)
    b = pkg.Batch(inst)
    done = 0
    for n in (1, 10):
        b.run(n - 1 - done)
        prev = [(to_np(b.positions(i)).astype(np.float64), to_np(b.field(i, "alpha")).astype(np.complex128))
                for i in range(len(inst))]
        b.run(1)
        done = n
        for i, it in enumerate(inst):
            prm = oparams(**it["params"])
            rec = {}
            Xo, ao = osipf.step(prev[i][0], osipf.full_spectrum(prev[i][1]), n, prm, record=rec)
            X1 = to_np(b.positions(i)).astype(np.float64)
            A1 = to_np(b.field(i, "alpha"))
            assert rel_l2(A1, osipf.half_spectrum(ao)) < 1e-5, (n, i)
            drift = prm.chi * prm.dt * np.abs(rec["v"]).max()
            assert np.abs(osipf.min_image(X1 - Xo, 2.0)).max() < 1e-6 + 1e-5 * drift, (n, i)
    b.close()


def test_ensemble_workload_sampled():
    """The 64-instance ensemble in the benchmark's launch configuration: every
    instance stays finite with its step count, and the two smallest instances
    are advanced by the oracle from the GPU state for one step."""
    ens = workloads.ensemble(64, seed=0)
    say("ensemble 64 instances, total P", sum(e["P"] for e in ens))
    inst = [dict(params=e["params"], X0=e["X0"].astype(np.float32)) for e in ens]
    b = pkg.Batch(inst)
    b.run(5)
    small = sorted(range(64), key=lambda i: ens[i]["P"])[:2]
    prev = {i: (to_np(b.positions(i)).astype(np.float64), to_np(b.field(i, "alpha")).astype(np.complex128))
            for i in small}
    b.run(1)
    for i in range(64):
        assert b.step_count(i) == 6
    for i in small:
        prm = oparams(**ens[i]["params"])
        rec = {}
        Xo, ao = osipf.step(prev[i][0], osipf.full_spectrum(prev[i][1]), 6, prm, record=rec)
        X1 = to_np(b.positions(i)).astype(np.float64)
        assert rel_l2(to_np(b.field(i, "alpha")), osipf.half_spectrum(ao)) < 1e-5, i
        drift = prm.chi * prm.dt * np.abs(rec["v"]).max()
        assert np.abs(osipf.min_image(X1 - Xo, 2.0)).max() < 1e-6 + 1e-5 * drift, i
    for i in range(0, 64, 9):
        assert torch.isfinite(b.positions(i)).all()
    b.close()


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-11), ("fp32", 1e-5)])
def test_graph_replay_matches_eager(precision, tol):
    say("graph vs eager", precision)
    X0 = workloads.blob(3000, 0.15, seed=5).astype(np.float32 if precision == "fp32" else np.float64)
    kw = dict(L=2.0, chi=2.0, mu=1.0, eps=1.0, k=1.0, M0=60.0, dt=1e-3, H=16, precision=precision, seed=3,
              resort_every=2)
    a = pkg.Sim(X0, **kw)
    e = pkg.Sim(X0, **kw)
    e.use_graphs(False)
    for chunk in (3, 9, 1, 8):  # 21 steps: eager heads, graph replays of 4 steps, eager tails
        a.run(chunk)
        e.run(chunk)
    Xa, Xe = to_np(a.positions()).astype(np.float64), to_np(e.positions()).astype(np.float64)
    assert a.n == e.n == 21
    assert np.abs(osipf.min_image(Xa - Xe, 2.0)).max() < tol
    assert rel_l2(to_np(a.field("alpha")), to_np(e.field("alpha"))) < tol
    if precision == "fp64":
        Xo, _ = osipf.run(X0.astype(np.float64), oparams(**kw), 21)
        assert np.abs(osipf.min_image(Xa - Xo, 2.0)).max() < 1e-9
    a.close()
    e.close()


@pytest.mark.parametrize("resort,pp", [(1, "two_phase"), (2, "sorted"), (3, "two_phase"), (5, "sorted")])
def test_sort_counts_taken_by_the_particle_pass(resort, pp):
    """The step before each re-sort counts its particles' tiles in the particle
    pass and the sort skips its histogram; the sort's scan checks that the
    counts add up to P (a mismatch raises at the next read).  Graph replay,
    eager stepping, a batch and the adjoint (whose segment sorts take their own
    histogram after the forward) agree, in FP64 with the oracle."""
    say("counted sorts", resort, pp)
    X0 = workloads.mix(6000, 0.15, seed=7)
    kw = dict(L=2.0, chi=2.0, mu=1.0, eps=1.0, k=1.0, M0=60.0, dt=1e-3, H=32, seed=4, resort_every=resort,
              particle_pass=pp)
    # FP64: graph replay and eager stepping against the oracle
    a = pkg.Sim(X0, precision="fp64", **kw)
    e = pkg.Sim(X0, precision="fp64", **kw)
    e.use_graphs(False)
    for chunk in (4, 11, 2, 7):
        a.run(chunk)
        e.run(chunk)
    Xo, _ = osipf.run(X0, oparams(**kw), 24)
    for s in (a, e):
        X = to_np(s.positions()).astype(np.float64)
        assert np.abs(osipf.min_image(X - Xo, 2.0)).max() < 1e-9
        s.close()
    # FP32 batch of three instances (two grid sizes) against standalone contexts
    # (the workloads' time step: FP32 rounding differences between the two
    # sort orders stay at rounding level over the 17 steps)
    inst = [dict(params=dict(kw, H=H, instance=i, precision="fp32", dt=5e-5),
                 X0=workloads.blob(P, 0.15, seed=20 + i).astype(np.float32))
            for i, (H, P) in enumerate(((32, 5000), (16, 3001), (32, 777)))]
    b = pkg.Batch(inst)
    b.run(17)
    for i, it in enumerate(inst):
        sim = pkg.Sim(it["X0"], **it["params"])
        sim.run(17)
        Xb, Xs = to_np(b.positions(i)).astype(np.float64), to_np(sim.positions()).astype(np.float64)
        assert np.abs(osipf.min_image(Xb - Xs, 2.0)).max() < 1e-5, i
        sim.close()
    b.close()


def test_adjoint_after_a_counting_step():
    """A forward whose last step counted the tiles of a sort it never runs:
    the adjoint's own segment sorts start from clear counts."""
    kw = dict(L=2.0, chi=1.0, mu=1.0, eps=1.0, k=1.0, M0=40.0, dt=1e-3, H=16, seed=2, resort_every=3,
              precision="fp64")
    X0 = workloads.blob(2000, 0.15, seed=9)
    sim = pkg.Sim(X0, **kw)
    loss, dchi, dmu, dX0 = sim.adjoint(5, ckpt_every=2)  # steps 1..5: step 5 counts for the sort due at step 6
    sim.run(4)  # the restored context keeps stepping (its re-sort after the adjoint takes a histogram)
    X = to_np(sim.positions()).astype(np.float64)
    Xo, _ = osipf.run(X0, oparams(**kw), 9)
    assert np.abs(osipf.min_image(X - Xo, 2.0)).max() < 1e-9
    assert math.isfinite(loss) and math.isfinite(dchi) and math.isfinite(dmu)
    sim.close()


def test_snapshot_round_trip(tmp_path):
    say("save / load")
    X0 = workloads.blob(2000, 0.15, seed=9)
    kw = dict(L=2.0, chi=1.5, mu=1.0, eps=1.0, k=1.0, M0=50.0, dt=1e-3, H=16, precision="fp64", seed=21,
              instance=3)
    a = pkg.Sim(X0, **kw)
    a.run(7)
    path = tmp_path / "state.sipf"
    a.save(path)
    b = pkg.Sim.load(path)
    assert b.n == 7 and b.P == 2000 and b.H == 16
    assert b.params.instance == 3 and b.params.seed == 21 and b.params.chi == 1.5
    assert np.array_equal(to_np(a.positions()), to_np(b.positions()))
    assert rel_l2(to_np(a.field("alpha")), to_np(b.field("alpha"))) < 1e-15
    a.run(6)
    b.run(6)
    assert a.n == b.n == 13
    Xa, Xb = to_np(a.positions()), to_np(b.positions())
    assert np.abs(osipf.min_image(Xa - Xb, 2.0)).max() < 1e-11
    Xo, _ = osipf.run(X0, oparams(**kw), 13)
    assert np.abs(osipf.min_image(Xb - Xo, 2.0)).max() < 1e-9
    a.close()
    b.close()


def test_autotune_picks_valid_settings_that_keep_results():
    say("autotune")
    X0 = workloads.mix(40000, 0.15, seed=2).astype(np.float32)
    kw = dict(L=2.0, chi=1.0, mu=1.0, eps=1.0, k=1.0, M0=80.0, dt=5e-5, H=32, precision="fp32", seed=0)
    tuned, ms = pkg.autotune(X0, nsteps=4, **kw)
    say(" tuned", tuned, ms)
    assert ms > 0
    assert tuned["tile"] in (4, 8, 16, 32) and 32 // tuned["tile"] <= 16
    assert tuned["chunk"] in (1024, 2048, 3072, 4096)
    assert tuned["resort_every"] in (2, 4, 6, 8, 16)
    assert tuned["particle_pass"] in (1, 2)
    a = pkg.Sim(X0, **kw)
    t = pkg.Sim(X0, **kw, **tuned)
    a.run(10)
    t.run(10)
    Xa, Xt = to_np(a.positions()).astype(np.float64), to_np(t.positions()).astype(np.float64)
    assert np.abs(osipf.min_image(Xa - Xt, 2.0)).max() < 1e-5
    a.close()
    t.close()
