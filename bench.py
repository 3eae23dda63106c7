"""Throughput of the SIPF-PIC step on one MI355X.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--scheme strang|em]

A step is one pass of the whole hot path (particle pass: deposit, gather,
push; field passes: forward FFT, mode update, filtered gradient, inverse FFT;
the periodic tile sort) over the resident particles.  Inputs are resident in
HBM before timing starts.  Prints one JSON line.
"""

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "particle-steps/s + ms/step at P=1e7,H=128; fwd+adjoint vs fwd on same GPU"
HBM_PEAK_GBS = 8000.0


def algorithmic_bytes(phase, P, H, tsize):
    """Bytes the method itself must move per launch of a pass (every array of
    the step read or written once; the byte model of the step, Sec. 3.2's
    O(P + H^3 log H) count): 24 P + 40 H^3 per FP32 step in all.  Particle
    ids, the re-sort and the intermediate spectra of the transforms are
    implementation overhead and are not counted here."""
    grid = tsize * H ** 3
    if phase == "particles":
        return 6 * tsize * P + grid + 3 * grid     # X read + write, deposit out, 3 gradient grids in
    if phase == "fwd_planes":
        return grid                                # deposit in
    if phase == "xpencils":
        return 2 * 2 * tsize * H * H * (H // 2 + 1)  # alpha read + write (half spectrum)
    if phase == "inv_planes":
        return 3 * grid                            # 3 gradient grids out
    return 0                                       # the re-sort moves no algorithmic bytes


def step_algorithmic_bytes(P, H, tsize):
    """24 P + 40 H^3 (FP32): X read + write, deposit write + read, alpha
    read + write, three gradient grids write + read."""
    return 6 * tsize * P + 2 * tsize * H ** 3 + 2 * 2 * tsize * H * H * (H // 2 + 1) + 6 * tsize * H ** 3


def implementation_bytes(phase, P, H, tsize):
    """Bytes each pass of this implementation touches at least once: the
    algorithmic bytes plus ids (the noise counter), the half spectra passed
    between the transform passes, and the re-sort's scatter, which reads and
    writes X and the ids (the re-sorts of a 3-D run take their tile counts
    from the particle pass of the step before, so no histogram pass reads X
    again)."""
    spec = 2 * tsize * H * H * (H // 2 + 1)
    grid = tsize * H ** 3
    if phase == "particles":
        return 6 * tsize * P + 4 * P + grid + 3 * grid
    if phase == "fwd_planes":
        return grid + spec
    if phase == "xpencils":
        return spec + 2 * spec + 3 * spec
    if phase == "inv_planes":
        return 3 * spec + 3 * grid
    if phase == "sort":
        return 2 * (3 * tsize + 4) * P
    return 0


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "particles_ring_h128_traffic.md")
TRAFFIC_SOURCES = ["paper_2512_03452_amd/csrc/particles.hip", "paper_2512_03452_amd/csrc/pass_common.h",
                   "paper_2512_03452_amd/csrc/common.h", "paper_2512_03452_amd/csrc/internal.h"]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of the particle pass from the committed counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the
    summary is missing or the kernel's sources changed since it was taken."""
    if kernel != "particles" or workload != "fp32_ring_h128" or not os.path.exists(TRAFFIC_FILE):
        return None
    import hashlib
    h = hashlib.sha256()
    for src in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, src), "rb") as f:
            h.update(f.read())
    with open(TRAFFIC_FILE) as f:
        for line in f:
            if line.startswith("TRAFFIC "):
                kv = dict(t.split("=", 1) for t in line.split()[1:])
                if kv.get("kernel") == kernel and kv.get("sources_sha256") == h.hexdigest():
                    return int(kv["fetch_bytes"]) + int(kv["write_bytes"])
    return None


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_worker(args):
    """One oracle run on its own sample: an untimed first step, then `steps`
    timed steps (started together with the other workers)."""
    workload, sample_P, steps, seed, barrier = args
    import numpy as np
    from oracle import sipf as osipf
    from paper_2512_03452_amd import workloads
    cfg = workloads.CONFIGS[workload]
    prm = dict(cfg["params"])
    prm.pop("precision", None)
    p = osipf.Params(**prm)
    X = cfg["init"](sample_P, seed=seed)
    alpha = np.zeros((p.H, p.H, p.H), dtype=np.complex128)
    ids = np.arange(sample_P, dtype=np.uint64)
    X, alpha = osipf.step(X, alpha, 1, p, ids)
    if barrier is not None:
        barrier.wait()
    t0 = time.perf_counter()
    for n in range(2, 2 + steps):
        X, alpha = osipf.step(X, alpha, n, p, ids)
    return time.perf_counter() - t0


def cpu_baseline(workload, H, sample_P, steps, workers):
    """The FP64 oracle on the host: `workers` concurrent processes (the host's
    cores), each stepping its own sample of sample_P particles of the same
    workload on the full grid, and one process alone.  numpy's FFT and
    bincount in the oracle are single-threaded, so one process uses one core."""
    import multiprocessing as mp
    nproc = os.cpu_count()
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = nproc
    ctx = mp.get_context("spawn")
    one = _oracle_worker((workload, sample_P, steps, 1, None))
    out = {"unit": "particle-steps/s", "kind": "oracle", "cpu_model": _cpu_model(), "nproc": nproc,
           "cores_available": avail,
           "one_core": {"value": sample_P * steps / one, "cores": 1, "wall_s": one}}
    if workers > 1:
        with ctx.Manager() as man:
            bar = man.Barrier(workers)
            with ctx.Pool(workers) as pool:
                walls = pool.map(_oracle_worker, [(workload, sample_P, steps, 1 + w, bar) for w in range(workers)])
        wall = max(walls)
        out.update(value=workers * sample_P * steps / wall, cores=workers, wall_s=wall)
    else:
        out.update(value=sample_P * steps / one, cores=1, wall_s=one)
    out["sample"] = (f"{out['cores']} concurrent oracle processes, each {sample_P} particles of the {workload} "
                     f"workload on the H={H} grid (own seed), {steps} timed steps after 1 untimed step; "
                     f"one_core: one process alone on the same sample")
    return out


def adjoint_ratio(pkg, workloads, np, torch):
    """fwd+adjoint time over forward time on the adjoint workload (same GPU),
    in FP64 and in the workload's FP32.  Each adjoint runs twice from the same
    inputs (the faster run is timed): the relative difference of the two dL/dX0
    shows how far rounding (summation order of the deposit) is amplified along
    the trajectory.  The headline ratio is FP64's: over these 100 steps the
    gradient is ill-conditioned (inputs perturbed at the float32 rounding level
    change it by O(1) even in FP64), so only FP64 gives it reproducibly and at
    the oracle's accuracy."""
    cfg = workloads.CONFIGS["fp32_adjoint_h64"]
    P, N, K = cfg["P"], cfg["steps"], 10
    out = {"workload": "fp32_adjoint_h64", "P": P, "H": cfg["params"]["H"], "steps": N, "ckpt_every": K}
    for prec in ("fp64", "fp32"):
        params = dict(cfg["params"], precision=prec)
        X0 = cfg["init"](P).astype(np.float32 if prec == "fp32" else np.float64)
        sim = pkg.Sim(X0, **params)
        sim.run(9)
        sim.sync()
        sim.close()
        sim = pkg.Sim(X0, **params)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run(N)
        sim.sync()
        t_fwd = time.perf_counter() - t0
        sim.close()
        runs = []
        for rep in range(2):
            sim = pkg.Sim(X0, **params)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            loss, dchi, dmu, dX0 = sim.adjoint(N, K)
            torch.cuda.synchronize()
            runs.append((time.perf_counter() - t0, loss, dchi, dmu, dX0.double()))
            sim.close()
        t_adj = min(r[0] for r in runs)
        a, b = runs[0][4], runs[1][4]
        out[prec] = {"fwd_ms": 1e3 * t_fwd, "fwd_adj_ms": 1e3 * t_adj, "ratio": t_adj / t_fwd,
                     "loss": runs[0][1], "dchi": [runs[0][2], runs[1][2]], "dmu": [runs[0][3], runs[1][3]],
                     "dX0_rel_diff_between_runs": float(torch.linalg.norm(a - b) / torch.linalg.norm(a)),
                     "grad_finite": bool(np.isfinite(runs[0][2]) and torch.isfinite(a).all().item())}
    out["ratio"] = out["fp64"]["ratio"]
    out["ratio_precision"] = "fp64"
    return out


def ensemble_throughput(pkg, workloads, np, torch, steps=40):
    """64-instance ensemble (uneven P, H, chi): one batch versus the same
    instances advanced one context after another (same GPU, same steps)."""
    ens = workloads.ensemble(64, seed=0)
    inst = [dict(params=e["params"], X0=e["X0"].astype(np.float32)) for e in ens]
    total_P = sum(e["P"] for e in ens)
    b = pkg.Batch(inst)
    b.run(9)
    b.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.run(steps)
    b.sync()
    t_batch = time.perf_counter() - t0
    b.profile(True)
    b.run(8)
    prof = b.profile_read()
    b.profile(False)
    b.close()
    del b
    t_seq = 0.0
    for it in inst:
        sim = pkg.Sim(it["X0"], **it["params"])
        sim.run(9)
        sim.sync()
        t0 = time.perf_counter()
        sim.run(steps)
        sim.sync()
        t_seq += time.perf_counter() - t0
        sim.close()
    return {"workload": "ensemble64_h32_h64", "instances": 64, "total_P": total_P, "steps": steps,
            "batched_ms_per_step": 1e3 * t_batch / steps, "batched_particle_steps_per_s": total_P * steps / t_batch,
            "sequential_ms_per_step": 1e3 * t_seq / steps, "sequential_particle_steps_per_s": total_P * steps / t_seq,
            "speedup": t_seq / t_batch,
            "phases_us_per_step": {k: 1e3 * v[0] / 8 for k, v in prof.items() if v[1]}}


def algorithmic_bytes_2d(phase, P, H, tsize):
    """Bytes each 2-D pass must move (every array read or written once)."""
    spec = 2 * tsize * H * (H // 2 + 1)
    grid = tsize * H * H
    if phase == "particles":
        # X read + write (2 coordinates), id read, deposit out, 2 gradient grids in
        return 4 * tsize * P + 4 * P + grid + 2 * grid
    if phase == "fwd_planes":
        return grid + spec
    if phase == "xpencils":
        return spec + 2 * spec + 2 * spec
    if phase == "inv_planes":
        return 2 * spec + 2 * grid
    return 0


def two_d_section(pkg, workloads, np, torch, level, steps=100, warmup=20):
    """The 2-D parabolic-elliptic runs of Sec. 5.2: step throughput at the
    critical-mass configuration (P = 2^22, H = 2048, L = 8), then the
    critical-mass and second-moment studies (full: the paper's sizes)."""
    from paper_2512_03452_amd import critical2d
    P, H, L = 1 << 22, 2048, 8.0
    prm = dict(critical2d.PARAMS_2D, L=L, H=H, M0=25.0, dt=5e-4, precision="fp32", seed=0)
    sim = pkg.Sim(workloads.disk(P, 1.0, seed=0).astype(np.float32), **prm)
    sim.run(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(steps)
    sim.sync()
    el = time.perf_counter() - t0
    sim.profile(True)
    sim.run(steps)
    prof = sim.profile_read()
    sim.profile(False)
    sim.close()
    phases = {k: {"us_avg": 1e3 * v[0] / v[1]} for k, v in prof.items() if v[1]}
    avg = prof["particles"][0] / prof["particles"][1] / 1e3
    ab = algorithmic_bytes_2d("particles", P, H, 4)
    out = {"workload": "disk_2d_elliptic_h2048", "P": P, "H": H, "L": L, "M0": 25.0, "dt": 5e-4, "steps": steps,
           "ms_per_step": 1e3 * el / steps, "particle_steps_per_s": P * steps / el, "phases": phases,
           "roofline": {"bound": "hbm", "kernel": "particles", "achieved": ab / avg / 1e9, "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": ab / avg / 1e9 / HBM_PEAK_GBS, "algorithmic_bytes_per_launch": ab,
                        "avg_launch_us": avg * 1e6}}
    if level == "full":
        cm, secs = critical2d.critical_mass_study()
        out["critical_mass"] = {"gpu_seconds": secs, "L": 8.0, "H": 2048, "P": 1 << 22, "T": 2.0,
                                "final": {str(M0): {"t": s[-1][0], "rho_max": s[-1][1], "hf_share": s[-1][2],
                                                    "m2": s[-1][3], "rho_max_t0": s[0][1]} for M0, s in cm.items()}}
        rows, secs = critical2d.second_moment_study()
        out["second_moment"] = {"gpu_seconds": secs, "T": 2.0, "P": 1 << 20, "rows": rows}
    else:
        cm, secs = critical2d.critical_mass_study(M0s=(22.0, 27.0), H=1024, P=1 << 20, T=0.5, every=250)
        out["critical_mass"] = {"gpu_seconds": secs, "L": 8.0, "H": 1024, "P": 1 << 20, "T": 0.5,
                                "final": {str(M0): {"t": s[-1][0], "rho_max": s[-1][1], "hf_share": s[-1][2],
                                                    "m2": s[-1][3], "rho_max_t0": s[0][1]} for M0, s in cm.items()}}
        rows, secs = critical2d.second_moment_study(Ls=(10.0, 20.0), M0s=(25.0,), P=1 << 18, T=0.5)
        out["second_moment"] = {"gpu_seconds": secs, "T": 0.5, "P": 1 << 18, "rows": rows}
    return out


def positivity_section(pkg, torch, X0, params, plain_ms, steps=20):
    """Step time with the positivity-preserving deposit (deposit, rounds, push as
    separate passes, no graphs) against the fused step, and its switch counts."""
    sim = pkg.Sim(X0, **dict(params, positivity=1))
    sim.run(3)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(steps)
    sim.sync()
    torch.cuda.synchronize()
    ms = 1e3 * (time.perf_counter() - t0) / steps
    switched, rounds = sim.positivity_stats()
    sim.close()
    return {"steps": steps, "ms_per_step": ms, "ratio_to_plain_step": ms / plain_ms,
            "switched_last_step": switched, "rounds_last_step": rounds, "P": int(X0.shape[0])}


def scheme_section(pkg, torch, X0, params, scheme, steps=100, warmup=20):
    """The same workload stepped with another push scheme (graph-replayed
    sipf_run, as the headline timing)."""
    sim = pkg.Sim(X0, **dict(params, scheme=scheme))
    sim.run(warmup)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(steps)
    sim.sync()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    sim.close()
    return {"scheme": scheme, "steps": steps, "ms_per_step": 1e3 * el / steps,
            "particle_steps_per_s": X0.shape[0] * steps / el}


def full_run_section(pkg, torch, X0, params, steps):
    """The workload's whole run (the configuration's step count from step 0,
    graph-replayed) with each FP32 particle pass: the torus contracts over
    the run and the pass that wins early is not the one that wins after the
    collapse."""
    out = {"steps": steps}
    for pp in ("two_phase", "sorted"):
        sim = pkg.Sim(X0, **dict(params, particle_pass=pp))
        sim.prepare_run(steps)
        sim.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.run(steps)
        sim.sync()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        rho_max = sim.diagnostics()["rho_max"]
        sim.close()
        out[pp] = {"ms_total": 1e3 * el, "ms_per_step": 1e3 * el / steps,
                   "particle_steps_per_s": X0.shape[0] * steps / el, "rho_max_end": rho_max}
    return out


def calibrate_copy(torch, nbytes=1 << 30, reps=5):
    """A plain device copy of nbytes, reps times: the reference whose HBM
    counters (FETCH_SIZE, WRITE_SIZE) scale those of the step's kernels."""
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"calibration": "device copy", "bytes_read": nbytes, "bytes_written": nbytes, "reps": reps}),
          flush=True)


def e1_study(size):
    """Convergence study of Sec. 5.1 against the stored radial reference:
    mean truncated quantile discrepancy per (P, H) and the log2 slopes."""
    from paper_2512_03452_amd import convergence
    q_ref = convergence.load_reference(os.path.join(ROOT, "tests", "golden", "radial_e1_quantiles.txt"))
    if size == "full":
        Ps, Hs, hmax, nsim = [2 ** e for e in range(11, 21)], [8, 16, 32, 64, 128], 128, 30
    else:
        Ps, Hs, hmax, nsim = [2 ** 11, 2 ** 13, 2 ** 15], [8, 16, 32], 64, 8
    pH = Ps[-1] if size == "full" else 2 ** 17
    configs = [(P, hmax) for P in Ps] + [(pH, H) for H in Hs if (pH, H) != (Ps[-1], hmax)]
    res, secs = convergence.run_study(configs, nsim, q_ref)
    eP = [res[(P, hmax)]["mean"] for P in Ps]
    eH = [res[(pH, H)]["mean"] for H in Hs]
    runs = nsim * len(configs)
    return {"nsim": nsim, "runs": runs, "steps": 2000, "gpu_seconds": secs,
            "particle_steps_per_s": nsim * sum(P for P, _ in configs) * 2000 / secs,
            "slope_P": convergence.slope(Ps, eP), "slope_H": convergence.slope(Hs, eH),
            "P": Ps, "E_vs_P": eP, "H_at_P": pH, "H": Hs, "E_vs_H": eH,
            "paper_slopes": {"P": -0.512, "H": -1.327}}


def e2_study(size):
    """SIPF (direct, Algorithm 1) against SIPF-PIC with P = H^3 in the setup of
    the convergence study: mean error and time of one run per grid size."""
    from paper_2512_03452_amd import convergence

    def log(msg):
        print("#   " + msg, file=sys.stderr, flush=True)
    q_ref = convergence.load_reference(os.path.join(ROOT, "tests", "golden", "radial_e1_quantiles.txt"))
    # the grid sizes of the paper's comparison (P = H^3), mixed-radix ones included
    if size == "full":
        rows = convergence.cost_error_study((8, 12, 16, 22, 32, 46, 64, 90, 128), 8, q_ref, max_direct_H=46,
                                            timing_steps=10, log=log)
    else:
        rows = convergence.cost_error_study((8, 12, 16, 22, 32, 46, 64), 4, q_ref, max_direct_H=32, timing_steps=10,
                                            log=log)
    return {"steps": 2000, "rows": rows}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="fp32_ring_h128")
    ap.add_argument("--scheme", default="strang", choices=["strang", "em"])
    ap.add_argument("--particle-pass", default="default", choices=["default", "sorted", "two_phase"],
                    help="FP32 particle pass of the timed workload (sipf_params.particle_pass)")
    ap.add_argument("--cpu-sample", type=int, default=1_000_000)
    ap.add_argument("--cpu-steps", type=int, default=2)
    ap.add_argument("--cpu-workers", type=int, default=0,
                    help="concurrent oracle processes (default: the usable host cores, at most 16)")
    ap.add_argument("--steady-steps", type=int, default=0,
                    help="steps of the steady-state reference run after the timed one (default: 4 graph periods)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-positivity", action="store_true")
    ap.add_argument("--no-other-scheme", action="store_true")
    ap.add_argument("--no-full-run", action="store_true",
                    help="skip the whole-run timing of the workload with each particle pass")
    ap.add_argument("--e1", default="reduced", choices=["none", "reduced", "full"],
                    help="convergence study of Sec. 5.1: 8 runs of 6 configurations, or the full 30 x 14")
    ap.add_argument("--e2", default="quick", choices=["none", "quick", "full"],
                    help="SIPF (direct) against SIPF-PIC with P = H^3: error and time per run")
    ap.add_argument("--two-d", default="quick", choices=["none", "quick", "full"],
                    help="2-D parabolic-elliptic runs of Sec. 5.2 (throughput, critical mass, second moment)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and exit")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU only (asked for --gpus {args.gpus}); "
              "the multi-GPU decomposition is a design note, not an implemented path.", file=sys.stderr)
        sys.exit(2)

    if args.steady_steps <= 0:
        args.steady_steps = 96
    if args.cpu_workers <= 0:
        try:
            args.cpu_workers = min(16, len(os.sched_getaffinity(0)))
        except AttributeError:
            args.cpu_workers = min(16, os.cpu_count() or 1)

    import numpy as np
    import torch

    if args.calibrate_copy:
        calibrate_copy(torch)
        return

    import paper_2512_03452_amd as pkg
    from paper_2512_03452_amd import workloads

    cfg = workloads.CONFIGS[args.workload]
    P = cfg["P"]
    params = dict(cfg["params"], scheme=args.scheme, particle_pass=args.particle_pass)
    H = params["H"]
    fp32 = params["precision"] == "fp32"
    tsize = 4 if fp32 else 8
    torch.cuda.set_device(0)
    print(f"# workload {args.workload}: P={P} H={H} scheme={args.scheme}", file=sys.stderr, flush=True)
    X0 = cfg["init"](P).astype(np.float32 if fp32 else np.float64)
    sim = pkg.Sim(X0, **params)

    sim.run(args.warmup)
    # capture the HIP graphs the timed run replays (runs no step), so that the
    # timed window holds graph replays only
    sim.prepare_run(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(args.steps)
    sim.sync()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    print(f"# timed {args.steps} steps in {elapsed:.4f} s", file=sys.stderr, flush=True)
    # steady state for reference: whole graph periods after the timed run
    sim.prepare_run(args.steady_steps)
    sim.sync()
    t0 = time.perf_counter()
    sim.run(args.steady_steps)
    sim.sync()
    steady = time.perf_counter() - t0

    # run-time diagnostics of the state (one call = deposit, three FFT passes, reductions)
    sim.diagnostics()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(5):
        diag = sim.diagnostics()
    diag = dict(diag, ms_per_call=1e3 * (time.perf_counter() - t0) / 5)
    sim.close()

    # per-kernel durations with HIP events on the library's stream, over the
    # timed steps again: a fresh context from the same input (the same seeded
    # trajectory up to rounding) runs the warm-up, then the timed steps with
    # phase timing on, so that the durations belong to the same states as the
    # timed window (the torus contracts as it runs, and the pass slows down
    # once it has collapsed)
    sim = pkg.Sim(X0, **params)
    del X0
    sim.run(args.warmup)
    sim.profile(True)
    sim.run(args.steps)
    prof = sim.profile_read()
    sim.profile(False)
    sim.sync()
    sim.close()
    phases = {k: {"ms_total": v[0], "launches": v[1], "us_avg": (1e3 * v[0] / v[1]) if v[1] else None}
              for k, v in prof.items()}
    dom = max((k for k in phases if phases[k]["launches"]), key=lambda k: phases[k]["ms_total"])
    avg_s = phases[dom]["ms_total"] / phases[dom]["launches"] / 1e3
    abytes = algorithmic_bytes(dom, P, H, tsize)
    achieved = abytes / avg_s / 1e9
    print(f"# phases: " + ", ".join(f"{k}={v['us_avg']:.1f}us" for k, v in phases.items() if v['launches']),
          file=sys.stderr, flush=True)

    ms_per_step = 1e3 * elapsed / args.steps
    step_bytes = step_algorithmic_bytes(P, H, tsize)
    impl_step_bytes = sum(implementation_bytes(k, P, H, tsize) * v["launches"] / args.steps
                          for k, v in phases.items())
    traffic = measured_traffic(dom, args.workload)
    out = {
        "metric": METRIC,
        "value": P * args.steps / elapsed,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if fp32 else "f64",
        "data": "synthetic",
        "config": {"workload": args.workload, "P": P, "H": H, "scheme": args.scheme, "particle_pass": args.particle_pass,
                   "dt": params["dt"], "M0": params["M0"], "init": "torus R=0.5 sd=0.05"
                   if "ring" in args.workload else args.workload},
        # dominant kernel: algorithmic bytes per launch (24 P + 16 H^3 for the
        # particle pass) over its average launch time (HIP events on the
        # library's stream); traffic = counter-measured HBM bytes per launch
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_over_algorithmic": (traffic / abytes) if traffic else None,
                     "algorithmic_bytes_per_launch": abytes, "avg_launch_us": avg_s * 1e6},
        # the whole step: 24 P + 40 H^3 over the timed ms per step
        "step_roofline": {"algorithmic_bytes_per_step": step_bytes,
                          "frac": step_bytes / (ms_per_step / 1e3) / 1e9 / HBM_PEAK_GBS,
                          "implementation_bytes_per_step": impl_step_bytes,
                          "overhead_bytes_per_step": impl_step_bytes - step_bytes},
        "steady_state": {"steps": args.steady_steps, "ms_per_step": 1e3 * steady / args.steady_steps,
                         "particle_steps_per_s": P * args.steady_steps / steady},
        "phases": phases,
        # every pass: algorithmic and implementation bytes per launch over its average duration
        "phase_roofline": {k: {"algorithmic_bytes": algorithmic_bytes(k, P, H, tsize),
                               "implementation_bytes": implementation_bytes(k, P, H, tsize),
                               "GB_s": algorithmic_bytes(k, P, H, tsize) / (v["us_avg"] * 1e3),
                               "frac": algorithmic_bytes(k, P, H, tsize) / (v["us_avg"] * 1e3) / HBM_PEAK_GBS,
                               "implementation_GB_s": implementation_bytes(k, P, H, tsize) / (v["us_avg"] * 1e3)}
                           for k, v in phases.items() if v["launches"]},
    }
    out["diagnostics"] = diag
    if not args.no_positivity:
        print("# positivity-preserving deposit on the same workload", file=sys.stderr, flush=True)
        X0 = cfg["init"](P).astype(np.float32 if fp32 else np.float64)  # the same seeded input as the timed run
        out["positivity"] = positivity_section(pkg, torch, X0, params, ms_per_step)
        del X0
    if fp32 and not args.no_full_run:
        print(f"# the whole {cfg['steps']}-step run with each particle pass", file=sys.stderr, flush=True)
        X0 = cfg["init"](P).astype(np.float32)
        out["full_run"] = full_run_section(pkg, torch, X0, params, cfg["steps"])
        del X0
    if not args.no_other_scheme:
        other = "em" if args.scheme == "strang" else "strang"
        print(f"# the same workload with the {other} push", file=sys.stderr, flush=True)
        X0 = cfg["init"](P).astype(np.float32 if fp32 else np.float64)
        out["other_scheme"] = scheme_section(pkg, torch, X0, params, other)
        del X0
    if args.e1 != "none":
        print(f"# convergence study of Sec. 5.1 ({args.e1})", file=sys.stderr, flush=True)
        out["e1"] = e1_study(args.e1)
    if args.e2 != "none":
        print(f"# SIPF against SIPF-PIC ({args.e2})", file=sys.stderr, flush=True)
        out["e2"] = e2_study(args.e2)
    if args.two_d != "none":
        print(f"# 2-D parabolic-elliptic runs ({args.two_d})", file=sys.stderr, flush=True)
        out["two_d"] = two_d_section(pkg, workloads, np, torch, args.two_d)
    if not args.no_adjoint:
        print("# fwd+adjoint vs fwd on the adjoint workload", file=sys.stderr, flush=True)
        out["adjoint"] = adjoint_ratio(pkg, workloads, np, torch)
    if not args.no_ensemble:
        print("# batched 64-instance ensemble vs one context at a time", file=sys.stderr, flush=True)
        out["ensemble"] = ensemble_throughput(pkg, workloads, np, torch)
    if not args.no_cpu_baseline:
        print("# timing the oracle on the host", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(args.workload, H, min(args.cpu_sample, P), args.cpu_steps,
                                           args.cpu_workers)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
