"""Convergence study of Sec. 5.1 on the GPU.

Initial density uniform in the unit ball (M0 = 80) in the periodic box of side
L = 8, mu = chi = 1, eps = 1e-4, k = 0.1, tau = 1e-5, 2000 steps to T = 0.02,
filter H0 = ceil(8 H^(8/13) L^(5/13)).  For every (P, H) the study runs
``nsim`` statistically independent simulations -- independent initial samples
and independent Brownian increments -- and evaluates, per run, the truncated
quantile discrepancy

    E = (1/(m+1)) sum_{j=0..m} |q_{j/n} - qhat_{j/n}|,   n = 1000, m = 749,

between the mass-fraction quantiles q of a radial reference solution (supplied
by the caller) and the empirical quantiles qhat of |X_p| at the final time.
The figure the paper reports is the mean of E over the runs; the slopes of
log2 E against log2 P (at the finest H) and against log2 H (at the largest P)
are the measured convergence orders.

All runs of a study are advanced together as instances of one batch (one
particle launch and one launch per FFT phase and grid size per step), split
into several batches only when the particle budget asks for it.  The empirical
quantiles are computed on the device from the final positions (a sort of the
radii; linear interpolation between order statistics).
"""

import math
import time

import numpy as np
import torch

from . import workloads
from .sim import Batch

N_QUANT = 1000
M_QUANT = math.ceil(3 * N_QUANT / 4) - 1


def probabilities():
    """j / n for j = 0 .. m (the truncated quantile levels)."""
    return np.arange(M_QUANT + 1) / N_QUANT


def empirical_quantiles(X, probs):
    """Quantiles of |X_p| at levels probs (float64 on the device): sorted radii,
    linear interpolation at (P - 1) p."""
    r, _ = torch.sort(torch.linalg.vector_norm(X.to(torch.float64), dim=1))
    P = r.shape[0]
    h = torch.as_tensor(probs, dtype=torch.float64, device=r.device) * (P - 1)
    lo = torch.floor(h).long().clamp_(0, P - 1)
    hi = (lo + 1).clamp_(max=P - 1)
    return r[lo] + (h - lo.to(torch.float64)) * (r[hi] - r[lo])


def discrepancy(q_ref, q_hat):
    return float(np.mean(np.abs(np.asarray(q_ref, dtype=np.float64) - np.asarray(q_hat, dtype=np.float64))))


def slope(x, y):
    """Least-squares slope of log2 y against log2 x."""
    lx, ly = np.log2(np.asarray(x, dtype=np.float64)), np.log2(np.asarray(y, dtype=np.float64))
    return float(np.polyfit(lx, ly, 1)[0])


def grid_bytes(H, precision="fp32"):
    """Device bytes of one 3-D instance's grids: deposit and 3 gradient grids
    (H^3 reals each) and 5 half spectra (B1, alpha, 3 gradient spectra)."""
    t = 4 if precision == "fp32" else 8
    return 4 * H ** 3 * t + 5 * H * H * (H // 2 + 1) * 2 * t


def run_study(configs, nsim, q_ref, steps=workloads.E1_STEPS, seed=0, precision="fp32",
              max_particles=400_000_000, max_grid_bytes=160e9, log=None):
    """Run nsim independent simulations for each (P, H) in configs.

    q_ref: reference quantiles at probabilities() (length m + 1).
    Returns {(P, H): {"E": per-run discrepancies, "mean", "std"}} and the
    elapsed GPU wall time of the runs (seconds, batches' steps only).
    """
    q_ref = np.asarray(q_ref, dtype=np.float64)
    if q_ref.shape != (M_QUANT + 1,):
        raise ValueError(f"q_ref must hold {M_QUANT + 1} quantiles")
    probs = probabilities()
    jobs = [(c, l) for c in range(len(configs)) for l in range(nsim)]
    out = {tuple(c): {"E": np.zeros(nsim)} for c in configs}
    elapsed = 0.0
    dt = np.float32 if precision == "fp32" else np.float64
    start = 0
    while start < len(jobs):
        # largest prefix within the particle and grid-memory budgets and the batch size limit
        end, total, gbytes = start, 0, 0.0
        while end < len(jobs) and end - start < 1024:
            P, H = configs[jobs[end][0]]
            gb = grid_bytes(H, precision)
            if end > start and (total + P > max_particles or gbytes + gb > max_grid_bytes):
                break
            total += P
            gbytes += gb
            end += 1
        if log:
            log(f"sampling {end - start} initial ensembles")
        inst = []
        for j in range(start, end):
            c, l = jobs[j]
            P, H = configs[c]
            prm = dict(workloads.E1_PARAMS, H=H, precision=precision, seed=seed, instance=j)
            X0 = workloads.ball(P, 1.0, seed=seed * 1_000_003 + 1000 * c + l).astype(dt)
            inst.append(dict(params=prm, X0=X0))
        if log:
            log(f"batch of {end - start} instances, {total} particles, {steps} steps")
        b = Batch(inst)
        del inst
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done = 0
        while done < steps:
            chunk = min(500, steps - done)
            b.run(chunk)
            done += chunk
            if log:
                b.sync()
                log(f"  step {done}")
        b.sync()
        elapsed += time.perf_counter() - t0
        for j in range(start, end):
            c, l = jobs[j]
            qh = empirical_quantiles(b.positions(j - start), probs).cpu().numpy()
            out[tuple(configs[c])]["E"][l] = discrepancy(q_ref, qh)
            assert b.step_count(j - start) == steps
        b.close()
        start = end
    for v in out.values():
        v["mean"] = float(np.mean(v["E"]))
        v["std"] = float(np.std(v["E"]))
    return out, elapsed


def _run_single(method, H, P, seed, instance, steps, precision):
    """One run of the study's setup with P particles on grid H: final
    positions and the GPU time of the steps (seconds)."""
    from .sim import Sim
    dt = np.float32 if precision == "fp32" else np.float64
    prm = dict(workloads.E1_PARAMS, H=H, precision=precision, seed=seed, instance=instance)
    if method == "direct":
        # Algorithm 1 as printed: Euler-Maruyama push, unfiltered gradient sum
        prm.update(method="direct", scheme="em", H0=-1.0)
    sim = Sim(workloads.ball(P, 1.0, seed=seed * 1_000_003 + instance).astype(dt), **prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.run(steps)
    sim.sync()
    secs = time.perf_counter() - t0
    X = sim.positions()
    sim.close()
    return X, secs


def cost_error_study(Hs, nsim, q_ref, methods=("pic", "direct"), steps=workloads.E1_STEPS, seed=0,
                     precision="fp32", max_direct_H=64, timing_steps=None, log=None):
    """Sec. 5.1 comparison of SIPF and SIPF-PIC: P = H^3 particles, the
    setup of the convergence study, nsim runs per (method, H): mean truncated
    quantile discrepancy and mean time of one run.  Runs of the direct method
    above max_direct_H are only timed over timing_steps steps and scaled to the
    full run (no error reported)."""
    probs = probabilities()
    out = []
    for method in methods:
        for H in Hs:
            P = H ** 3
            if method == "direct" and H > max_direct_H:
                if not timing_steps:
                    continue
                _, secs = _run_single(method, H, P, seed, 0, timing_steps, precision)
                out.append(dict(method=method, H=H, P=P, runs=0, E=None, seconds_per_run=secs * steps / timing_steps,
                                timed_steps=timing_steps))
                continue
            E, T = [], []
            for l in range(nsim):
                X, secs = _run_single(method, H, P, seed, 1000 * H + l, steps, precision)
                E.append(discrepancy(q_ref, empirical_quantiles(X, probs).cpu().numpy()))
                T.append(secs)
                if log and secs > 2.0:
                    log(f"{method} H={H} run {l}: {secs:.3g} s")
            out.append(dict(method=method, H=H, P=P, runs=nsim, E=float(np.mean(E)), E_std=float(np.std(E)),
                            seconds_per_run=float(np.mean(T)), timed_steps=steps))
            if log:
                log(f"{method} H={H} E={np.mean(E):.4g} s/run={np.mean(T):.3g}")
    return out


def load_reference(path):
    """Read a reference quantile table ("p q_p" lines, '#' comments)."""
    data = np.loadtxt(path)
    if data.shape != (M_QUANT + 1, 2) or not np.allclose(data[:, 0], probabilities()):
        raise ValueError(f"{path}: expected {M_QUANT + 1} rows at probabilities j/{N_QUANT}")
    return data[:, 1]


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="Convergence study of Sec. 5.1 (uniform ball, T = 0.02)")
    ap.add_argument("--reference", required=True, help="reference quantile table (p q_p lines)")
    ap.add_argument("--nsim", type=int, default=30)
    ap.add_argument("--hmax", type=int, default=128)
    ap.add_argument("--pmin-log2", type=int, default=11)
    ap.add_argument("--pmax-log2", type=int, default=20)
    ap.add_argument("--hmin", type=int, default=8)
    ap.add_argument("--steps", type=int, default=workloads.E1_STEPS)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--out", default=None, help="write the results as JSON here")
    a = ap.parse_args(argv)
    q_ref = load_reference(a.reference)
    Ps = [2 ** e for e in range(a.pmin_log2, a.pmax_log2 + 1)]
    Hs = [h for h in (8, 16, 32, 64, 128, 256) if a.hmin <= h <= a.hmax]
    configs = [(P, a.hmax) for P in Ps] + [(Ps[-1], H) for H in Hs if H != a.hmax]
    res, secs = run_study(configs, a.nsim, q_ref, steps=a.steps, seed=a.seed,
                          log=lambda s: print(s, flush=True))
    eP = [res[(P, a.hmax)]["mean"] for P in Ps]
    eH = [res[(Ps[-1], H)]["mean"] for H in Hs]
    report = {
        "nsim": a.nsim, "steps": a.steps, "seconds": secs,
        "particle_steps_per_s": a.nsim * sum(P for P, _ in configs) * a.steps / secs,
        "slope_P": slope(Ps, eP), "slope_H": slope(Hs, eH),
        "E_vs_P": {str(P): [res[(P, a.hmax)]["mean"], res[(P, a.hmax)]["std"]] for P in Ps},
        "E_vs_H": {str(H): [res[(Ps[-1], H)]["mean"], res[(Ps[-1], H)]["std"]] for H in Hs},
    }
    print(json.dumps(report, indent=1), flush=True)
    if a.out:
        with open(a.out, "w") as f:
            json.dump(report, f, indent=1)


if __name__ == "__main__":
    main()
