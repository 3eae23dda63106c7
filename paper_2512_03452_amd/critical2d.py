"""The two-dimensional parabolic-elliptic experiments of Sec. 5.2 on the GPU.

System (k, eps, mu, chi) = (0, 0, 1, 1) in two dimensions, initial density
uniform on the unit disk with mass M0, periodic square [-L/2, L/2)^2.

Second moment.  For this system in the whole plane the second moment per unit
mass obeys d/dt m2 = 4 mu - chi M0 / (2 pi) (eq. ``second_moment`` divided by
M0), so m2(2) = 17/2 - M0/pi from the unit disk (m2(0) = 1/2).  On the periodic
square the zero-mean Green's function of -Lap is -(1/2 pi) ln|x| + |x|^2/(4 L^2)
plus terms of order |x|^4/L^4, which adds chi M0/L^2 (m2 - |xbar|^2) to the
rate: with a = 4 mu - chi M0/(2 pi) and b = chi M0 / L^2,
    m2(t) = (m2(0) + a/b) e^{b t} - a/b        (xbar = 0),
which tends to the whole-plane law as L grows.  The paper's study (fixed
L/H = 5/512, L = 10, 20, 40, P = 2^20, tau = 5e-4, T = 2) shows the numerical
m2 approaching the whole-plane value as L grows; ``second_moment_study`` runs
those configurations as one batch and reports both predictions next to the
measured m2.

Critical mass.  ``critical_mass_study`` runs M0 = 22 .. 27 (L = 8, H = 2048,
P = 2^22, tau = 5e-4, T = 2) as one batch and records, every ``every`` steps,
the maximum of the regularised density, the high-frequency energy share of
c_hat and m2 (the indicators of Sec. 5.2).
"""

import math
import time

import numpy as np
import torch

from . import workloads
from .sim import Batch

PARAMS_2D = dict(chi=1.0, mu=1.0, eps=0.0, k=0.0, dim=2)


def whole_plane_m2(m0, M0, t, mu=1.0, chi=1.0):
    """m2(t) = m2(0) + (4 mu - chi M0 / (2 pi)) t (eq. second_moment per unit mass)."""
    return m0 + (4.0 * mu - chi * M0 / (2.0 * math.pi)) * t


def periodic_m2(m0, M0, L, t, mu=1.0, chi=1.0):
    """m2(t) on the periodic square to order L^-2 (see the module docstring)."""
    a = 4.0 * mu - chi * M0 / (2.0 * math.pi)
    b = chi * M0 / L ** 2
    return (m0 + a / b) * math.exp(b * t) - a / b


def _run(configs, P, tau, steps, precision, seed, every, log):
    inst = []
    for i, (L, H, M0) in enumerate(configs):
        prm = dict(PARAMS_2D, L=L, H=H, M0=M0, dt=tau, precision=precision, seed=seed, instance=i)
        X0 = workloads.disk(P, 1.0, seed=seed * 1000 + i).astype(np.float32 if precision == "fp32" else np.float64)
        inst.append(dict(params=prm, X0=X0))
    b = Batch(inst)
    series = [[] for _ in configs]
    d0 = b.diagnostics()
    for i, d in enumerate(d0):
        series[i].append(d)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gpu = 0.0
    done = 0
    while done < steps:
        k = min(every, steps - done)
        b.run(k)
        b.sync()
        done += k
        gpu += time.perf_counter() - t0
        for i, d in enumerate(b.diagnostics()):
            series[i].append(d)
        if log:
            log(f"  step {done}")
        t0 = time.perf_counter()
    b.close()
    return series, gpu


def second_moment_study(Ls=(10.0, 20.0, 40.0), M0s=(24.6, 25.0, 25.4), P=1 << 20, tau=5e-4, T=2.0,
                        h=5.0 / 512.0, precision="fp32", seed=0, log=None):
    """m2(T) for every (L, M0) with H = L / h, against both predictions."""
    steps = int(round(T / tau))
    configs = [(L, int(round(L / h)), M0) for L in Ls for M0 in M0s]
    series, secs = _run(configs, P, tau, steps, precision, seed, max(steps // 4, 1), log)
    rows = []
    for (L, H, M0), s in zip(configs, series):
        m0, mT = s[0]["m2"], s[-1]["m2"]
        rows.append(dict(L=L, H=H, M0=M0, m2_0=m0, m2_T=mT, whole_plane=whole_plane_m2(m0, M0, T),
                         periodic=periodic_m2(m0, M0, L, T), paper_line=17.0 / 2.0 - M0 / math.pi))
    return rows, secs


def critical_mass_study(M0s=(22.0, 23.0, 24.0, 25.0, 26.0, 27.0), L=8.0, H=2048, P=1 << 22, tau=5e-4, T=2.0,
                        every=400, precision="fp32", seed=0, log=None):
    """Indicator time series for every M0: lists of (t, rho_max, hf_share, m2)."""
    steps = int(round(T / tau))
    configs = [(L, H, M0) for M0 in M0s]
    series, secs = _run(configs, P, tau, steps, precision, seed, every, log)
    out = {}
    for (L, H, M0), s in zip(configs, series):
        out[M0] = [(d["step"] * tau, d["rho_max"], d["hf_share"], d["m2"]) for d in s]
    return out, secs
