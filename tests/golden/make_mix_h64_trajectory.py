"""Write the oracle's positions of sampled particles after 100 steps of the
mixed workload at its full size (Algorithm 4 with the Strang splitting).

Workload: box [-1, 1]^3, H = 64, P = 1,000,000 particles, half uniform on the
box and half N(0, 0.15^2 I), M0 = 80, chi = mu = eps = k = 1, tau = 5e-5,
c(x, 0) = 0, Philox seed 0.  The initial positions are the seeded draw of
``workloads.CONFIGS["fp32_mix_h64"]`` rounded to float32 (the precision the
GPU path is given them in) and widened back; the oracle then runs in FP64.
Stored: the ids of 1024 particles drawn with numpy seed 2024, their positions
after 100 steps, and the coefficients alpha_q of c for 0 <= q_x, q_y, q_z <= 3.
Calls only the oracle (and the seeded input generator, loaded from its file).

    python tests/golden/make_mix_h64_trajectory.py     (about 10 minutes)
"""

import importlib.util
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

from oracle import sipf as osipf  # noqa: E402

OUT = os.path.join(HERE, "mix_h64_p1e6_100steps.txt")
STEPS = 100
NSAMPLE = 1024


def _workloads():
    spec = importlib.util.spec_from_file_location(
        "_sipf_workloads", os.path.join(ROOT, "paper_2512_03452_amd", "workloads.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def sample_ids(P):
    return np.sort(np.random.default_rng(2024).choice(P, NSAMPLE, replace=False))


def main():
    wl = _workloads()
    cfg = wl.CONFIGS["fp32_mix_h64"]
    P = cfg["P"]
    kw = {k: v for k, v in cfg["params"].items() if k not in ("precision", "tile", "resort_every", "chunk")}
    prm = osipf.Params(**kw)
    X0 = cfg["init"](P).astype(np.float32).astype(np.float64)
    t0 = time.time()
    X, a = osipf.run(X0, prm, STEPS)
    ids = sample_ids(P)
    with open(OUT, "w") as f:
        f.write("# Oracle (FP64) state after %d steps of the mixed workload at full size:\n" % STEPS)
        f.write("# H = 64, P = %d (half uniform, half N(0, 0.15^2 I)), M0 = 80, chi = mu = eps = k = 1,\n" % P)
        f.write("# tau = 5e-5, Strang splitting, Philox seed 0; written by make_mix_h64_trajectory.py.\n")
        for qx in range(4):
            for qy in range(4):
                for qz in range(4):
                    v = a[qx, qy, qz]
                    f.write("# alpha %d %d %d %.17e %.17e\n" % (qx, qy, qz, v.real, v.imag))
        f.write("# id x y z\n")
        for i in ids:
            f.write("%d %.17e %.17e %.17e\n" % (i, X[i, 0], X[i, 1], X[i, 2]))
    print("wrote", OUT, "in %.0f s" % (time.time() - t0))


if __name__ == "__main__":
    main()
