"""Write the radial reference quantiles of the convergence study (Sec. 5.1).

Runs oracle.radial.solve with the parameters of Sec. 5.1 (uniform ball of
radius 1, M0 = 80, mu = chi = 1, eps = 1e-4, k = 0.1, T = 0.02, tau = 1e-5,
L = 8, N = 4e5 finite volumes) and stores the mass-fraction quantiles
q_{j/n}, j = 0 .. 749 (n = 1000), and the 0.999 quantile, in
radial_e1_quantiles.txt next to this script.  Calls only the oracle.

    python tests/golden/make_radial_reference.py [N]
"""

import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import radial  # noqa: E402


def main():
    N = int(sys.argv[1]) if len(sys.argv) > 1 else 400_000
    t0 = time.time()
    g, psi, c = radial.solve(N=N)
    p = radial.truncation(1000)
    q = radial.quantiles_reference(g, psi, p)
    q999 = float(radial.quantiles_reference(g, psi, [0.999])[0])
    out = os.path.join(HERE, "radial_e1_quantiles.txt")
    with open(out, "w") as f:
        f.write("# Radial reference of the convergence study of Sec. 5.1 (uniform ball, M0 = 80,\n")
        f.write("# mu = chi = 1, eps = 1e-4, k = 0.1, T = 0.02, tau = 1e-5, L = 8, R_ball = %.6f,\n" % g.R)
        f.write("# N = %d finite volumes), written by tests/golden/make_radial_reference.py.\n" % N)
        f.write("# q999 %.8f\n" % q999)
        f.write("# mass %.15f\n" % float(np.sum(psi * g.V)))
        f.write("# p q_p\n")
        for pi, qi in zip(p, q):
            f.write("%.3f %.10f\n" % (pi, qi))
    print(f"N={N} q999={q999:.6f} wall {time.time() - t0:.1f} s -> {out}")


if __name__ == "__main__":
    main()
