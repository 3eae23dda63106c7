"""FP64 CPU oracle for the SIPF-PIC time step.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute anything in this package: only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with
the HIP library (``paper_2512_03452_amd``) and imports nothing from it.

The oracle is a plain, slow, literal reading of the paper
(Hu, Wang, Xin, Zhang, "A fast stochastic interacting particle-field method
for 3D parabolic-parabolic chemotaxis systems", arXiv:2512.03452):

* ``philox``   -- the counter-based normal stream that drives the Brownian
                  increments.  The paper does not name a generator (it only
                  says the increments are i.i.d. Gaussian, Algorithm 4); the
                  generator is Philox4x32-10 from its published definition
                  (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller.
* ``stencil``  -- the particle/grid weights of Sec. 3.1: the trilinear
                  ``F^(2)`` (eq. ``2ord``) and the 32-node fourth-order
                  ``F^(4)`` (eq. ``4ord``), plus their lambda-derivatives for
                  the adjoint.
* ``sipf``     -- P2G (Definition ``particle2grid``, Algorithm 2), G2P
                  (Definition ``grid2particle``, Algorithm 3), the F_H
                  transform convention (Sec. 3.1), the implicit mode update
                  (eq. ``alpha_hat_update``), the Gaussian filter and spectral
                  gradient (Algorithm 4), the split push (Algorithm 4) and the
                  Euler-Maruyama push (eq. ``rho_hat_update``); the direct
                  O(PH^3) SIPF step (Algorithm 1) used as a brute-force check.
* ``sipf2d``   -- the step in two dimensions and the elliptic (eps = 0)
                  field update used by the 2-D experiments of Sec. 5.2.
* ``adjoint``  -- hand-written reverse mode of the SIPF-PIC step with the noise
                  held fixed (pathwise gradient of a final-density loss).
* ``radial``   -- radially symmetric finite-volume reference solution and the
                  truncated quantile discrepancy of the convergence study
                  (Sec. 5.1).
* ``diagnostics`` -- the run-time indicators of Sec. 5 (maximum of the
                  regularised density, high-frequency energy share, R_num,
                  second moment, mass and integral of c_hat).

Every floating-point quantity is float64.  Where the paper is silent or
ambiguous the reading taken is stated at the function that implements it.
"""

from . import philox, stencil, sipf, sipf2d, adjoint, radial, diagnostics  # noqa: F401
from .sipf import Params  # noqa: F401
