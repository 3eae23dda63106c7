"""SIPF-PIC time step on AMD Instinct MI355X (gfx950).

The method (stochastic interacting particle-field method with particle-in-cell
acceleration, arXiv:2512.03452, Algorithm 4) runs in the hand-written HIP
kernels of ``libsipf.so``; this package only marshals arguments to its C ABI
(``include/sipf.h``) and uses torch for device memory and streams.
"""

from ._lib import SipfError, load as load_library  # noqa: F401
from . import workloads  # noqa: F401


def __getattr__(name):
    # torch-dependent front end, imported on first use
    if name in ("Sim", "Batch", "Rollout", "autotune", "dbg_philox", "dbg_cells", "dbg_deposit"):
        from . import sim
        return getattr(sim, name)
    raise AttributeError(name)
