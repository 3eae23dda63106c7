"""The allocation-free deposit entry point (sipf_deposit_noalloc) against the
allocating one (sipf_dbg_deposit), through the C ABI, on two calls in a row
with the second on fewer particles.  Both run the same kernels, so the grids
agree to the deposit's parity bar: 1e-5 relative L2 in FP32 (float atomics
add the work items' windows in a different order), 1e-12 in FP64.  The mass
M0 is checked on each grid as well."""

import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():  # pragma: no cover - CPU containers
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2512_03452_amd import _lib, workloads  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _deposit(name, prm, X):
    out = torch.full((prm.H, prm.H, prm.H), float("nan"), dtype=X.dtype, device=X.device)
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    lib = _lib.load()
    rc = getattr(lib, name)(ctypes.byref(prm), int(X.shape[0]), ctypes.c_void_p(X.data_ptr()),
                            ctypes.c_void_p(out.data_ptr()), stream)
    assert rc == 0, lib.sipf_last_error().decode()
    torch.cuda.synchronize()
    return out.double().cpu().numpy()


def _rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-5), ("fp64", 1e-12)])
def test_noalloc_deposit_matches_the_allocating_deposit(precision, tol):
    dtype = torch.float32 if precision == "fp32" else torch.float64
    torch.cuda.set_device(0)
    # a clustered blob on H = 64, then a smaller mixed sample on H = 32 (the
    # second call reuses the scratch the first one left behind)
    cases = [(64, 80.0, workloads.blob(300001, 0.1, seed=11)), (32, 60.0, workloads.mix(20011, 0.15, seed=12))]
    for H, M0, Xn in cases:
        say(f"noalloc deposit: {precision} H={H} P={Xn.shape[0]}")
        prm = _lib.default_params(L=2.0, M0=M0, H=H, precision=precision)
        X = torch.as_tensor(Xn).to(device="cuda", dtype=dtype).contiguous()
        got = _deposit("sipf_deposit_noalloc", prm, X)
        ref = _deposit("sipf_dbg_deposit", prm, X)
        assert np.isfinite(got).all()
        err = _rel_l2(got, ref)
        say(f"  rel L2 {err:.3e}  mass {got.sum():.10g} (M0 {M0})")
        assert err < tol
        assert abs(got.sum() - M0) < (1e-5 if precision == "fp32" else 1e-12) * M0


def test_noalloc_deposit_rejects_counts_beyond_its_scratch():
    prm = _lib.default_params(L=2.0, M0=1.0, H=32, precision="fp32")
    X = torch.zeros((2, 3), dtype=torch.float32, device="cuda")
    phi = torch.zeros((32, 32, 32), dtype=torch.float32, device="cuda")
    lib = _lib.load()
    rc = lib.sipf_deposit_noalloc(ctypes.byref(prm), (1 << 19) + 1, ctypes.c_void_p(X.data_ptr()),
                                  ctypes.c_void_p(phi.data_ptr()), ctypes.c_void_p(0))
    assert rc == _lib.SIPF_EINVAL
    assert b"524288" in lib.sipf_last_error()
