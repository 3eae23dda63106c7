"""Host-only checks of the C ABI (no GPU needed, no compute calls)."""

import ctypes
import os
import re
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sipf.h")


def _lib():
    from paper_2512_03452_amd import _lib
    return _lib


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sipf_[a-z_0-9]+)\s*\(", src)))


def test_library_loads_and_exports_every_declared_symbol():
    lib = _lib().load()
    names = _declared_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(lib, n), n
    # every declared function has a binding signature
    assert set(names) <= set(_lib().SIGNATURES)


def test_params_struct_layout_matches_c(tmp_path):
    cc = shutil.which("gcc")
    if cc is None:
        pytest.skip("gcc not available")
    L = _lib()
    fields = [f for f, _ in L.SipfParams._fields_]
    prog = "#include <stdio.h>\n#include <stddef.h>\n#include \"sipf.h\"\nint main(void){\n"
    prog += 'printf("%zu\\n", sizeof(sipf_params));\n'
    for f in fields:
        prog += f'printf("%zu\\n", offsetof(sipf_params, {f}));\n'
    prog += "return 0;}\n"
    src = tmp_path / "layout.c"
    src.write_text(prog)
    exe = tmp_path / "layout"
    subprocess.run([cc, "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    vals = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert vals[0] == ctypes.sizeof(L.SipfParams)
    for f, off in zip(fields, vals[1:]):
        assert getattr(L.SipfParams, f).offset == off, f


def test_defaults():
    p = _lib().default_params()
    assert (p.L, p.H, p.p2g_order, p.g2p_order, p.scheme, p.precision) == (2.0, 64, 4, 2, 0, 0)


@pytest.mark.parametrize("field,value", [
    ("H", 48), ("H", 4), ("H", 512), ("dt", 0.0), ("dt", float("nan")), ("eps", -1.0), ("mu", -1.0),
    ("chi", float("inf")), ("M0", -2.0), ("L", 0.0), ("p2g_order", 2), ("g2p_order", 4),
    ("scheme", 7), ("precision", 3), ("tile", 3), ("tile", 4096), ("chunk", 17), ("dim", 1), ("dim", 4), ("propagator", 2), ("method", 2),
    ("positivity", 2), ("positivity", -1), ("particle_pass", 3), ("particle_pass", -1),
])
def test_invalid_parameters_rejected_before_device(field, value):
    L = _lib()
    lib = L.load()
    p = L.default_params(**{field: value})
    X = np.zeros((4, 3), np.float32)
    h = ctypes.c_void_p()
    rc = lib.sipf_init(ctypes.byref(p), 4, X.ctypes.data_as(ctypes.c_void_p), 0, None, 0, None, ctypes.byref(h))
    assert rc == L.SIPF_EINVAL
    assert h.value is None
    assert lib.sipf_last_error()


@pytest.mark.parametrize("H,tile", [(4, 0), (8192, 0), (48, 0), (1024, 8), (64, 3)])
def test_invalid_2d_parameters_rejected(H, tile):
    L = _lib()
    lib = L.load()
    p = L.default_params(dim=2, H=H, tile=tile)
    X = np.zeros((4, 2), np.float32)
    h = ctypes.c_void_p()
    rc = lib.sipf_init(ctypes.byref(p), 4, X.ctypes.data_as(ctypes.c_void_p), 0, None, 0, None, ctypes.byref(h))
    assert rc == L.SIPF_EINVAL
    assert h.value is None


def test_exponential_propagator_needs_positive_eps():
    L = _lib()
    lib = L.load()
    p = L.default_params(eps=0.0, propagator="exp")
    X = np.zeros((4, 3), np.float32)
    h = ctypes.c_void_p()
    rc = lib.sipf_init(ctypes.byref(p), 4, X.ctypes.data_as(ctypes.c_void_p), 0, None, 0, None, ctypes.byref(h))
    assert rc == L.SIPF_EINVAL and h.value is None


@pytest.mark.parametrize("kw", [
    dict(H=24), dict(H=90, precision="fp64"), dict(H=12, tile=13), dict(H=90, tile=5), dict(H=46, tile=2),
    dict(H=22, tile=-11),
])
def test_mixed_radix_parameters_rejected(kw):
    """3-D grids take 12, 22, 46 and 90 besides powers of two; a tile then
    leaves at most 16 tiles per axis, the last one possibly partial."""
    L = _lib()
    p = L.default_params(**kw)
    h = ctypes.c_void_p()
    X = np.zeros((4, 3), np.float64 if kw.get("precision") == "fp64" else np.float32)
    rc = L.load().sipf_init(ctypes.byref(p), 4, X.ctypes.data_as(ctypes.c_void_p), 0, None, 0, None, ctypes.byref(h))
    assert rc == L.SIPF_EINVAL and h.value is None


@pytest.mark.parametrize("kw", [dict(positivity=1, dim=2, H=64), dict(positivity=1, method="direct", H=8)])
def test_positivity_option_is_for_the_3d_pic_step(kw):
    L = _lib()
    p = L.default_params(**kw)
    h = ctypes.c_void_p()
    X = np.zeros((4, p.dim if p.dim else 3), np.float32)
    rc = L.load().sipf_init(ctypes.byref(p), 4, X.ctypes.data_as(ctypes.c_void_p), 0, None, 0, None, ctypes.byref(h))
    assert rc == L.SIPF_EINVAL and h.value is None
    lib = L.load()
    sw, r = ctypes.c_int64(), ctypes.c_int32()
    assert lib.sipf_positivity_stats(None, ctypes.byref(sw), ctypes.byref(r)) == L.SIPF_EINVAL


@pytest.mark.parametrize("kw", [dict(H=256, precision="fp64"), dict(H=256, method="direct"), dict(H=512)])
def test_h256_limits(kw):
    """H = 256 runs SIPF-PIC in FP32 only; the direct method stops at 128."""
    L = _lib()
    p = L.default_params(**kw)
    h = ctypes.c_void_p()
    X = np.zeros((4, 3), np.float64 if kw.get("precision") == "fp64" else np.float32)
    rc = L.load().sipf_init(ctypes.byref(p), 4, X.ctypes.data_as(ctypes.c_void_p), 0, None, 0, None, ctypes.byref(h))
    assert rc == L.SIPF_EINVAL and h.value is None


def test_fp64_h128_rejected():
    L = _lib()
    p = L.default_params(H=128, precision="fp64")
    h = ctypes.c_void_p()
    X = np.zeros((4, 3))
    rc = L.load().sipf_init(ctypes.byref(p), 4, X.ctypes.data_as(ctypes.c_void_p), 0, None, 0, None, ctypes.byref(h))
    assert rc == L.SIPF_EINVAL


def test_bad_particle_count_and_null_pointers():
    L = _lib()
    lib = L.load()
    p = L.default_params()
    h = ctypes.c_void_p()
    X = np.zeros((4, 3), np.float32)
    assert lib.sipf_init(ctypes.byref(p), 0, X.ctypes.data_as(ctypes.c_void_p), 0, None, 0, None, ctypes.byref(h)) == L.SIPF_EINVAL
    assert lib.sipf_init(ctypes.byref(p), 4, None, 0, None, 0, None, ctypes.byref(h)) == L.SIPF_EINVAL
    assert lib.sipf_init(None, 4, X.ctypes.data_as(ctypes.c_void_p), 0, None, 0, None, ctypes.byref(h)) == L.SIPF_EINVAL
    assert lib.sipf_step(None) == L.SIPF_EINVAL
    assert lib.sipf_run(None, 3) == L.SIPF_EINVAL
    assert lib.sipf_prepare_run(None, 3) == L.SIPF_EINVAL
    assert lib.sipf_destroy(None) == L.SIPF_OK


def test_non_finite_host_positions_rejected_before_device():
    L = _lib()
    lib = L.load()
    p = L.default_params()
    X = np.zeros((5, 3), np.float32)
    X[3, 1] = np.nan
    h = ctypes.c_void_p()
    rc = lib.sipf_init(ctypes.byref(p), 5, X.ctypes.data_as(ctypes.c_void_p), 0, None, 0, None, ctypes.byref(h))
    assert rc == L.SIPF_ENUMERIC


def test_load_of_missing_snapshot_is_eio(tmp_path):
    L = _lib()
    h = ctypes.c_void_p()
    rc = L.load().sipf_load(str(tmp_path / "nope.bin").encode(), None, ctypes.byref(h))
    assert rc == L.SIPF_EIO
    assert h.value is None


def _snap_header_type():
    L = _lib()

    class Hdr(ctypes.Structure):
        _fields_ = [("magic", ctypes.c_char * 8), ("version", ctypes.c_uint32), ("tsize", ctypes.c_uint32),
                    ("prm", L.SipfParams), ("P", ctypes.c_int64), ("n", ctypes.c_int64)]
    return Hdr


@pytest.mark.parametrize("damage", ["magic", "version", "truncated", "oversized", "tsize"])
def test_load_of_corrupt_snapshot_is_eio(tmp_path, damage):
    L = _lib()
    Hdr = _snap_header_type()
    p = L.default_params(H=8)
    P = 10
    h = Hdr(b"SIPFSNAP", 4, 4, p, P, 3)
    payload = bytes(P * 3 * 4 + 8 * 8 * 5 * 2 * 4)
    if damage == "magic":
        h.magic = b"SIPFSNAQ"
    elif damage == "version":
        h.version = 3  # the layout before the particle_pass field
    elif damage == "tsize":
        h.tsize = 8
    elif damage == "truncated":
        payload = payload[:-1]
    elif damage == "oversized":
        payload = payload + b"\0"
    f = tmp_path / "snap.bin"
    f.write_bytes(bytes(h) + payload)
    out = ctypes.c_void_p()
    rc = L.load().sipf_load(str(f).encode(), None, ctypes.byref(out))
    assert rc == L.SIPF_EIO
    assert out.value is None


def _batch_init(L, prms, Ps, Xs, on_device=0):
    n = len(prms)
    arr = (L.SipfParams * max(n, 1))()
    for i, p in enumerate(prms):
        arr[i] = p
    P = (ctypes.c_int64 * max(n, 1))(*Ps)
    ptrs = (ctypes.c_void_p * max(n, 1))(*[X.ctypes.data for X in Xs])
    h = ctypes.c_void_p()
    rc = L.load().sipf_batch_init(n, arr, P, ptrs, on_device, None, ctypes.byref(h))
    return rc, h


@pytest.mark.parametrize("case", ["empty", "mixed_precision", "mixed_scheme", "bad_instance", "bad_count",
                                  "non_finite", "mixed_positivity", "mixed_pass"])
def test_batch_init_rejects_before_device(case):
    L = _lib()
    a = L.default_params(H=16)
    b = L.default_params(H=32, chi=2.0, instance=1)
    Xa = np.zeros((7, 3), np.float32)
    Xb = np.zeros((9, 3), np.float32)
    prms, Ps, Xs = [a, b], [7, 9], [Xa, Xb]
    want = L.SIPF_EINVAL
    if case == "empty":
        prms, Ps, Xs = [], [], []
    elif case == "mixed_precision":
        prms[1] = L.default_params(H=32, precision="fp64")
    elif case == "mixed_scheme":
        prms[1] = L.default_params(H=32, scheme="em")
    elif case == "bad_instance":
        prms[1] = L.default_params(H=48)
    elif case == "bad_count":
        Ps[0] = 0
    elif case == "mixed_positivity":
        prms[1] = L.default_params(H=32, positivity=1)
    elif case == "mixed_pass":
        prms[1] = L.default_params(H=32, particle_pass="two_phase")
    elif case == "non_finite":
        Xb[4, 2] = np.inf
        want = L.SIPF_ENUMERIC
    rc, h = _batch_init(L, prms, Ps, Xs)
    assert rc == want
    assert h.value is None
    assert L.load().sipf_last_error()


def test_batch_and_tuning_null_handles():
    L = _lib()
    lib = L.load()
    n = ctypes.c_int64()
    assert lib.sipf_batch_run(None, 1) == L.SIPF_EINVAL
    assert lib.sipf_batch_prepare_run(None, 1) == L.SIPF_EINVAL
    assert lib.sipf_batch_sync(None) == L.SIPF_EINVAL
    assert lib.sipf_batch_get_step(None, 0, ctypes.byref(n)) == L.SIPF_EINVAL
    assert lib.sipf_batch_get_positions(None, 0, None, 1) == L.SIPF_EINVAL
    assert lib.sipf_batch_use_graphs(None, 1) == L.SIPF_EINVAL
    assert lib.sipf_batch_destroy(None) == L.SIPF_OK
    assert lib.sipf_use_graphs(None, 0) == L.SIPF_EINVAL
    assert lib.sipf_get_params(None, None, None) == L.SIPF_EINVAL
    d = L.SipfDiag()
    assert lib.sipf_diagnostics(None, ctypes.byref(d)) == L.SIPF_EINVAL
    assert lib.sipf_batch_diagnostics(None, ctypes.byref(d)) == L.SIPF_EINVAL
    assert ctypes.sizeof(L.SipfDiag) == 7 * 8
    p = L.default_params(H=24)
    best = L.SipfParams()
    ms = ctypes.c_double()
    X = np.zeros((4, 3), np.float32)
    assert lib.sipf_autotune(ctypes.byref(p), 4, X.ctypes.data_as(ctypes.c_void_p), 0, 4, None, ctypes.byref(best),
                             ctypes.byref(ms)) == L.SIPF_EINVAL
