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
    ("H", 48), ("H", 4), ("H", 256), ("dt", 0.0), ("dt", float("nan")), ("eps", 0.0), ("mu", -1.0),
    ("chi", float("inf")), ("M0", -2.0), ("L", 0.0), ("p2g_order", 2), ("g2p_order", 4),
    ("scheme", 7), ("precision", 3), ("tile", 3), ("tile", 4096), ("chunk", 17), ("reserved", 1),
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
