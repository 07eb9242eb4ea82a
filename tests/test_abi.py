"""The C ABI of include/spaimg.h, checked on the host (no GPU needed).

The shared library loads, exports every function the header declares (and
no other mg_ symbol), and rejects bad arguments on the host before any GPU
work: invalid sizes, dimensions and coefficients in mg_setup, and a null
handle in every entry point that takes one, each with MG_EINVAL and a
message from mg_last_error.
"""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "spaimg.h")
LIB = os.path.join(ROOT, "paper_2206_05543_amd", "libspaimg.so")
MG_EINVAL = -1


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|void|const char\s*\*)\s*(mg_\w+)\s*\(", text,
                                 flags=re.M)))


def _lib():
    if not os.path.exists(LIB):
        pytest.skip("libspaimg.so is not built")
    L = ctypes.CDLL(LIB)
    L.mg_last_error.restype = ctypes.c_char_p
    return L


def test_header_declares_the_entry_points():
    names = _declared()
    for must in ("mg_setup", "mg_vcycle", "mg_solve", "mg_vcycle_adjoint", "mg_destroy",
                 "mg_last_error"):
        assert must in names
    assert len(names) >= 15


def test_library_exports_exactly_the_declared_symbols():
    L = _lib()
    names = _declared()
    for n in names:
        assert hasattr(L, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True,
                         check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines()
                if ln.split() and ln.split()[-1].startswith("mg_")}
    assert exported == set(names)


def _msg(L):
    return L.mg_last_error().decode()


@pytest.mark.parametrize("N,d,nc,what", [(64, 1, 3, "d must be"), (64, 4, 3, "d must be"),
                                         (2, 2, 3, "power of two"), (48, 2, 3, "power of two"),
                                         (1 << 17, 2, 3, "too large"), (4096, 3, 2, "too large"),
                                         (64, 2, 2, "coefficients"), (64, 3, 3, "coefficients")])
def test_setup_rejects_bad_arguments(N, d, nc, what):
    L = _lib()
    h = ctypes.c_void_p(1)
    c = (ctypes.c_double * nc)(*([0.1] * nc))
    rc = L.mg_setup(N, d, c, nc, ctypes.byref(h))
    assert rc == MG_EINVAL
    assert h.value is None
    assert what in _msg(L)


def test_setup_rejects_non_finite_coefficients():
    L = _lib()
    h = ctypes.c_void_p()
    c = (ctypes.c_double * 3)(0.2, float("nan"), 0.0)
    assert L.mg_setup(64, 2, c, 3, ctypes.byref(h)) == MG_EINVAL
    assert "finite" in _msg(L)
    assert L.mg_setup(64, 2, c, 3, None) == MG_EINVAL


def test_null_handle_is_rejected_everywhere():
    L = _lib()
    vp, i, dbl = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    null = vp()
    p = vp(1)  # never dereferenced: the handle check comes first
    calls = {
        "mg_set_option": (null, i(1), dbl(0.0)),
        "mg_set_coeffs": (null, p, i(3)),
        "mg_vcycle": (null, p, p, null),
        "mg_solve": (null, p, p, dbl(1e-10), null, null),
        "mg_vcycle_adjoint": (null, p, p, i(0), p, p, p, p, null),
        "mg_checkpoint": (null, p, p, i(0), null),
        "mg_sweep": (null, i(0), i(0), i(0), p, p, p, null),
        "mg_sweep_correct": (null, i(0), i(0), p, p, p, p, null),
        "mg_sweep_zero_restrict": (null, i(0), i(0), p, p, p, null),
        "mg_sweep_smooth_restrict": (null, i(0), i(0), p, p, p, p, null),
        "mg_sweep_post_pre_restrict": (null, i(0), i(0), p, p, p, p, p, p, null),
        "mg_coarse_cycle": (null, i(0), i(0), p, p, null),
        "mg_residual_norm": (null, p, p, p, null),
        "mg_get_timing": (null, i(0), i(0), p, p),
        "mg_reset_timing": (null,),
        "mg_num_levels": (null,),
    }
    for name, args in calls.items():
        assert getattr(L, name)(*args) == MG_EINVAL, name
    L.mg_destroy(null)  # a no-op
    # every entry point that can fail is covered here or in mg_setup's test
    assert set(calls) | {"mg_setup", "mg_destroy", "mg_last_error"} == set(_declared())
