"""Host-side checks of the C-ABI library (no GPU needed): the shared library
loads, exports every function declared in include/sd.h, and its host FP64
construction of the triangle weight bases (App. C.3) agrees with the oracle's
independent pseudoinverse solution."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sd.h")
LIB = os.path.join(ROOT, "paper_2108_10480_amd", "libsd.so")


def _declared():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sd_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def libsd():
    if not os.path.exists(LIB):
        pytest.fail("libsd.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_library_exports_every_declared_symbol(libsd):
    names = _declared()
    assert "sd_build_bvh" in names and "sd_eval_grad" in names
    missing = [n for n in names if not hasattr(libsd, n)]
    assert not missing, missing


def test_python_binding_names_match_header():
    from paper_2108_10480_amd import api, surrogate
    declared = set(_declared())
    for n in declared:
        if n in ("sd_last_error", "sd_free_scene", "sd_scene_info_get"):
            continue
        if n.startswith("sd_surrogate_"):
            meth = {"create": "__init__"}.get(n[len("sd_surrogate_"):], n[len("sd_surrogate_"):])
            assert hasattr(surrogate.Surrogate, meth), n
        else:
            assert hasattr(api, n) or hasattr(surrogate, n), n
        assert n in api.EXPORTED, n


def test_triangle_weight_basis_matches_oracle(libsd, oracle_mod):
    O = oracle_mod
    B = np.empty((3, 64), np.float64)
    libsd.sd_triangle_weight_basis.restype = ctypes.c_int
    assert libsd.sd_triangle_weight_basis(ctypes.c_void_p(B.ctypes.data)) == 0
    B = B.reshape(3, 8, 8)
    for (v, e) in [(6, 2), (5, 2), (3, 3), (2, 1), (9, 4)]:
        lib_c = B[0] / v + B[1] / e + B[2] * (v - 1) / v
        ref = O.triangle_weight_coeffs(v, e)
        assert np.abs(lib_c - ref).max() < 1e-9 * max(1, np.abs(ref).max()), (v, e)
    # isolated triangle: (1, 1, 1) gives the constant 1 exactly up to rounding
    one = B.sum(0)
    ref = np.zeros((8, 8)); ref[0, 0] = 1
    assert np.abs(one - ref).max() < 1e-9


def test_null_and_bad_arguments_rejected_on_host(libsd):
    """Argument validation happens on the host before any device work."""
    libsd.sd_build_bvh.restype = ctypes.c_int
    libsd.sd_last_error.restype = ctypes.c_char_p
    out = ctypes.c_void_p()
    # negative size
    rc = libsd.sd_build_bvh(None, ctypes.c_int64(-1), None, ctypes.c_int64(0), None, ctypes.c_int64(0),
                            None, ctypes.c_int64(0), ctypes.c_uint32(0), None, ctypes.byref(out))
    assert rc == -1 and b"negative" in libsd.sd_last_error()
    # null vertex array with triangles
    rc = libsd.sd_build_bvh(None, ctypes.c_int64(3), None, ctypes.c_int64(0), None, ctypes.c_int64(0),
                            None, ctypes.c_int64(1), ctypes.c_uint32(0), None, ctypes.byref(out))
    assert rc == -1
    # eval on a null scene
    libsd.sd_eval.restype = ctypes.c_int

    class P(ctypes.Structure):
        _fields_ = [("alpha", ctypes.c_float), ("alpha_u", ctypes.c_float),
                    ("beta", ctypes.c_float), ("flags", ctypes.c_uint32)]
    p = P(10.0, 0.0, 0.5, 0)
    assert libsd.sd_eval(None, None, ctypes.c_int64(0), ctypes.byref(p), None, None) == -1
    assert libsd.sd_rigid_adjoint(None, ctypes.c_int64(-1), None, ctypes.c_int64(1), None, None,
                                  None, None, None, None) == -1


def test_memory_budget_entry_points_on_host(libsd):
    """sd_set_memory_budget / sd_memory_in_use touch no device: the count
    starts at zero in a process that has allocated nothing, a null output is
    rejected, and any budget (or none) is accepted."""
    libsd.sd_memory_in_use.restype = ctypes.c_int
    libsd.sd_set_memory_budget.restype = ctypes.c_int
    n = ctypes.c_int64(-7)
    assert libsd.sd_memory_in_use(ctypes.byref(n)) == 0 and n.value == 0
    assert libsd.sd_memory_in_use(None) == -1
    for b in (0, 1 << 30, -1):
        assert libsd.sd_set_memory_budget(ctypes.c_int64(b)) == 0
