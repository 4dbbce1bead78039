"""The C ABI library: builds, loads without a GPU, and exports every entry
point that include/skipm.h declares with the signature the binding uses."""
import ctypes
import re
from pathlib import Path

import pytest

import paper_2003_08072_amd as sk

HEADER = Path(__file__).resolve().parents[1] / "include" / "skipm.h"


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\([^;{]*\)\s*;",
                       text, flags=re.M)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("lp_create", "lp_destroy", "ipm_step", "pcg_solve", "sketch_apply",
                     "lp_solve", "sketch_hash"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = sk.load()
    for name in declared_functions():
        assert hasattr(lib, name), name
        assert name in sk.SIGNATURES, name


def test_struct_layouts_match_header():
    # sizes follow the C layout of the header structs on x86-64
    assert ctypes.sizeof(sk.Params) == 6 * 8 + 6 * 4 + 8
    assert ctypes.sizeof(sk.Problem) == 3 * 8 + 2 * 4 + 8 + 8 + 4 * 8
    assert ctypes.sizeof(sk.Result) == 4 * 4 + 6 * 8
    assert ctypes.sizeof(sk.StepInfo) == 11 * 8 + 4 * 4


def test_params_default_values():
    p = sk.default_params()
    assert p.sigma == 0.5 and p.gamma == 0.999 and p.tol_cg == 1e-5
    assert p.s == 1 and p.w == 0 and p.resketch == 1 and p.precision == sk.SKIPM_PREC_FP64


def test_argument_validation_without_device():
    lib = sk.load()
    assert lib.skipm_params_default(None) == sk.SKIPM_EINVAL
    h = ctypes.c_void_p()
    prm = sk.default_params()
    assert lib.lp_create(ctypes.byref(h), None, ctypes.byref(prm), None) == sk.SKIPM_EINVAL
    prob = sk.Problem(m=0, n=10)
    assert lib.lp_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(prm), None) == \
        sk.SKIPM_EINVAL
    prob = sk.Problem(m=5, n=3)
    assert lib.lp_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(prm), None) == \
        sk.SKIPM_EINVAL
    assert b"m <= n" in lib.skipm_last_error()
    assert lib.lp_destroy(None) == sk.SKIPM_OK
    for bad in (dict(sigma=0.9), dict(gamma=1.0), dict(s=3, w=200), dict(w=2)):
        p = sk.default_params(**bad)
        prob = sk.Problem(m=10, n=100, format=sk.SKIPM_DENSE, a_dtype=sk.SKIPM_F64,
                          a_vals=1, b=1, c=1)
        assert lib.lp_create(ctypes.byref(h), ctypes.byref(prob), ctypes.byref(p), None) == \
            sk.SKIPM_EINVAL, bad
    assert lib.sketch_hash(0, 0, 3, 10, 10, None, None, None) == sk.SKIPM_EINVAL
