"""C-ABI surface of libdks on the CPU: the library loads, exports every entry
point include/dks.h declares, and rejects bad arguments with the documented
status codes before touching a device."""
import ctypes as ct
import math
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dks.h")
LIB = os.path.join(ROOT, "paper_1211_1446_amd", "libdks.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dks_[a-z_A-Z0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.fail("libdks.so is not built (run __graft_entry__.build())")
    return ct.CDLL(LIB)


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert {"dks_init_basis", "dks_apply_H", "dks_apply_filter", "dks_lobpcgf_solve",
            "dks_free_basis", "dks_basis_info"} <= set(names)
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (dks_\w+)", out))
    missing = [n for n in names if n not in exported]
    assert not missing, missing
    for n in names:
        getattr(lib, n)


def test_default_options(lib):
    import paper_1211_1446_amd as dk
    o = dk.default_opts()
    assert math.isnan(o.C) and math.isnan(o.Omega)
    assert o.n_init == 3 and o.tol == 1e-8 and o.use_filter == 1 and o.mode == dk.MODE_FP64


def test_host_validation_status_codes(lib):
    EINVAL = -1
    vp = ct.c_void_p
    lib.dks_init_basis.argtypes = [vp, ct.c_int, ct.c_int, ct.POINTER(vp)]
    out = vp()
    assert lib.dks_init_basis(None, 0, 0, ct.byref(out)) == EINVAL
    assert out.value is None
    lib.dks_last_error.restype = ct.c_char_p
    assert lib.dks_last_error()
    lib.dks_basis_info.argtypes = [vp, ct.c_int, vp, vp, vp]
    assert lib.dks_basis_info(None, 0, None, None, None) == EINVAL
    lib.dks_apply_H.argtypes = [vp, ct.c_int, vp, vp, ct.c_int, ct.c_int, vp]
    assert lib.dks_apply_H(None, 0, None, None, 1, 0, None) == EINVAL
    lib.dks_apply_filter.argtypes = [vp, ct.c_int, vp, vp, ct.c_int, ct.c_double, ct.c_double,
                                     ct.c_int, vp]
    assert lib.dks_apply_filter(None, 0, None, None, 1, 0.0, 1.0, 0, None) == EINVAL
    lib.dks_lobpcgf_solve.argtypes = [vp] + [ct.c_int] * 2 + [vp] * 6
    assert lib.dks_lobpcgf_solve(None, 0, 1, None, None, None, None, None, None) == EINVAL
    lib.dks_filter_constants.argtypes = [vp, ct.c_int, vp, vp]
    assert lib.dks_filter_constants(None, 0, None, None) == EINVAL
    lib.dks_num_systems.argtypes = [vp]
    assert lib.dks_num_systems(None) == 0
    lib.dks_free_basis.argtypes = [vp]
    lib.dks_free_basis(None)


def test_product_has_no_oracle_dependency():
    """The product package and its sources never import or name the oracle."""
    pkg = os.path.join(ROOT, "paper_1211_1446_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "sysgen" not in text, f
