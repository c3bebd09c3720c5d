"""The C-ABI library loads and exports every symbol the header declares
(no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

import paper_2602_14454_amd as dwf

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", fn)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(dwf_[a-z0-9_]+)\s*\(", txt))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    if not os.path.exists(dwf.LIB_PATH):
        pytest.skip("libdwf.so not built")
    lib = dwf.load()
    declared = _declared()
    assert len(declared) >= 15
    missing = [n for n in declared if not hasattr(lib, n)]
    assert not missing, missing
    # and the binding marshals every one of them
    assert set(declared) <= set(dwf.SIGNATURES), set(declared) - set(dwf.SIGNATURES)


def test_status_strings_and_params_default():
    if not os.path.exists(dwf.LIB_PATH):
        pytest.skip("libdwf.so not built")
    lib = dwf.load()
    assert lib.dwf_status_string(0) == b"ok"
    assert lib.dwf_status_string(-2) == b"unsupported dimensions"
    p = dwf.default_params()
    assert p.tol == 1e-10 and p.check_every == 1 and p.algo == dwf.ALGO_CGNR


def test_bad_dims_rejected_before_any_device_call():
    if not os.path.exists(dwf.LIB_PATH):
        pytest.skip("libdwf.so not built")
    with pytest.raises(dwf.DwfError) as e:
        dwf.Lattice((4, 3, 4, 4))
    assert e.value.status == -2
