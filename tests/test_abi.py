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


def test_params_struct_matches_header():
    """The ctypes mirror of dwf_solve_params has the size the library fills."""
    if not os.path.exists(dwf.LIB_PATH):
        pytest.skip("libdwf.so not built")
    p = dwf.default_params()
    assert p.autotune == 1 and p.use_graph == 1 and p.restart == 16


def test_tune_cache_round_trip(tmp_path, monkeypatch):
    """Tile-tuner cache: an entry written to the file named by DWF_TUNE_CACHE
    is read back after the in-memory copy is dropped (host code only)."""
    if not os.path.exists(dwf.LIB_PATH):
        pytest.skip("libdwf.so not built")
    path = tmp_path / "tune.txt"
    monkeypatch.setenv("DWF_TUNE_CACHE", str(path))
    dwf.tune_cache_reload()
    key = "gfx950|p1|16x16x16x32s12r12"
    assert dwf.tune_cache_get(key) is None
    dwf.tune_cache_put(key, 4, 1, 0.8125)
    dwf.tune_cache_put("gfx950|p2|8x8x8x8s8r1", 1, 0, 0.03)
    lines = path.read_text().splitlines()
    assert f"{key} 4 1 0.8125" in lines and len(lines) == 2
    dwf.tune_cache_reload()
    assert dwf.tune_cache_get(key) == (4, 1, 0.8125)
    # a corrupt line is ignored, the rest is kept
    path.write_text(path.read_text() + "garbage line here\n" + "k 0 0 1.0\n")
    dwf.tune_cache_reload()
    assert dwf.tune_cache_get(key) == (4, 1, 0.8125) and dwf.tune_cache_get("k") is None
    with pytest.raises(dwf.DwfError):
        dwf.tune_cache_put("bad key", 1, 0, 1.0)
    with pytest.raises(dwf.DwfError):
        dwf.tune_cache_put("k2", 0, 0, 1.0)
    monkeypatch.setenv("DWF_TUNE_CACHE", "off")
    dwf.tune_cache_reload()
    assert dwf.tune_cache_get(key) is None
