"""The C-ABI library loads without a GPU and exports every entry point that
include/*.h declares; host-side validation works without device calls."""
import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b((?:lbm|sg)_[a-z0-9_]+)\s*\(", text):
            names.add(m.group(1))
    return sorted(names)


def test_headers_declare_something():
    assert "lbm_step" in declared_functions()


def test_library_exports_all_declared_symbols():
    from paper_2408_01081_amd import _lib
    L = _lib.load()
    missing = [n for n in declared_functions() if not hasattr(L, n)]
    assert not missing, missing
    bound = {n for n, _, _ in _lib.SIGNATURES}
    assert set(declared_functions()) <= bound | set(getattr(_lib, "EXTRA_BOUND", ()))


def test_host_validation_without_gpu():
    from paper_2408_01081_amd import _lib
    L = _lib.load()
    P = _lib.LbmParams
    ok = P(64, 32, 1.0 / 64, 0.25 / 64 / 2.0, 1.0, 1.0, 1.0, 0, 0, 0)
    assert L.lbm_workspace_bytes(ctypes.byref(ok)) > 2 * 20 * 64 * 32 * 4
    bad_cfl = P(64, 32, 1.0, 1.0, 1.0, 1.0, 1.0, 0, 0, 0)
    assert L.lbm_workspace_bytes(ctypes.byref(bad_cfl)) == 0
    h = ctypes.c_void_p()
    st = L.lbm_create(ctypes.byref(bad_cfl), ctypes.c_void_p(256), 1 << 30, None, ctypes.byref(h))
    assert st == 2 and b"CFL" in L.lbm_last_error()
    neg = P(0, 32, 1.0, 0.1, 1.0, 1.0, 1.0, 0, 0, 0)
    st = L.lbm_create(ctypes.byref(neg), ctypes.c_void_p(256), 1 << 30, None, ctypes.byref(h))
    assert st == 1
    small = L.lbm_create(ctypes.byref(ok), ctypes.c_void_p(256), 16, None, ctypes.byref(h))
    assert small == 4


def test_product_path_has_no_oracle_dependency():
    # the library and its binding never import or load the oracle
    pkg = os.path.join(ROOT, "paper_2408_01081_amd")
    for path in glob.glob(os.path.join(pkg, "**", "*"), recursive=True):
        if path.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
            text = open(path).read()
            assert "oracle" not in text.replace("Oracle", ""), path
