"""The C-ABI library loads without a GPU and exports every entry point that
include/*.h declares; host-side validation works without device calls."""
import ctypes
import math
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


def test_blocked_variants_take_large_row_major_grids():
    # row base addresses of the blocked kernel are formed in 64 bits, so an
    # 8192^2 row-major lattice (row offsets up to 5.4 GB) may use it; in the
    # plane-major layout one row's 20 planes span more than 2^31 bytes at
    # this size, beyond the 32-bit offsets inside a row, and it is refused
    from paper_2408_01081_amd import _lib
    L = _lib.load()
    N = 8192
    for flags, want in ((0, 0), (1, 1)):
        p = _lib.LbmParams(N, N, 1.0 / N, 0.125 / N, 1.0, 1.0, 1.0, 0, 0, flags)
        nb = L.lbm_workspace_bytes(ctypes.byref(p))
        assert nb >= 2 * 80 * N * N
        h = ctypes.c_void_p()
        assert L.lbm_create(ctypes.byref(p), ctypes.c_void_p(256), nb, None, ctypes.byref(h)) == 0
        try:
            assert L.lbm_set_tblock_config(h, 40) == want, L.lbm_last_error()
        finally:
            L.lbm_destroy(h)


def test_zero_shear_modulus_is_admitted_with_the_gradient_initialisation():
    # mu = 0 (c_mu = 0) passes set-up; the stress initialisation, which
    # divides by c_mu, refuses it before any device work; batched instances
    # (initialised from stress) refuse it at planning
    from paper_2408_01081_amd import _lib
    L = _lib.load()
    p = _lib.LbmParams(32, 32, 1.0 / 32, 0.4 / 32, 1.5, 0.0, 1.0, 0, 0, 0)
    nb = L.lbm_workspace_bytes(ctypes.byref(p))
    assert nb > 0
    h = ctypes.c_void_p()
    assert L.lbm_create(ctypes.byref(p), ctypes.c_void_p(256), nb, None, ctypes.byref(h)) == 0
    try:
        kK, km, c = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
        assert L.lbm_lattice_constants(h, ctypes.byref(kK), ctypes.byref(km), ctypes.byref(c)) == 0
        assert km.value == 0.0 and abs(kK.value - math.sqrt(1.5) * 0.4) < 1e-15
        fake = ctypes.c_void_p(4096)
        assert L.lbm_init(h, fake, fake, None) == 1
        assert b"lbm_init_from_gradient" in L.lbm_last_error()
    finally:
        L.lbm_destroy(h)
    arr = (_lib.LbmParams * 2)(_lib.LbmParams(32, 32, 1.0 / 32, 0.4 / 32, 1.0, 0.5, 1.0, 0, 0, 0), p)
    assert L.lbm_batch_workspace_bytes(2, ctypes.cast(arr, ctypes.c_void_p)) == 0
    neg = _lib.LbmParams(32, 32, 1.0 / 32, 0.4 / 32, 1.5, -0.1, 1.0, 0, 0, 0)
    assert L.lbm_workspace_bytes(ctypes.byref(neg)) == 0


def test_split_dirichlet_launch_rule():
    # which blocked launches of a Dirichlet lattice run split (interior with
    # the periodic kernel's code, wall band with the Dirichlet rule): the
    # variant has a split kernel (T, store type, prefetch), the interior
    # strips [1, (nx - T) // (64 - 2T)) are one or more and ny >= 33; modes
    # -1 (the default) and 1 split every such variant, 0 none; periodic
    # lattices never; host logic only (no device work)
    from paper_2408_01081_amd import _lib
    L = _lib.load()
    kernels = {(7, 0, 1), (7, 0, 2), (6, 0, 1), (6, 0, 2), (5, 0, 1)}
    info = []
    for i in range(L.lbm_tblock_config_count()):
        t, sr, nt, pf = (ctypes.c_int32() for _ in range(4))
        assert L.lbm_tblock_config_info(i, ctypes.byref(t), ctypes.byref(sr), ctypes.byref(nt),
                                        ctypes.byref(pf)) == 0
        info.append((t.value, nt.value, pf.value))
    for nx, ny, bc in ((2048, 1024, 1), (130, 33, 1), (130, 32, 1), (100, 40, 1), (64, 64, 1),
                       (2048, 1024, 0)):
        p = _lib.LbmParams(nx, ny, 1.0 / nx, 0.2 / nx, 1.0, 0.5, 1.0, bc, 0, 0)
        nb = L.lbm_workspace_bytes(ctypes.byref(p))
        h = ctypes.c_void_p()
        assert L.lbm_create(ctypes.byref(p), ctypes.c_void_p(256), nb, None, ctypes.byref(h)) == 0
        try:
            for mode in (1, -1, 0):
                assert L.lbm_set_tblock_split(h, mode) == 0
                for i, (T, nt, pf) in enumerate(info):
                    fits = (bc == 1 and (T, nt, pf) in kernels and (nx - T) // (64 - 2 * T) > 1
                            and ny >= 33)
                    want = fits and mode != 0
                    assert L.lbm_tblock_split_active(h, i) == int(want), (nx, ny, bc, mode, i)
            assert L.lbm_set_tblock_split(h, 2) != 0
            assert L.lbm_tblock_split_active(h, len(info)) == -1
        finally:
            L.lbm_destroy(h)


def test_launch_selection_calls_reject_null_arguments():
    # host-side argument checks of the launch-selection calls (no device work)
    from paper_2408_01081_amd import _lib
    L = _lib.load()
    out = ctypes.c_int32(7)
    assert L.lbm_select_for_steps(None, 20, ctypes.byref(out)) == 1
    assert L.lbm_get_tblock_remainder(None, 4, ctypes.byref(out)) == 1
    assert L.lbm_tblock_split_active(None, 0) == -1
    assert out.value == 7
