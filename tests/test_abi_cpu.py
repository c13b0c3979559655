"""Host-side checks of the C ABI (no device work): every function declared
in include/mde.h is exported by libmde.so, and the argument validation of
the setup calls behaves as documented."""
import ctypes as C
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "mde.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mde_[a-z_0-9]+)\s*\(", txt)))


def _lib():
    from paper_1106_2456_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmde.so not built")
    return _lib


def test_every_declared_symbol_is_exported():
    L = _lib()
    lib = L.lib()
    decl = _declared()
    assert len(decl) >= 30
    for name in decl:
        assert hasattr(lib, name), name
    assert set(decl) == set(L.exported_symbols())


def test_build_targets_gfx950_only():
    import subprocess
    so = os.path.join(ROOT, "paper_1106_2456_amd", "libmde.so")
    if not os.path.exists(so):
        pytest.skip("not built")
    out = subprocess.run(["/opt/rocm/llvm/bin/llvm-readelf", "-S", so], capture_output=True, text=True).stdout
    assert ".hip_fatbin" in out


def _desc(L, n=(2, 2), no=(5, 5), W=4, max_order=4, prec=0):
    d = L.MdeDesc()
    d.n_elec[0], d.n_elec[1] = n
    d.n_orb[0], d.n_orb[1] = no
    d.max_walkers = W
    d.max_order = max_order
    d.refresh_every = 4
    d.precision = prec
    return d


def _arr(x, t=np.int32):
    a = np.ascontiguousarray(x, t)
    return a, a.ctypes.data


def test_validation_of_setup_calls():
    L = _lib()
    lib = L.lib()
    h = C.c_void_p()
    bad = _desc(L, n=(0, 2))
    assert lib.mde_create(C.byref(bad), None, C.byref(h)) == L.MDE_UNSUPPORTED
    bad = _desc(L, max_order=9)
    assert lib.mde_create(C.byref(bad), None, C.byref(h)) == L.MDE_INVALID
    d = _desc(L)
    assert lib.mde_create(C.byref(d), None, C.byref(h)) == 0
    try:
        # reference must come first and be empty
        off, po = _arr([0, 1]); hs, ph = _arr([0]); ps, pp = _arr([2])
        assert lib.mde_set_excitations(h, 0, 1, po, ph, pp) == L.MDE_INVALID
        # particle out of range
        off, po = _arr([0, 0, 1]); hs, ph = _arr([0]); ps, pp = _arr([7])
        assert lib.mde_set_excitations(h, 0, 2, po, ph, pp) == L.MDE_INVALID
        assert b"out of range" in lib.mde_error_string(h)
        # hole used as particle
        ps, pp = _arr([1])
        assert lib.mde_set_excitations(h, 0, 2, po, ph, pp) == L.MDE_INVALID
        # duplicate excitations
        off, po = _arr([0, 0, 1, 2]); hs, ph = _arr([0, 0]); ps, pp = _arr([2, 2])
        assert lib.mde_set_excitations(h, 0, 3, po, ph, pp) == L.MDE_INVALID
        # non-ascending holes
        off, po = _arr([0, 0, 2]); hs, ph = _arr([1, 0]); ps, pp = _arr([2, 3])
        assert lib.mde_set_excitations(h, 0, 2, po, ph, pp) == L.MDE_INVALID
        # CI before excitations
        c, pc = _arr([1.0], np.float64); i0, pi0 = _arr([0])
        assert lib.mde_set_ci(h, 1, pc, pi0, pi0) == L.MDE_STATE
        # a valid expansion
        off, po = _arr([0, 0, 1, 3]); hs, ph = _arr([1, 0, 1]); ps, pp = _arr([2, 3, 4])
        for s in (0, 1):
            assert lib.mde_set_excitations(h, s, 3, po, ph, pp) == 0
        c, pc = _arr([1.0, 0.5, -0.2], np.float64)
        u, pu = _arr([0, 1, 2]); dd, pd = _arr([0, 2, 5])
        assert lib.mde_set_ci(h, 3, pc, pu, pd) == L.MDE_INVALID
        dd, pd = _arr([0, 2, 1])
        assert lib.mde_set_ci(h, 3, pc, pu, pd) == 0
        b = C.c_size_t()
        assert lib.mde_workspace_bytes(h, 5, C.byref(b)) == L.MDE_INVALID
        assert lib.mde_workspace_bytes(h, 4, C.byref(b)) == 0
        assert b.value > 0
        # evaluation before binding is a state error
        assert lib.mde_init(h, 1, None, None, None, None, None) == L.MDE_STATE
        assert lib.mde_accept(h, 0, None) == L.MDE_STATE
        assert lib.mde_backward(h, None, None, None, None, None) == L.MDE_STATE
        tile, ie, thr = C.c_int32(), C.c_int32(), C.c_int32()
        assert lib.mde_get_plan(h, 0, C.byref(tile), C.byref(ie), C.byref(thr)) == 0
        assert tile.value in (1, 2, 4, 8, 16, 32, 64) and thr.value % 64 == 0
        assert lib.mde_set_plan(h, 0, 3, 0, 0) == L.MDE_INVALID
        assert lib.mde_set_plan(h, 0, 4, 128, 256) == 0
    finally:
        lib.mde_destroy(h)
