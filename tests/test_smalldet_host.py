"""Host build of the small-determinant routines the determinant kernel uses
(the same header compiled with g++): det S and the bordered-form vector
y_j = det(S with column j replaced by c) against numpy determinants, for the
written-out orders 1..4, the elimination path 5..8 and the run form (prefix
cofactors applied to the last column)."""
import ctypes as C
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "..", "paper_1106_2456_amd", "csrc", "host_test", "smalldet_host.cpp")


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("sd") / "libsd.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", SRC, "-o", out], check=True)
    L = C.CDLL(out)
    P = C.POINTER(C.c_double)
    for name in ("mde_host_small_det", "mde_host_small_det_generic", "mde_host_run_form"):
        f = getattr(L, name)
        f.argtypes = [C.c_int, P, P, P]
        f.restype = C.c_double
    return L


def _call(f, S, c):
    k = S.shape[0]
    S = np.ascontiguousarray(S, np.float64)
    c = np.ascontiguousarray(c, np.float64)
    y = np.zeros(k)
    P = C.POINTER(C.c_double)
    d = f(k, S.ctypes.data_as(P), c.ctypes.data_as(P), y.ctypes.data_as(P))
    return d, y


def _ref(S, c):
    k = S.shape[0]
    y = np.empty(k)
    for j in range(k):
        M = S.copy()
        M[:, j] = c
        y[j] = np.linalg.det(M)
    return np.linalg.det(S), y


@pytest.mark.parametrize("k", range(1, 9))
def test_small_det_and_bordered_vector(lib, k):
    rng = np.random.default_rng(100 + k)
    for _ in range(20):
        S = rng.normal(size=(k, k))
        c = rng.normal(size=k)
        d_ref, y_ref = _ref(S, c)
        scale = np.prod(np.abs(S).sum(1))   # bound on |det| of S and its column swaps
        for f in (lib.mde_host_small_det, lib.mde_host_small_det_generic):
            d, y = _call(f, S, c)
            assert abs(d - d_ref) <= 1e-13 * scale
            assert np.abs(y - y_ref).max() <= 1e-13 * scale * (1 + np.abs(c).max())


@pytest.mark.parametrize("k", [1, 2, 3, 4])
def test_run_form(lib, k):
    rng = np.random.default_rng(200 + k)
    for _ in range(50):
        S = rng.normal(size=(k, k))
        c = rng.normal(size=k)
        d_ref, y_ref = _ref(S, c)
        d, y = _call(lib.mde_host_run_form, S, c)
        scale = np.prod(np.abs(S).sum(1)) * (1 + np.abs(c).max())
        assert abs(d - d_ref) <= 1e-13 * scale
        assert np.abs(y - y_ref).max() <= 1e-13 * scale


def test_run_form_singular_and_structured(lib):
    # rank-deficient S: det 0 exactly representable, y still finite and right
    S = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [0.5, -1.0, 2.0]])
    c = np.array([1.0, -2.0, 0.25])
    d, y = _call(lib.mde_host_run_form, S, c)
    d_ref, y_ref = _ref(S, c)
    assert abs(d) <= 1e-14 and np.allclose(y, y_ref, atol=1e-13)
    # identity: det 1, y = c
    for k in (1, 2, 3, 4):
        d, y = _call(lib.mde_host_run_form, np.eye(k), np.arange(1.0, k + 1))
        assert d == 1.0 and np.array_equal(y, np.arange(1.0, k + 1))
