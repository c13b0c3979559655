"""Pins for the oracle's LU determinant and inverse: brute force (Leibniz),
a library routine (numpy slogdet), closed forms (triangular, permutation),
and the singular case."""
import itertools

import numpy as np
import pytest

import oracle
from tests._util import leibniz, perm_sign


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_lu_matches_leibniz(n):
    rng = np.random.default_rng(100 + n)
    for _ in range(5):
        M = rng.standard_normal((n, n))
        s, l = oracle.slogdet(M)
        ref = leibniz(M)
        assert s == np.sign(ref)
        assert abs(s * np.exp(l) - ref) <= 1e-12 * max(1.0, abs(ref)) * 10


@pytest.mark.parametrize("n", [7, 16, 32, 64, 100])
def test_lu_matches_numpy(n):
    rng = np.random.default_rng(200 + n)
    M = rng.standard_normal((n, n))
    s, l = oracle.slogdet(M)
    s2, l2 = np.linalg.slogdet(M)
    assert s == s2
    assert abs(l - l2) < 1e-11 * max(1.0, abs(l2))


def test_triangular_and_permutation_closed_forms():
    rng = np.random.default_rng(3)
    U = np.triu(rng.standard_normal((6, 6))) + 3 * np.eye(6)
    s, l = oracle.slogdet(U)
    d = np.prod(np.diag(U))
    assert s == np.sign(d) and abs(l - np.log(abs(d))) < 1e-13
    L = U.T.copy()
    s, l = oracle.slogdet(L)
    assert s == np.sign(d) and abs(l - np.log(abs(d))) < 1e-13
    for p in itertools.permutations(range(4)):
        P = np.eye(4)[list(p)]
        s, l = oracle.slogdet(P)
        assert s == perm_sign(p) and abs(l) < 1e-15


def test_singular_gives_zero_sign():
    M = np.array([[1.0, 2.0, 3.0], [2.0, 4.0, 6.0], [0.0, 1.0, 5.0]])
    s, l = oracle.slogdet(M)
    assert s == 0.0 and l == -np.inf


def test_inverse():
    rng = np.random.default_rng(5)
    for n in (1, 2, 5, 17, 64):
        M = rng.standard_normal((n, n))
        X = oracle.inverse(M)
        assert np.abs(X @ M - np.eye(n)).max() < 1e-10 * np.linalg.cond(M)
