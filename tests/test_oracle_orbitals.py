"""Pins of the oracle's orbital evaluator against facts that do not come
from its own code: special points of one Gaussian (at its centre, on an
axis), a permutation of the MO matrix that a transposed contraction would
undo the wrong way, linearity in the MO coefficients, invariance and
covariance under a rotation of the whole system, and a numpy closed form
of the same orbitals."""
import numpy as np

import oracle
import synth


def _system(centres, expo, mo):
    nb = len(expo)
    n_orb = mo.shape[0]
    ex = synth.Excitations(np.zeros(2, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32))
    return synth.System((1, 1), (n_orb, n_orb), np.zeros((1, 3)), np.asarray(centres, float),
                        np.asarray(expo, float), np.asarray(mo, float), (ex, ex),
                        np.ones(1), np.zeros(1, np.int32), np.zeros(1, np.int32))


def test_single_gaussian_special_points():
    a = 0.7
    c = np.array([[0.3, -1.1, 2.0]])
    s = _system(c, [a], np.ones((1, 1)))
    # at the centre: value 1, gradient 0, laplacian -6a
    f = oracle.orbitals(s, 0, c)[0, :, 0]
    assert np.allclose(f, [1.0, 0.0, 0.0, 0.0, -6 * a], rtol=0, atol=1e-15)
    # on the y axis at distance d: exp(-a d^2), d/dy = -2 a d exp(..),
    # laplacian = (4 a^2 d^2 - 6 a) exp(..)
    d = 0.9
    f = oracle.orbitals(s, 0, c + [[0.0, d, 0.0]])[0, :, 0]
    v = np.exp(-a * d * d)
    assert np.allclose(f, [v, 0.0, -2 * a * d * v, 0.0, (4 * a * a * d * d - 6 * a) * v],
                       rtol=1e-14, atol=1e-15)


def test_mo_contraction_orientation():
    """mo[p][b] selects basis function b for orbital p.  With a cyclic
    permutation (p -> b = p + 1 mod nb) orbital p evaluated at the centre of
    basis function p + 1 is 1; the transposed contraction would pick
    b = p - 1 instead and give a much smaller value."""
    nb = 5
    rng = np.random.default_rng(3)
    centres = rng.normal(0, 3.0, (nb, 3))
    expo = rng.uniform(0.5, 2.0, nb)
    mo = np.zeros((nb, nb))
    for p in range(nb):
        mo[p, (p + 1) % nb] = 1.0
    s = _system(centres, expo, mo)
    for p in range(nb):
        f = oracle.orbitals(s, 0, centres[(p + 1) % nb][None])[0]
        assert abs(f[0, p] - 1.0) < 1e-15
        assert np.all(np.abs(f[1:4, p]) < 1e-15)
        assert abs(f[4, p] + 6 * expo[(p + 1) % nb]) < 1e-13


def test_rectangular_mo_and_linearity():
    """n_orb != nb exercises the [n_orb][nb] layout; the orbitals are linear
    in the MO coefficients."""
    rng = np.random.default_rng(5)
    nb, no = 7, 3
    centres = rng.normal(0, 1.0, (nb, 3))
    expo = np.exp(rng.uniform(np.log(0.1), np.log(20.0), nb))
    m1 = rng.normal(size=(no, nb))
    m2 = rng.normal(size=(no, nb))
    pts = rng.normal(0, 1.0, (6, 3))
    f1 = oracle.orbitals(_system(centres, expo, m1), 0, pts)
    f2 = oracle.orbitals(_system(centres, expo, m2), 0, pts)
    f12 = oracle.orbitals(_system(centres, expo, m1 - 2.5 * m2), 0, pts)
    assert f1.shape == (6, 5, no)
    scale = np.abs(f1).max() + np.abs(f2).max()
    assert np.abs(f12 - (f1 - 2.5 * f2)).max() <= 1e-13 * scale


def test_rotation_invariance_and_covariance():
    """Rotating centres and positions together leaves values and laplacians
    unchanged and rotates the gradients."""
    rng = np.random.default_rng(9)
    nb, no = 6, 4
    centres = rng.normal(0, 1.5, (nb, 3))
    expo = np.exp(rng.uniform(np.log(0.2), np.log(5.0), nb))
    mo = rng.normal(size=(no, nb))
    pts = rng.normal(0, 1.5, (5, 3))
    Q = synth.haar_orthogonal(rng, 3)
    f = oracle.orbitals(_system(centres, expo, mo), 0, pts)
    g = oracle.orbitals(_system(centres @ Q.T, expo, mo), 0, pts @ Q.T)
    sc = np.abs(f).max()
    assert np.abs(g[:, 0] - f[:, 0]).max() <= 1e-13 * sc
    assert np.abs(g[:, 4] - f[:, 4]).max() <= 1e-12 * sc
    rot = np.einsum("ij,qjp->qip", Q, f[:, 1:4])
    assert np.abs(g[:, 1:4] - rot).max() <= 1e-12 * sc


def test_numpy_closed_form_water_basis():
    wl = synth.water_like(1, W=2, n_det=10)
    s = wl.system
    pts = wl.walkers.pos.reshape(-1, 3)
    f = oracle.orbitals(s, 0, pts)
    d = pts[:, None, :] - s.centres[None, :, :]           # [P, nb, 3]
    r2 = (d * d).sum(-1)
    chi = np.exp(-s.expo[None] * r2)
    grad = -2 * s.expo[None, :, None] * d * chi[..., None]
    lap = (4 * s.expo[None] ** 2 * r2 - 6 * s.expo[None]) * chi
    mo = s.mo_spin(0)                                      # [n_orb, nb]
    ref = np.concatenate([(chi @ mo.T)[:, None], np.einsum("qbk,pb->qkp", grad, mo),
                          (lap @ mo.T)[:, None]], axis=1)
    assert np.abs(f - ref).max() <= 1e-13 * np.abs(ref).max()
