"""Pins for the oracle's derivatives: finite differences of its own values
(orbitals, log|Psi|), with Richardson extrapolation for the laplacian."""
import numpy as np
import pytest

import oracle
import synth


def test_orbital_derivatives_by_fd():
    wl = synth.water_like(1, W=1, n_det=10)
    sysm = wl.system
    rng = np.random.default_rng(0)
    pts = synth.WATER_NUCLEI[rng.integers(0, 3, 6)] + 0.7 * rng.standard_normal((6, 3))
    f = oracle.orbitals(sysm, 0, pts)
    h = 1e-5
    for d in range(3):
        e = np.zeros(3); e[d] = h
        fd = (oracle.orbitals(sysm, 0, pts + e)[:, 0] - oracle.orbitals(sysm, 0, pts - e)[:, 0]) / (2 * h)
        scale = np.abs(f[:, 0]).max() * 400
        assert np.abs(fd - f[:, 1 + d]).max() < 1e-7 * scale

    def lap(hh):
        acc = -6 * oracle.orbitals(sysm, 0, pts)[:, 0]
        for d in range(3):
            e = np.zeros(3); e[d] = hh
            acc = acc + oracle.orbitals(sysm, 0, pts + e)[:, 0] + oracle.orbitals(sysm, 0, pts - e)[:, 0]
        return acc / hh ** 2
    L = (4 * lap(5e-4) - lap(1e-3)) / 3
    assert np.abs(L - f[:, 4]).max() < 1e-5 * np.abs(f[:, 4]).max()


@pytest.mark.parametrize("e", [0, 4, 7])
def test_grad_lap_log_psi_by_fd(e):
    wl = synth.water_like(1, W=3, n_det=120)
    sysm = wl.system
    pos = wl.walkers.pos
    g, L = oracle.grad_lap(sysm, pos, e)
    s0, l0 = oracle.log_psi(sysm, pos)

    def ratio(delta):
        p = pos.copy()
        p[:, e] += delta
        s, l = oracle.log_psi(sysm, p)
        return s * s0 * np.exp(l - l0)

    h = 1e-5
    for d in range(3):
        dd = np.zeros(3); dd[d] = h
        fd = (ratio(dd) - ratio(-dd)) / (2 * h)
        assert np.all(np.abs(fd - g[:, d]) < 1e-7 * (1 + np.abs(g[:, d])))

    def lap(hh):
        acc = -6.0
        for d in range(3):
            dd = np.zeros(3); dd[d] = hh
            acc = acc + ratio(dd) + ratio(-dd)
        return acc / hh ** 2
    Lfd = (4 * lap(5e-4) - lap(1e-3)) / 3
    assert np.all(np.abs(Lfd - L) < 1e-5 * (1 + np.abs(L)))


def test_move_grad_is_grad_at_new_position():
    wl = synth.water_like(1, W=2, n_det=60)
    sysm, pos = wl.system, wl.walkers.pos
    new = pos[:, 1] + 0.25
    mv = oracle.move(sysm, pos, 1, new)
    p2 = pos.copy(); p2[:, 1] = new
    g, L = oracle.grad_lap(sysm, p2, 1)
    assert np.allclose(mv["grad"], g, rtol=1e-12, atol=1e-13)
    assert np.allclose(mv["lap"], L, rtol=1e-12, atol=1e-12)
    s0, l0 = oracle.log_psi(sysm, pos)
    s1, l1 = oracle.log_psi(sysm, p2)
    assert np.allclose(mv["ratio"], s0 * s1 * np.exp(l1 - l0), rtol=1e-12)
