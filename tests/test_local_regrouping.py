"""The algebra behind the all-electron derivatives, checked on the CPU
before any kernel: for every electron i, grad^a_i Psi / Psi equals
sum_q d^a_i[q] M[i][q] with M = [A^-T - Z T_V^T | Z], Z = A^-T (dN/dT_V) / N,
where dN/dT_V comes from the oracle's table adjoint (Jacobi's formula on full
matrices) and the reference values from the oracle's row-replacement LUs."""
import numpy as np

import oracle
import synth


def _check(wl, W):
    s = wl.system
    pos = wl.walkers.pos[:W]
    ou, od = oracle.walker_orbitals(s, pos)
    T = []
    for sp, orb in ((0, ou), (1, od)):
        n = s.n_elec[sp]
        T.append(np.stack([np.linalg.solve(o[:, 0, :n], o[:, 0, n:]) for o in orb]))
    _, _, _, gu, gd = oracle.tables(s, T[0], T[1])    # dlog|N|/dT = (dN/dT) / N
    nu = s.n_elec[0]
    for e in range(sum(s.n_elec)):
        sp = 0 if e < nu else 1
        i = e if sp == 0 else e - nu
        orb = (ou, od)[sp]
        g = (gu, gd)[sp]
        n = s.n_elec[sp]
        ref_g, ref_l, sc_g, sc_l = oracle.grad_lap(s, pos, e, scales=True)
        for w in range(W):
            Ainv = np.linalg.inv(orb[w, :, 0, :n])
            Z = Ainv.T @ g[w]
            M = np.concatenate([Ainv.T - Z @ T[sp][w].T, Z], axis=1)
            d = orb[w, i, 1:5, :]                       # grad x, y, z, laplacian rows
            v = d @ M[i]
            assert np.all(np.abs(v[:3] - ref_g[w]) <= 1e-10 * sc_g[w]), (e, w)
            assert abs(v[3] - ref_l[w]) <= 1e-10 * sc_l[w], (e, w)


def test_regrouping_water_like():
    _check(synth.water_like(2, W=4, n_det=600), 4)


def test_regrouping_molecular():
    _check(synth.molecular(3, W=2, n_det=200, n_moves=1, n=12, m=40, nb=64, n_nuc=6, box=6.0), 2)
