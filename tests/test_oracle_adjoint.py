"""Pins for the oracle's adjoints: Euler identities (degree-1 homogeneity
in c, degree-k homogeneity of each k x k determinant in table entries),
central finite differences, and agreement of two independent routes
(explicit tables vs. orbital matrix chained through Phi_V = A T_V)."""
import numpy as np

import oracle
import synth


def _tables_from_orbitals(sysm, ou, od):
    Ts = []
    for s, orb in ((0, ou), (1, od)):
        n = sysm.n_elec[s]
        Phi = orb[:, :, 0, :]
        Ts.append(np.stack([np.linalg.solve(P[:, :n], P[:, n:]) for P in Phi]))
    return Ts


def _setup(W=3, n_det=150):
    wl = synth.water_like(1, W=W, n_det=n_det)
    sysm = wl.system
    ou, od = oracle.walker_orbitals(sysm, wl.walkers.pos)
    Tu, Td = _tables_from_orbitals(sysm, ou, od)
    return sysm, ou, od, Tu, Td


def test_euler_identities():
    sysm, ou, od, Tu, Td = _setup()
    s, l, gc, gu, gd = oracle.tables(sysm, Tu, Td)
    assert np.allclose(gc @ sysm.coef, 1.0, rtol=0, atol=1e-12)
    ku = sysm.exc[0].orders()[sysm.det_up]
    kd = sysm.exc[1].orders()[sysm.det_dn]
    # c_I grad_c[I] = c_I R_up R_dn / N: the share of determinant I
    share = gc * sysm.coef[None, :]
    assert np.allclose((gu * Tu).sum(axis=(1, 2)), share @ ku, rtol=1e-10, atol=1e-10)
    assert np.allclose((gd * Td).sum(axis=(1, 2)), share @ kd, rtol=1e-10, atol=1e-10)


def test_finite_differences():
    sysm, ou, od, Tu, Td = _setup(W=2, n_det=80)
    s, l, gc, gu, gd = oracle.tables(sysm, Tu, Td)
    h = 1e-6
    rng = np.random.default_rng(1)
    for I in rng.choice(sysm.n_det, 12, replace=False):
        cp = sysm.coef.copy(); cp[I] += h
        cm = sysm.coef.copy(); cm[I] -= h
        fd = (oracle.tables(sysm, Tu, Td, coef=cp)[1] - oracle.tables(sysm, Tu, Td, coef=cm)[1]) / (2 * h)
        assert np.allclose(fd, gc[:, I], rtol=1e-6, atol=1e-8)
    for (r, p) in [(0, 0), (1, 3), (4, 19), (2, 7)]:
        for which in (0, 1):
            Tp = [Tu.copy(), Td.copy()]; Tm = [Tu.copy(), Td.copy()]
            Tp[which][:, r, p] += h; Tm[which][:, r, p] -= h
            fd = (oracle.tables(sysm, *Tp)[1] - oracle.tables(sysm, *Tm)[1]) / (2 * h)
            g = (gu, gd)[which][:, r, p]
            assert np.allclose(fd, g, rtol=1e-6, atol=1e-8)


def test_two_routes_agree():
    """dlog|Psi|/dT_V = A^T dlog|Psi|/dPhi_V (A held fixed) and
    dlog|Psi|/dc from the orbital route equals the table route."""
    sysm, ou, od, Tu, Td = _setup(W=3, n_det=200)
    s, l, gc, gu, gd = oracle.tables(sysm, Tu, Td)
    for w in range(3):
        out2, gc2, gphi_u, gphi_d = oracle.psi_adjoint(sysm, ou[w, :, :, :], od[w, :, :, :])
        assert np.allclose(gc2, gc[w], rtol=1e-10, atol=1e-12)
        for s_, gphi, gT in ((0, gphi_u, gu), (1, gphi_d, gd)):
            n = sysm.n_elec[s_]
            A = (ou, od)[s_][w, :, 0, :n]
            ref = A.T @ gphi[:, n:]
            assert np.allclose(ref, gT[w], rtol=1e-8, atol=1e-9 * np.abs(gT[w]).max())
        # log|Psi| = log|D0_up| + log|D0_dn| + log|N|
        su, lu = np.linalg.slogdet(ou[w, :, 0, :5])
        sd, ld = np.linalg.slogdet(od[w, :, 0, :5])
        assert abs(out2[1] - (lu + ld + l[w])) < 1e-10 * abs(out2[1])


def test_singular_excited_table_matrix():
    """The table route's fallback for a singular excited matrix X_u (its
    cofactors by column replacement): a double excitation whose two table
    columns are exactly proportional has det X_u = 0, yet contributes
    cofactors to dlog|N|/dT.  Checked against central differences of the
    oracle's own forward, which takes no such branch."""
    ex_u = synth.Excitations(np.array([0, 0, 1, 3, 4], np.int32),
                             np.array([2, 0, 1, 1], np.int32),
                             np.array([5, 3, 4, 6], np.int32))
    ex_d = synth.Excitations(np.array([0, 0, 1], np.int32),
                             np.array([1], np.int32), np.array([3], np.int32))
    det_up = np.array([0, 1, 2, 0, 2, 3], np.int32)
    det_dn = np.array([0, 0, 0, 1, 1, 1], np.int32)
    coef = np.array([1.0, 0.4, -0.7, 0.3, 0.25, -0.5])
    ex = synth.Excitations(np.zeros(2, np.int32), np.zeros(0, np.int32), np.zeros(0, np.int32))
    sysm = synth.System((3, 2), (7, 5), np.zeros((1, 3)), np.zeros((1, 3)), np.ones(1),
                        np.zeros((7, 1)), (ex_u, ex_d), coef, det_up, det_dn)
    # dyadic entries: the double (0,1 -> 3,4) reads columns 0 and 1 of T_up,
    # and column 1 = 1.5 x column 0 exactly, so X_u is singular in floating point
    Tu = np.array([[[0.5, 0.75, -0.25, 1.0],
                    [-1.0, -1.5, 0.5, 0.25],
                    [0.25, 0.375, 2.0, -0.5]]])
    Td = np.array([[[0.5, -0.25, 1.5], [1.25, 0.75, -1.0]]])
    s, l, gc, gu, gd = oracle.tables(sysm, Tu, Td)
    assert s[0] != 0.0
    # the double's ratio is exactly zero
    assert gc[0, 2] == 0.0
    h = 1e-6
    for r in range(3):
        for p in range(4):
            Tp, Tm = Tu.copy(), Tu.copy()
            Tp[0, r, p] += h
            Tm[0, r, p] -= h
            fd = (oracle.tables(sysm, Tp, Td)[1] - oracle.tables(sysm, Tm, Td)[1]) / (2 * h)
            assert abs(fd[0] - gu[0, r, p]) <= 1e-8 * (1 + abs(fd[0])), (r, p, fd, gu[0, r, p])
    # the cofactors reached through the fallback are not zero: the singular
    # double is the only determinant holding hole 1 with particle 4
    assert abs(gu[0, 1, 1]) > 1e-3
