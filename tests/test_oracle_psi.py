"""Pins for the oracle's multi-determinant sum: a hand-worked example,
Leibniz brute force on tiny systems (all determinants), antisymmetry,
the single-determinant and one-electron-per-spin special cases, the
linear-combination-virtuals closed form, and the table read-off
(Sec. III) computed by numpy as an independent route."""
import numpy as np
import pytest

import oracle
import synth
from tests._util import brute_psi, exc_columns, leibniz, load_golden, system_from_json


def test_hand_example():
    d = load_golden("hand_example.json")
    sysm = system_from_json(d)
    ou = np.asarray(d["orb_up"], np.float64)[None]
    od = np.asarray(d["orb_dn"], np.float64)[None]
    r = oracle.mds(sysm, ou, od, e_deriv=0, shift=np.zeros(1), ratios=True)
    assert abs(r["psi"][0] - d["psi"]) < 1e-12
    assert np.allclose(r["dpsi"][0] / r["psi"][0], d["dpsi_over_psi_e0"], rtol=0, atol=1e-14)
    assert np.allclose(r["ratio_up"][0], d["ratio_up"], atol=1e-14)
    assert np.allclose(r["ratio_dn"][0], d["ratio_dn"], atol=1e-14)
    s, l, gc, gu, gd = oracle.tables(sysm, np.asarray(d["T_up"])[None], np.asarray(d["T_dn"])[None])
    assert s[0] == 1.0 and abs(np.exp(l[0]) - d["N"]) < 1e-12


@pytest.mark.parametrize("seed,nu,nd,m", [(1, 2, 2, 2), (2, 3, 2, 2), (3, 2, 1, 3), (4, 3, 3, 2)])
def test_brute_force_all_determinants(seed, nu, nd, m):
    wl = synth.tiny_system(seed, nu, nd, m, 0, W=3, all_dets=True)
    sysm = wl.system
    ou, od = oracle.walker_orbitals(sysm, wl.walkers.pos)
    r = oracle.mds(sysm, ou, od, shift=np.zeros(3))
    for w in range(3):
        ref = brute_psi(sysm, ou[w], od[w])
        scale = sum(abs(c) for c in sysm.coef) * np.abs(ou[w, :, 0]).max() ** nu * np.abs(od[w, :, 0]).max() ** nd
        assert abs(r["psi"][w] - ref) <= 1e-13 * max(scale, abs(ref))
    # derivative rows: every electron, every component
    for e in range(nu + nd):
        r = oracle.mds(sysm, ou, od, e_deriv=e, shift=np.zeros(3))
        for w in range(3):
            for c in range(4):
                ref = brute_psi(sysm, ou[w], od[w], row=e, comp=c + 1)
                assert abs(r["dpsi"][w, c] - ref) <= 1e-11 * max(1.0, abs(ref))


def test_antisymmetry_same_spin_swap():
    wl = synth.tiny_system(7, 3, 3, 4, 40, W=4)
    sysm = wl.system
    pos = wl.walkers.pos
    s0, l0 = oracle.log_psi(sysm, pos)
    p2 = pos.copy()
    p2[:, [0, 2]] = p2[:, [2, 0]]          # swap two up electrons
    s1, l1 = oracle.log_psi(sysm, p2)
    assert np.all(s1 == -s0) and np.allclose(l1, l0, atol=1e-12)
    p3 = pos.copy()
    p3[:, [3, 5]] = p3[:, [5, 3]]          # swap two down electrons
    s2, l2 = oracle.log_psi(sysm, p3)
    assert np.all(s2 == -s0) and np.allclose(l2, l0, atol=1e-12)


def test_single_determinant_reduction():
    wl = synth.water_like(1, W=5, n_det=50)
    sysm = synth.with_coef(wl.system, np.r_[1.0, np.zeros(wl.system.n_det - 1)])
    ou, od = oracle.walker_orbitals(sysm, wl.walkers.pos)
    s, l = oracle.log_psi(sysm, wl.walkers.pos)
    for w in range(5):
        su, lu = np.linalg.slogdet(ou[w, :, 0, :5])
        sd, ld = np.linalg.slogdet(od[w, :, 0, :5])
        assert s[w] == su * sd and abs(l[w] - (lu + ld)) < 1e-12 * max(1, abs(lu + ld))


def test_one_electron_per_spin_closed_form():
    wl = synth.tiny_system(9, 1, 1, 3, 12, W=4, max_order=2)
    sysm = wl.system
    ou, od = oracle.walker_orbitals(sysm, wl.walkers.pos)
    r = oracle.mds(sysm, ou, od, e_deriv=0, shift=np.zeros(4))
    for w in range(4):
        psi = 0.0
        dpsi = np.zeros(4)
        for I in range(sysm.n_det):
            pu = exc_columns(sysm.exc[0], int(sysm.det_up[I]), 1)[0]
            pd = exc_columns(sysm.exc[1], int(sysm.det_dn[I]), 1)[0]
            psi += sysm.coef[I] * ou[w, 0, 0, pu] * od[w, 0, 0, pd]
            dpsi += sysm.coef[I] * ou[w, 0, 1:, pu] * od[w, 0, 0, pd]
        assert abs(r["psi"][w] - psi) < 1e-13 * max(1, abs(psi))
        assert np.allclose(r["dpsi"][w], dpsi, rtol=1e-12, atol=1e-14)


def test_lincomb_virtuals_closed_form():
    """phi_p = sum_b w[p,b] phi_b for virtual p: every excited determinant is
    the reference times det of w entries, for every configuration, so the
    Psi ratio of any move equals the reference ratio and the derivatives are
    those of the reference determinant alone."""
    wl = synth.water_like(1, W=3, n_det=60)
    sysm, ws = synth.lincomb_virtuals(wl.system)
    n = sysm.n_elec[0]
    ou, od = oracle.walker_orbitals(sysm, wl.walkers.pos)
    r = oracle.mds(sysm, ou, od, ratios=True)
    for s, key in ((0, "ratio_up"), (1, "ratio_dn")):
        ex = sysm.exc[s]
        for u in range(ex.n_exc):
            h, p = ex.get(u)
            S = np.array([[ws[s][pl - n, hj] for pl in p] for hj in h]).reshape(len(h), len(p))
            assert np.allclose(r[key][:, u], leibniz(S), rtol=1e-9, atol=1e-11)
    # move: ratio equals the reference-determinant ratio; derivatives those of D0
    pos = wl.walkers.pos
    new = pos[:, 2] + np.array([0.2, -0.1, 0.3])
    mv = oracle.move(sysm, pos, 2, new)
    ref = synth.with_coef(sysm, np.r_[1.0, np.zeros(sysm.n_det - 1)])
    mv0 = oracle.move(ref, pos, 2, new)
    assert np.allclose(mv["ratio"], mv0["ratio"], rtol=1e-10)
    assert np.allclose(mv["grad"], mv0["grad"], rtol=1e-9, atol=1e-12)
    assert np.allclose(mv["lap"], mv0["lap"], rtol=1e-9, atol=1e-10)


def test_table_readoff_independent_route():
    """Oracle's full-LU ratios D_u/D_0 equal det S_u with S_u[j,l] = T[h_j,p_l],
    T = A^-1 Phi computed by numpy (Sec. III table and r x r read-off)."""
    wl = synth.water_like(2, W=3, n_det=400)
    sysm = wl.system
    ou, od = oracle.walker_orbitals(sysm, wl.walkers.pos)
    r = oracle.mds(sysm, ou, od, ratios=True)
    for w in range(3):
        for s, orb, key in ((0, ou, "ratio_up"), (1, od, "ratio_dn")):
            n = sysm.n_elec[s]
            Phi = orb[w, :, 0, :]
            T = np.linalg.solve(Phi[:, :n], Phi)
            ex = sysm.exc[s]
            for u in range(ex.n_exc):
                h, p = ex.get(u)
                S = T[np.ix_(h, p)]
                ref = np.linalg.det(S) if len(h) else 1.0
                scale = np.prod(np.abs(S).max(axis=1)) * max(1, len(h)) ** 2 if len(h) else 1.0
                assert abs(r[key][w, u] - ref) <= 1e-10 * max(scale, abs(ref)) * np.linalg.cond(Phi[:, :n])


def test_zero_length_move_ratio_is_one():
    wl = synth.water_like(1, W=4, n_det=80)
    pos = wl.walkers.pos
    mv = oracle.move(wl.system, pos, 3, pos[:, 3].copy())
    assert np.allclose(mv["ratio"], 1.0, rtol=0, atol=1e-14)


def test_water_geometry_of_nuclei():
    """The water-like nuclei reproduce r_OH = 0.9572 A and the H-O-H angle of
    104.52 deg (Sec. VI) to the precision of their two-decimal bohr values."""
    O, H1, H2 = synth.WATER_NUCLEI
    r = np.linalg.norm(H1 - O) / synth.BOHR_PER_ANGSTROM
    ang = np.degrees(np.arccos(np.dot(H1 - O, H2 - O) / np.linalg.norm(H1 - O) / np.linalg.norm(H2 - O)))
    assert abs(r - 0.9572) < 0.005 and abs(ang - 104.52) < 0.5
