"""Pins of the oracle's first-order error scales for FP32 table entries.

The scales claim: if every FP32-stored table quantity (the table T' at R',
the other spin's table, the moving spin's table at R, c' and g^a) carries a
relative error of at most eps against its magnitude E, each output moves by
at most eps * X (to first order).  These tests build that situation with
independent numpy code -- tables by numpy.linalg, entries rounded to float32
or formed by a float32 matrix product, small determinants by
numpy.linalg.det -- and check the observed error against u32 * X.  They
also check the table-route values against the plain full-LU route and a
closed form of the scale for a one-determinant expansion of singles."""
import numpy as np
import pytest

import oracle
import synth

U32 = 2.0 ** -24


def _f32(x):
    return np.asarray(x, np.float32).astype(np.float64)


def _fp32_route(sysm, pos, e, new_r, kind):
    """ratio, grad, lap of one move from FP32-stored table quantities."""
    nu = sysm.n_elec[0]
    ms = 0 if e < nu else 1
    os_ = 1 - ms
    row = e if ms == 0 else e - nu
    ou, od = oracle.walker_orbitals(sysm, pos)
    blk = oracle.orbitals(sysm, ms, new_r)
    W = pos.shape[0]
    out = np.empty((W, 5))
    for w in range(W):
        orb = (ou[w], od[w])
        tabs = {}
        for s, phi, key in ((ms, orb[ms][:, 0].copy(), "R"), (ms, None, "Rp"),
                            (os_, orb[os_][:, 0].copy(), "O")):
            n = sysm.n_elec[s]
            if key == "Rp":
                phi = orb[ms][:, 0].copy()
                phi[row] = blk[w, 0]
            B = np.linalg.inv(phi[:, :n])
            if kind == "round":
                T = _f32(B @ phi[:, n:])
            else:
                T = (B.astype(np.float32) @ phi[:, n:].astype(np.float32)).astype(np.float64)
            tabs[key] = (B, T, phi)
        n = sysm.n_elec[ms]
        Bp, Tp, phip = tabs["Rp"]
        cp = _f32(Bp[:, row])
        rho_a, g = [], []
        if kind == "round":
            # the rank-one form: T' = T - c' q^T in FP64 from the stored FP32
            # table, q = a'^T T - phi'_V, then rounded; g^a = w^a + (k^a/rho) q
            B0, T0 = tabs["R"][0], tabs["R"][1]
            c = B0[:, row]
            a_new = blk[w, 0]
            rho = a_new[:n] @ c
            q = a_new[:n] @ T0 - a_new[n:]
            Tp = _f32(T0 - np.outer(c / rho, q))
        for a in range(4):
            d = blk[w, 1 + a]
            rho_a.append(d[:n] @ Bp[:, row])
            if kind == "round":
                wa = d[n:] - d[:n] @ T0
                g.append(_f32(wa + (d[:n] @ c) / rho * q))
            else:
                ea = (d[:n] @ Bp).astype(np.float32)
                g.append(_f32(d[n:] - (ea @ phip[:, n:].astype(np.float32)).astype(np.float64)))

        def ratios(s, T, deriv=False):
            ex = sysm.exc[s]
            nn = sysm.n_elec[s]
            R = np.empty(ex.n_exc)
            G = np.empty((ex.n_exc, 4))
            for u in range(ex.n_exc):
                h, p = ex.get(u)
                S = T[np.ix_(h, p - nn)]
                R[u] = np.linalg.det(S) if len(h) else 1.0
                if deriv:
                    for a in range(4):
                        M = np.empty((len(h) + 1, len(h) + 1))
                        M[0, 0] = rho_a[a]
                        M[0, 1:] = -g[a][p - nn]
                        M[1:, 0] = cp[h]
                        M[1:, 1:] = S
                        G[u, a] = np.linalg.det(M)
            return R, G

        R0, _ = ratios(ms, tabs["R"][1])
        R1, G1 = ratios(ms, Tp, deriv=True)
        Ro, _ = ratios(os_, tabs["O"][1])
        um = sysm.det_up if ms == 0 else sysm.det_dn
        uo = sysm.det_dn if ms == 0 else sysm.det_up
        c = sysm.coef
        N0 = np.sum(c * R0[um] * Ro[uo])
        N1 = np.sum(c * R1[um] * Ro[uo])
        A = (c[:, None] * G1[um] * Ro[uo][:, None]).sum(0)
        rho = np.linalg.det(phip[:, :n]) / np.linalg.det(tabs["R"][2][:, :n])
        out[w, 0] = rho * N1 / N0
        out[w, 1:] = A / N1
    return out


@pytest.mark.parametrize("kind", ["round", "gemm"])
def test_fp32_entries_stay_within_first_order_scale(kind):
    cases = [(synth.water_like(2, W=12, n_det=800, n_moves=2), 3),
             (synth.water_like(2, W=12, n_det=800, n_moves=2), 7),
             (synth.molecular(3, W=4, n_det=150, n_moves=2, n=12, m=40, nb=64, n_nuc=6, box=6.0), 14)]
    worst, seen = 0.0, []
    for wl, e in cases:
        s = wl.system
        pos = wl.walkers.pos
        new_r = pos[:, e] + wl.moves.disp[0]
        ref = oracle.move(s, pos, e, new_r)
        exact = np.column_stack([ref["ratio"], ref["grad"], ref["lap"]])
        X = oracle.mixed_scales(s, pos, e, new_r)[kind]
        got = _fp32_route(s, pos, e, new_r, kind)
        rel = np.abs(got - exact) / (U32 * X)
        # first order: at most 1 for rounding; a float32 product of length
        # n adds up to (n + 2) u32 per entry against |A^-1| |Phi_V|
        bound = 1.5 if kind == "round" else 1.5 * (s.n_elec[0] + 3)
        worst = max(worst, rel.max())
        seen.append(rel.ravel())
        assert rel.max() <= bound, (kind, e, rel.max())
    # the scale is not vacuous: typical errors are a visible share of it
    assert np.median(np.concatenate(seen)) > (1e-3 if kind == "round" else 1e-4)


def test_table_route_values_equal_full_lu_route():
    wl = synth.molecular(3, W=5, n_det=300, n_moves=2, n=12, m=40, nb=64, n_nuc=6, box=6.0)
    s = wl.system
    pos = wl.walkers.pos
    for e in (0, 17):
        new_r = pos[:, e] + wl.moves.disp[1]
        ref = oracle.move(s, pos, e, new_r)
        v = oracle.mixed_scales(s, pos, e, new_r)["vals"]
        assert np.all(np.abs(v[:, 0] - ref["ratio"]) <= 1e-12 * ref["scale_ratio"])
        assert np.all(np.abs(v[:, 1:4] - ref["grad"]) <= 1e-12 * ref["scale_grad"])
        assert np.all(np.abs(v[:, 4] - ref["lap"]) <= 1e-12 * ref["scale_lap"])


def test_single_determinant_closed_form():
    """One determinant: the reference in the moving (up) spin and a single
    excitation in the other.  Every output is then proportional to one table
    entry of the other spin (P = |entry|), read at R and R' alike, so each
    scale is 2 |x|: X = |x| (1 + 1) for the ratio, (|x| + |x|) for the
    derivatives (the reference's derivative factor rho^a is FP64)."""
    wl = synth.water_like(2, W=6, n_det=400, n_moves=2)
    s = wl.system
    ex_u, ex_d = s.exc
    I = next(i for i in range(s.n_det) if ex_u.order(s.det_up[i]) == 0 and ex_d.order(s.det_dn[i]) == 1)
    one = synth.with_coef(s, np.where(np.arange(s.n_det) == I, 1.0, 0.0))
    pos = wl.walkers.pos
    new_r = pos[:, 2] + wl.moves.disp[0]
    m = oracle.mixed_scales(one, pos, 2, new_r)
    for kind in ("round", "gemm"):
        X = m[kind]
        if kind == "round":
            assert np.allclose(X, 2 * np.abs(m["vals"]), rtol=1e-12)
        # the product-formed entry's magnitude |A^-1| |Phi_V| bounds |entry|
        assert np.all(X >= 2 * np.abs(m["vals"]) * (1 - 1e-12))


def test_propagated_errors_cover_a_committed_sequence():
    """Tables kept in FP32 across commits (the rank-one form): along a
    sequence of committed moves the float32 emulation stays within the
    scale whose entry magnitudes are propagated by StoredTableErrors."""
    wl = synth.molecular(3, W=3, n_det=150, n_moves=6, n=12, m=40, nb=64, n_nuc=6, box=6.0)
    s = wl.system
    pos = wl.walkers.pos.copy()
    nu = s.n_elec[0]
    # stored FP32 tables of both spins, emulated along the sequence
    ou, od = oracle.walker_orbitals(s, pos)
    T32 = [np.stack([_f32(np.linalg.solve(o[:, 0, :s.n_elec[sp]], o[:, 0, s.n_elec[sp]:]))
                     for o in orb]) for sp, orb in ((0, ou), (1, od))]
    B = [np.stack([np.linalg.inv(o[:, 0, :s.n_elec[sp]]) for o in orb]) for sp, orb in ((0, ou), (1, od))]
    track = oracle.StoredTableErrors(s, pos)
    worst = 0.0
    for k, e in enumerate([0, 3, 14, 5, 20, 1]):
        sp = 0 if e < nu else 1
        row = e if sp == 0 else e - nu
        n = s.n_elec[sp]
        new_r = pos[:, e] + wl.moves.disp[k]
        blk = oracle.orbitals(s, sp, new_r)
        ref = oracle.move(s, pos, e, new_r)
        X = track.scales(pos, e, new_r)["round"]
        for w in range(pos.shape[0]):
            c = B[sp][w][:, row]
            a = blk[w, 0]
            rho = a[:n] @ c
            q = a[:n] @ T32[sp][w] - a[n:]
            Tp = _f32(T32[sp][w] - np.outer(c / rho, q))
            ex = s.exc[sp]
            def dets(T, spin):
                exs = s.exc[spin]
                nn = s.n_elec[spin]
                return np.array([np.linalg.det(T[np.ix_(exs.get(u)[0], exs.get(u)[1] - nn)])
                                 if exs.order(u) else 1.0 for u in range(exs.n_exc)])
            R0, R1, Ro = dets(T32[sp][w], sp), dets(Tp, sp), dets(T32[1 - sp][w], 1 - sp)
            um = s.det_up if sp == 0 else s.det_dn
            uo = s.det_dn if sp == 0 else s.det_up
            ratio = rho * np.sum(s.coef * R1[um] * Ro[uo]) / np.sum(s.coef * R0[um] * Ro[uo])
            rel = abs(ratio - ref["ratio"][w]) / (U32 * X[w, 0])
            worst = max(worst, rel)
            assert rel <= 1.5, (k, w, rel)
            if wl.moves.accept[k, w]:
                T32[sp][w] = Tp
                B[sp][w] = B[sp][w] - np.outer(c / rho, a[:n] @ B[sp][w] - np.eye(n)[row])
        track.commit(wl.moves.accept[k])
        pos[:, e] = new_r
    assert worst > 1e-3

