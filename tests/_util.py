"""Helpers shared by the tests (no method arithmetic beyond brute force)."""
import itertools
import json
import os

import numpy as np

import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def perm_sign(p):
    s = 1
    p = list(p)
    for i in range(len(p)):
        for j in range(i + 1, len(p)):
            if p[i] > p[j]:
                s = -s
    return s


def leibniz(M):
    """Determinant as the sum over all n! permutations (brute force)."""
    M = np.asarray(M, dtype=np.float64)
    n = M.shape[0]
    if n == 0:
        return 1.0
    tot = 0.0
    for p in itertools.permutations(range(n)):
        t = float(perm_sign(p))
        for i in range(n):
            t *= M[i, p[i]]
        tot += t
    return tot


def exc_columns(ex, u, n):
    col = list(range(n))
    h, p = ex.get(u)
    for a, b in zip(h, p):
        col[a] = b
    return col


def system_from_json(d):
    ex = []
    for key in ("exc_up", "exc_dn"):
        e = d[key]
        ex.append(synth.Excitations(np.asarray(e["offsets"], np.int32),
                                    np.asarray(e["holes"], np.int32),
                                    np.asarray(e["particles"], np.int32)))
    nb = 1
    return synth.System(tuple(d["n_elec"]), tuple(d["n_orb"]), np.zeros((1, 3)),
                        np.zeros((nb, 3)), np.ones(nb), np.zeros((max(d["n_orb"]), nb)),
                        tuple(ex), np.asarray(d["coef"], np.float64),
                        np.asarray(d["det_up"], np.int32), np.asarray(d["det_dn"], np.int32))


def load_golden(name):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def brute_psi(sysm, orb_up1, orb_dn1, coef=None, row=None, comp=0):
    """Psi of one walker by Leibniz determinants of the full excited
    matrices; optionally electron `row` (global index) takes orbital
    component `comp` (derivative row replacement)."""
    coef = sysm.coef if coef is None else coef
    nu, nd = sysm.n_elec
    tot = 0.0
    for I in range(sysm.n_det):
        dets = []
        for s, (orb, idx) in enumerate(((orb_up1, sysm.det_up[I]), (orb_dn1, sysm.det_dn[I]))):
            n = sysm.n_elec[s]
            col = exc_columns(sysm.exc[s], int(idx), n)
            M = np.empty((n, n))
            for i in range(n):
                gi = i if s == 0 else nu + i
                c = comp if (row is not None and gi == row) else 0
                M[i] = orb[i, c, col]
            dets.append(leibniz(M))
        tot += coef[I] * dets[0] * dets[1]
    return tot
