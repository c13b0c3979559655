"""CPU FP64 oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` (plain C,
``oracle.c``), which evaluates every determinant by LU of the full excited
n x n matrix (Sec. II definitions; Sec. IV derivatives by row
replacement).  It shares no code with the GPU library.

Functions whose results have no independent pin say so in their docstring
("parity unpinned"); all of the ones below are pinned by ``tests/test_oracle_*``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

_dp = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_ip = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O3 -march=native -fopenmp)."""
    if force or not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
        tmp = _SO + ".tmp"
        cmd = ["gcc", "-O3", "-march=native", "-fopenmp", "-fPIC", "-shared",
               "-std=c11", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _SO)
    return _SO


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(_SO)
        L.oracle_orbitals.argtypes = [C.c_int, _dp, _dp, C.c_int, _dp, C.c_int, _dp, _dp]
        L.oracle_slogdet.argtypes = [C.c_int, _dp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        L.oracle_inverse.argtypes = [C.c_int, _dp, _dp, C.POINTER(C.c_double), C.POINTER(C.c_double)]
        exc = [C.c_int, _ip, _ip, _ip]
        L.oracle_mds_batch.argtypes = ([C.c_int] * 5 + [_dp, _dp] + exc + exc +
                                       [C.c_int64, _dp, _ip, _ip, C.c_int, _dp, _dp,
                                        C.c_void_p, C.c_void_p])
        L.oracle_psi_adjoint.argtypes = ([C.c_int] * 4 + [_dp, _dp] + exc + exc +
                                         [C.c_int64, _dp, _ip, _ip, _dp, _dp, _dp, _dp])
        L.oracle_tables_batch.argtypes = ([C.c_int] * 5 + [_dp, _dp] + exc + exc +
                                          [C.c_int64, _dp, _ip, _ip, _dp, _dp, _dp, _dp])
        L.oracle_mixed_scales_batch.argtypes = ([C.c_int] * 5 + [_dp, _dp, C.c_int, _dp] + exc + exc +
                                                [C.c_int64, _dp, _ip, _ip, C.c_void_p, C.c_void_p,
                                                 C.c_void_p, _dp, _dp])
        L.oracle_num_threads.restype = C.c_int
        _lib = L
    return _lib


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _exc_args(ex):
    return [int(ex.n_exc), _i32(ex.offsets), _i32(ex.holes), _i32(ex.particles)]


# ---------------------------------------------------------------------------
# orbitals
# ---------------------------------------------------------------------------

def orbitals(sysm, spin: int, pos: np.ndarray) -> np.ndarray:
    """phi_p and its derivatives at positions ``pos`` [..., 3] -> [..., 5, n_orb]
    (component 0 value, 1..3 gradient, 4 laplacian)."""
    pos = _f64(pos)
    shp = pos.shape[:-1]
    P = int(np.prod(shp)) if shp else 1
    mo = _f64(sysm.mo_spin(spin))
    no = mo.shape[0]
    out = np.empty((P, 5, no))
    lib().oracle_orbitals(int(sysm.nb), _f64(sysm.centres), _f64(sysm.expo), no, mo, P,
                          pos.reshape(P, 3), out)
    return out.reshape(*shp, 5, no)


def walker_orbitals(sysm, pos: np.ndarray):
    """Orbital blocks of every electron: (up [W, n_up, 5, no_up], dn [...])."""
    pos = _f64(pos)
    nu = sysm.n_elec[0]
    return orbitals(sysm, 0, pos[:, :nu]), orbitals(sysm, 1, pos[:, nu:])


# ---------------------------------------------------------------------------
# dense linear algebra (exposed for the pins)
# ---------------------------------------------------------------------------

def slogdet(M: np.ndarray):
    M = _f64(M)
    s, l = C.c_double(), C.c_double()
    lib().oracle_slogdet(int(M.shape[0]), M, C.byref(s), C.byref(l))
    return s.value, l.value


def inverse(M: np.ndarray) -> np.ndarray:
    M = _f64(M)
    out = np.zeros_like(M)
    s, l = C.c_double(), C.c_double()
    lib().oracle_inverse(int(M.shape[0]), M, out, C.byref(s), C.byref(l))
    return out


# ---------------------------------------------------------------------------
# Psi and its derivatives
# ---------------------------------------------------------------------------

def mds(sysm, orb_up: np.ndarray, orb_dn: np.ndarray, e_deriv: int = -1,
        shift: Optional[np.ndarray] = None, ratios: bool = False, coef=None):
    """Multi-determinant sum for W walkers.

    Returns a dict with ``shift`` [W] (log scale L*), ``psi`` [W]
    (= Psi exp(-L*)), ``dpsi`` [W, 4] (the same sum with electron e_deriv's
    row replaced by d/dx, d/dy, d/dz, laplacian), ``sign0``/``log0`` [W, 2]
    of the reference determinants and, if ``ratios``, the per-excitation
    ratios D_u / D_0 of each spin."""
    orb_up = _f64(orb_up); orb_dn = _f64(orb_dn)
    W = orb_up.shape[0]
    nu, nd = sysm.n_elec
    nou, nod = sysm.n_orb
    assert orb_up.shape == (W, nu, 5, nou) and orb_dn.shape == (W, nd, 5, nod)
    ex_u, ex_d = sysm.exc
    coef = _f64(sysm.coef if coef is None else coef)
    sh = np.full(W, np.nan) if shift is None else _f64(np.broadcast_to(shift, (W,)))
    out = np.empty((W, 15))
    ru = np.empty((W, ex_u.n_exc)) if ratios else None
    rd = np.empty((W, ex_d.n_exc)) if ratios else None
    rc = lib().oracle_mds_batch(W, nu, nd, nou, nod, orb_up, orb_dn,
                                *_exc_args(ex_u), *_exc_args(ex_d),
                                int(coef.shape[0]), coef, _i32(sysm.det_up),
                                _i32(sysm.det_dn), int(e_deriv), sh, out,
                                ru.ctypes.data if ratios else None,
                                rd.ctypes.data if ratios else None)
    if rc != 0:
        raise RuntimeError("oracle_mds_batch failed")
    res = dict(shift=out[:, 0].copy(), psi=out[:, 1].copy(), dpsi=out[:, 2:6].copy(),
               sign0=out[:, [6, 8]].copy(), log0=out[:, [7, 9]].copy(),
               psi_abs=out[:, 10].copy(), dpsi_abs=out[:, 11:15].copy())
    if ratios:
        res["ratio_up"], res["ratio_dn"] = ru, rd
    return res


def log_psi(sysm, pos: np.ndarray):
    """(sign Psi, log|Psi|) per walker at positions pos [W, n_tot, 3]."""
    ou, od = walker_orbitals(sysm, pos)
    r = mds(sysm, ou, od)
    return np.sign(r["psi"]), np.log(np.abs(r["psi"])) + r["shift"]


def move(sysm, pos: np.ndarray, e: int, new_r: np.ndarray, coef=None):
    """Quantities of one proposed move of electron e to new_r [W, 3]:
    ratio Psi(R')/Psi(R), grad_e ln Psi(R') [W, 3], lap_e Psi(R')/Psi(R') [W]
    (Sec. II ratio eq., Sec. IV eq. gradMDS).  Both sums use the same log
    shift, taken at R."""
    ou, od = walker_orbitals(sysm, pos)
    r0 = mds(sysm, ou, od, coef=coef)
    pos2 = pos.copy()
    pos2[:, e] = new_r
    ou2, od2 = walker_orbitals(sysm, pos2)
    r1 = mds(sysm, ou2, od2, e_deriv=e, shift=r0["shift"], coef=coef)
    ratio = r1["psi"] / r0["psi"]
    grad = r1["dpsi"][:, :3] / r1["psi"][:, None]
    lap = r1["dpsi"][:, 3] / r1["psi"]
    # condition-aware scales of x = sum(a) / sum(b):
    #   X = (sum|a| + |x| sum|b|) / |sum b|
    sc_ratio = (r1["psi_abs"] + np.abs(ratio) * r0["psi_abs"]) / np.abs(r0["psi"])
    sc_d = (r1["dpsi_abs"] + np.abs(r1["dpsi"] / r1["psi"][:, None]) * r1["psi_abs"][:, None]) \
        / np.abs(r1["psi"])[:, None]
    return dict(ratio=ratio, grad=grad, lap=lap, psi_old=r0, psi_new=r1,
                scale_ratio=sc_ratio, scale_grad=sc_d[:, :3], scale_lap=sc_d[:, 3])


def grad_lap(sysm, pos: np.ndarray, e: int, coef=None, scales: bool = False):
    """grad_e ln Psi and lap_e Psi / Psi at R (no move).  With ``scales`` also
    their condition-aware scales (as in ``move``)."""
    ou, od = walker_orbitals(sysm, pos)
    r = mds(sysm, ou, od, e_deriv=e, coef=coef)
    g = r["dpsi"][:, :3] / r["psi"][:, None]
    lap = r["dpsi"][:, 3] / r["psi"]
    if not scales:
        return g, lap
    sc = (r["dpsi_abs"] + np.abs(r["dpsi"] / r["psi"][:, None]) * r["psi_abs"][:, None]) \
        / np.abs(r["psi"])[:, None]
    return g, lap, sc[:, :3], sc[:, 3]


# ---------------------------------------------------------------------------
# adjoints
# ---------------------------------------------------------------------------

def psi_adjoint(sysm, orb_up1: np.ndarray, orb_dn1: np.ndarray, coef=None):
    """One walker: (sign, log|Psi|), dlog|Psi|/dc [n_det] and
    dlog|Psi|/dPhi_sigma [n_sigma, n_orb_sigma] (values only), by Jacobi's
    formula on each full excited matrix."""
    ex_u, ex_d = sysm.exc
    coef = _f64(sysm.coef if coef is None else coef)
    nu, nd = sysm.n_elec
    nou, nod = sysm.n_orb
    out2 = np.empty(2)
    gc = np.empty(coef.shape[0])
    gu = np.empty((nu, nou)); gd = np.empty((nd, nod))
    rc = lib().oracle_psi_adjoint(nu, nd, nou, nod, _f64(orb_up1), _f64(orb_dn1),
                                  *_exc_args(ex_u), *_exc_args(ex_d),
                                  int(coef.shape[0]), coef, _i32(sysm.det_up),
                                  _i32(sysm.det_dn), out2, gc, gu, gd)
    if rc != 0:
        raise RuntimeError("oracle_psi_adjoint failed")
    return out2, gc, gu, gd


def tables(sysm, T_up: np.ndarray, T_dn: np.ndarray, coef=None):
    """N = sum_I c_I det X_up,I det X_dn,I from explicit virtual tables
    T_sigma [W, n, m] (X_u = identity with column h_j replaced by the table
    column of p_j), by full n x n LU.  Returns sign [W], log|N| [W],
    dlog|N|/dc [W, n_det], dlog|N|/dT_up [W, n, m], dlog|N|/dT_dn."""
    ex_u, ex_d = sysm.exc
    coef = _f64(sysm.coef if coef is None else coef)
    T_up = _f64(T_up); T_dn = _f64(T_dn)
    W, nu, mu = T_up.shape
    _, nd, md = T_dn.shape
    out2 = np.empty((W, 2))
    gc = np.empty((W, coef.shape[0]))
    gu = np.empty_like(T_up); gd = np.empty_like(T_dn)
    rc = lib().oracle_tables_batch(W, nu, nd, mu, md, T_up, T_dn,
                                   *_exc_args(ex_u), *_exc_args(ex_d),
                                   int(coef.shape[0]), coef, _i32(sysm.det_up),
                                   _i32(sysm.det_dn), out2, gc, gu, gd)
    if rc != 0:
        raise RuntimeError("oracle_tables_batch failed")
    return out2[:, 0], out2[:, 1], gc, gu, gd


# ---------------------------------------------------------------------------
# error scales of the FP32-table forms
# ---------------------------------------------------------------------------

def mixed_scales(sysm, pos: np.ndarray, e: int, new_r: np.ndarray, coef=None, err=None):
    """First-order error scales of one proposed move (as ``move``) for forms
    that keep table entries in FP32.  A relative perturbation eps of every
    FP32-stored entry moves each output x by at most eps * X to first order.

    Returns ``round`` [W, 5] (entries rounded to FP32: E = |entry|, or the
    propagated magnitudes ``err`` = (err_up [W, n, m], err_dn) of tables
    kept in FP32 across commits), ``gemm`` [W, 5] (entries formed by an FP32
    product of A^-1 and Phi_V: E = |A^-1| |Phi_V|), columns (ratio, d/dx,
    d/dy, d/dz, laplacian), ``vals`` [W, 5], the same outputs computed
    through the tables (pinned against ``move``), and ``err_next``
    [W, n, m], the moving spin's table magnitudes after a commit of this
    move (only with ``err``)."""
    pos = _f64(pos)
    W = pos.shape[0]
    nu, nd = sysm.n_elec
    nou, nod = sysm.n_orb
    ou, od = walker_orbitals(sysm, pos)
    spin = 0 if e < nu else 1
    blk = _f64(orbitals(sysm, spin, _f64(new_r)))
    ex_u, ex_d = sysm.exc
    coef = _f64(sysm.coef if coef is None else coef)
    out = np.empty((W, 2, 5))
    vals = np.empty((W, 5))
    e_ms = e_os = e_next = None
    if err is not None:
        e_ms = _f64(err[spin])
        e_os = _f64(err[1 - spin])
        e_next = np.empty_like(e_ms)
    ptr = lambda a: None if a is None else a.ctypes.data  # noqa: E731
    rc = lib().oracle_mixed_scales_batch(W, nu, nd, nou, nod, ou, od, int(e), blk,
                                         *_exc_args(ex_u), *_exc_args(ex_d),
                                         int(coef.shape[0]), coef, _i32(sysm.det_up),
                                         _i32(sysm.det_dn), ptr(e_ms), ptr(e_os), ptr(e_next),
                                         out, vals)
    if rc != 0:
        raise RuntimeError("oracle_mixed_scales_batch failed (singular reference?)")
    res = dict(round=out[:, 0].copy(), gemm=out[:, 1].copy(), vals=vals)
    if err is not None:
        res["err_next"] = e_next
    return res


def table_magnitudes(sysm, pos: np.ndarray):
    """|T_V| of both spins at positions pos [W, n_tot, 3]: the entry
    magnitudes of tables just computed from scratch and rounded once
    (T = A^-1 Phi_V, Sec. III)."""
    ou, od = walker_orbitals(sysm, pos)
    out = []
    for s, orb in ((0, ou), (1, od)):
        n = sysm.n_elec[s]
        T = np.stack([np.linalg.solve(o[:, 0, :n], o[:, 0, n:]) for o in orb])
        out.append(np.abs(T))
    return out


class StoredTableErrors:
    """Entrywise first-order error magnitudes (units of eps) of the two
    spins' tables kept in FP32 across commits, along a trajectory: one
    rounding after a from-scratch evaluation, propagated through each
    committed table update (see oracle_mixed_scales_batch)."""

    def __init__(self, sysm, pos):
        self.sysm = sysm
        self.err = table_magnitudes(sysm, pos)

    def scales(self, pos, e, new_r):
        self._last = mixed_scales(self.sysm, pos, e, new_r, err=self.err)
        self._spin = 0 if e < self.sysm.n_elec[0] else 1
        return self._last

    def commit(self, accepted):
        acc = np.asarray(accepted, bool)
        self.err[self._spin][acc] = self._last["err_next"][acc]

    def refresh(self, pos):
        self.err = table_magnitudes(self.sysm, pos)
