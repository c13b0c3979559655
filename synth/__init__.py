"""Seeded synthetic inputs for the multi-determinant evaluation.

This module only draws random numbers and lays them out: nuclei, an
s-Gaussian basis (centres, exponents), a molecular-orbital coefficient
matrix, electron positions, particle-hole excitation lists, CI
coefficients, move displacements and acceptance masks.  It evaluates no
orbital, determinant, table or ratio: both the CPU oracle and the GPU
library take these arrays and do all of the method's arithmetic
themselves.

Notation follows the paper (Sec. II): for each spin there are ``n``
electrons and ``n + m`` orbitals; orbitals ``0..n-1`` fill the reference
determinant, ``n..n+m-1`` are the virtual orbitals.  An excitation
replaces holes ``h_j`` (occupied) by particles ``p_j`` (virtual); the
particle ``p_j`` takes the column of hole ``h_j``.  Holes and particles are
listed in ascending order and paired in that order.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

ROOT_SEED = 11062456
BOHR_PER_ANGSTROM = 1.0 / 0.529177210903

# Streams spawned from the root SeedSequence, in this fixed order.
_STREAMS = ("basis", "mo", "nuclei", "electrons", "ci_structure",
            "ci_coef", "moves", "accept")

# Water-like nuclei (bohr): O at the origin, H at (+-1.43, 1.11, 0).
WATER_NUCLEI = np.array([[0.0, 0.0, 0.0],
                         [1.43, 1.11, 0.0],
                         [-1.43, 1.11, 0.0]])

ORDER_QUOTA = (0.10, 0.50, 0.30, 0.10)   # share of excitation orders 1..4


@dataclass
class Excitations:
    """Unique per-spin excitation list in CSR form.

    Entry 0 is always the empty excitation (the reference determinant).
    ``holes[offsets[u]:offsets[u+1]]`` are the holes of excitation ``u``,
    ascending; ``particles[...]`` the matching particles, ascending.
    """
    offsets: np.ndarray     # int32 [n_exc + 1]
    holes: np.ndarray       # int32 [offsets[-1]]
    particles: np.ndarray   # int32 [offsets[-1]]

    @property
    def n_exc(self) -> int:
        return int(self.offsets.shape[0] - 1)

    def order(self, u: int) -> int:
        return int(self.offsets[u + 1] - self.offsets[u])

    def orders(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.int32)

    def get(self, u: int) -> Tuple[np.ndarray, np.ndarray]:
        a, b = int(self.offsets[u]), int(self.offsets[u + 1])
        return self.holes[a:b], self.particles[a:b]


@dataclass
class System:
    """One molecular-shaped system and its multi-determinant expansion."""
    n_elec: Tuple[int, int]          # electrons per spin (up, down)
    n_orb: Tuple[int, int]           # orbitals per spin = n + m
    nuclei: np.ndarray               # [n_nuc, 3]
    centres: np.ndarray              # [nb, 3] basis centres
    expo: np.ndarray                 # [nb] Gaussian exponents
    mo: np.ndarray                   # [n_orb_max, nb]; orbital p = sum_b mo[p,b] chi_b
    exc: Tuple[Excitations, Excitations]
    coef: np.ndarray                 # [n_det] float64, coef[0] = 1
    det_up: np.ndarray               # [n_det] int32 index into exc[0]
    det_dn: np.ndarray               # [n_det] int32 index into exc[1]
    mo_dn: Optional[np.ndarray] = None   # separate down-spin MOs (None: same as up)

    @property
    def n_det(self) -> int:
        return int(self.coef.shape[0])

    @property
    def nb(self) -> int:
        return int(self.expo.shape[0])

    def mo_spin(self, s: int) -> np.ndarray:
        mo = self.mo if (s == 0 or self.mo_dn is None) else self.mo_dn
        return np.ascontiguousarray(mo[: self.n_orb[s]])


@dataclass
class Walkers:
    pos: np.ndarray                  # [W, n_up + n_dn, 3]

    @property
    def W(self) -> int:
        return int(self.pos.shape[0])


@dataclass
class Moves:
    electron: np.ndarray             # [n_moves] int32 electron index
    disp: np.ndarray                 # [n_moves, W, 3]
    accept: np.ndarray               # [n_moves, W] uint8 (all ones)
    accept_half: np.ndarray          # [n_moves, W] uint8 (seeded 50 % mask)


@dataclass
class Workload:
    name: str
    system: System
    walkers: Walkers
    moves: Moves
    meta: dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# primitive draws
# --------------------------------------------------------------------------

def _streams(key: Sequence[int]) -> dict:
    ss = np.random.SeedSequence([ROOT_SEED, *key])
    kids = ss.spawn(len(_STREAMS))
    return {name: np.random.Generator(np.random.PCG64(k))
            for name, k in zip(_STREAMS, kids)}


def haar_orthogonal(rng: np.random.Generator, n: int) -> np.ndarray:
    """Haar-random orthogonal n x n matrix (QR of a Gaussian matrix with the
    column signs fixed by diag(R))."""
    z = rng.standard_normal((n, n))
    q, r = np.linalg.qr(z)
    q = q * np.sign(np.diag(r))[None, :]
    return q


def draw_basis(rng: np.random.Generator, nuclei: np.ndarray, nb: int,
               a_lo: float = 0.1, a_hi: float = 20.0):
    """Basis function b sits on nucleus b mod n_nuc; exponents are
    log-uniform in [a_lo, a_hi]."""
    n_nuc = nuclei.shape[0]
    centres = nuclei[np.arange(nb) % n_nuc].copy()
    expo = np.exp(rng.uniform(math.log(a_lo), math.log(a_hi), size=nb))
    return centres, expo


def draw_positions(rng: np.random.Generator, nuclei: np.ndarray, W: int,
                   n_tot: int, sigma: float = 1.0) -> np.ndarray:
    """Each electron picks a nucleus uniformly and sits at a Gaussian offset."""
    which = rng.integers(0, nuclei.shape[0], size=(W, n_tot))
    return nuclei[which] + sigma * rng.standard_normal((W, n_tot, 3))


def _quota_split(total: int, shares: Sequence[float]) -> List[int]:
    """Largest-remainder rounding of total * shares."""
    raw = [total * s for s in shares]
    base = [int(math.floor(x)) for x in raw]
    rest = total - sum(base)
    order = sorted(range(len(raw)), key=lambda i: (-(raw[i] - base[i]), i))
    for i in order[:rest]:
        base[i] += 1
    return base


def _n_spin_exc(n: int, m: int, k: int) -> int:
    if k < 0 or k > n or k > m:
        return 0
    return math.comb(n, k) * math.comb(m, k)


def _capacity(n_up, n_dn, m_up, m_dn, k) -> int:
    return sum(_n_spin_exc(n_up, m_up, ku) * _n_spin_exc(n_dn, m_dn, k - ku)
               for ku in range(k + 1))


def _enumerate_spin(n: int, m: int, k: int):
    from itertools import combinations
    for h in combinations(range(n), k):
        for p in combinations(range(n, n + m), k):
            yield (h, p)


def draw_expansion(rng_struct: np.random.Generator, rng_coef: np.random.Generator,
                   n_elec: Tuple[int, int], n_virt: Tuple[int, int], n_det: int,
                   max_order: int = 4, shares: Sequence[float] = ORDER_QUOTA,
                   decay: Optional[float] = None):
    """Random CI expansion: n_det distinct determinants including the
    reference (index 0, c_0 = 1).  Orders 1..max_order follow ``shares`` of
    n_det - 1 (largest-remainder rounding); a quota above the number of
    distinct determinants of that order is capped and its shortfall moves to
    the next order.  The total order k is split k_up ~ Binomial(k, 1/2),
    redrawn until both spins can hold it; holes and particles are drawn
    uniformly without replacement.  c_I = z_I exp(-decay I), z ~ N(0,1),
    decay = 10 / n_det unless given."""
    n_up, n_dn = n_elec
    m_up, m_dn = n_virt
    shares = list(shares)[:max_order]
    quotas = _quota_split(n_det - 1, [s / sum(shares) for s in shares])
    dets = [((), (), (), ())]
    seen = {dets[0]}
    carry = 0
    realized = []
    for k in range(1, max_order + 1):
        want = quotas[k - 1] + carry
        cap = _capacity(n_up, n_dn, m_up, m_dn, k)
        take = min(want, cap)
        carry = want - take
        got = []
        if take > 0 and take * 2 >= cap:
            # dense regime: enumerate every order-k determinant, sample subset
            allk = []
            for ku in range(k + 1):
                kd = k - ku
                ups = list(_enumerate_spin(n_up, m_up, ku))
                dns = list(_enumerate_spin(n_dn, m_dn, kd))
                for a in ups:
                    for b in dns:
                        allk.append((a[0], a[1], b[0], b[1]))
            pick = rng_struct.choice(len(allk), size=take, replace=False)
            got = [allk[i] for i in np.sort(pick)]
            for d in got:
                seen.add(d)
        else:
            while len(got) < take:
                while True:
                    ku = int(rng_struct.binomial(k, 0.5))
                    kd = k - ku
                    if (ku <= min(n_up, m_up)) and (kd <= min(n_dn, m_dn)):
                        break
                hu = tuple(sorted(rng_struct.choice(n_up, ku, replace=False).tolist()))
                pu = tuple(sorted((n_up + rng_struct.choice(m_up, ku, replace=False)).tolist()))
                hd = tuple(sorted(rng_struct.choice(n_dn, kd, replace=False).tolist()))
                pd = tuple(sorted((n_dn + rng_struct.choice(m_dn, kd, replace=False)).tolist()))
                d = (hu, pu, hd, pd)
                if d in seen:
                    continue
                seen.add(d)
                got.append(d)
        dets.extend(got)
        realized.append(len(got))
    nd = len(dets)
    if decay is None:
        decay = 10.0 / nd
    z = rng_coef.standard_normal(nd)
    coef = z * np.exp(-decay * np.arange(nd))
    coef[0] = 1.0

    def build(spin):
        index = {}
        offs, hs, ps = [0], [], []
        idx = np.empty(nd, dtype=np.int32)
        for I, d in enumerate(dets):
            key = (d[2 * spin], d[2 * spin + 1])
            if key not in index:
                index[key] = len(index)
                hs.extend(key[0])
                ps.extend(key[1])
                offs.append(len(hs))
            idx[I] = index[key]
        ex = Excitations(np.asarray(offs, np.int32), np.asarray(hs, np.int32),
                         np.asarray(ps, np.int32))
        return ex, idx

    ex_up, i_up = build(0)
    ex_dn, i_dn = build(1)
    meta = {"order_quota": quotas, "order_realized": realized,
            "n_exc_up": ex_up.n_exc, "n_exc_dn": ex_dn.n_exc}
    return (ex_up, ex_dn), coef.astype(np.float64), i_up, i_dn, meta


def draw_moves(rng_moves: np.random.Generator, rng_acc: np.random.Generator,
               n_moves: int, W: int, n_tot: int, step: float,
               electron_order: Optional[np.ndarray] = None) -> Moves:
    """Move s displaces electron s mod n_tot (up electrons first) by
    N(0, step^2) in each direction, independently per walker."""
    if electron_order is None:
        electron = (np.arange(n_moves) % n_tot).astype(np.int32)
    else:
        electron = np.asarray(electron_order, np.int32)
    disp = step * rng_moves.standard_normal((n_moves, W, 3))
    acc = np.ones((n_moves, W), np.uint8)
    half = (rng_acc.random((n_moves, W)) < 0.5).astype(np.uint8)
    return Moves(electron, disp, acc, half)


# --------------------------------------------------------------------------
# systems and workloads
# --------------------------------------------------------------------------

def make_system(key: Sequence[int], n_elec: Tuple[int, int], n_virt: Tuple[int, int],
                nuclei: np.ndarray, nb: int, n_det: int, max_order: int = 4,
                shares: Sequence[float] = ORDER_QUOTA, decay: Optional[float] = None,
                streams: Optional[dict] = None):
    rs = streams if streams is not None else _streams(key)
    centres, expo = draw_basis(rs["basis"], nuclei, nb)
    n_orb = (n_elec[0] + n_virt[0], n_elec[1] + n_virt[1])
    if max(n_orb) > nb:
        raise ValueError("need at least as many basis functions as orbitals")
    q = haar_orthogonal(rs["mo"], nb)
    mo = np.ascontiguousarray(q[: max(n_orb)])
    exc, coef, iu, idn, meta = draw_expansion(rs["ci_structure"], rs["ci_coef"],
                                              n_elec, n_virt, n_det, max_order,
                                              shares, decay)
    sysm = System(tuple(n_elec), n_orb, nuclei.copy(), centres, expo, mo, exc,
                  coef, iu, idn)
    return sysm, rs, meta


def make_workload(key: Sequence[int], name: str, n_elec, n_virt, nuclei, nb, n_det,
                  W, n_moves, step=0.3, max_order=4, shares=ORDER_QUOTA, decay=None,
                  electron_order=None) -> Workload:
    sysm, rs, meta = make_system(key, n_elec, n_virt, nuclei, nb, n_det, max_order,
                                 shares, decay)
    n_tot = n_elec[0] + n_elec[1]
    pos = draw_positions(rs["electrons"], nuclei, W, n_tot)
    mv = draw_moves(rs["moves"], rs["accept"], n_moves, W, n_tot, step, electron_order)
    meta.update(dict(W=W, n_moves=n_moves, key=list(key)))
    return Workload(name, sysm, Walkers(pos), mv, meta)


def water_like(cfg: int = 1, W: Optional[int] = None, n_det: Optional[int] = None,
               n_moves: Optional[int] = None) -> Workload:
    """Water-like system: 5 up + 5 down electrons, 5 occupied + 20 virtual
    orbitals per spin from 40 s-Gaussians on the three water nuclei.
    cfg 1: one walker, 200 determinants, 1000 moves.
    cfg 2: 4096 walkers, 10 000 determinants (cfg 4 uses 1024 walkers)."""
    defaults = {1: (1, 200, 1000), 2: (4096, 10000, 100), 4: (1024, 10000, 10)}
    dW, dN, dM = defaults[cfg]
    W = dW if W is None else W
    n_det = dN if n_det is None else n_det
    n_moves = dM if n_moves is None else n_moves
    key = (cfg if cfg != 4 else 2,)
    return make_workload(key, f"water-like cfg{cfg}", (5, 5), (20, 20),
                         WATER_NUCLEI, 40, n_det, W, n_moves)


def molecular(cfg: int = 3, W: int = 2048, n_det: int = 100000, n_moves: int = 64,
              n: int = 32, m: int = 224, nb: int = 512, n_nuc: int = 20,
              box: float = 12.0, electron_order=None) -> Workload:
    """Molecular-shaped system: n electrons per spin, n + m orbitals from nb
    s-Gaussians on n_nuc nuclei uniform in a box of side ``box`` bohr.
    electron_order: the moving electron of each move (default: move s moves
    electron s mod 2n)."""
    rs = _streams((cfg,))
    nuclei = rs["nuclei"].uniform(0.0, box, size=(n_nuc, 3))
    sysm, rs, meta = make_system((cfg,), (n, n), (m, m), nuclei, nb, n_det,
                                 streams=rs)
    pos = draw_positions(rs["electrons"], nuclei, W, 2 * n)
    mv = draw_moves(rs["moves"], rs["accept"], n_moves, W, 2 * n, 0.3, electron_order)
    meta.update(dict(W=W, n_moves=n_moves, key=[cfg]))
    return Workload(f"molecular n={n} m={m} ndet={n_det}", sysm, Walkers(pos), mv, meta)


def uneven_instances(n_inst: int = 64, W: int = 256, n_moves: int = 4,
                     n_lo: int = 5, n_hi: int = 64,
                     ndet_lo: float = 1e2, ndet_hi: float = 2e5,
                     only: Optional[Sequence[int]] = None) -> List[Workload]:
    """Uneven batch: instance j has n ~ U{n_lo..n_hi} electrons per spin,
    m = 4n virtuals, N_det log-uniform in [ndet_lo, ndet_hi], 2(n+m) basis
    functions on max(3, round(0.625 n)) nuclei in a box of side
    12 (n/32)^(1/3) bohr."""
    top = np.random.Generator(np.random.PCG64(np.random.SeedSequence([ROOT_SEED, 5])))
    ns = top.integers(n_lo, n_hi + 1, size=n_inst)
    nds = np.round(np.exp(top.uniform(math.log(ndet_lo), math.log(ndet_hi), size=n_inst))).astype(int)
    out = []
    for j in range(n_inst):
        if only is not None and j not in only:
            continue
        n = int(ns[j]); m = 4 * n; nd = int(nds[j])
        rs = _streams((5, j))
        n_nuc = max(3, int(round(0.625 * n)))
        box = 12.0 * (n / 32.0) ** (1.0 / 3.0)
        nuclei = rs["nuclei"].uniform(0.0, box, size=(n_nuc, 3))
        sysm, rs, meta = make_system((5, j), (n, n), (m, m), nuclei, 2 * (n + m), nd,
                                     streams=rs)
        pos = draw_positions(rs["electrons"], nuclei, W, 2 * n)
        mv = draw_moves(rs["moves"], rs["accept"], n_moves, W, 2 * n, 0.3)
        meta.update(dict(W=W, n_moves=n_moves, key=[5, j], n=n, m=m))
        out.append(Workload(f"uneven[{j}] n={n} ndet={nd}", sysm, Walkers(pos), mv, meta))
    return out


def tiny_system(seed: int, n_up: int, n_dn: int, m: int, n_det: int, W: int = 1,
                nb: Optional[int] = None, max_order: int = 4, n_moves: int = 4,
                step: float = 0.3, all_dets: bool = False) -> Workload:
    """Small system for brute-force checks (n <= 3, m <= 3 typically).
    all_dets=True lists every determinant reachable up to max_order."""
    nb = nb if nb is not None else max(n_up, n_dn) + m + 2
    key = (1000 + seed,)
    rs = _streams(key)
    nuclei = WATER_NUCLEI
    if all_dets:
        cap = 1 + sum(_capacity(n_up, n_dn, m, m, k) for k in range(1, max_order + 1))
        n_det = cap
        shares = [1.0] * max_order
        # every quota >= capacity -> enumeration of all determinants
        sysm, rs, meta = make_system(key, (n_up, n_dn), (m, m), nuclei, nb, 10 ** 7,
                                     max_order, shares, decay=0.1, streams=rs)
    else:
        sysm, rs, meta = make_system(key, (n_up, n_dn), (m, m), nuclei, nb, n_det,
                                     max_order, streams=rs)
    pos = draw_positions(rs["electrons"], nuclei, W, n_up + n_dn)
    mv = draw_moves(rs["moves"], rs["accept"], n_moves, W, n_up + n_dn, step)
    meta.update(dict(W=W, key=list(key)))
    return Workload(f"tiny seed={seed}", sysm, Walkers(pos), mv, meta)


def lincomb_virtuals(sysm: System, rng_seed: int = 7) -> Tuple[System, List[np.ndarray]]:
    """Copy of ``sysm`` whose virtual MO rows are random linear combinations
    of its occupied MO rows: phi_p = sum_{b<n} w[p,b] phi_b.  Returns the new
    system and, per spin, the weights w [m, n] (inputs only)."""
    rng = np.random.Generator(np.random.PCG64(rng_seed))
    if sysm.n_elec[0] != sysm.n_elec[1] or sysm.n_orb[0] != sysm.n_orb[1]:
        raise ValueError("lincomb fixture assumes equal spin shapes")
    n, no = sysm.n_elec[0], sysm.n_orb[0]
    mo = sysm.mo.copy()
    w = rng.standard_normal((no - n, n))
    mo[n:no] = w @ mo[:n]
    s2 = System(sysm.n_elec, sysm.n_orb, sysm.nuclei, sysm.centres, sysm.expo, mo,
                sysm.exc, sysm.coef, sysm.det_up, sysm.det_dn)
    return s2, [w, w]


def with_coef(sysm: System, coef: np.ndarray) -> System:
    return System(sysm.n_elec, sysm.n_orb, sysm.nuclei, sysm.centres, sysm.expo,
                  sysm.mo, sysm.exc, np.asarray(coef, np.float64), sysm.det_up,
                  sysm.det_dn, sysm.mo_dn)
