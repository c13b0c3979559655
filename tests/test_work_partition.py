"""Host-side checks of the determinant kernel's work decomposition (no
device work): for several plans, the work items of every walker tile cover
each excitation exactly once, the staged record ranges respect the LDS
capacity, the dense block (orders 1 and 2 filled when most of them are
present) is handed out in whole hole-set units, and on 64-walker tiles the
per-wave ranges of an item cover its excitations exactly once.  A mistake
here would make the kernel skip or double-count excitations (or read
records it did not stage), which the sampled GPU parity tests might miss."""
import ctypes as C
import os

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ITEM_MAX = 1024


def _lib():
    from paper_1106_2456_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        pytest.skip("libmde.so not built")
    return _lib


def _ptr(a):
    return a.ctypes.data


def _context(L, s):
    lib = L.lib()
    d = L.MdeDesc()
    d.n_elec[0], d.n_elec[1] = s.n_elec
    d.n_orb[0], d.n_orb[1] = s.n_orb
    d.max_walkers = 4096
    d.max_order = 4
    d.refresh_every = 10
    d.precision = 0
    h = C.c_void_p()
    assert lib.mde_create(C.byref(d), None, C.byref(h)) == 0
    keep = []
    for sp in (0, 1):
        e = s.exc[sp]
        off = np.ascontiguousarray(e.offsets, np.int32)
        ho = np.ascontiguousarray(e.holes, np.int32)
        pa = np.ascontiguousarray(e.particles, np.int32)
        keep += [off, ho, pa]
        assert lib.mde_set_excitations(h, sp, off.shape[0] - 1, _ptr(off), _ptr(ho), _ptr(pa)) == 0
    co = np.ascontiguousarray(s.coef, np.float64)
    du = np.ascontiguousarray(s.det_up, np.int32)
    dd = np.ascontiguousarray(s.det_dn, np.int32)
    assert lib.mde_set_ci(h, co.shape[0], _ptr(co), _ptr(du), _ptr(dd)) == 0
    return h


def _items(L, h, spin, W, wt, item_exc, threads):
    lib = L.lib()
    ni, nr = C.c_int32(), C.c_int32()
    layout = np.zeros(4, np.int32)
    rc = lib.mde_debug_items(h, spin, W, wt, item_exc, threads, None, 0, C.byref(ni), None, 0,
                             C.byref(nr), _ptr(layout))
    assert rc in (0, L.MDE_NOMEM)
    items = np.zeros((max(ni.value, 1), 10), np.int32)
    ranges = np.zeros(max(nr.value, 1), np.int32)
    assert lib.mde_debug_items(h, spin, W, wt, item_exc, threads, _ptr(items), ni.value,
                               C.byref(ni), _ptr(ranges), nr.value, C.byref(nr), _ptr(layout)) == 0
    return items[:ni.value], ranges[:nr.value], layout


def _check(items, ranges, layout, s, spin, W, wt, threads):
    U, da, db, dk = (int(x) for x in layout)
    n = s.n_elec[spin]
    m = s.n_orb[spin] - n
    n_tiles = (W + wt - 1) // wt
    nslot = threads // 64
    if db > da:
        # dense block: singles (m per hole) then doubles (one hole pair each)
        assert dk == 3 or dk == 1
        b1 = da + n * m if dk & 1 else da
        starts = list(range(da, b1, m))
        if dk & 2:
            NP = m * (m - 1) // 2
            assert db == b1 + NP * n * (n - 1) // 2
            starts += list(range(b1, db, NP))
        units = set(starts + [db])
    for t in range(n_tiles):
        mine = items[items[:, 2] == t]
        if wt == 64:
            # exactly one item of the tile (its first slot) forms the move's quantities
            assert (mine[:, 3] == 1).sum() == 1
            assert mine[mine[:, 3] == 1][0, 6] == mine[:, 6].min()
        cover = np.zeros(U, np.int32)
        for it in mine:
            u0, u1, slot, wb, d0, d1 = (int(x) for x in it[4:10])
            assert 1 <= u0 <= u1 <= U
            assert u1 - u0 <= ITEM_MAX
            cover[u0:u1] += 1
            if wt == 64:
                if d1 > d0:
                    assert da <= d0 < d1 <= db and d0 in units and d1 in units
                    cover[d0:d1] += 1
                    assert u0 >= db          # sparse records after the dense block
                # per-wave ranges: exactly the item's excitations, dense ones in units
                w = ranges[wb:wb + 2 * nslot].reshape(nslot, 2)
                wc = np.zeros(U, np.int32)
                for j0, j1 in w:
                    if j1 <= j0:
                        continue
                    in_sparse = u0 <= j0 and j1 <= u1
                    in_dense = d0 <= j0 and j1 <= d1
                    assert in_sparse or in_dense, (j0, j1, u0, u1, d0, d1)
                    if in_dense and not in_sparse:
                        assert j0 in units and j1 in units
                    wc[j0:j1] += 1
                want = np.zeros(U, np.int32)
                want[u0:u1] = 1
                want[d0:d1] += 1
                assert np.array_equal(wc, want)
            else:
                assert d0 == d1 == 0 or d1 <= d0
                assert 1 <= it[3] <= 8            # one order per item
        assert cover[0] == 0 and np.all(cover[1:] == 1), t


@pytest.mark.parametrize("plan", [(64, 700, 512), (64, 1332, 512), (64, 300, 256),
                                  (64, 20000, 512), (64, 50, 512), (32, 400, 1024), (16, 300, 256)])
def test_water_partition(plan):
    L = _lib()
    s = synth.water_like(2, W=8, n_moves=1).system
    h = _context(L, s)
    try:
        W = 4096
        for spin in (0, 1):
            items, ranges, layout = _items(L, h, spin, W, *plan)
            # the water-like expansion has most doubles: the dense block exists
            assert layout[3] == 3 and layout[2] > layout[1]
            _check(items, ranges, layout, s, spin, W, *plan[::2][:1], plan[2])
    finally:
        L.lib().mde_destroy(h)


def test_sparse_expansion_has_no_dense_block():
    L = _lib()
    s = synth.water_like(1, W=8, n_moves=1).system      # 200 determinants
    h = _context(L, s)
    try:
        for plan in [(64, 40, 512), (64, 5, 256), (8, 40, 256)]:
            items, ranges, layout = _items(L, h, 0, 1000, *plan)
            assert layout[1] == layout[2]
            _check(items, ranges, layout, s, 0, 1000, plan[0], plan[2])
    finally:
        L.lib().mde_destroy(h)
