"""Seeded input generator: reproducibility and structural validity."""
import numpy as np

import synth


def test_seeds_reproduce_bitwise():
    a = synth.water_like(1, W=3, n_det=100, n_moves=5)
    b = synth.water_like(1, W=3, n_det=100, n_moves=5)
    for x, y in ((a.walkers.pos, b.walkers.pos), (a.system.mo, b.system.mo),
                 (a.system.coef, b.system.coef), (a.moves.disp, b.moves.disp),
                 (a.system.exc[0].holes, b.system.exc[0].holes)):
        assert np.array_equal(x, y)


def test_mo_orthogonal():
    wl = synth.water_like(1, W=1, n_det=10)
    q = wl.system.mo
    assert np.allclose(q @ q.T, np.eye(q.shape[0]), atol=1e-12)


def test_expansion_valid_and_distinct():
    wl = synth.water_like(2, W=1)
    s = wl.system
    assert s.n_det == 10000 and s.coef[0] == 1.0
    assert s.det_up[0] == 0 and s.det_dn[0] == 0
    # realized histogram with the singles cap (200 distinct singles exist)
    assert wl.meta["order_realized"] == [200, 5799, 3000, 1000]
    seen = set()
    for I in range(s.n_det):
        key = []
        for sp, idx in ((0, s.det_up[I]), (1, s.det_dn[I])):
            h, p = s.exc[sp].get(int(idx))
            n = s.n_elec[sp]
            assert len(set(h.tolist())) == len(h) and len(set(p.tolist())) == len(p)
            assert np.all((h >= 0) & (h < n)) and np.all((p >= n) & (p < s.n_orb[sp]))
            assert np.all(np.diff(h) > 0) and np.all(np.diff(p) > 0)
            key.append((tuple(h), tuple(p)))
        key = tuple(key)
        assert key not in seen
        seen.add(key)
    for sp in (0, 1):
        ex = s.exc[sp]
        assert ex.order(0) == 0
        keys = {tuple(ex.holes[ex.offsets[u]:ex.offsets[u + 1]]) + (-1,) +
                tuple(ex.particles[ex.offsets[u]:ex.offsets[u + 1]]) for u in range(ex.n_exc)}
        assert len(keys) == ex.n_exc


def test_moves_schedule():
    wl = synth.water_like(1, W=2, n_det=20, n_moves=25)
    assert list(wl.moves.electron[:12]) == [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 0, 1]
    assert wl.moves.disp.shape == (25, 2, 3)
    assert set(np.unique(wl.moves.accept_half)) <= {0, 1}
