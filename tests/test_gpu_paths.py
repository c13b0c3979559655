"""GPU parity of the entry points and branches the trajectory tests do not
reach: derivatives at the current positions (mde_grad_lap), excitation
orders 5-8 (elimination path, on 64-walker and on small walker tiles),
per-walker status bits forced from the host, captured group sweeps, the
autograd Function over two forwards that share tables, and a group whose
member changed its plan."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import dev, gpu_orbitals, make_ctx, say, scaled_err

pytestmark = pytest.mark.gpu


def test_grad_lap_matches_oracle():
    """grad_e ln Psi(R) and lap_e Psi(R)/Psi(R) at the current positions,
    after init and after a few committed moves, every electron."""
    wl = synth.water_like(2, W=70, n_det=1500, n_moves=6)
    s = wl.system
    ctx = make_ctx(wl)
    pos = wl.walkers.pos.copy()
    ctx.init(*gpu_orbitals(ctx, pos))
    worst = 0.0
    for phase in range(2):
        if phase == 1:
            for k in range(6):
                e = int(wl.moves.electron[k])
                new_r = pos[:, e] + wl.moves.disp[k]
                ctx.propose(e, ctx.sgauss_eval(ctx.spin_of(e), dev(new_r)))
                mask = wl.moves.accept_half[k]
                ctx.accept(e, dev(mask, torch.uint8))
                pos[mask.astype(bool), e] = new_r[mask.astype(bool)]
        for e in range(sum(s.n_elec)):
            cur = ctx.sgauss_eval(ctx.spin_of(e), dev(pos[:, e]))
            g, lap, st = ctx.grad_lap(e, cur)
            rg, rl, sg, sl = oracle.grad_lap(s, pos, e, scales=True)
            eg = scaled_err(g.cpu().numpy(), rg, sg).max()
            el = scaled_err(lap.cpu().numpy(), rl, sl).max()
            worst = max(worst, eg, el)
            assert not st.cpu().numpy().any()
            assert eg <= 1e-10 and el <= 1e-10, (phase, e, eg, el)
    say(f"grad_lap: worst scaled error {worst:.2e}")


def _high_order_workload(W):
    """8 + 8 electrons, 10 virtuals per spin, excitation orders up to 8 per
    spin (one order-8 up excitation appended to the drawn expansion)."""
    wl = synth.make_workload((77,), "high orders", (8, 8), (10, 10), synth.WATER_NUCLEI, 24, 400,
                             W, 16, max_order=8, shares=[1, 2, 2, 2, 2, 2, 2, 2])
    s = wl.system
    ex = s.exc[0]
    holes = np.concatenate([ex.holes, np.arange(8, dtype=np.int32)])
    parts = np.concatenate([ex.particles, np.arange(9, 17, dtype=np.int32)])
    offs = np.concatenate([ex.offsets, [ex.offsets[-1] + 8]]).astype(np.int32)
    s.exc = (synth.Excitations(offs, holes, parts), s.exc[1])
    s.det_up = np.concatenate([s.det_up, [ex.n_exc]]).astype(np.int32)
    s.det_dn = np.concatenate([s.det_dn, [0]]).astype(np.int32)
    s.coef = np.concatenate([s.coef, [0.05]])
    return wl


@pytest.mark.parametrize("walker_tile", [64, 4])
def test_orders_5_to_8(walker_tile):
    wl = _high_order_workload(W=70)
    s = wl.system
    orders = np.concatenate([s.exc[0].orders(), s.exc[1].orders()])
    assert orders.max() == 8 and (orders >= 5).sum() > 50
    ctx = make_ctx(wl, max_order=8, bind=False)
    for sp in (0, 1):
        ctx.set_plan(sp, walker_tile=walker_tile)
    ctx.bind(70)
    pos = wl.walkers.pos.copy()
    la, sg, st = ctx.init(*gpu_orbitals(ctx, pos))
    ref_s, ref_l = oracle.log_psi(s, pos)
    assert np.abs(la.cpu().numpy() - ref_l).max() <= 1e-10 * np.abs(ref_l).max()
    assert np.array_equal(sg.cpu().numpy(), ref_s)
    ou, od = oracle.walker_orbitals(s, pos)
    ref = oracle.mds(s, ou, od, ratios=True)
    for sp, key in ((0, "ratio_up"), (1, "ratio_dn")):
        r = ctx.export("ratios", sp).cpu().numpy()
        assert np.abs(r - ref[key]).max() <= 1e-9 * np.abs(ref[key]).max(), sp
    worst = 0.0
    for k in range(16):
        e = int(wl.moves.electron[k])
        new_r = pos[:, e] + wl.moves.disp[k]
        ratio, grad, lap, st = ctx.propose(e, ctx.sgauss_eval(ctx.spin_of(e), dev(new_r)))
        mask = wl.moves.accept_half[k]
        ctx.accept(e, dev(mask, torch.uint8))
        r = oracle.move(s, pos, e, new_r)
        er = scaled_err(ratio.cpu().numpy(), r["ratio"], r["scale_ratio"]).max()
        eg = scaled_err(grad.cpu().numpy(), r["grad"], r["scale_grad"]).max()
        el = scaled_err(lap.cpu().numpy(), r["lap"], r["scale_lap"]).max()
        worst = max(worst, er, eg, el)
        assert er <= 1e-10 and eg <= 1e-10 and el <= 1e-10, (k, er, eg, el)
        assert not st.cpu().numpy().any()
        pos[mask.astype(bool), e] = new_r[mask.astype(bool)]
    say(f"orders 5-8, walker tile {walker_tile}: worst scaled error {worst:.2e}")


def test_status_bits_forced_from_host():
    """SINGULAR_REF from two up electrons at the same position (other
    walkers unaffected); SMALL_RATIO and ZERO_PSI from a proposed orbital
    block of zeros; NONFINITE from a NaN in a proposed block."""
    from paper_1106_2456_amd._lib import (ST_NONFINITE, ST_SINGULAR_REF, ST_SMALL_RATIO,
                                          ST_ZERO_PSI)
    W = 70
    wl = synth.water_like(2, W=W, n_det=600, n_moves=2)
    s = wl.system
    pos = wl.walkers.pos.copy()
    pos[5, 1] = pos[5, 0]            # walker 5: up electrons 0 and 1 coincide
    ctx = make_ctx(wl)
    la, sg, st = ctx.init(*gpu_orbitals(ctx, pos))
    st = st.cpu().numpy()
    assert st[5] & ST_SINGULAR_REF
    others = np.arange(W) != 5
    assert not st[others].any()
    ref_s, ref_l = oracle.log_psi(s, pos[others])
    assert np.abs(la.cpu().numpy()[others] - ref_l).max() <= 1e-10 * np.abs(ref_l).max()
    # proposals from clean positions
    pos = wl.walkers.pos.copy()
    ctx.init(*gpu_orbitals(ctx, pos))
    e = 2
    new_r = pos[:, e] + wl.moves.disp[0]
    blk = ctx.sgauss_eval(0, dev(new_r))
    blk[11].zero_()                  # walker 11: every orbital value zero
    blk[23, 0, 7] = float("nan")     # walker 23: one NaN orbital value
    ratio, grad, lap, st = ctx.propose(e, blk)
    st = st.cpu().numpy()
    assert st[11] & ST_SMALL_RATIO and st[11] & ST_ZERO_PSI, st[11]
    assert ratio.cpu().numpy()[11] == 0.0
    assert st[23] & ST_NONFINITE, st[23]
    clean = np.ones(W, bool)
    clean[[11, 23]] = False
    assert not st[clean].any()
    ref = oracle.move(s, pos, e, new_r)
    er = scaled_err(ratio.cpu().numpy()[clean], ref["ratio"][clean], ref["scale_ratio"][clean])
    assert er.max() <= 1e-10


def test_group_capture_replay_matches_eager():
    """A group sweep captured into a HIP graph and replayed (twice, with eager
    re-initialisation in between) gives the eager sweep's results bit for bit
    (on a side stream: the legacy default stream cannot be captured)."""
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        _group_capture_body(stream)


def _group_capture_body(stream):
    from paper_1106_2456_amd import Group
    wls = [synth.water_like(2, W=40, n_det=600, n_moves=12),
           synth.tiny_system(21, 3, 3, 9, 150, W=33, n_moves=12)]
    ctxs = [make_ctx(w, bind=False, stream=stream) for w in wls]
    g = Group(ctxs, [w.walkers.W for w in wls])
    n_moves = 12
    inputs = []
    for k in range(n_moves):
        es, blks, masks = [], [], []
        for c, w in zip(ctxs, wls):
            e = int(w.moves.electron[k])
            # every move displaces the initial positions: inputs stay fixed
            r = w.walkers.pos[:, e] + w.moves.disp[k]
            es.append(e)
            blks.append(c.sgauss_eval(c.spin_of(e), dev(r)))
            masks.append(dev(w.moves.accept_half[k], torch.uint8))
        inputs.append((es, blks, masks))
    outs = [[(torch.zeros(w.walkers.W, dtype=torch.float64, device="cuda"),
              torch.zeros((w.walkers.W, 3), dtype=torch.float64, device="cuda"),
              torch.zeros(w.walkers.W, dtype=torch.float64, device="cuda"),
              torch.zeros(w.walkers.W, dtype=torch.int32, device="cuda")) for w in wls]
            for _ in range(n_moves)]

    def reinit():
        for c, w in zip(ctxs, wls):
            c.init(*gpu_orbitals(c, w.walkers.pos))

    def sweep():
        for k, (es, blks, masks) in enumerate(inputs):
            g.propose(es, blks, outs[k])
            g.accept(es, masks)

    def clear():
        for ok in outs:
            for o in ok:
                for x in o:
                    x.zero_()

    def snapshot():
        stream.synchronize()
        return [[x.cpu().numpy().copy() for o in ok for x in o] for ok in outs]

    reinit()
    sweep()
    eager = snapshot()
    assert any(np.abs(x).max() > 0 for a in eager for x in a)
    clear()
    reinit()
    stream.synchronize()
    with g.capture() as cap:
        sweep()
    for rep in range(2):
        clear()
        reinit()
        stream.synchronize()
        cap.graph.launch()
        got = snapshot()
        for a, b in zip(eager, got):
            for x, y in zip(a, b):
                assert np.array_equal(x, y), rep


def test_autograd_two_forwards_sharing_tables():
    """Two forwards through one context with the same tables and different
    coefficients: the first forward's backward must use its own
    coefficients."""
    from paper_1106_2456_amd import MultiDetLogPsi
    W = 64
    wl = synth.water_like(2, W=W, n_det=500)
    s = wl.system
    ctx = make_ctx(wl)
    rng = np.random.default_rng(8)
    Tu, Td = rng.normal(0, 0.6, (W, 5, 20)), rng.normal(0, 0.6, (W, 5, 20))
    c1 = s.coef.copy()
    c2 = s.coef * rng.uniform(0.5, 1.5, s.n_det)
    tu, td = dev(Tu).requires_grad_(True), dev(Td)
    k1 = dev(c1).requires_grad_(True)
    k2 = dev(c2).requires_grad_(True)
    la1, _ = MultiDetLogPsi.apply(ctx, k1, tu, td)
    la2, _ = MultiDetLogPsi.apply(ctx, k2, tu, td)
    la1.sum().backward()
    _, _, gc_o, gu_o, _ = oracle.tables(s, Tu, Td, coef=c1)
    e_c = np.abs(k1.grad.cpu().numpy() - gc_o.sum(0)).max() / np.abs(gc_o.sum(0)).max()
    e_t = np.abs(tu.grad.cpu().numpy() - gu_o).max() / np.abs(gu_o).max()
    assert e_c <= 1e-10 and e_t <= 1e-10, (e_c, e_t)
    del la2


def test_group_member_plan_change_rebuilds():
    """A member re-planned after the group was built (mde_set_plan + init):
    the group rebuilds its work items and still matches the member alone."""
    from paper_1106_2456_amd import Group
    wls = [synth.water_like(2, W=64, n_det=600, n_moves=2),
           synth.water_like(2, W=64, n_det=300, n_moves=2)]
    ctxs = [make_ctx(w, bind=False) for w in wls]
    g = Group(ctxs, [64, 64])
    for c, w in zip(ctxs, wls):
        c.init(*gpu_orbitals(c, w.walkers.pos))
    wt = ctxs[0].get_plan(0)["walker_tile"]
    item = ctxs[0].get_plan(0)["item_exc"]
    # coarser items: fewer than the workspace was sized for
    ctxs[0].set_plan(0, walker_tile=wt, item_exc=2 * item)
    ctxs[0].set_plan(1, walker_tile=wt, item_exc=2 * item)
    ctxs[0].init(*gpu_orbitals(ctxs[0], wls[0].walkers.pos))
    es = [int(w.moves.electron[0]) for w in wls]
    blks = [c.sgauss_eval(c.spin_of(e), dev(w.walkers.pos[:, e] + w.moves.disp[0]))
            for c, w, e in zip(ctxs, wls, es)]
    outs = [(torch.zeros(64, dtype=torch.float64, device="cuda"),
             torch.zeros((64, 3), dtype=torch.float64, device="cuda"),
             torch.zeros(64, dtype=torch.float64, device="cuda"),
             torch.zeros(64, dtype=torch.int32, device="cuda")) for _ in wls]
    g.propose(es, blks, outs)
    torch.cuda.synchronize()
    for c, w, e, o in zip(ctxs, wls, es, outs):
        ref = oracle.move(w.system, w.walkers.pos, e, w.walkers.pos[:, e] + w.moves.disp[0])
        err = scaled_err(o[0].cpu().numpy(), ref["ratio"], ref["scale_ratio"]).max()
        assert err <= 1e-10, err


def test_mixed_tile_group_tuned_and_captured():
    """Members of different walker tiles in one group (one launch per tile
    class inside each group call), equal to the oracle; after mde_group_tune
    (which re-evaluates the members from their orbitals) still equal to it."""
    from paper_1106_2456_amd import Group
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        wls = [synth.water_like(2, W=64, n_det=600, n_moves=8),
               synth.molecular(3, W=9, n_det=300, n_moves=8, n=12, m=40, nb=64, n_nuc=6, box=6.0),
               synth.molecular(3, W=5, n_det=200, n_moves=8, n=32, m=64, nb=96, n_nuc=8, box=8.0)]
        ctxs = [make_ctx(w, bind=False, stream=stream) for w in wls]
        g = Group(ctxs, [w.walkers.W for w in wls], common_tile=False)
        tiles = sorted({c.get_plan(0)["walker_tile"] for c in ctxs})
        say("mixed-tile group tiles", tiles)
        assert len(tiles) >= 2
        pos = [w.walkers.pos.copy() for w in wls]
        for c, p in zip(ctxs, pos):
            c.init(*gpu_orbitals(c, p))

        def step(k, check):
            es, blks, outs, masks, news = [], [], [], [], []
            for c, w, p in zip(ctxs, wls, pos):
                e = int(w.moves.electron[k])
                r = p[:, e] + w.moves.disp[k]
                es.append(e)
                news.append(r)
                blks.append(c.sgauss_eval(c.spin_of(e), dev(r)))
                outs.append((torch.zeros(c.W, dtype=torch.float64, device="cuda"),
                             torch.zeros((c.W, 3), dtype=torch.float64, device="cuda"),
                             torch.zeros(c.W, dtype=torch.float64, device="cuda"),
                             torch.zeros(c.W, dtype=torch.int32, device="cuda")))
                masks.append(dev(w.moves.accept_half[k], torch.uint8))
            g.propose(es, blks, outs)
            g.accept(es, masks)
            stream.synchronize()
            if check:
                for i, (w, p) in enumerate(zip(wls, pos)):
                    ref = oracle.move(w.system, p, es[i], news[i])
                    er = scaled_err(outs[i][0].cpu().numpy(), ref["ratio"], ref["scale_ratio"]).max()
                    eg = scaled_err(outs[i][1].cpu().numpy(), ref["grad"], ref["scale_grad"]).max()
                    assert er <= 1e-10 and eg <= 1e-10, (k, i, er, eg)
            for i, (w, p) in enumerate(zip(wls, pos)):
                acc = w.moves.accept_half[k].astype(bool)
                p[acc, es[i]] = news[i][acc]
            return es, blks

        for k in range(3):
            es, blks = step(k, True)
        g.tune(es, blks)
        say("after tune", [c.get_plan(0) for c in ctxs])
        # the tuner re-evaluates from the kept orbitals (the current positions)
        for k in range(3, 6):
            step(k, True)
