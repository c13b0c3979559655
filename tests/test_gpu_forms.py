"""GPU parity of the other forms: FP64 and mixed precision at n = 32
(small walker tiles, MFMA table GEMM), the adjoint (eval_tables/backward and
the autograd Function), uneven groups, and HIP-graph replay."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import (MIXED_TOL, dev, gpu_orbitals, make_ctx, output_errors, report_errors, say,
                        scaled_err)

pytestmark = pytest.mark.gpu


def _traj(wl, ctx, n_moves, precision, mask_key="accept_half"):
    s = wl.system
    pos = wl.walkers.pos.copy()
    ou, od = gpu_orbitals(ctx, pos)
    ctx.init(ou, od)
    scaled, plain = [], []
    masks = getattr(wl.moves, mask_key)
    n_tot = sum(s.n_elec)
    track = oracle.StoredTableErrors(s, pos) if precision != "fp64" else None
    for k in range(n_moves):
        e = int(wl.moves.electron[k])
        spin = 0 if e < s.n_elec[0] else 1
        new_r = pos[:, e] + wl.moves.disp[k]
        ratio, grad, lap, st = ctx.propose(e, ctx.sgauss_eval(spin, dev(new_r)))
        ctx.accept(e, dev(masks[k], torch.uint8))
        ref = oracle.move(s, pos, e, new_r)
        ms = track.scales(pos, e, new_r) if track else None
        a, b = output_errors(precision, (ratio.cpu().numpy(), grad.cpu().numpy(), lap.cpu().numpy()),
                             ref, ms)
        scaled.append(a)
        plain.append(b)
        assert np.all(st.cpu().numpy() == 0), (k, st)
        acc = masks[k].astype(bool)
        pos[acc, e] = new_r[acc]
        if track:
            track.commit(acc)
            if (k + 1) % n_tot == 0:     # the library's from-scratch refresh
                track.refresh(pos)
    return np.concatenate(scaled), np.concatenate(plain)


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_gemm", "mixed_gemm_ksum64"])
def test_molecular_n32(precision):
    """FP64: every sample within 1e-10 of the condition-aware scale.  The
    FP32-table forms: within 1e-5 of the first-order scale of FP32 table
    entries (rounded entries for the rank-one form, product-formed entries
    for the GEMM forms); the plain relative error is printed beside it."""
    wl = synth.molecular(3, W=6, n_det=1500, n_moves=40)
    ctx = make_ctx(wl, precision=precision)
    say(f"n=32 {precision} plan", ctx.get_plan(0))
    scaled, plain = _traj(wl, ctx, 40, precision)
    report_errors(f"n=32 {precision}", scaled, plain)
    tol = 1e-10 if precision == "fp64" else MIXED_TOL
    assert scaled.max() <= tol, (precision, scaled.max())


def test_adjoint_against_oracle_and_fd():
    from paper_1106_2456_amd import MultiDetLogPsi
    wl = synth.water_like(2, W=70, n_det=1500)
    s = wl.system
    ctx = make_ctx(wl)
    rng = np.random.default_rng(4)
    W = 70
    Tu = rng.normal(0, 0.6, (W, 5, 20))
    Td = rng.normal(0, 0.6, (W, 5, 20))
    go = rng.normal(0, 1, W)
    sg_o, la_o, gc_o, gu_o, gd_o = oracle.tables(s, Tu, Td)
    coef = dev(s.coef).requires_grad_(True)
    tu = dev(Tu).requires_grad_(True)
    td = dev(Td).requires_grad_(True)
    la, sg = MultiDetLogPsi.apply(ctx, coef, tu, td)
    assert np.allclose(sg.detach().cpu().numpy(), sg_o)
    assert np.abs(la.detach().cpu().numpy() - la_o).max() <= 1e-11 * (1 + np.abs(la_o).max())
    (la * dev(go)).sum().backward()
    gc = coef.grad.cpu().numpy()
    ref_gc = (go[:, None] * gc_o).sum(0)
    scale_gc = (np.abs(go[:, None] * gc_o)).sum(0) + 1e-300
    e_gc = (np.abs(gc - ref_gc) / scale_gc).max()
    e_gu = np.abs(tu.grad.cpu().numpy() - go[:, None, None] * gu_o).max() / np.abs(go[:, None, None] * gu_o).max()
    e_gd = np.abs(td.grad.cpu().numpy() - go[:, None, None] * gd_o).max() / np.abs(go[:, None, None] * gd_o).max()
    say(f"adjoint: grad_c {e_gc:.2e} grad_T_up {e_gu:.2e} grad_T_dn {e_gd:.2e}")
    assert e_gc <= 1e-10 and e_gu <= 1e-10 and e_gd <= 1e-10
    # central finite differences of the library's own forward (h = 1e-6)
    h = 1e-6
    for (w, r, p) in [(0, 0, 0), (3, 2, 7), (69, 4, 19)]:
        Tp, Tm = Tu.copy(), Tu.copy()
        Tp[w, r, p] += h
        Tm[w, r, p] -= h
        lp = ctx.eval_tables(dev(Tp), dev(Td), dev(s.coef))[0].cpu().numpy()[w]
        lm = ctx.eval_tables(dev(Tm), dev(Td), dev(s.coef))[0].cpu().numpy()[w]
        fd = (lp - lm) / (2 * h)
        assert abs(fd - gu_o[w, r, p]) <= 1e-6 * (1 + abs(fd))
    for I in [0, 5, 1499]:
        cp, cm = s.coef.copy(), s.coef.copy()
        cp[I] += h
        cm[I] -= h
        lp = ctx.eval_tables(dev(Tu), dev(Td), dev(cp))[0].cpu().numpy()
        lm = ctx.eval_tables(dev(Tu), dev(Td), dev(cm))[0].cpu().numpy()
        fd = ((lp - lm) / (2 * h) * go).sum()
        assert abs(fd - ref_gc[I]) <= 1e-6 * (1 + abs(fd))


def test_adjoint_deterministic():
    wl = synth.water_like(2, W=64, n_det=800)
    ctx = make_ctx(wl)
    rng = np.random.default_rng(5)
    Tu, Td = dev(rng.normal(0, 0.6, (64, 5, 20))), dev(rng.normal(0, 0.6, (64, 5, 20)))
    go = dev(rng.normal(0, 1, 64))
    outs = []
    for _ in range(2):
        ctx.eval_tables(Tu, Td, dev(wl.system.coef))
        outs.append([x.cpu().numpy() for x in ctx.backward(go)])
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


@pytest.mark.parametrize("by_tile, precision", [(False, "fp64"), (True, "fp64"), (True, "mixed")])
def test_group_matches_oracle_and_single_contexts(by_tile, precision):
    """Groups (one launch for all instances, or one per walker-tile size)
    equal each instance run alone with the same plan, bit for bit, and the
    oracle: FP64 within 1e-10 (condition-aware scale), the mixed form within
    1e-5 of the first-order FP32-entry scale."""
    from paper_1106_2456_amd import Group
    wls = [synth.water_like(2, W=40, n_det=600, n_moves=6),
           synth.tiny_system(21, 3, 3, 9, 150, W=33, n_moves=6),
           synth.molecular(3, W=5, n_det=300, n_moves=6, n=12, m=40, nb=64, n_nuc=6, box=6.0)]
    tol = 1e-10 if precision == "fp64" else MIXED_TOL
    ctxs = [make_ctx(w, precision=precision, bind=False) for w in wls]
    Ws = [w.walkers.W for w in wls]
    if by_tile:
        groups = Group.by_tile(ctxs, Ws)
    else:
        groups = [(Group(ctxs, Ws), list(range(len(ctxs))))]
    plans = [c.get_plan(0) for c in ctxs]
    say("group plans", plans)
    # twins with the same plan, run one at a time
    twins = [make_ctx(w, precision=precision, bind=False) for w in wls]
    for t, c, w in zip(twins, ctxs, wls):
        for sp in (0, 1):
            p = c.get_plan(sp)
            t.set_plan(sp, p["walker_tile"], p["item_exc"], p["threads"])
        t.bind(w.walkers.W)
    pos = [w.walkers.pos.copy() for w in wls]
    for c, t, w, p in zip(ctxs, twins, wls, pos):
        ou, od = gpu_orbitals(c, p)
        c.init(ou, od)
        t.init(ou, od)
    tracks = [oracle.StoredTableErrors(w.system, p) if precision != "fp64" else None
              for w, p in zip(wls, pos)]
    for k in range(6):
        es, news, outs, masks = [], [], [], []
        for i, (c, w, p) in enumerate(zip(ctxs, wls, pos)):
            e = int(w.moves.electron[k])
            es.append(e)
            news.append(c.sgauss_eval(c.spin_of(e), dev(p[:, e] + w.moves.disp[k])))
            outs.append((torch.empty(c.W, dtype=torch.float64, device="cuda"),
                         torch.empty((c.W, 3), dtype=torch.float64, device="cuda"),
                         torch.empty(c.W, dtype=torch.float64, device="cuda"),
                         torch.zeros(c.W, dtype=torch.int32, device="cuda")))
            masks.append(dev(w.moves.accept_half[k], torch.uint8))
        for grp, idx in groups:
            grp.propose([es[i] for i in idx], [news[i] for i in idx], [outs[i] for i in idx])
            grp.accept([es[i] for i in idx], [masks[i] for i in idx])
        for i, (t, w, p) in enumerate(zip(twins, wls, pos)):
            r1 = t.propose(es[i], news[i])
            t.accept(es[i], masks[i])
            for a, b in zip(outs[i][:3], r1[:3]):
                assert torch.equal(a, b), (k, i)
            new_r = p[:, es[i]] + w.moves.disp[k]
            ref = oracle.move(w.system, p, es[i], new_r)
            ms = tracks[i].scales(p, es[i], new_r) if tracks[i] else None
            sc, _ = output_errors(precision, tuple(o.cpu().numpy() for o in outs[i][:3]), ref, ms)
            assert sc.max() <= tol, (k, i, sc.max(axis=0))
            acc = w.moves.accept_half[k].astype(bool)
            p[acc, es[i]] = new_r[acc]
            if tracks[i]:
                tracks[i].commit(acc)
                if (k + 1) % sum(w.system.n_elec) == 0:
                    tracks[i].refresh(p)


def test_graph_replay_matches_eager():
    wl = synth.water_like(2, W=64, n_det=500, n_moves=10)
    s = wl.system
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        from paper_1106_2456_amd import Context
        ctxs = []
        for _ in range(2):
            c = Context(s.n_elec, s.n_orb, 64, max_order=4, stream=stream)
            c.set_expansion(s.exc[0], s.exc[1], s.coef, s.det_up, s.det_dn)
            for sp in (0, 1):
                c.set_basis(sp, s.centres, s.expo, s.mo_spin(sp))
            c.bind(64)
            ctxs.append(c)
        g_ctx, e_ctx = ctxs
        pos = wl.walkers.pos
        for c in ctxs:
            ou, od = gpu_orbitals(c, pos)
            c.init(ou, od)
        news = [g_ctx.sgauss_eval(g_ctx.spin_of(int(e)), dev(pos[:, int(e)] + wl.moves.disp[k]))
                for k, e in enumerate(wl.moves.electron[:10])]
        mask = dev(wl.moves.accept_half[0], torch.uint8)
        outs = [(torch.empty(64, dtype=torch.float64, device="cuda"),
                 torch.empty((64, 3), dtype=torch.float64, device="cuda"),
                 torch.empty(64, dtype=torch.float64, device="cuda"),
                 torch.zeros(64, dtype=torch.int32, device="cuda")) for _ in range(10)]
        stream.synchronize()
        with g_ctx.capture() as cap:
            for k, e in enumerate(wl.moves.electron[:10]):
                g_ctx.propose(int(e), news[k], outs[k])
                g_ctx.accept(int(e), mask)
        for rep in range(3):
            cap.graph.launch()
            stream.synchronize()
            for k, e in enumerate(wl.moves.electron[:10]):
                r = e_ctx.propose(int(e), news[k])
                e_ctx.accept(int(e), mask)
                for a, b in zip(outs[k][:3], r[:3]):
                    assert torch.equal(a, b), (rep, k)
            _ = torch.ones(10, device="cuda").sum().item()   # eager work between replays


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_profiled_repeats_leave_results_unchanged(precision):
    """A profiled proposal issues the determinant kernel several times back to
    back between its events; the results must equal an unprofiled twin's."""
    wl = synth.water_like(2, W=128, n_det=800, n_moves=4)
    s = wl.system
    ctxs = [make_ctx(wl, precision=precision) for _ in range(2)]
    pos = wl.walkers.pos.copy()
    for c in ctxs:
        ou, od = gpu_orbitals(c, pos)
        c.init(ou, od)
    ctxs[0].profile_enable(16, 4)
    for k in range(4):
        e = int(wl.moves.electron[k])
        no = ctxs[0].sgauss_eval(ctxs[0].spin_of(e), dev(pos[:, e] + wl.moves.disp[k]))
        mask = dev(wl.moves.accept_half[k], torch.uint8)
        r0 = ctxs[0].propose(e, no)
        r1 = ctxs[1].propose(e, no)
        for a, b in zip(r0[:3], r1[:3]):
            assert torch.equal(a, b), k
        for c in ctxs:
            c.accept(e, mask)
    torch.cuda.synchronize()
    ms, n = ctxs[0].profile_read()
    ctxs[0].profile_disable()
    say(f"{precision}: {n} profiled launches, {ms / max(n, 1) * 1e3:.1f} us each")
    assert n == 16 and ms > 0.0

