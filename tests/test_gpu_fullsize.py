"""Parity at the full sizes of the five workloads, in the launch
configurations the benchmark uses, on sampled outputs the oracle computes one
walker at a time:

* water-like batched (5+5 electrons, 10 000 determinants, 4 096 walkers, FP64),
  one full sweep with the autotuned plan, 32 walkers spread over the tiles;
* molecular-shaped (n = 32, m = 224, 100 000 determinants, 2 048 walkers),
  FP64 and the three FP32-table forms, 32 walkers x 10 moves against stored
  oracle values;
* the adjoint on the water-like system (1 024 walkers, FP64), every walker;
* the uneven batch (64 instances, n = 5..64, m = 4n, 10^2..2*10^5
  determinants, 256 walkers each) in one group launch, FP64, sampled
  (instance, walker) pairs.

Gates as in the other parity tests: FP64 1e-10 under the condition-aware
scale; FP32-table forms 1e-5 under the first-order FP32-entry scale."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import (MIXED_TOL, dev, gpu_orbitals, make_ctx, output_errors, report_errors, say,
                        scaled_err)

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _check_move(s, pos_sample, e, new_sample, got, tol, tag):
    ratio, grad, lap = got
    ref = oracle.move(s, pos_sample, e, new_sample)
    er = scaled_err(ratio, ref["ratio"], ref["scale_ratio"]).max()
    eg = scaled_err(grad, ref["grad"], ref["scale_grad"]).max()
    el = scaled_err(lap, ref["lap"], ref["scale_lap"]).max()
    say(f"  {tag}: ratio {er:.2e} grad {eg:.2e} lap {el:.2e}")
    assert er <= tol and eg <= tol and el <= tol, (tag, er, eg, el)
    return max(er, eg, el)


def test_water_batched_full_size():
    wl = synth.water_like(2, W=4096, n_moves=10)
    s = wl.system
    W = wl.walkers.W
    n_tot = sum(s.n_elec)
    ctx = make_ctx(wl, refresh_every=n_tot)
    pos = wl.walkers.pos.copy()
    ou, od = gpu_orbitals(ctx, pos)
    nu = s.n_elec[0]
    up = ctx.sgauss_eval(0, dev(pos[:, 0] + wl.moves.disp[0]))
    dn = ctx.sgauss_eval(1, dev(pos[:, nu] + wl.moves.disp[nu]))
    ctx.init(ou, od)
    ctx.autotune(up, dn)
    say("plan", ctx.get_plan(0), ctx.get_plan(1))
    ctx.init(ou, od)
    sample = np.unique(np.concatenate([np.arange(0, W, 131), [63, 64, W - 1]]))
    for k in range(n_tot):
        e = int(wl.moves.electron[k])
        sp = ctx.spin_of(e)
        new_r = pos[:, e] + wl.moves.disp[k]
        ratio, grad, lap, st = ctx.propose(e, ctx.sgauss_eval(sp, dev(new_r)))
        mask = wl.moves.accept_half[k]
        ctx.accept(e, dev(mask, torch.uint8))
        assert np.all(st.cpu().numpy() == 0)
        got = (ratio.cpu().numpy()[sample], grad.cpu().numpy()[sample], lap.cpu().numpy()[sample])
        _check_move(s, pos[sample].copy(), e, new_r[sample], got, 1e-10, f"move {k} e={e}")
        acc = mask.astype(bool)
        pos[acc, e] = new_r[acc]


def _golden_module():
    import importlib.util
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "make_molecular_sample.py")
    spec = importlib.util.spec_from_file_location("make_molecular_sample", path)
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.parametrize("precision", ["fp64", "mixed", "mixed_gemm", "mixed_gemm_ksum64"])
def test_molecular_full_size(precision):
    """n = 32, m = 224, 100 000 determinants, 2 048 walkers, default launch
    plan: 10 moves alternating the spins, 32 sampled walkers (one per
    64-walker tile) against the oracle's stored values
    (tests/golden/molecular_n32_sample.npz, written by the oracle alone)."""
    gm = _golden_module()
    wl, g = gm.load()
    assert str(g["fingerprint"]) == gm.fingerprint(wl), "generator drifted: rewrite the golden file"
    s = wl.system
    ctx = make_ctx(wl, precision=precision)
    say(f"n=32 full size {precision} plan", ctx.get_plan(0), ctx.get_plan(1))
    pos = wl.walkers.pos.copy()
    ctx.init(*gpu_orbitals(ctx, pos))
    sample = g["sample"]
    scaled_all, plain_all = [], []
    for k, e in enumerate(g["electrons"]):
        e = int(e)
        new_r = pos[:, e] + wl.moves.disp[k]
        ratio, grad, lap, st = ctx.propose(e, ctx.sgauss_eval(ctx.spin_of(e), dev(new_r)))
        mask = wl.moves.accept_half[k]
        ctx.accept(e, dev(mask, torch.uint8))
        assert not st.cpu().numpy()[sample].any()
        ref = dict(ratio=g["ratio"][k], grad=g["grad"][k], lap=g["lap"][k],
                   scale_ratio=g["sc_ratio"][k], scale_grad=g["sc_grad"][k], scale_lap=g["sc_lap"][k])
        ms = dict(round=g["x_round"][k], gemm=g["x_gemm"][k])
        got = (ratio.cpu().numpy()[sample], grad.cpu().numpy()[sample], lap.cpu().numpy()[sample])
        sc, pl = output_errors(precision, got, ref, ms)
        scaled_all.append(sc)
        plain_all.append(pl)
        acc = mask.astype(bool)
        pos[acc, e] = new_r[acc]
    scaled_all = np.concatenate(scaled_all)
    plain_all = np.concatenate(plain_all)
    report_errors(f"n=32 full size {precision}", scaled_all, plain_all)
    tol = 1e-10 if precision == "fp64" else MIXED_TOL
    assert scaled_all.max() <= tol, (precision, scaled_all.max(axis=0))


def test_adjoint_full_size():
    from paper_1106_2456_amd import MultiDetLogPsi
    wl = synth.water_like(2, W=1024)
    s = wl.system
    ctx = make_ctx(wl)
    ou, od = gpu_orbitals(ctx, wl.walkers.pos)
    ctx.init(ou, od)
    # the walkers' own tables
    Tu = ctx.export("table", 0).cpu().numpy()
    Td = ctx.export("table", 1).cpu().numpy()
    go = np.random.default_rng(44).normal(0, 1, 1024)
    coef = dev(s.coef).requires_grad_(True)
    tu = dev(Tu).requires_grad_(True)
    td = dev(Td).requires_grad_(True)
    la, sg = MultiDetLogPsi.apply(ctx, coef, tu, td)
    (la * dev(go)).sum().backward()
    sg_o, la_o, gc_o, gu_o, gd_o = oracle.tables(s, Tu, Td)
    assert np.array_equal(sg.detach().cpu().numpy(), sg_o)
    e_la = np.abs(la.detach().cpu().numpy() - la_o).max()
    ref_gc = (go[:, None] * gc_o).sum(0)
    scale_gc = np.abs(go[:, None] * gc_o).sum(0) + 1e-300
    e_gc = (np.abs(coef.grad.cpu().numpy() - ref_gc) / scale_gc).max()
    e_gu = np.abs(tu.grad.cpu().numpy() - go[:, None, None] * gu_o).max() / np.abs(go[:, None, None] * gu_o).max()
    e_gd = np.abs(td.grad.cpu().numpy() - go[:, None, None] * gd_o).max() / np.abs(go[:, None, None] * gd_o).max()
    say(f"adjoint full size: log|N| {e_la:.2e} grad_c {e_gc:.2e} grad_T_up {e_gu:.2e} grad_T_dn {e_gd:.2e}")
    assert e_la <= 1e-11 * (1 + np.abs(la_o).max())
    assert e_gc <= 1e-10 and e_gu <= 1e-10 and e_gd <= 1e-10


def test_uneven_group_full_size():
    from paper_1106_2456_amd import Group
    say("generating 64 instances")
    wls = synth.uneven_instances(W=256, n_moves=1)
    ctxs = [make_ctx(w, bind=False) for w in wls]
    grp = Group(ctxs, [256] * len(wls))
    say("group plan", ctxs[0].get_plan(0), "instances", len(ctxs))
    pos = [w.walkers.pos.copy() for w in wls]
    for c, p in zip(ctxs, pos):
        ou, od = gpu_orbitals(c, p)
        c.init(ou, od)
    es, news, outs, masks, new_r = [], [], [], [], []
    for c, w, p in zip(ctxs, wls, pos):
        e = int(w.moves.electron[0])
        es.append(e)
        r = p[:, e] + w.moves.disp[0]
        new_r.append(r)
        news.append(c.sgauss_eval(c.spin_of(e), dev(r)))
        outs.append((torch.empty(256, dtype=torch.float64, device="cuda"),
                     torch.empty((256, 3), dtype=torch.float64, device="cuda"),
                     torch.empty(256, dtype=torch.float64, device="cuda"),
                     torch.zeros(256, dtype=torch.int32, device="cuda")))
        masks.append(dev(w.moves.accept_half[0], torch.uint8))
    grp.propose(es, news, outs)
    grp.accept(es, masks)
    torch.cuda.synchronize()
    ns = np.array([w.meta["n"] for w in wls])
    nd = np.array([w.system.n_det for w in wls])
    picks = sorted(set([int(np.argmin(ns)), int(np.argmax(ns)), int(np.argmin(nd)), int(np.argmax(nd)), 7, 40]))
    for i in picks:
        w = wls[i]
        wsel = np.array([0, 255]) if nd[i] < 20000 else np.array([100])
        got = tuple(o.cpu().numpy()[wsel] for o in outs[i][:3])
        assert np.all(outs[i][3].cpu().numpy() == 0)
        _check_move(w.system, pos[i][wsel].copy(), es[i], new_r[i][wsel], got, 1e-10,
                    f"instance {i} n={ns[i]} ndet={nd[i]}")
