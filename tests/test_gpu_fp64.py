"""FP64 path on the GPU vs the CPU oracle (parity).  Every comparison is
element by element on the same seeded inputs; the gate for a ratio of sums
x = sum(a)/sum(b) is |dx| <= tol * (sum|a| + |x| sum|b|)/|sum b| (equals
tol*|x| when nothing cancels), tol = 1e-10."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import dev, gpu_orbitals, make_ctx, say, scaled_err

pytestmark = pytest.mark.gpu
TOL = 1e-10


def test_orbital_provider_matches_oracle():
    wl = synth.water_like(1, W=3, n_det=20)
    ctx = make_ctx(wl)
    ou, od = gpu_orbitals(ctx, wl.walkers.pos)
    ru, rd = oracle.walker_orbitals(wl.system, wl.walkers.pos)
    for g, r in ((ou, ru), (od, rd)):
        g = g.cpu().numpy()
        assert np.abs(g - r).max() <= 1e-13 * max(1.0, np.abs(r).max())


@pytest.mark.parametrize("W,n_det", [(1, 200), (7, 300), (70, 400)])
def test_init_logpsi_and_ratios(W, n_det):
    say(f"init W={W} n_det={n_det}")
    wl = synth.water_like(1, W=W, n_det=n_det)
    s = wl.system
    ctx = make_ctx(wl)
    ou, od = gpu_orbitals(ctx, wl.walkers.pos)
    la, sg, st = ctx.init(ou, od)
    torch.cuda.synchronize()
    rou, rod = oracle.walker_orbitals(s, wl.walkers.pos)
    r = oracle.mds(s, rou, rod, ratios=True)
    ref_la = np.log(np.abs(r["psi"])) + r["shift"]
    assert np.all(st.cpu().numpy() == 0)
    assert np.all(sg.cpu().numpy() == np.sign(r["psi"]))
    # log|Psi| error in absolute terms ~ relative error of Psi
    scale = r["psi_abs"] / np.abs(r["psi"])
    assert np.all(np.abs(la.cpu().numpy() - ref_la) <= TOL * scale)
    for spin, key in ((0, "ratio_up"), (1, "ratio_dn")):
        g = ctx.export("ratios", spin).cpu().numpy()
        ref = r[key]
        sc = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max(axis=1, keepdims=True))
        err = np.abs(g - ref) / sc
        say(f"  spin {spin}: max scaled ratio error {err.max():.2e}")
        assert err.max() <= TOL
        B = ctx.export("inverse", spin).cpu().numpy()
        n = s.n_elec[spin]
        A = (rou, rod)[spin][:, :, 0, :n]
        for w in range(min(W, 5)):
            assert np.abs(B[w] @ A[w] - np.eye(n)).max() <= 1e-12 * np.linalg.cond(A[w])


def _run_trajectory(wl, n_moves, mask_key, ctx, check_every=1):
    s = wl.system
    pos = wl.walkers.pos.copy()
    ou, od = gpu_orbitals(ctx, pos)
    ctx.init(ou, od)
    worst = {"ratio": 0.0, "grad": 0.0, "lap": 0.0}
    mask_all = getattr(wl.moves, mask_key)
    for k in range(n_moves):
        e = int(wl.moves.electron[k])
        spin = 0 if e < s.n_elec[0] else 1
        new_r = pos[:, e] + wl.moves.disp[k]
        no = ctx.sgauss_eval(spin, dev(new_r))
        ratio, grad, lap, st = ctx.propose(e, no)
        mask = mask_all[k]
        ctx.accept(e, dev(mask, torch.uint8))
        if k % check_every == 0:
            ref = oracle.move(s, pos, e, new_r)
            er = scaled_err(ratio.cpu().numpy(), ref["ratio"], ref["scale_ratio"]).max()
            eg = scaled_err(grad.cpu().numpy(), ref["grad"], ref["scale_grad"]).max()
            el = scaled_err(lap.cpu().numpy(), ref["lap"], ref["scale_lap"]).max()
            worst["ratio"] = max(worst["ratio"], er)
            worst["grad"] = max(worst["grad"], eg)
            worst["lap"] = max(worst["lap"], el)
            assert np.all(st.cpu().numpy() == 0), (k, st)
            assert er <= TOL and eg <= TOL and el <= TOL, (k, e, er, eg, el)
        acc = mask.astype(bool)
        pos[acc, e] = new_r[acc]
    return worst, pos


@pytest.mark.parametrize("mask_key", ["accept", "accept_half"])
def test_trajectory_water_single_walker(mask_key):
    wl = synth.water_like(1, W=1, n_moves=200)
    ctx = make_ctx(wl)
    worst, pos = _run_trajectory(wl, 200, mask_key, ctx)
    say(f"cfg1 W=1 200 moves ({mask_key}): worst scaled errors {worst}")


def test_trajectory_batched_walkers_and_state():
    wl = synth.water_like(2, W=96, n_det=2000, n_moves=25)
    ctx = make_ctx(wl)
    worst, pos = _run_trajectory(wl, 25, "accept_half", ctx)
    say(f"batched W=96 n_det=2000 25 moves: {worst}")
    # state after the moves: inverse and log det vs fresh LU of the final positions
    rou, rod = oracle.walker_orbitals(wl.system, pos)
    for spin, orb in ((0, rou), (1, rod)):
        n = wl.system.n_elec[spin]
        B = ctx.export("inverse", spin).cpu().numpy()
        ld = ctx.export("logdet", spin).cpu().numpy()
        for w in range(0, 96, 17):
            A = orb[w, :, 0, :n]
            assert np.abs(B[w] @ A - np.eye(n)).max() <= 1e-11 * np.linalg.cond(A)
            assert abs(ld[w] - np.linalg.slogdet(A)[1]) <= 1e-11 * np.linalg.cond(A)
    # the CI sum N = Psi / (D0_up D0_dn): the periodic FP64 refreshes (after
    # moves 10 and 20) keep the N of the moves instead of re-summing it
    r = oracle.mds(wl.system, rou, rod)
    scale = np.exp(r["shift"] - r["log0"][:, 0] - r["log0"][:, 1])
    n_ref = r["psi"] * r["sign0"][:, 0] * r["sign0"][:, 1] * scale
    n_abs = r["psi_abs"] * scale
    n_gpu = ctx.export("N").cpu().numpy()
    err = (np.abs(n_gpu - n_ref) / n_abs).max()
    say(f"N after 25 moves: scaled error {err:.2e}")
    assert err <= 1e-10


@pytest.mark.parametrize("n", [1, 2, 4, 6, 8])
def test_refresh_state_small_spins(n):
    """The refresh of spins with at most 8 electrons (eight lanes per walker,
    pivoting across the lane group): inverse, log|det| and table after a
    commit and its refresh, 70 walkers (a partial second tile), against a
    fresh LU of the final positions."""
    wl = synth.tiny_system(40 + n, n, n, 6, 60, W=70, n_moves=2)
    ctx = make_ctx(wl, refresh_every=1)
    pos = wl.walkers.pos.copy()
    ou, od = gpu_orbitals(ctx, pos)
    ctx.init(ou, od)
    e = int(wl.moves.electron[0])
    new_r = pos[:, e] + wl.moves.disp[0]
    ctx.propose(e, ctx.sgauss_eval(ctx.spin_of(e), dev(new_r)))
    mask = wl.moves.accept_half[0]
    ctx.accept(e, dev(mask, torch.uint8))      # refresh after every commit
    acc = mask.astype(bool)
    pos[acc, e] = new_r[acc]
    rou, rod = oracle.walker_orbitals(wl.system, pos)
    worst = 0.0
    for spin, orb in ((0, rou), (1, rod)):
        B = ctx.export("inverse", spin).cpu().numpy()
        ld = ctx.export("logdet", spin).cpu().numpy()
        T = ctx.export("table", spin).cpu().numpy()
        for w in range(wl.walkers.W):
            A = orb[w, :, 0, :n]
            cond = np.linalg.cond(A)
            ref_T = np.linalg.solve(A, orb[w, :, 0, n:])
            e_B = np.abs(B[w] @ A - np.eye(n)).max()
            e_ld = abs(ld[w] - np.linalg.slogdet(A)[1])
            e_T = np.abs(T[w] - ref_T).max() / (1.0 + np.abs(ref_T).max())
            worst = max(worst, e_B / cond, e_ld / cond, e_T / cond)
            assert e_B <= 1e-11 * cond and e_ld <= 1e-11 * cond and e_T <= 1e-11 * cond, (spin, w)
    say(f"n={n}: refresh state, worst condition-scaled error {worst:.2e}")


def test_sizing_query_after_bind_keeps_state():
    """Regression: a workspace-size query on a bound context must not touch
    its device descriptors (it once replaced them with null pointers)."""
    wl = synth.water_like(1, W=4, n_det=120, n_moves=3)
    ctx = make_ctx(wl)
    assert ctx.workspace_bytes(4) > 0
    pos = wl.walkers.pos.copy()
    ou, od = gpu_orbitals(ctx, pos)
    la, sg, st = ctx.init(ou, od)
    e = int(wl.moves.electron[0])
    new_r = pos[:, e] + wl.moves.disp[0]
    ratio, grad, lap, st = ctx.propose(e, ctx.sgauss_eval(0, dev(new_r)))
    ref = oracle.move(wl.system, pos, e, new_r)
    assert scaled_err(ratio.cpu().numpy(), ref["ratio"], ref["scale_ratio"]).max() <= TOL
