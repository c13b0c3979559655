"""GPU parity of the all-electron derivatives (mde_local_derivs): every
electron's grad ln Psi and lap Psi / Psi at the current positions against
the oracle's row-replacement LUs, after init and after committed moves (a
from-scratch refresh among them), on 64-walker tiles and on small tiles;
and agreement with the per-electron mde_grad_lap."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import dev, gpu_orbitals, make_ctx, say, scaled_err

pytestmark = pytest.mark.gpu


def _all_electrons(ctx, s, pos):
    ou, od = gpu_orbitals(ctx, pos)
    g, lap, st = ctx.local_derivs(ou, od)
    return g.cpu().numpy(), lap.cpu().numpy(), st.cpu().numpy()


def _compare(s, pos, g, lap, tag):
    worst = 0.0
    for e in range(sum(s.n_elec)):
        rg, rl, sg, sl = oracle.grad_lap(s, pos, e, scales=True)
        eg = scaled_err(g[:, e], rg, sg).max()
        el = scaled_err(lap[:, e], rl, sl).max()
        worst = max(worst, eg, el)
        assert eg <= 1e-10 and el <= 1e-10, (tag, e, eg, el)
    say(f"local derivs {tag}: worst scaled error {worst:.2e}")


@pytest.mark.parametrize("case", ["water", "molecular12", "molecular32"])
def test_local_derivs_match_oracle(case):
    if case == "water":
        wl = synth.water_like(2, W=70, n_det=1500, n_moves=12)
    elif case == "molecular12":
        wl = synth.molecular(3, W=9, n_det=400, n_moves=30, n=12, m=40, nb=64, n_nuc=6, box=6.0)
    else:
        wl = synth.molecular(3, W=6, n_det=1500, n_moves=12)
    s = wl.system
    ctx = make_ctx(wl)
    say(f"{case} plan", ctx.get_plan(0))
    pos = wl.walkers.pos.copy()
    ctx.init(*gpu_orbitals(ctx, pos))
    g, lap, st = _all_electrons(ctx, s, pos)
    assert not st.any()
    _compare(s, pos, g, lap, f"{case} init")
    n_tot = sum(s.n_elec)
    n_moves = min(12, wl.moves.disp.shape[0]) if case != "molecular12" else 30
    for k in range(n_moves):
        e = int(wl.moves.electron[k])
        new_r = pos[:, e] + wl.moves.disp[k]
        ctx.propose(e, ctx.sgauss_eval(ctx.spin_of(e), dev(new_r)))
        mask = wl.moves.accept_half[k]
        ctx.accept(e, dev(mask, torch.uint8))
        pos[mask.astype(bool), e] = new_r[mask.astype(bool)]
    assert n_moves >= min(n_tot, 12)
    g, lap, st = _all_electrons(ctx, s, pos)
    assert not st.any()
    _compare(s, pos, g, lap, f"{case} after {n_moves} moves")
    # the same quantity one electron at a time
    for e in (0, n_tot - 1):
        cur = ctx.sgauss_eval(ctx.spin_of(e), dev(pos[:, e]))
        g1, l1, _ = ctx.grad_lap(e, cur)
        assert np.allclose(g1.cpu().numpy(), g[:, e], rtol=1e-9, atol=1e-12)
        assert np.allclose(l1.cpu().numpy(), lap[:, e], rtol=1e-9, atol=1e-12)
