"""Stability remedies of the paper's Sec. V on the GPU: reference switching
(mde_set_reference) and the proposal read through the bordered determinant
(the generalized determinant lemma, never dividing by det A'/det A).

Walkers are placed on the node of the up reference determinant by bisection
of its sign along a line (host side, with the oracle's orbitals): there the
table of the original reference has entries of order 1/det A, and the
rebased context, whose reference is a determinant that does not vanish
there, keeps full accuracy."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_1106_2456_amd._lib import ST_REF_ILLCOND
from tests._gpu import dev, gpu_orbitals, make_ctx, say, scaled_err

pytestmark = pytest.mark.gpu


def _ref_det(s, pos_w, e, r):
    """det of the up reference matrix of one walker with electron e at r."""
    p = pos_w[: s.n_elec[0]].copy()
    p[e] = r
    A = oracle.orbitals(s, 0, p)[:, 0, : s.n_elec[0]]
    return np.linalg.det(A)


def _node_point(s, pos_w, e, direction, t_max=2.0, offset=1e-11):
    """A point r_e + t d within `offset` bohr of the node of the up reference
    determinant (not on it: the oracle takes logarithms of determinants)."""
    f = lambda t: _ref_det(s, pos_w, e, pos_w[e] + t * direction)  # noqa: E731
    ts = np.linspace(-t_max, t_max, 81)
    vals = [f(t) for t in ts]
    for a, b, fa, fb in zip(ts[:-1], ts[1:], vals[:-1], vals[1:]):
        if fa == 0.0:
            return pos_w[e] + (a + offset) * direction
        if np.sign(fa) != np.sign(fb):
            for _ in range(70):
                mid = 0.5 * (a + b)
                fm = f(mid)
                if fm == 0.0 or b - a < 1e-16:
                    break
                if np.sign(fm) == np.sign(fa):
                    a, fa = mid, fm
                else:
                    b = mid
            return pos_w[e] + (0.5 * (a + b) + offset) * direction
    return None


def _near_node_positions(s, pos, e, rng):
    out = pos.copy()
    for w in range(pos.shape[0]):
        for _ in range(20):
            d = rng.normal(size=3)
            d /= np.linalg.norm(d)
            r = _node_point(s, pos[w], e, d)
            if r is not None:
                out[w, e] = r
                break
        else:
            raise RuntimeError("no node found")
    return out


def _traj_check(ctx, s, pos, moves, tol, tag):
    worst = 0.0
    for e, disp, mask in moves:
        new_r = pos[:, e] + disp
        ratio, grad, lap, st = ctx.propose(e, ctx.sgauss_eval(ctx.spin_of(e), dev(new_r)))
        ctx.accept(e, dev(mask, torch.uint8))
        ref = oracle.move(s, pos, e, new_r)
        er = scaled_err(ratio.cpu().numpy(), ref["ratio"], ref["scale_ratio"]).max()
        eg = scaled_err(grad.cpu().numpy(), ref["grad"], ref["scale_grad"]).max()
        el = scaled_err(lap.cpu().numpy(), ref["lap"], ref["scale_lap"]).max()
        worst = max(worst, er, eg, el)
        assert er <= tol and eg <= tol and el <= tol, (tag, e, er, eg, el)
        acc = mask.astype(bool)
        pos[acc, e] = new_r[acc]
    say(f"{tag}: worst scaled error {worst:.2e}")


def test_rebased_context_matches_oracle():
    """A context whose reference is another determinant (a double up, a
    single down) gives the caller's Psi, ratios, derivatives and
    all-electron derivatives."""
    wl = synth.water_like(2, W=40, n_det=600, n_moves=12)
    s = wl.system
    ex_u, ex_d = s.exc
    ref_up = next(u for u in range(ex_u.n_exc) if ex_u.order(u) == 2)
    ref_dn = next(u for u in range(ex_d.n_exc) if ex_d.order(u) == 1)
    ctx = make_ctx(wl, max_order=8, bind=False)
    ctx.set_reference(ref_up, ref_dn)
    ctx.bind(40)
    pos = wl.walkers.pos.copy()
    la, sg, st = ctx.init(*gpu_orbitals(ctx, pos))
    ref_s, ref_l = oracle.log_psi(s, pos)
    assert np.abs(la.cpu().numpy() - ref_l).max() <= 1e-10 * np.abs(ref_l).max()
    assert np.array_equal(sg.cpu().numpy(), ref_s)
    moves = [(int(wl.moves.electron[k]), wl.moves.disp[k], wl.moves.accept_half[k]) for k in range(12)]
    _traj_check(ctx, s, pos, moves, 1e-10, "rebased (double up, single down)")
    g, lap, st = ctx.local_derivs(*gpu_orbitals(ctx, pos))
    for e in (0, 7):
        rg, rl, sgs, sls = oracle.grad_lap(s, pos, e, scales=True)
        assert scaled_err(g.cpu().numpy()[:, e], rg, sgs).max() <= 1e-10
        assert scaled_err(lap.cpu().numpy()[:, e], rl, sls).max() <= 1e-10


def test_reference_switch_on_the_reference_node():
    wl = synth.water_like(2, W=16, n_det=600, n_moves=6)
    s = wl.system
    rng = np.random.default_rng(12)
    pos = _near_node_positions(s, wl.walkers.pos, 4, rng)
    ou, od = oracle.walker_orbitals(s, pos)
    rel_det = np.array([abs(np.linalg.det(o[:, 0, :5])) / np.prod(np.linalg.norm(o[:, 0, :5], axis=1))
                        for o in ou])
    say(f"reference determinant / Hadamard bound on the node: max {rel_det.max():.1e}")
    ref_s, ref_l = oracle.log_psi(s, pos)
    plain = make_ctx(wl)
    la, sg, st = plain.init(*gpu_orbitals(plain, pos))
    st = st.cpu().numpy()
    assert np.all(st & ST_REF_ILLCOND), st
    err_plain = np.abs(la.cpu().numpy() - ref_l) / np.abs(ref_l)
    say(f"original reference on its node: log|Psi| relative error max {err_plain.max():.1e}")
    # the new reference: the up excitation whose ratio to the vanishing
    # reference is largest for the worst walker
    R = np.abs(plain.export("ratios", 0).cpu().numpy())
    ref_up = int(np.argmax(R[:, 1:].min(axis=0))) + 1
    rebased = make_ctx(wl, max_order=8, bind=False)
    rebased.set_reference(ref_up, 0)
    rebased.bind(16)
    la, sg, st = rebased.init(*gpu_orbitals(rebased, pos))
    st = st.cpu().numpy()
    assert not (st & ST_REF_ILLCOND).any()
    err = np.abs(la.cpu().numpy() - ref_l) / np.abs(ref_l)
    say(f"switched reference (up excitation {ref_up}): log|Psi| relative error max {err.max():.1e}")
    assert err.max() <= 1e-10
    assert np.array_equal(sg.cpu().numpy(), ref_s)
    moves = [(int(wl.moves.electron[k]), wl.moves.disp[k], wl.moves.accept[k]) for k in range(6)]
    _traj_check(rebased, s, pos.copy(), moves, 1e-10, "switched reference, moves off the node")


def test_proposal_onto_the_reference_node():
    """A proposal that lands on the node of the reference determinant
    (det A'/det A ~ 0): ratio, gradient and laplacian are read through the
    bordered determinants, with nothing divided by det A'/det A, and keep
    full accuracy."""
    wl = synth.water_like(2, W=16, n_det=600, n_moves=2)
    s = wl.system
    pos = wl.walkers.pos.copy()
    rng = np.random.default_rng(3)
    target = _near_node_positions(s, pos, 4, rng)
    ctx = make_ctx(wl)
    ctx.init(*gpu_orbitals(ctx, pos))
    new_r = target[:, 4]
    ratio, grad, lap, st = ctx.propose(4, ctx.sgauss_eval(0, dev(new_r)))
    ref = oracle.move(s, pos, 4, new_r)
    er = scaled_err(ratio.cpu().numpy(), ref["ratio"], ref["scale_ratio"]).max()
    eg = scaled_err(grad.cpu().numpy(), ref["grad"], ref["scale_grad"]).max()
    el = scaled_err(lap.cpu().numpy(), ref["lap"], ref["scale_lap"]).max()
    say(f"proposal onto the reference node: ratio {er:.1e} grad {eg:.1e} lap {el:.1e}")
    assert er <= 1e-10 and eg <= 1e-10 and el <= 1e-10
