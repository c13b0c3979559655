"""The allocation-free entry point mde_local_derivs_noalloc, called through
the C ABI: two calls in a row (the second on a context with fewer walkers)
give the outputs of mde_local_derivs on the same state, and the oracle's."""
import ctypes as C

import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import gpu_orbitals, make_ctx, scaled_err

pytestmark = pytest.mark.gpu


def _call(fn, ctx, ou, od):
    W, nt = ctx.W, sum(ctx.n_elec)
    g = torch.full((W, nt, 3), float("nan"), dtype=torch.float64, device="cuda")
    lap = torch.full((W, nt), float("nan"), dtype=torch.float64, device="cuda")
    st = torch.zeros(W, dtype=torch.int32, device="cuda")
    rc = fn(ctx._h, C.c_void_p(ou.data_ptr()), C.c_void_p(od.data_ptr()), C.c_void_p(g.data_ptr()),
            C.c_void_p(lap.data_ptr()), C.c_void_p(st.data_ptr()))
    assert rc == 0, rc
    torch.cuda.synchronize()
    return g.cpu().numpy(), lap.cpu().numpy(), st.cpu().numpy()


def test_noalloc_matches_workspace_variant():
    from paper_1106_2456_amd import lib
    L = lib()
    for W in (70, 23):
        wl = synth.water_like(2, W=W, n_det=900, n_moves=3)
        s = wl.system
        ctx = make_ctx(wl)
        pos = wl.walkers.pos.copy()
        ou, od = gpu_orbitals(ctx, pos)
        ctx.init(ou, od)
        g0, l0, s0 = _call(L.mde_local_derivs, ctx, ou, od)
        g1, l1, s1 = _call(L.mde_local_derivs_noalloc, ctx, ou, od)
        assert not s0.any() and not s1.any()
        assert np.array_equal(g0, g1) and np.array_equal(l0, l1), W
        for e in (0, 9):
            rg, rl, sg, sl = oracle.grad_lap(s, pos, e, scales=True)
            assert scaled_err(g1[:, e], rg, sg).max() <= 1e-10
            assert scaled_err(l1[:, e], rl, sl).max() <= 1e-10
