"""GPU parity of the on-device Metropolis loop with drift (mde_vmc) against
the same loop driven on the host with the oracle: identical accept/reject
decisions for every move and the same final positions, with the random
numbers given to both sides."""
import numpy as np
import pytest
import torch

import oracle
import synth
from tests._gpu import dev, gpu_orbitals, make_ctx, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64"])
def test_vmc_loop_matches_host_oracle_loop(precision):
    W, n_steps, tau = 32, 2, 0.05
    wl = synth.water_like(2, W=W, n_det=600, n_moves=1)
    s = wl.system
    n_tot = sum(s.n_elec)
    rng = np.random.default_rng(2024)
    chi = rng.standard_normal((n_steps, n_tot, W, 3))
    u = rng.random((n_steps, n_tot, W))
    ctx = make_ctx(wl, precision=precision)
    pos0 = wl.walkers.pos.copy()
    ctx.init(*gpu_orbitals(ctx, pos0))
    pos = dev(pos0)
    acc = torch.zeros(W, dtype=torch.int32, device="cuda")
    st = ctx.vmc(n_steps, tau, dev(chi), dev(u), pos, acc)
    torch.cuda.synchronize()
    assert not st.cpu().numpy().any()
    # the same loop on the host, every quantity from the oracle
    p = pos0.copy()
    acc_ref = np.zeros(W, np.int64)
    for step in range(n_steps):
        for e in range(n_tot):
            g0, _ = oracle.grad_lap(s, p, e)
            cur = p[:, e].copy()
            newp = cur + tau * g0 + np.sqrt(tau) * chi[step, e]
            ref = oracle.move(s, p, e, newp)
            fwd = ((newp - cur - tau * g0) ** 2).sum(1)
            rev = ((cur - newp - tau * ref["grad"]) ** 2).sum(1)
            prob = ref["ratio"] ** 2 * np.exp((fwd - rev) / (2 * tau))
            a = u[step, e] < prob
            p[a, e] = newp[a]
            acc_ref += a
    got = acc.cpu().numpy()
    say(f"vmc: {got.sum()} of {W * n_steps * n_tot} moves accepted (oracle loop {acc_ref.sum()})")
    assert np.array_equal(got, acc_ref)
    dp = np.abs(pos.cpu().numpy() - p).max()
    say(f"vmc: final positions differ by at most {dp:.1e} bohr")
    assert dp <= 1e-10
    # the library's state follows the walkers: log|Psi| at the final positions
    la, sg, _ = ctx.refresh()
    ref_s, ref_l = oracle.log_psi(s, p)
    assert np.abs(la.cpu().numpy() - ref_l).max() <= 1e-10 * np.abs(ref_l).max()
