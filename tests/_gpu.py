"""GPU test helpers: wire a seeded workload into a libmde context and run
the oracle on the same inputs.  Inputs to the GPU path are the generator's
arrays; orbital values on the GPU side come from the library's own s-Gaussian
provider, on the oracle side from the oracle's own evaluator."""
import sys

import numpy as np
import torch

import oracle


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_ctx(wl, precision="fp64", W=None, refresh_every=None, max_order=None, bind=True):
    from paper_1106_2456_amd import Context
    s = wl.system
    W = W if W is not None else wl.walkers.W
    mo = max_order or max(int(s.exc[0].orders().max()), int(s.exc[1].orders().max()), 1)
    ctx = Context(s.n_elec, s.n_orb, W, max_order=mo, refresh_every=refresh_every,
                  precision=precision)
    ctx.set_expansion(s.exc[0], s.exc[1], s.coef, s.det_up, s.det_dn)
    for sp in (0, 1):
        ctx.set_basis(sp, s.centres, s.expo, s.mo_spin(sp))
    if bind:
        ctx.bind(W)
    return ctx


def dev(x, dtype=torch.float64):
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda:0")


def gpu_orbitals(ctx, pos):
    """pos [W, n_tot, 3] numpy -> (orb_up, orb_dn) device tensors from the
    library's provider."""
    nu = ctx.n_elec[0]
    p = dev(pos)
    ou = ctx.sgauss_eval(0, p[:, :nu].contiguous())
    od = ctx.sgauss_eval(1, p[:, nu:].contiguous())
    return ou, od


def scaled_err(x, ref, scale):
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    scale = np.maximum(np.asarray(scale, np.float64), np.finfo(float).tiny)
    return np.abs(x - ref) / scale
