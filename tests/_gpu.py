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


def make_ctx(wl, precision="fp64", W=None, refresh_every=None, max_order=None, bind=True,
             stream=None):
    from paper_1106_2456_amd import Context
    s = wl.system
    W = W if W is not None else wl.walkers.W
    mo = max_order or max(int(s.exc[0].orders().max()), int(s.exc[1].orders().max()), 1)
    ctx = Context(s.n_elec, s.n_orb, W, max_order=mo, refresh_every=refresh_every,
                  precision=precision, stream=stream)
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


# FP32-table forms and the first-order scale kind that bounds them: tables
# kept in FP32 across commits (rank-one table updates; pass the scales of
# oracle.StoredTableErrors along the trajectory), or entries formed by an
# FP32 product of A^-1 and Phi_V (tables rebuilt by the MFMA GEMM)
MIXED_SCALE_KIND = {"mixed": "round", "mixed_gemm": "gemm", "mixed_gemm_ksum64": "gemm"}
MIXED_TOL = 1e-5


def output_errors(precision, got, ref, ms=None):
    """Errors of (ratio [W], grad [W,3], lap [W]) against oracle.move's dict.
    FP64: condition-aware scale; FP32-table forms: the oracle's first-order
    FP32-entry scale (oracle.mixed_scales) of the matching kind.  Returns
    (scaled [W,5], plain relative [W,5])."""
    vals = np.column_stack([np.asarray(got[0]), np.asarray(got[1]), np.asarray(got[2])])
    exact = np.column_stack([ref["ratio"], ref["grad"], ref["lap"]])
    if precision == "fp64":
        scale = np.column_stack([ref["scale_ratio"], ref["scale_grad"], ref["scale_lap"]])
    else:
        scale = ms[MIXED_SCALE_KIND[precision]]
    d = np.abs(vals - exact)
    return d / np.maximum(scale, np.finfo(float).tiny), d / np.maximum(np.abs(exact), np.finfo(float).tiny)


def report_errors(tag, scaled, plain):
    names = ("ratio", "grad", "lap")
    cols = (slice(0, 1), slice(1, 4), slice(4, 5))
    for nm, c in zip(names, cols):
        s, p = scaled[:, c].ravel(), plain[:, c].ravel()
        say(f"  {tag} {nm}: scaled max {s.max():.2e} p99 {np.quantile(s, 0.99):.2e} | plain relative "
            f"max {p.max():.2e} median {np.median(p):.2e}, {int((p > 1e-5).sum())}/{p.size} above 1e-5")
