"""torch.autograd.Function over the library's table-form forward and its
hand-written adjoint kernels.

    log|N| = MultiDetLogPsi.apply(ctx, coef, T_up, T_dn)

N_w = sum_I coef_I det S_up,I(T_up[w]) det S_dn,I(T_dn[w]) (Sec. III r x r
read-off of the tables); log|Psi_w| = log|D0_up| + log|D0_dn| + log|N_w| and
the reference determinants do not depend on the tables or coefficients, so
the gradients below are those of log|Psi| as well.
"""
from __future__ import annotations

import torch


class MultiDetLogPsi(torch.autograd.Function):
    @staticmethod
    def forward(fctx, mctx, coef, T_up, T_dn):
        coef = coef.contiguous()
        T_up = T_up.contiguous()
        T_dn = T_dn.contiguous()
        la, sg, st = mctx.eval_tables(T_up, T_dn, coef)
        fctx.mctx = mctx
        fctx.state_seq = mctx.state_seq
        fctx.save_for_backward(coef, T_up, T_dn)
        fctx.mark_non_differentiable(sg)
        return la, sg

    @staticmethod
    def backward(fctx, go, gsign):
        mctx = fctx.mctx
        coef, T_up, T_dn = fctx.saved_tensors
        # the context holds the state of its last call; unless that call was
        # this forward, evaluate this forward's tables and coefficients again
        # (cheap relative to the backward)
        if mctx.state_seq != fctx.state_seq:
            mctx.eval_tables(T_up, T_dn, coef)
        gc, gu, gd = mctx.backward(go.contiguous().to(torch.float64),
                                   want_coef=fctx.needs_input_grad[1],
                                   want_T=fctx.needs_input_grad[2] or fctx.needs_input_grad[3])
        return None, gc, gu, gd
