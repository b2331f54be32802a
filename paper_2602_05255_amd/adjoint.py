"""Differentiated log-psi through the low-rank chain: a torch.autograd.Function
whose forward and backward are the library's hand-written kernels.

For samples s with occupancies occ_s, M_s = Phi[occ_s] + B_s C_s^T and
logdet_s = log det M_s (complex log: log|det| + i arg det).  Forward:
FP64/complex128 factorisation of A_s = Phi[occ_s] (``lrx_det_init_inverse``),
then ``lrx_det_lowrank_fwd`` (matrix determinant lemma, Sec. II.A).  The
factorised state is the checkpoint saved for backward (a flushed inverse, not
one inverse per step).  Backward: ``lrx_det_lowrank_bwd`` (Woodbury, Eq.
det_inv) returns dPhi, dB, dC.
"""
from __future__ import annotations

import torch

from . import lrx


class LowRankLogDet(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi, b, c, occ, bulk_dtype):
        W, n = occ.shape
        r = b.shape[-1]
        sites = phi.shape[0]
        st = lrx.State(lrx.LRX_DET, bulk_dtype, W, n, k_max=1, delay=0, device=phi.device)
        wide = st.wide
        lrx.lrx_det_init_inverse(st, phi.detach().to(wide).contiguous(), sites, occ)
        bb = b.detach().to(st.dtype).contiguous()
        cc = c.detach().to(st.dtype).contiguous()
        P = torch.empty(W, n, r, dtype=st.dtype, device=phi.device)
        Q = torch.empty_like(P)
        Rinv = torch.empty(W, r, r, dtype=st.dtype, device=phi.device)
        logabs = torch.empty(W, dtype=torch.float64, device=phi.device)
        phase = torch.empty(W, dtype=wide, device=phi.device)
        lrx.lrx_det_lowrank_fwd(st, r, bb, cc, P, Q, Rinv, logabs, phase)
        ctx.st, ctx.r, ctx.sites = st, r, sites
        ctx.phi_dtype, ctx.b_dtype, ctx.c_dtype = phi.dtype, b.dtype, c.dtype
        ctx.save_for_backward(occ, P, Q, Rinv)
        if torch.is_complex(phase):
            out = torch.complex(logabs, torch.angle(phase))
        else:
            out = logabs
        ctx.mark_non_differentiable(phase)
        return out, phase

    @staticmethod
    def backward(ctx, g_out, _g_phase):
        occ, P, Q, Rinv = ctx.saved_tensors
        st = ctx.st
        W, n, r = P.shape
        g = g_out.to(st.wide).contiguous()
        dphi = torch.empty(ctx.sites, n, dtype=st.dtype, device=P.device)
        dB = torch.empty_like(P)
        dC = torch.empty_like(P)
        nbytes = lrx.lrx_det_lowrank_work_bytes(st, r, ctx.sites)
        work = torch.empty(nbytes, dtype=torch.uint8, device=P.device)
        lrx.lrx_det_lowrank_bwd(st, r, occ, ctx.sites, P, Q, Rinv, g, dphi, dB, dC, work)
        return dphi.to(ctx.phi_dtype), dB.to(ctx.b_dtype), dC.to(ctx.c_dtype), None, None


def lowrank_logdet(phi, b, c, occ, bulk_dtype=None):
    """log det (Phi[occ_s] + B_s C_s^T) for every sample s, differentiable in Phi, B, C.

    Returns (logdet [S] (complex for complex inputs, else log|det|), phase [S]).
    """
    bulk = bulk_dtype if bulk_dtype is not None else phi.dtype
    return LowRankLogDet.apply(phi, b, c, occ, bulk)
