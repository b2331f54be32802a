"""Differentiated log-psi through the low-rank chain: torch.autograd.Functions whose
forward and backward are the library's hand-written kernels.

Determinants (Sec. II.A): for samples s with occupancies occ_s,
M_s = Phi[occ_s] + B_s C_s^T and logdet_s = log det M_s (complex log:
log|det| + i arg det).  The forward reads A_s^-1 from a walker state -- the
checkpoint, flushed or in the delayed form of Sec. II.C (no flush, no new
factorisation) -- and applies the matrix determinant lemma
(``lrx_det_lowrank_fwd``); the backward (``lrx_det_lowrank_bwd``, Woodbury,
Eq. det_inv) returns dPhi, dB, dC.

Pfaffians (Sec. III.A, Appendix A): M_s = F[occ_s][:, occ_s] - U_s J U_s^T and
log pf M_s by the Pfaffian low-rank identity (``lrx_pf_lowrank_fwd``), with the
gradient d log pf / dM_ij = (1/2) (M^-1)_ji (Eq. pf_grad) for dF and dU
(``lrx_pf_lowrank_bwd``); and the stand-alone batched ``logpf`` / ``slogpf`` /
``pf`` of dense skew matrices (Parlett-Reid factorisation of ``lrx_pf_init_inverse``,
gradient by ``lrx_pf_grad``).

All arithmetic runs in liblrx; this module allocates outputs and marshals calls.
"""
from __future__ import annotations

import torch

from . import lrx


def _out_log(logabs, phase):
    if torch.is_complex(phase):
        return torch.complex(logabs, torch.angle(phase))
    return logabs


class _DetLowRank(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi, b, c, st, occ):
        W, n, r = st.walkers, st.n, b.shape[-1]
        bb = b.detach().to(st.dtype).contiguous()
        cc = c.detach().to(st.dtype).contiguous()
        P = torch.empty(W, n, r, dtype=st.dtype, device=b.device)
        Q = torch.empty_like(P)
        Rinv = torch.empty(W, r, r, dtype=st.dtype, device=b.device)
        logabs = torch.empty(W, dtype=torch.float64, device=b.device)
        phase = torch.empty(W, dtype=st.wide, device=b.device)
        lrx.lrx_det_lowrank_fwd(st, r, bb, cc, P, Q, Rinv, logabs, phase)
        ctx.st, ctx.r, ctx.sites = st, r, phi.shape[0]
        ctx.dtypes = (phi.dtype, b.dtype, c.dtype)
        ctx.save_for_backward(occ, P, Q, Rinv)
        ctx.mark_non_differentiable(phase)
        return _out_log(logabs, phase), phase

    @staticmethod
    def backward(ctx, g_out, _g_phase):
        occ, P, Q, Rinv = ctx.saved_tensors
        st, r = ctx.st, ctx.r
        g = g_out.to(st.wide).contiguous()
        dphi = torch.empty(ctx.sites, st.n, dtype=st.dtype, device=P.device)
        dB = torch.empty_like(P)
        dC = torch.empty_like(P)
        work = torch.empty(lrx.lrx_det_lowrank_work_bytes(st, r, ctx.sites), dtype=torch.uint8, device=P.device)
        lrx.lrx_det_lowrank_bwd(st, r, occ, ctx.sites, P, Q, Rinv, g, dphi, dB, dC, work)
        pd, bd, cd = ctx.dtypes
        return dphi.to(pd), dB.to(bd), dC.to(cd), None, None


class _PfLowRank(torch.autograd.Function):
    @staticmethod
    def forward(ctx, f, u, st, occ):
        W, n, r = st.walkers, st.n, u.shape[-1]
        uu = u.detach().to(st.dtype).contiguous()
        P = torch.empty(W, n, r, dtype=st.dtype, device=u.device)
        Rinv = torch.empty(W, r, r, dtype=st.dtype, device=u.device)
        logabs = torch.empty(W, dtype=torch.float64, device=u.device)
        phase = torch.empty(W, dtype=st.wide, device=u.device)
        lrx.lrx_pf_lowrank_fwd(st, r, uu, P, Rinv, logabs, phase)
        ctx.st, ctx.r, ctx.sites = st, r, f.shape[0]
        ctx.dtypes = (f.dtype, u.dtype)
        ctx.save_for_backward(occ, P, Rinv)
        ctx.mark_non_differentiable(phase)
        return _out_log(logabs, phase), phase

    @staticmethod
    def backward(ctx, g_out, _g_phase):
        occ, P, Rinv = ctx.saved_tensors
        st, r = ctx.st, ctx.r
        g = g_out.to(st.wide).contiguous()
        dF = torch.empty(ctx.sites, ctx.sites, dtype=st.dtype, device=P.device)
        dU = torch.empty_like(P)
        work = torch.empty(lrx.lrx_pf_lowrank_work_bytes(st, r, ctx.sites), dtype=torch.uint8, device=P.device)
        lrx.lrx_pf_lowrank_bwd(st, r, occ, ctx.sites, P, Rinv, g, dF, dU, work)
        fd, ud = ctx.dtypes
        return dF.to(fd), dU.to(ud), None, None


class _LogPf(torch.autograd.Function):
    @staticmethod
    def forward(ctx, a, bulk_dtype):
        W, n, _ = a.shape
        st = lrx.State(lrx.LRX_PF, bulk_dtype, W, n, device=a.device)
        lrx.lrx_pf_init_inverse(st, a.detach().to(st.wide).contiguous(), n, None)
        ctx.st = st
        ctx.a_dtype = a.dtype
        logabs, phase = st.logabs.clone(), st.phase.clone()
        ctx.mark_non_differentiable(phase)
        return _out_log(logabs, phase), phase

    @staticmethod
    def backward(ctx, g_out, _g_phase):
        st = ctx.st
        dA = torch.empty(st.walkers, st.n, st.n, dtype=st.dtype, device=g_out.device)
        lrx.lrx_pf_grad(st, g_out.to(st.wide).contiguous(), dA)
        return dA.to(ctx.a_dtype), None


def lowrank_logdet(phi, b, c, occ, bulk_dtype=None):
    """log det (Phi[occ_s] + B_s C_s^T) for every sample s, differentiable in Phi, B, C.

    Factorises A_s = Phi[occ_s] in FP64 / complex128 first (a fresh state); use
    walker_lowrank_logdet to start from an existing walker state instead.
    Returns (logdet [S] (complex for complex inputs, else log|det|), phase [S]).
    """
    bulk = bulk_dtype if bulk_dtype is not None else phi.dtype
    W, n = occ.shape
    st = lrx.State(lrx.LRX_DET, bulk, W, n, k_max=1, delay=0, device=phi.device)
    lrx.lrx_det_init_inverse(st, phi.detach().to(st.wide).contiguous(), phi.shape[0], occ)
    return _DetLowRank.apply(phi, b, c, st, occ)


def walker_lowrank_logdet(walkers, b, c, phi=None):
    """log det (Phi[occ_w] + B_w C_w^T) of every walker of a determinant Walkers batch,
    with A_w^-1 taken from the walkers' state as it stands (the checkpoint: flushed or
    mid-window in the delayed form).  phi (default: the walkers' orbital table) is the
    tensor that receives dPhi; its values must be those the state was built from.
    The state must not change until the backward pass has run."""
    phi = walkers.table if phi is None else phi
    return _DetLowRank.apply(phi, b, c, walkers.st, walkers.occ)


def lowrank_logpf(f, u, occ, bulk_dtype=None):
    """log pf (F[occ_s][:, occ_s] - U_s J U_s^T) for every sample s, differentiable in F
    and U (U: [S][n][2k]); factorises A_s by Parlett-Reid first (a fresh state).
    Returns (logpf [S] (complex for complex inputs, else log|pf|), phase [S])."""
    bulk = bulk_dtype if bulk_dtype is not None else f.dtype
    W, n = occ.shape
    st = lrx.State(lrx.LRX_PF, bulk, W, n, k_max=1, delay=0, device=f.device)
    lrx.lrx_pf_init_inverse(st, f.detach().to(st.wide).contiguous(), f.shape[0], occ)
    return _PfLowRank.apply(f, u, st, occ)


def walker_lowrank_logpf(walkers, u, f=None):
    """lowrank_logpf for every walker of a Pfaffian Walkers batch, with A_w^-1 from the
    walkers' state as it stands (flushed or in the delayed form)."""
    f = walkers.table if f is None else f
    return _PfLowRank.apply(f, u, walkers.st, walkers.occ)


def logpf(a, bulk_dtype=None):
    """Batched log Pfaffian of dense skew matrices a [W][n][n] (n even): complex log pf for
    complex input, log|pf| for real input; differentiable (Eq. pf_grad)."""
    bulk = bulk_dtype if bulk_dtype is not None else a.dtype
    return _LogPf.apply(a, bulk)[0]


def slogpf(a, bulk_dtype=None):
    """(phase, log|pf|) of dense skew matrices; log|pf| is differentiable."""
    bulk = bulk_dtype if bulk_dtype is not None else a.dtype
    lp, phase = _LogPf.apply(a, bulk)
    return phase, (lp.real if torch.is_complex(lp) else lp)


def pf(a, bulk_dtype=None):
    """Batched Pfaffian of dense skew matrices, differentiable."""
    bulk = bulk_dtype if bulk_dtype is not None else a.dtype
    lp, phase = _LogPf.apply(a, bulk)
    if torch.is_complex(lp):
        return torch.exp(lp)
    return phase * torch.exp(lp)
