"""torch.autograd.Function wrappers of the banded operators.

Every forward and backward runs the library's HIP kernels; the functions here
only allocate outputs and route sensitivities (Table 1 of the paper).

Tensors are FP64 bands of shape (n, l+u+1) in record-major storage (row j =
column j of the band, slot u+i-j holds B[i,j]; lower-banded and symmetric
matrices use u = 0).  Symmetric inputs (the precision Q) are given by their
lower band, and their gradients are with respect to those stored entries: an
off-diagonal stored value stands for both Q_ij and Q_ji.

  chol(Q)            -> (L, logdet)        Algorithm 1 / Algorithm 2
  trsv(L, b, trans)  -> L^{-1} b or L^{-T} b      Table 1, solve row
  subset_inv(L)      -> band of (L L^T)^{-1}       Algorithm 3 / Algorithm 4
  gbmm(A, B, ...)    -> band of op(A) op(B)        Table 1, product row
  gbmv(A, x, tA)     -> op(A) x                    Table 1, product row
  outer_band(m, v)   -> band of m v^T              Table 1, outer-product row
  gauss_loss(plan, Q, y, S) -> per-problem logdet Q - y^T Q^{-1} y + tr(Q^{-1} S)
                                  (fused forward and backward over a batch)
  solve_band_mat(L, R, lr, u) -> band (k, u) of L^{-1} R   Algorithm 5 / Table 1
  vi_kl(plan, Lq, Lp, mq, mp) -> per-problem KL(q || p) of the variational
                                  objective (Eq. (KL), Algorithm 7; batched)
"""
from __future__ import annotations

import torch

from . import bandops as bo


def _band(t: torch.Tensor, l: int, u: int = 0) -> bo.Band:
    if t.dtype != torch.float64:
        raise TypeError("the autograd wrappers take FP64 bands")
    return bo.Band(t.contiguous(), l, u)


def _vec(t: torch.Tensor) -> torch.Tensor:
    if t.dtype != torch.float64:
        raise TypeError("the autograd wrappers take FP64 vectors")
    return t.contiguous()


def _check_info(info: torch.Tensor):
    r = int(info.max().item())
    if r != 0:
        raise bo.BandOpsError(f"matrix is not positive definite (leading minor of order {r})")


class Chol(torch.autograd.Function):
    """Q (lower band, k = Q.shape[1]-1) -> (L, log det Q)."""

    @staticmethod
    def forward(ctx, Q):
        k = Q.shape[1] - 1
        L, _, logdet, info = bo.bo_chol(_band(Q, k))
        _check_info(info)
        ctx.save_for_backward(L.band)
        ctx.k = k
        return L.band, logdet.reshape(())

    @staticmethod
    def backward(ctx, gL, glogdet):
        (Lt,) = ctx.saved_tensors
        L = bo.Band(Lt, ctx.k)
        Lbar = bo.Band(gL.contiguous().clone() if gL is not None else torch.zeros_like(Lt), ctx.k)
        if glogdet is not None:
            bo.bo_logdet_bwd(L, glogdet, out=Lbar, accumulate=True)
        return bo.bo_chol_bwd(L, Lbar).band


class Trsv(torch.autograd.Function):
    """x = L^{-1} b (trans = 0) or L^{-T} b (trans = 1)."""

    @staticmethod
    def forward(ctx, L, b, trans: int = 0):
        k = L.shape[1] - 1
        Lb = _band(L, k)
        x = bo.bo_trsv(Lb, _vec(b), trans)
        ctx.save_for_backward(Lb.band, x)
        ctx.k, ctx.trans = k, trans
        return x

    @staticmethod
    def backward(ctx, gx):
        Lt, x = ctx.saved_tensors
        bbar, Lbar = bo.bo_trsv_bwd(bo.Band(Lt, ctx.k), x, gx.contiguous(), ctx.trans)
        return Lbar.band, bbar, None


class SubsetInv(torch.autograd.Function):
    """Lower band (width k) of (L L^T)^{-1}."""

    @staticmethod
    def forward(ctx, L):
        k = L.shape[1] - 1
        Lb = _band(L, k)
        S = bo.bo_subset_inv(Lb)
        ctx.save_for_backward(Lb.band, S.band)
        ctx.k = k
        return S.band

    @staticmethod
    def backward(ctx, gS):
        Lt, St = ctx.saved_tensors
        k = ctx.k
        return bo.bo_subset_inv_bwd(bo.Band(Lt, k), bo.Band(St, k), bo.Band(gS.contiguous(), k)).band


class Gbmm(torch.autograd.Function):
    """Band (l, u) of op(A) op(B) for (la, ua)- and (lb, ub)-banded A, B."""

    @staticmethod
    def forward(ctx, A, B, la, ua, lb, ub, tA, tB, l, u):
        Ab, Bb = _band(A, la, ua), _band(B, lb, ub)
        C = bo.bo_gbmm(Ab, Bb, tA, tB, l, u)
        ctx.save_for_backward(Ab.band, Bb.band)
        ctx.meta = (la, ua, lb, ub, tA, tB, l, u)
        return C.band

    @staticmethod
    def backward(ctx, gC):
        At, Bt = ctx.saved_tensors
        la, ua, lb, ub, tA, tB, l, u = ctx.meta
        A, B, Cb = bo.Band(At, la, ua), bo.Band(Bt, lb, ub), bo.Band(gC.contiguous(), l, u)
        gA = gB = None
        if ctx.needs_input_grad[0]:
            # d/dA of <Cbar, op(A) op(B)>: band_A(Cbar op(B)^T), transposed when tA
            gA = (bo.bo_gbmm(Cb, B, 0, 1 - tB, la, ua) if not tA
                  else bo.bo_gbmm(B, Cb, tB, 1, la, ua)).band
        if ctx.needs_input_grad[1]:
            gB = (bo.bo_gbmm(A, Cb, 1 - tA, 0, lb, ub) if not tB
                  else bo.bo_gbmm(Cb, A, 1, tA, lb, ub)).band
        return gA, gB, None, None, None, None, None, None, None, None


class Gbmv(torch.autograd.Function):
    """op(A) x for an (l, u)-banded A."""

    @staticmethod
    def forward(ctx, A, x, l, u, tA):
        Ab = _band(A, l, u)
        y = bo.bo_gbmv(Ab, _vec(x), tA)
        ctx.save_for_backward(Ab.band, x)
        ctx.meta = (l, u, tA)
        return y

    @staticmethod
    def backward(ctx, gy):
        At, x = ctx.saved_tensors
        l, u, tA = ctx.meta
        A, gy = bo.Band(At, l, u), gy.contiguous()
        gA = gx = None
        if ctx.needs_input_grad[0]:
            gA = (bo.bo_outer_band(gy, x, l, u) if not tA else bo.bo_outer_band(x, gy, l, u)).band
        if ctx.needs_input_grad[1]:
            gx = bo.bo_gbmv(A, gy, 1 - tA)
        return gA, gx, None, None, None


class OuterBand(torch.autograd.Function):
    """Band (l, u) of m v^T."""

    @staticmethod
    def forward(ctx, m, v, l, u):
        O = bo.bo_outer_band(_vec(m), _vec(v), l, u)
        ctx.save_for_backward(m, v)
        ctx.meta = (l, u)
        return O.band

    @staticmethod
    def backward(ctx, gO):
        m, v = ctx.saved_tensors
        l, u = ctx.meta
        Ob = bo.Band(gO.contiguous(), l, u)
        gm = bo.bo_gbmv(Ob, v, 0) if ctx.needs_input_grad[0] else None
        gv = bo.bo_gbmv(Ob, m, 1) if ctx.needs_input_grad[1] else None
        return gm, gv, None, None


def _scale(plan, kind, g, t):
    """g[p] * t on every problem p's records or entries, in the library."""
    return plan.scale(bo.F64, kind, g.contiguous(), t, torch.empty_like(t))


class GaussLoss(torch.autograd.Function):
    """Per-problem loss_p = log det Q_p - y_p^T Q_p^{-1} y_p + tr(Q_p^{-1} S_p)
    over a plan's batch.  Q, S: packed lower bands (all problems' records back
    to back); y: packed vectors.  The forward pass runs the library's fused
    forward and backward passes once: it writes the losses and d loss / dQ,
    dy, dS, which backward scales by the upstream sensitivities (the library's
    per-problem scaling)."""

    @staticmethod
    def forward(ctx, plan, Q, y, S):
        Q, y, S = _vec(Q), _vec(y), _vec(S)
        dev = Q.device
        E, N = Q.numel(), y.numel()
        bufs = {nm: torch.empty(E, dtype=torch.float64, device=dev) for nm in ("L", "Sig", "Lbar", "Qbar", "Sbar")}
        z = torch.empty(N, dtype=torch.float64, device=dev)
        ybar = torch.empty(N, dtype=torch.float64, device=dev)
        parts = torch.empty((plan.nprob, 3), dtype=torch.float64, device=dev)
        loss = torch.empty(plan.nprob, dtype=torch.float64, device=dev)
        info = torch.zeros(plan.nprob, dtype=torch.int32, device=dev)
        io = plan.io(Q=Q, y=y, S=S, z=z, x=ybar, parts=parts, info=info, loss=loss, **bufs)
        plan.gauss_loss(bo.F64, io)
        _check_info(info)
        ctx.save_for_backward(bufs["Qbar"], ybar, bufs["Sbar"])
        ctx.plan = plan
        return loss

    @staticmethod
    def backward(ctx, g):
        Qbar, ybar, Sbar = ctx.saved_tensors
        plan = ctx.plan
        gQ = _scale(plan, bo.SCALE_BAND, g, Qbar) if ctx.needs_input_grad[1] else None
        gy = _scale(plan, bo.SCALE_VEC, g, ybar) if ctx.needs_input_grad[2] else None
        gS = _scale(plan, bo.SCALE_BAND, g, Sbar) if ctx.needs_input_grad[3] else None
        return None, gQ, gy, gS


class SolveBandMat(torch.autograd.Function):
    """Band (k, u) of L^{-1} R (Algorithm 5) and its reverse mode (Table 1,
    solve matrix-matrix).  L: (n, k+1) lower band; R: (n, lr+u+1) band with lr
    lower and u upper diagonals; output (n, k+u+1)."""

    @staticmethod
    def forward(ctx, L, R, lr: int, u: int):
        k = L.shape[1] - 1
        Lb, Rb = _band(L, k), _band(R, lr, u)
        O = bo.bo_solve_band_mat(Lb, Rb)
        ctx.save_for_backward(L, O.band)
        ctx.lr, ctx.u = lr, u
        return O.band

    @staticmethod
    def backward(ctx, gO):
        L, O = ctx.saved_tensors
        k = L.shape[1] - 1
        Rbar, Lbar = bo.bo_solve_band_mat_bwd(_band(L, k), _band(O, k, ctx.u), _band(gO, k, ctx.u), ctx.lr)
        return Lbar.band, Rbar.band, None, None


class ViKL(torch.autograd.Function):
    """Per-problem KL(q_p || p_p) of the variational objective (Eq. (KL),
    Algorithm 7) over a plan's batch: q = N(m_q, (L_q L_q^T)^{-1}),
    p = N(m_p, (L_p L_p^T)^{-1}).  Lq, Lp: packed lower bands; mq, mp: packed
    vectors.  The forward pass runs the fused forward and reverse passes once
    and keeps the four gradients for backward."""

    @staticmethod
    def forward(ctx, plan, Lq, Lp, mq, mp):
        Lq, Lp, mq, mp = _vec(Lq), _vec(Lp), _vec(mq), _vec(mp)
        dev = Lq.device
        E, N = Lq.numel(), mq.numel()
        bufs = {nm: torch.empty(E, dtype=torch.float64, device=dev) for nm in ("Sig", "Lqbar", "Lpbar")}
        bufs.update({nm: torch.empty(N, dtype=torch.float64, device=dev) for nm in ("mqbar", "mpbar")})
        parts = torch.zeros((plan.nprob, 4), dtype=torch.float64, device=dev)
        plan.vi_kl(bo.F64, plan.kl_io(Lq=Lq, Lp=Lp, mq=mq, mp=mp, parts=parts, **bufs))
        ctx.save_for_backward(bufs["Lqbar"], bufs["Lpbar"], bufs["mqbar"], bufs["mpbar"])
        ctx.plan = plan
        return parts[:, 0]

    @staticmethod
    def backward(ctx, g):
        Lqbar, Lpbar, mqbar, mpbar = ctx.saved_tensors
        plan = ctx.plan
        return (None, _scale(plan, bo.SCALE_BAND, g, Lqbar) if ctx.needs_input_grad[1] else None,
                _scale(plan, bo.SCALE_BAND, g, Lpbar) if ctx.needs_input_grad[2] else None,
                _scale(plan, bo.SCALE_VEC, g, mqbar) if ctx.needs_input_grad[3] else None,
                _scale(plan, bo.SCALE_VEC, g, mpbar) if ctx.needs_input_grad[4] else None)


class Whiten(torch.autograd.Function):
    """Whitened GMRF samples F = L^{-T} v, L = C(Q) (Section 3.2, Algorithm
    6), over a plan's batch, FP64: Q packed lower bands, v packed vectors.
    Backward runs the library's reverse mode (Table 1, Algorithm 2)."""

    @staticmethod
    def forward(ctx, plan, Q, v):
        Q, v = _vec(Q), _vec(v)
        L = torch.empty_like(Q)
        F = torch.empty_like(v)
        info = torch.zeros(plan.nprob, dtype=torch.int32, device=Q.device)
        plan.whiten(bo.F64, plan.wh_io(Q=Q, v=v, L=L, F=F, info=info))
        _check_info(info)
        ctx.save_for_backward(L, F)
        ctx.plan = plan
        return F

    @staticmethod
    def backward(ctx, Fbar):
        L, F = ctx.saved_tensors
        plan = ctx.plan
        vbar = torch.empty_like(F)
        Qbar = torch.empty_like(L)
        plan.whiten_bwd(bo.F64, plan.wh_io(L=L, F=F, Fbar=_vec(Fbar), vbar=vbar, Qbar=Qbar))
        return None, Qbar if ctx.needs_input_grad[1] else None, vbar if ctx.needs_input_grad[2] else None


def whiten(plan, Q, v):
    return Whiten.apply(plan, Q, v)


class MargLik(torch.autograd.Function):
    """Per-problem log marginal likelihood with partial observations (Eq.
    (marg_lik), Algorithm 8) over a plan's batch, FP64: Q packed lower bands,
    mask and b = E^T Y packed vectors, tau2 one per problem.  The forward pass
    runs the library's call once and keeps the gradients in Q, b and tau2."""

    @staticmethod
    def forward(ctx, plan, Q, mask, b, tau2):
        Q, mask, b, tau2 = _vec(Q), _vec(mask), _vec(b), _vec(tau2)
        dev = Q.device
        E, N, P = Q.numel(), b.numel(), plan.nprob
        bufs = {nm: torch.empty(E, dtype=torch.float64, device=dev) for nm in ("L", "Sig", "Qbar")}
        bufs.update({nm: torch.empty(N, dtype=torch.float64, device=dev) for nm in ("x", "bbar")})
        tau2bar = torch.empty(P, dtype=torch.float64, device=dev)
        parts = torch.empty((P, 4), dtype=torch.float64, device=dev)
        info = torch.zeros(P, dtype=torch.int32, device=dev)
        plan.marglik(bo.F64, plan.ml_io(Q=Q, mask=mask, b=b, tau2=tau2, tau2bar=tau2bar, parts=parts, info=info,
                                         **bufs))
        _check_info(info)
        ctx.save_for_backward(bufs["Qbar"], bufs["bbar"], tau2bar)
        ctx.plan = plan
        return parts[:, 0]

    @staticmethod
    def backward(ctx, g):
        Qbar, bbar, tau2bar = ctx.saved_tensors
        plan = ctx.plan
        return (None, _scale(plan, bo.SCALE_BAND, g, Qbar) if ctx.needs_input_grad[1] else None, None,
                _scale(plan, bo.SCALE_VEC, g, bbar) if ctx.needs_input_grad[3] else None,
                _scale(plan, bo.SCALE_PROBLEM, g, tau2bar) if ctx.needs_input_grad[4] else None)


def marglik(plan, Q, mask, b, tau2):
    return MargLik.apply(plan, Q, mask, b, tau2)


class NatGP(torch.autograd.Function):
    """Per-problem GP regression value a(eta_pr, Lam_pr) - a(eta_po, Lam_po)
    in banded natural parameters (Appendix C.5, Algorithm 10) over a plan's
    batch, FP64: Lpr, Llik packed lower bands, etapr, etalik packed vectors.
    The forward pass keeps the four gradients."""

    @staticmethod
    def forward(ctx, plan, Lpr, etapr, Llik, etalik):
        Lpr, etapr, Llik, etalik = _vec(Lpr), _vec(etapr), _vec(Llik), _vec(etalik)
        dev = Lpr.device
        E, N, P = Lpr.numel(), etapr.numel(), plan.nprob
        bufs = {nm: torch.empty(E, dtype=torch.float64, device=dev) for nm in ("L", "Sig", "Lprbar", "Llikbar")}
        bufs.update({nm: torch.empty(N, dtype=torch.float64, device=dev) for nm in ("x", "etaprbar")})
        parts = torch.empty((P, 5), dtype=torch.float64, device=dev)
        info = torch.zeros(P, dtype=torch.int32, device=dev)
        plan.natgp(bo.F64, plan.ng_io(Lpr=Lpr, etapr=etapr, Llik=Llik, etalik=etalik, parts=parts, info=info, **bufs))
        _check_info(info)
        ctx.save_for_backward(bufs["Lprbar"], bufs["etaprbar"], bufs["Llikbar"], bufs["x"])
        ctx.plan = plan
        return parts[:, 0]

    @staticmethod
    def backward(ctx, g):
        Lprbar, etaprbar, Llikbar, x = ctx.saved_tensors
        plan = ctx.plan
        return (None, _scale(plan, bo.SCALE_BAND, g, Lprbar) if ctx.needs_input_grad[1] else None,
                _scale(plan, bo.SCALE_VEC, g, etaprbar) if ctx.needs_input_grad[2] else None,
                _scale(plan, bo.SCALE_BAND, g, Llikbar) if ctx.needs_input_grad[3] else None,
                _scale(plan, bo.SCALE_VEC, g, x) if ctx.needs_input_grad[4] else None)


def natgp(plan, Lpr, etapr, Llik, etalik):
    return NatGP.apply(plan, Lpr, etapr, Llik, etalik)


def chol(Q):
    return Chol.apply(Q)


def trsv(L, b, trans: int = 0):
    return Trsv.apply(L, b, trans)


def subset_inv(L):
    return SubsetInv.apply(L)


def gbmm(A, B, la, ua, lb, ub, tA=0, tB=0, l=None, u=None):
    lA, uA = (ua, la) if tA else (la, ua)
    lB, uB = (ub, lb) if tB else (lb, ub)
    l = lA + lB if l is None else l
    u = uA + uB if u is None else u
    return Gbmm.apply(A, B, la, ua, lb, ub, tA, tB, l, u)


def gbmv(A, x, l, u=0, tA=0):
    return Gbmv.apply(A, x, l, u, tA)


def outer_band(m, v, l, u=0):
    return OuterBand.apply(m, v, l, u)


def gauss_loss(plan, Q, y, S):
    return GaussLoss.apply(plan, Q, y, S)


def solve_band_mat(L, R, lr: int, u: int):
    return SolveBandMat.apply(L, R, lr, u)


def vi_kl(plan, Lq, Lp, mq, mp):
    return ViKL.apply(plan, Lq, Lp, mq, mp)
