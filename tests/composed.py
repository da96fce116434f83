"""Single-problem compositions of the separate differentiable operators, used
by the tests as references for the fused batched calls (the arithmetic that
joins the operators is torch's here, which is why this lives with the tests
and not in the package)."""
import torch

from paper_1902_10078_amd import autograd as ag


def gauss_loss_composed(Q, y, S):
    """logdet Q - y^T Q^{-1} y + tr(Q^{-1} S) for one problem, composed from
    the separate operators (Table 1 compositions through autograd): the
    log-determinant from C, the quadratic term from S, the trace from I."""
    k = Q.shape[1] - 1
    L, logdet = ag.chol(Q)
    z = ag.trsv(L, y, 0)
    Sig = ag.subset_inv(L)
    w = torch.full((k + 1,), 2.0, dtype=torch.float64, device=Q.device)
    w[0] = 1.0
    return logdet - (z * z).sum() + (Sig * S * w).sum()


def vi_kl_composed(Lq, Lp, mq, mp):
    """KL(q || p) for one problem composed from the separate operators as
    Algorithm 7 writes it: tr(I(L_q) P(L_p, L_p^T)) as the weighted sum over
    the band, the log-diagonals, ||P(L_p^T, m_p - m_q)||^2."""
    k = Lq.shape[1] - 1
    n = Lq.shape[0]
    Sig = ag.subset_inv(Lq)
    Qp = ag.gbmm(Lp, Lp, k, 0, k, 0, 0, 1, k, 0)
    w = torch.full((k + 1,), 2.0, dtype=torch.float64, device=Lq.device)
    w[0] = 1.0
    tr = (Sig * Qp * w).sum()
    v = ag.gbmv(Lp, mp - mq, k, 0, 1)
    return 0.5 * (tr + 2.0 * (torch.log(Lq[:, 0]).sum() - torch.log(Lp[:, 0]).sum()) + (v * v).sum() - n)
