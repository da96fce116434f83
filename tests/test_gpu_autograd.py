"""torch.autograd.Function wrappers: every backward (the library's adjoint
kernels) checked against central finite differences (torch.autograd.gradcheck
on the device, FP64) and against a dense reference gradient computed with
torch-CPU float64 autograd through dense Cholesky / solve / inverse / matmul.

Dense references differentiate through the band -> dense construction, so
their gradients are with respect to the stored band entries, as the library's
are (a stored off-diagonal entry of a symmetric band stands for Q_ij and Q_ji).
"""
import numpy as np
import pytest
import torch

import oracle
import composed
from bandutil import band_mask
from paper_1902_10078_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-10


@pytest.fixture(scope="module")
def ag():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1902_10078_amd import autograd, bandops
    bandops.lib()
    return autograd


def spd_band(n, k, seed):
    rng = np.random.default_rng(seed)
    L0 = inputs.random_lower_band(n, k, rng)
    Q = oracle.gbmm(L0, k, 0, L0, k, 0, tB=1, lc=k, uc=0)
    return Q, L0, rng


def cuda(a, grad=False):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda", requires_grad=grad)


def cpu(a, grad=False):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float64, requires_grad=grad)


# ---- dense helpers in torch (CPU, differentiable) ----

def t_gen_to_dense(B, l, u):
    n = B.shape[0]
    M = torch.zeros((n, n), dtype=torch.float64)
    for s in range(l + u + 1):
        d = s - u
        for j in range(n):
            i = j + d
            if 0 <= i < n:
                M = M.index_put((torch.tensor([i]), torch.tensor([j])), B[j, s].reshape(1))
    return M


def t_sym_to_dense(B, k):
    M = t_gen_to_dense(B, k, 0)
    return M + torch.tril(M, -1).T


def t_dense_to_gen(M, l, u):
    n = M.shape[0]
    rows = []
    for j in range(n):
        rec = []
        for s in range(l + u + 1):
            i = j + s - u
            rec.append(M[i, j] if 0 <= i < n else torch.zeros((), dtype=torch.float64))
        rows.append(torch.stack(rec))
    return torch.stack(rows)


# ------------------------------------------------------------ gradcheck (FD)

@pytest.mark.parametrize("n,k", [(7, 2), (9, 3), (6, 0)])
def test_chol_gradcheck(ag, n, k):
    Q, _, _ = spd_band(n, k, 10 + n)
    Qt = cuda(Q, True)
    assert torch.autograd.gradcheck(lambda q: ag.chol(q), (Qt,), eps=1e-6, atol=1e-6, rtol=1e-5)


@pytest.mark.parametrize("trans", [0, 1])
def test_trsv_gradcheck(ag, trans):
    _, L0, rng = spd_band(8, 2, 21)
    b = rng.normal(size=8)
    assert torch.autograd.gradcheck(lambda L, x: ag.trsv(L, x, trans), (cuda(L0, True), cuda(b, True)),
                                    eps=1e-6, atol=1e-6, rtol=1e-5)


def test_subset_inv_gradcheck(ag):
    _, L0, _ = spd_band(8, 3, 22)
    assert torch.autograd.gradcheck(lambda L: ag.subset_inv(L), (cuda(L0, True),),
                                    eps=1e-6, atol=1e-6, rtol=1e-5)


@pytest.mark.parametrize("la,ua,lb,ub,tA,tB", [(1, 0, 1, 0, 0, 1), (2, 1, 0, 2, 1, 0), (1, 2, 2, 1, 1, 1)])
def test_gbmm_gradcheck(ag, la, ua, lb, ub, tA, tB):
    rng = np.random.default_rng(23)
    n = 7
    A = rng.normal(size=(n, la + ua + 1)) * band_gen_mask(n, la, ua)
    B = rng.normal(size=(n, lb + ub + 1)) * band_gen_mask(n, lb, ub)
    assert torch.autograd.gradcheck(lambda a, b: ag.gbmm(a, b, la, ua, lb, ub, tA, tB),
                                    (cuda(A, True), cuda(B, True)), eps=1e-6, atol=1e-6, rtol=1e-5)


@pytest.mark.parametrize("l,u,tA", [(2, 1, 0), (1, 2, 1)])
def test_gbmv_and_outer_gradcheck(ag, l, u, tA):
    rng = np.random.default_rng(24)
    n = 7
    A = rng.normal(size=(n, l + u + 1)) * band_gen_mask(n, l, u)
    x, m = rng.normal(size=n), rng.normal(size=n)
    assert torch.autograd.gradcheck(lambda a, v: ag.gbmv(a, v, l, u, tA), (cuda(A, True), cuda(x, True)),
                                    eps=1e-6, atol=1e-6, rtol=1e-5)
    assert torch.autograd.gradcheck(lambda a, b: ag.outer_band(a, b, l, u), (cuda(m, True), cuda(x, True)),
                                    eps=1e-6, atol=1e-6, rtol=1e-5)


def band_gen_mask(n, l, u):
    m = np.zeros((n, l + u + 1))
    for s in range(l + u + 1):
        d = s - u
        for j in range(n):
            if 0 <= j + d < n:
                m[j, s] = 1.0
    return m


# ------------------------------------------------- dense autograd references

def test_chol_vs_dense_autograd(ag):
    n, k = 12, 3
    Q, _, rng = spd_band(n, k, 31)
    W = rng.normal(size=(n, k + 1)) * band_mask(n, k)
    c = 0.7
    Qg = cuda(Q, True)
    L, logdet = ag.chol(Qg)
    ((L * cuda(W)).sum() + c * logdet).backward()
    Qc = cpu(Q, True)
    Ld = torch.linalg.cholesky(t_sym_to_dense(Qc, k))
    Lb = t_dense_to_gen(Ld, k, 0)
    ((Lb * cpu(W)).sum() + c * 2 * torch.log(torch.diagonal(Ld)).sum()).backward()
    ref = Qc.grad.numpy() * band_mask(n, k)
    got = Qg.grad.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= TOL * max(1.0, np.max(np.abs(ref)))


def test_trsv_subset_inv_vs_dense_autograd(ag):
    n, k = 11, 2
    _, L0, rng = spd_band(n, k, 32)
    b = rng.normal(size=n)
    W = rng.normal(size=(n, k + 1)) * band_mask(n, k)
    wx, wx2 = rng.normal(size=n), rng.normal(size=n)
    Lg, bg = cuda(L0, True), cuda(b, True)
    f = ((ag.trsv(Lg, bg, 0) * cuda(wx)).sum() + (ag.trsv(Lg, bg, 1) * cuda(wx2)).sum()
         + (ag.subset_inv(Lg) * cuda(W)).sum())
    f.backward()
    Lc, bc = cpu(L0, True), cpu(b, True)
    Ld = t_gen_to_dense(Lc, k, 0)
    x0 = torch.linalg.solve_triangular(Ld, bc.reshape(-1, 1), upper=False).reshape(-1)
    x1 = torch.linalg.solve_triangular(Ld.T, bc.reshape(-1, 1), upper=True).reshape(-1)
    Sd = torch.cholesky_inverse(Ld)
    fr = (x0 * cpu(wx)).sum() + (x1 * cpu(wx2)).sum() + (t_dense_to_gen(Sd, k, 0) * cpu(W)).sum()
    fr.backward()
    for got, ref in ((Lg.grad, Lc.grad.numpy() * band_mask(n, k)), (bg.grad, bc.grad.numpy())):
        got = got.cpu().numpy()
        assert np.max(np.abs(got - ref)) <= TOL * max(1.0, np.max(np.abs(ref)))


def test_products_vs_dense_autograd(ag):
    n, la, ua, lb, ub = 9, 2, 1, 1, 2
    rng = np.random.default_rng(33)
    A = rng.normal(size=(n, la + ua + 1)) * band_gen_mask(n, la, ua)
    B = rng.normal(size=(n, lb + ub + 1)) * band_gen_mask(n, lb, ub)
    x = rng.normal(size=n)
    Wc = rng.normal(size=(n, 3 + 3 + 1))
    wy = rng.normal(size=n)
    Ag, Bg, xg = cuda(A, True), cuda(B, True), cuda(x, True)
    C = ag.gbmm(Ag, Bg, la, ua, lb, ub, 1, 0)          # A^T B: lower ua+lb = 2, upper la+ub = 4
    y = ag.gbmv(Ag, xg, la, ua, 0)
    f = (C * cuda(Wc[:, : C.shape[1]] * band_gen_mask(n, ua + lb, la + ub))).sum() + (y * cuda(wy)).sum()
    f.backward()
    Ac, Bc, xc = cpu(A, True), cpu(B, True), cpu(x, True)
    Ad, Bd = t_gen_to_dense(Ac, la, ua), t_gen_to_dense(Bc, lb, ub)
    Cr = t_dense_to_gen(Ad.T @ Bd, ua + lb, la + ub)
    fr = (Cr * cpu(Wc[:, : Cr.shape[1]] * band_gen_mask(n, ua + lb, la + ub))).sum() + ((Ad @ xc) * cpu(wy)).sum()
    fr.backward()
    for got, ref in ((Ag.grad, Ac.grad.numpy() * band_gen_mask(n, la, ua)),
                     (Bg.grad, Bc.grad.numpy() * band_gen_mask(n, lb, ub)), (xg.grad, xc.grad.numpy())):
        got = got.cpu().numpy()
        assert np.max(np.abs(got - ref)) <= TOL * max(1.0, np.max(np.abs(ref)))


# --------------------------------------------------------------- loss unit

def test_gauss_loss_batch_vs_dense_autograd_and_composed(ag):
    from paper_1902_10078_amd import bandops as bo
    ns, ks = [10, 37, 5], [2, 3, 1]
    Qs, ys, Ss = [], [], []
    for p, (n, k) in enumerate(zip(ns, ks)):
        Q, _, rng = spd_band(n, k, 40 + p)
        Qs.append(Q)
        ys.append(rng.normal(size=n))
        Ss.append(inputs.random_sym_band_dd(n, k, rng))
    plan = bo.Plan(ns, ks, device="cuda")
    Qg = cuda(np.concatenate([q.ravel() for q in Qs]), True)
    yg = cuda(np.concatenate(ys), True)
    Sg = cuda(np.concatenate([s.ravel() for s in Ss]), True)
    g = cuda(np.array([1.0, -0.5, 2.0]))
    loss = ag.gauss_loss(plan, Qg, yg, Sg)
    (loss * g).sum().backward()
    gQ, gy, gS = Qg.grad.cpu().numpy(), yg.grad.cpu().numpy(), Sg.grad.cpu().numpy()
    bo_, vo = 0, 0
    for p, (n, k) in enumerate(zip(ns, ks)):
        Qc, yc, Sc = cpu(Qs[p], True), cpu(ys[p], True), cpu(Ss[p], True)
        Qd = t_sym_to_dense(Qc, k)
        Sd = t_sym_to_dense(Sc, k)
        Qi = torch.linalg.inv(Qd)
        lr = torch.logdet(Qd) - yc @ Qi @ yc + torch.trace(Qi @ Sd)
        assert abs(loss[p].item() - lr.item()) <= 1e-11 * max(1.0, abs(lr.item()))
        (lr * float(g[p])).backward()
        m = band_mask(n, k)
        for got, ref in ((gQ[bo_:bo_ + n * (k + 1)].reshape(n, k + 1), Qc.grad.numpy() * m),
                         (gy[vo:vo + n], yc.grad.numpy()),
                         (gS[bo_:bo_ + n * (k + 1)].reshape(n, k + 1), Sc.grad.numpy() * m)):
            assert np.max(np.abs(got - ref)) <= 1e-10 * max(1.0, np.max(np.abs(ref)))
        # the same loss composed from separate operators through autograd
        Qp = cuda(Qs[p], True)
        lc = composed.gauss_loss_composed(Qp, cuda(ys[p]), cuda(Ss[p]))
        lc.backward()
        assert abs(lc.item() - loss[p].item()) <= 1e-11 * max(1.0, abs(lr.item()))
        ref = gQ[bo_:bo_ + n * (k + 1)].reshape(n, k + 1) / float(g[p])
        assert np.max(np.abs(Qp.grad.cpu().numpy() - ref)) <= 1e-10 * max(1.0, np.max(np.abs(ref)))
        bo_ += n * (k + 1)
        vo += n


def test_gauss_loss_finite_differences(ag):
    """Central differences along random stored-band directions of Q and y."""
    from paper_1902_10078_amd import bandops as bo
    n, k = 300, 3
    Q, _, rng = spd_band(n, k, 50)
    y = rng.normal(size=n)
    S = inputs.random_sym_band_dd(n, k, rng)
    plan = bo.Plan([n], [k], device="cuda")
    Qg, yg = cuda(Q.ravel(), True), cuda(y, True)
    St = cuda(S.ravel())
    ag.gauss_loss(plan, Qg, yg, St).sum().backward()
    m = band_mask(n, k).ravel()
    for trial in range(3):
        dQ = rng.normal(size=Q.size) * m
        dy = rng.normal(size=n)
        h = 1e-5
        fp = ag.gauss_loss(plan, cuda(Q.ravel() + h * dQ), cuda(y + h * dy), St).item()
        fm = ag.gauss_loss(plan, cuda(Q.ravel() - h * dQ), cuda(y - h * dy), St).item()
        fd = (fp - fm) / (2 * h)
        an = float(Qg.grad.cpu().numpy() @ dQ + yg.grad.cpu().numpy() @ dy)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))
