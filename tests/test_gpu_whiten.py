"""GPU parity of the whitened GMRF sample F = L^{-T} v, L = C(Q), and its
reverse mode (bo_plan_whiten, bo_plan_whiten_bwd; Section 3.2, Algorithm 6)
against the FP64 oracle, through the C ABI, on seeded batches over several
bandwidths (0 to 12), chunks and groups with ragged tails and the degenerate
sizes n = 0, n = 1, k >= n; the mixed format; the info code; and the autograd
Function against dense torch autograd.

Tolerances: FP64 1e-12 relative (max-norm per output array).  Mixed format:
against the oracle on the same FP32-rounded inputs (FP64 diagonals kept) at
1e-6 (L, F and vbar are stored in FP32)."""
import numpy as np
import pytest
import torch

import oracle
from bandutil import band_mask, rel_err
from paper_1902_10078_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12
TOL_MIXED = 1e-6


@pytest.fixture(scope="module")
def bo():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1902_10078_amd import bandops
    bandops.lib()
    return bandops


def draw(ns, ks, seed):
    rng = np.random.default_rng(seed)
    Qs, vs, Fbs = [], [], []
    for n, k in zip(ns, ks):
        if n:
            L0 = inputs.random_lower_band(n, k, rng)
            Qs.append(oracle.gbmm(L0, k, 0, L0, k, 0, tB=1, lc=k, uc=0))
        else:
            Qs.append(np.zeros((0, k + 1)))
        vs.append(rng.normal(size=n))
        Fbs.append(rng.normal(size=n))
    return Qs, vs, Fbs


def rounded(B):
    R = B.astype(np.float32).astype(np.float64)
    if B.shape[0]:
        R[:, 0] = B[:, 0]
    return R


def run_wh(bo, plan, Qs, vs, Fbs, prec=0, reuse=False):
    cat = lambda a: np.concatenate([x.ravel() for x in a])
    dt = torch.float64 if prec == 0 else torch.float32
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    t = dict(Q=dev(cat(Qs)), v=dev(cat(vs)), Fbar=dev(cat(Fbs)))
    E, N, P = t["Q"].numel(), plan.rows, plan.nprob
    for nm in ("L", "Qbar"):
        t[nm] = torch.full((E,), float("nan"), dtype=dt, device="cuda")
    for nm in ("F", "vbar"):
        t[nm] = torch.full((N,), float("nan"), dtype=dt, device="cuda")
    t["logdet"] = torch.full((P,), float("nan"), dtype=torch.float64, device="cuda")
    t["info"] = torch.full((P,), -7, dtype=torch.int32, device="cuda")
    if prec == 1:
        t["Qd"] = torch.tensor(np.concatenate([a[:, 0] for a in Qs]), dtype=torch.float64, device="cuda")
        for nm in ("Ld", "Qbard"):
            t[nm] = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
    io = plan.wh_io(reuse=reuse, **t)
    plan.whiten(prec, io)
    plan.whiten_bwd(prec, io)
    torch.cuda.synchronize()
    res = {k: v.detach().cpu().numpy() for k, v in t.items()}
    res = {k: (v if k == "info" else v.astype(np.float64)) for k, v in res.items()}
    if prec == 1:
        for nm in ("L", "Qbar"):
            for p, (n, k) in enumerate(zip(plan.ns, plan.ks)):
                o, v = plan.boff[p], plan.voff[p]
                res[nm][o:o + n * (k + 1):k + 1] = res[nm + "d"][v:v + n]
    return res


def check(plan, Qs, vs, Fbs, res, tol):
    for p, (n, k) in enumerate(zip(plan.ns, plan.ks)):
        assert res["info"][p] == 0, p
        if n == 0:
            continue
        L, F, info = oracle.whiten(Qs[p], k, vs[p])
        assert info == 0
        vbar, Qbar = oracle.whiten_bwd(L, k, F, Fbs[p])
        o, v = plan.boff[p], plan.voff[p]
        m = band_mask(n, k)
        got = lambda nm: res[nm][o:o + n * (k + 1)].reshape(n, k + 1)
        assert rel_err(got("L") * m, L * m) <= tol, (p, "L")
        assert rel_err(got("Qbar") * m, Qbar * m) <= tol, (p, "Qbar")
        assert np.all(got("Qbar")[m == 0] == 0), (p, "Qbar pads")
        assert rel_err(res["F"][v:v + n], F) <= tol, (p, "F")
        assert rel_err(res["vbar"][v:v + n], vbar) <= tol, (p, "vbar")
        ld = oracle.logdet(L, k)
        assert abs(res["logdet"][p] - ld) <= tol * max(1.0, np.abs(np.log(L[:, 0])).sum() * 2), (p, "logdet")


BATCHES = [
    ([3000, 1, 0, 700, 257, 4, 12000, 3], [3, 0, 2, 5, 11, 12, 1, 5]),
    ([20011, 5, 999, 4000], [5, 5, 11, 7]),
    ([1, 2, 3], [0, 1, 2]),
]


@pytest.mark.parametrize("ns,ks", BATCHES)
def test_whiten_fp64(bo, ns, ks):
    print(f"case whiten fp64 ns={ns} ks={ks}", flush=True)
    Qs, vs, Fbs = draw(ns, ks, 51 + len(ns))
    plan = bo.Plan(ns, ks, target_chunks=300)
    res = run_wh(bo, plan, Qs, vs, Fbs)
    check(plan, Qs, vs, Fbs, res, TOL)


@pytest.mark.parametrize("ns,ks", BATCHES[:2])
def test_whiten_mixed(bo, ns, ks):
    print(f"case whiten mixed ns={ns} ks={ks}", flush=True)
    Qs, vs, Fbs = draw(ns, ks, 61 + len(ns))
    plan = bo.Plan(ns, ks, target_chunks=300)
    res = run_wh(bo, plan, Qs, vs, Fbs, prec=1)
    r32 = lambda a: a.astype(np.float32).astype(np.float64)
    check(plan, [rounded(a) for a in Qs], [r32(a) for a in vs], [r32(a) for a in Fbs], res, TOL_MIXED)


@pytest.mark.parametrize("prec", [0, 1])
def test_whiten_bwd_reusing_chunk_products(bo, prec):
    """The backward call taking the chunk products the forward call left in
    the workspace (reuse) meets the same bar against the oracle."""
    ns, ks = BATCHES[0]
    print(f"case whiten reuse prec={prec}", flush=True)
    Qs, vs, Fbs = draw(ns, ks, 71 + prec)
    plan = bo.Plan(ns, ks, target_chunks=300)
    res = run_wh(bo, plan, Qs, vs, Fbs, prec=prec, reuse=True)
    if prec == 0:
        check(plan, Qs, vs, Fbs, res, TOL)
    else:
        r32 = lambda a: a.astype(np.float32).astype(np.float64)
        check(plan, [rounded(a) for a in Qs], [r32(a) for a in vs], [r32(a) for a in Fbs], res, TOL_MIXED)


def test_whiten_full_size_rows(bo):
    """Two problems of 3e5 rows (k = 5) in the default chunk schedule."""
    print("case whiten full size", flush=True)
    ns, ks = [300_000, 300_000], [5, 5]
    Qs, vs, Fbs = draw(ns, ks, 8)
    plan = bo.Plan(ns, ks)
    res = run_wh(bo, plan, Qs, vs, Fbs)
    check(plan, Qs, vs, Fbs, res, TOL)


def test_whiten_info(bo):
    print("case whiten info", flush=True)
    ns, ks = [400, 300], [3, 2]
    Qs, vs, Fbs = draw(ns, ks, 12)
    Qs[1][150, 0] = -1.0
    plan = bo.Plan(ns, ks, target_chunks=60)
    res = run_wh(bo, plan, Qs, vs, Fbs)
    assert res["info"][0] == 0 and res["info"][1] == 151


def test_whiten_autograd_vs_dense(bo):
    """The autograd Function against dense torch autograd (CPU, FP64) of
    F = L^{-T} v through the band -> symmetric -> Cholesky construction."""
    from paper_1902_10078_amd import autograd as ag
    ns, ks = [9, 23, 4], [2, 3, 1]
    Qs, vs, Fbs = draw(ns, ks, 3)
    plan = bo.Plan(ns, ks)
    cu = lambda a: torch.tensor(np.concatenate([x.ravel() for x in a]), dtype=torch.float64, device="cuda",
                                requires_grad=True)
    tQ, tv = cu(Qs), cu(vs)
    F = ag.whiten(plan, tQ, tv)
    w = torch.tensor(np.concatenate(Fbs), device="cuda")
    (F * w).sum().backward()
    gQ, gv = tQ.grad.cpu().numpy(), tv.grad.cpu().numpy()
    for p, (n, k) in enumerate(zip(ns, ks)):
        Qt = torch.tensor(Qs[p], requires_grad=True)
        vt = torch.tensor(vs[p], requires_grad=True)
        M = torch.zeros((n, n), dtype=torch.float64)
        for d in range(min(k, n - 1) + 1):
            idx = torch.arange(n - d)
            M = M.index_put((idx + d, idx), Qt[: n - d, d])
            if d:
                M = M.index_put((idx, idx + d), Qt[: n - d, d])
        Lt = torch.linalg.cholesky(M)
        Ft = torch.linalg.solve_triangular(Lt.T.contiguous(), vt.reshape(n, 1), upper=True).reshape(n)
        (Ft * torch.tensor(Fbs[p])).sum().backward()
        o, v = plan.boff[p], plan.voff[p]
        assert np.max(np.abs(F.detach().cpu().numpy()[v:v + n] - Ft.detach().numpy())) <= 1e-12
        m = band_mask(n, k)
        g = Qt.grad.numpy() * m
        assert np.max(np.abs(gQ[o:o + n * (k + 1)].reshape(n, k + 1) * m - g)) <= 1e-11 * max(1.0, np.abs(g).max())
        assert np.max(np.abs(gv[v:v + n] - vt.grad.numpy())) <= 1e-12 * max(1.0, np.abs(gv[v:v + n]).max())
