"""GPU parity of the log marginal likelihood with partial observations
(bo_plan_marglik; Section 3.1, Eq. (marg_lik), Algorithm 8) against the FP64
oracle, through the C ABI, on seeded batches that span many chunks and groups
of the chunked passes and end in ragged tails; with every node observed, none,
n = 0, n = 1, k = 0, k >= n, and the two failure kinds of the info code.

Tolerances: FP64 1e-12 relative (max-norm per output array; per part against
the sum of the magnitudes of its terms, which cancel).  The mixed format is
compared with the oracle on the same FP32-rounded inputs (FP64 diagonals
kept) at 1e-6: I(L), I(L_Q), x and L^{-1} b are stored in FP32 between the
passes."""
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


def draw(ns, ks, fracs, seed):
    rng = np.random.default_rng(seed)
    Q, mask, b = [], [], []
    for n, k, f in zip(ns, ks, fracs):
        if n:
            L0 = inputs.random_lower_band(n, k, rng)
            Q.append(oracle.gbmm(L0, k, 0, L0, k, 0, tB=1, lc=k, uc=0))
        else:
            Q.append(np.zeros((0, k + 1)))
        m = (rng.random(n) < f).astype(float)
        mask.append(m)
        b.append(rng.normal(size=n) * m)
    tau2 = rng.uniform(0.3, 2.0, size=len(ns))
    return Q, mask, b, tau2


def rounded(B):
    R = B.astype(np.float32).astype(np.float64)
    if B.shape[0]:
        R[:, 0] = B[:, 0]
    return R


def run_ml(bo, plan, Q, mask, b, tau2, prec=0):
    cat = lambda a: np.concatenate([x.ravel() for x in a]) if a else np.zeros(0)
    dt = torch.float64 if prec == 0 else torch.float32
    dev = lambda a, d=dt: torch.tensor(np.ascontiguousarray(a), dtype=d, device="cuda")
    Qf = cat(Q)
    E, N, P = Qf.size, plan.rows, plan.nprob
    t = dict(Q=dev(Qf), mask=dev(cat(mask)), b=dev(cat(b)), tau2=dev(tau2, torch.float64))
    for nm in ("L", "Sig", "Qbar"):
        t[nm] = torch.full((E,), float("nan"), dtype=dt, device="cuda")
    for nm in ("x", "bbar"):
        t[nm] = torch.full((N,), float("nan"), dtype=dt, device="cuda")
    t["tau2bar"] = torch.full((P,), float("nan"), dtype=torch.float64, device="cuda")
    t["parts"] = torch.full((P, 4), float("nan"), dtype=torch.float64, device="cuda")
    t["info"] = torch.full((P,), -7, dtype=torch.int32, device="cuda")
    if prec == 1:
        t["Qd"] = torch.tensor(np.concatenate([a[:, 0] for a in Q]) if Q else np.zeros(0),
                               dtype=torch.float64, device="cuda")
        for nm in ("Ld", "Sigd", "Qbard"):
            t[nm] = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
    plan.marglik(prec, plan.ml_io(**t))
    torch.cuda.synchronize()
    res = {k: v.detach().cpu().numpy() for k, v in t.items()}
    res = {k: (v if k == "info" else v.astype(np.float64)) for k, v in res.items()}
    if prec == 1:
        for nm in ("L", "Sig", "Qbar"):
            for p, (n, k) in enumerate(zip(plan.ns, plan.ks)):
                o, v = plan.boff[p], plan.voff[p]
                res[nm][o:o + n * (k + 1):k + 1] = res[nm + "d"][v:v + n]
    return res


def check(plan, Q, mask, b, tau2, res, tol):
    for p, (n, k) in enumerate(zip(plan.ns, plan.ks)):
        r = oracle.marglik(Q[p], k, mask[p], b[p], tau2[p])
        assert r["info"] == 0 and res["info"][p] == 0, p
        o, v = plan.boff[p], plan.voff[p]
        m = band_mask(n, k)
        # the log part is a sum of terms that cancel: scale by their magnitudes
        nm = mask[p].sum()
        t2 = tau2[p]
        terms = (0.5 * nm * np.log(2 * np.pi), abs(r["parts"][1]), abs(r["parts"][2]),
                 0.5 * nm * abs(np.log(t2)), b[p] @ b[p] / (2 * t2), r["parts"][3] / (2 * t2 * t2))
        scales = (sum(terms), abs(r["parts"][1]), abs(r["parts"][2]), abs(r["parts"][3]))
        for i in range(4):
            assert abs(res["parts"][p, i] - r["parts"][i]) <= tol * max(1.0, scales[i]), (p, i)
        tsc = abs(r["tau2bar"]) + nm / (2 * t2) + b[p] @ b[p] / (2 * t2 * t2) + r["parts"][3] / t2 ** 3
        assert abs(res["tau2bar"][p] - r["tau2bar"]) <= tol * max(1.0, tsc), (p, "tau2bar")
        got = res["Qbar"][o:o + n * (k + 1)].reshape(n, k + 1)
        assert rel_err(got * m, r["Qbar"] * m) <= tol, (p, "Qbar")
        assert np.all(got[m == 0] == 0), (p, "Qbar pads")
        assert rel_err(res["bbar"][v:v + n], r["bbar"]) <= tol, (p, "bbar")
        assert np.all(res["bbar"][v:v + n][mask[p] == 0] == 0), (p, "bbar unobserved")
        # the posterior factor, its band inverse and x = Q1^{-1} b
        if n:
            Q1 = Q[p].copy()
            Q1[:, 0] += mask[p] / t2
            L1, info = oracle.chol(Q1, k)
            assert info == 0
            gl = res["L"][o:o + n * (k + 1)].reshape(n, k + 1)
            assert rel_err(gl * m, L1 * m) <= tol, (p, "L")
            gs = res["Sig"][o:o + n * (k + 1)].reshape(n, k + 1)
            assert rel_err(gs * m, oracle.subset_inv(L1, k) * m) <= tol, (p, "Sig")
            xr = oracle.trsv(L1, k, oracle.trsv(L1, k, b[p]), trans=1)
            assert rel_err(res["x"][v:v + n], xr) <= tol, (p, "x")


BATCHES = [
    ([3000, 1, 0, 700, 257, 4, 12000, 3], [3, 0, 2, 5, 11, 12, 1, 5], [0.5, 1.0, 0.5, 0.0, 0.3, 1.0, 0.9, 0.5]),
    ([20011, 5, 999], [5, 5, 11], [0.2, 0.6, 1.0]),
    ([1, 2, 3], [0, 1, 2], [1.0, 0.5, 1.0]),
]


@pytest.mark.parametrize("ns,ks,fracs", BATCHES)
def test_marglik_fp64(bo, ns, ks, fracs):
    print(f"case marglik fp64 ns={ns} ks={ks}", flush=True)
    Q, mask, b, tau2 = draw(ns, ks, fracs, 11 + len(ns))
    plan = bo.Plan(ns, ks, target_chunks=300)
    res = run_ml(bo, plan, Q, mask, b, tau2)
    check(plan, Q, mask, b, tau2, res, TOL)


@pytest.mark.parametrize("ns,ks,fracs", BATCHES[:2])
def test_marglik_mixed(bo, ns, ks, fracs):
    print(f"case marglik mixed ns={ns} ks={ks}", flush=True)
    Q, mask, b, tau2 = draw(ns, ks, fracs, 23 + len(ns))
    plan = bo.Plan(ns, ks, target_chunks=300)
    res = run_ml(bo, plan, Q, mask, b, tau2, prec=1)
    Qr = [rounded(a) for a in Q]
    br = [a.astype(np.float32).astype(np.float64) for a in b]
    check(plan, Qr, mask, br, tau2, res, TOL_MIXED)


def test_marglik_full_size_rows(bo):
    """Two problems of 3e5 rows (k = 5, half the nodes observed) in the chunk
    schedule of the default plan: every output against the oracle."""
    ns, ks = [300_000, 300_000], [5, 5]
    print("case marglik full size", flush=True)
    Q, mask, b, tau2 = draw(ns, ks, [0.5, 0.5], 5)
    plan = bo.Plan(ns, ks)
    res = run_ml(bo, plan, Q, mask, b, tau2)
    check(plan, Q, mask, b, tau2, res, TOL)


def test_marglik_info_codes(bo):
    """A prior precision that is not positive definite: where the observations
    make Q1 positive definite the info is n + the failing row of C(Q); where Q1
    fails too, its own failing row.  The parts and tau2bar are NaN; the
    problems around them are unaffected."""
    print("case marglik info codes", flush=True)
    ns, ks, fracs = [400, 300, 500], [3, 2, 4], [0.5, 0.5, 0.5]
    Q, mask, b, tau2 = draw(ns, ks, fracs, 71)
    # problem 0: Q fails at row 123, which is observed with 1/tau2 large enough
    mask[0][123] = 1.0
    b[0][123] = 0.4
    tau2[0] = 0.01
    Q[0][123, 0] = -Q[0][123, 0] * 0.1
    # problem 1: Q1 fails at row 77 (unobserved)
    mask[1][77] = 0.0
    b[1][77] = 0.0
    Q[1][77, 0] = -1.0
    plan = bo.Plan(ns, ks, target_chunks=60)
    res = run_ml(bo, plan, Q, mask, b, tau2)
    for p in (0, 1):
        r = oracle.marglik(Q[p], ks[p], mask[p], b[p], tau2[p])
        assert r["info"] != 0
        assert res["info"][p] == r["info"], (p, res["info"][p], r["info"])
        assert np.all(np.isnan(res["parts"][p])) and np.isnan(res["tau2bar"][p])
    assert res["info"][0] > ns[0] and res["info"][1] <= ns[1]
    p = 2
    r = oracle.marglik(Q[p], ks[p], mask[p], b[p], tau2[p])
    assert res["info"][p] == 0
    assert abs(res["parts"][p, 0] - r["parts"][0]) <= 1e-12 * max(1.0, abs(r["parts"][1]) + abs(r["parts"][2]))


def test_marglik_autograd_vs_dense(bo):
    """The autograd Function against dense torch autograd (CPU, FP64) of
    log N(Y; 0, E Q^{-1} E^T + tau2 I) in the stored band of Q, in b at the
    observed nodes and in tau2, with per-problem output weights."""
    from paper_1902_10078_amd import autograd as ag
    ns, ks, fracs = [9, 23, 4], [2, 3, 1], [0.6, 0.5, 1.0]
    Q, mask, b, tau2 = draw(ns, ks, fracs, 91)
    plan = bo.Plan(ns, ks)
    cu = lambda a, rg=True: torch.tensor(np.concatenate([x.ravel() for x in a]) if isinstance(a, list) else a,
                                         dtype=torch.float64, device="cuda", requires_grad=rg)
    tQ, tb, tt = cu(Q), cu(b), cu(tau2)
    w = torch.tensor([1.0, -0.5, 2.0], dtype=torch.float64, device="cuda")
    lp = ag.marglik(plan, tQ, cu(mask, False), tb, tt)
    (lp * w).sum().backward()
    gQ, gb, gt = tQ.grad.cpu().numpy(), tb.grad.cpu().numpy(), tt.grad.cpu().numpy()
    for p, (n, k) in enumerate(zip(ns, ks)):
        obs = np.nonzero(mask[p])[0]
        Qt = torch.tensor(Q[p], requires_grad=True)
        bt = torch.tensor(b[p], requires_grad=True)
        t2 = torch.tensor(tau2[p], dtype=torch.float64, requires_grad=True)
        M = torch.zeros((n, n), dtype=torch.float64)
        for d in range(min(k, n - 1) + 1):
            idx = torch.arange(n - d)
            M = M.index_put((idx + d, idx), Qt[: n - d, d])
            if d:
                M = M.index_put((idx, idx + d), Qt[: n - d, d])
        E = torch.eye(n, dtype=torch.float64)[torch.tensor(obs)]
        C = E @ torch.linalg.inv(M) @ E.T + t2 * torch.eye(len(obs), dtype=torch.float64)
        Y = bt[torch.tensor(obs)]
        ref = -0.5 * len(obs) * np.log(2 * np.pi) - 0.5 * torch.logdet(C) - 0.5 * Y @ torch.linalg.solve(C, Y)
        assert abs(lp[p].item() - ref.item()) <= 1e-11 * max(1.0, abs(ref.item()))
        (ref * float(w[p])).backward()
        o, v = plan.boff[p], plan.voff[p]
        m = band_mask(n, k)
        g = Qt.grad.numpy() * m
        assert np.max(np.abs(gQ[o:o + n * (k + 1)].reshape(n, k + 1) * m - g)) <= 1e-10 * max(1.0, np.abs(g).max())
        gbr = bt.grad.numpy() * mask[p]
        assert np.max(np.abs(gb[v:v + n] * mask[p] - gbr)) <= 1e-10 * max(1.0, np.abs(gbr).max())
        assert abs(gt[p] - t2.grad.item()) <= 1e-10 * max(1.0, abs(t2.grad.item()))
