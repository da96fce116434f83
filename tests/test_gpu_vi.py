"""GPU parity of the variational KL term (bo_plan_vi_kl; Section 3.3, Eq. (KL),
Algorithm 7) against the FP64 oracle, through the C ABI, on seeded batches
that span many chunks and groups of the chunked passes and end in ragged
tails, with the degenerate sizes n = 0, n = 1, k = 0 and k >= n.

Tolerances: FP64 1e-12 relative (max-norm per output array, relative per
part).  The mixed format is compared with the oracle on the same FP32-rounded
inputs (FP64 diagonals kept) at 1e-6: intermediates (Sigma, Q_p / 2, v) are
stored in FP32."""
import numpy as np
import pytest
import torch

import oracle
import composed
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
    Lq = [inputs.random_lower_band(n, k, rng) if n else np.zeros((0, k + 1)) for n, k in zip(ns, ks)]
    Lp = [inputs.random_lower_band(n, k, rng) if n else np.zeros((0, k + 1)) for n, k in zip(ns, ks)]
    mq = [rng.normal(size=n) for n in ns]
    mp = [rng.normal(size=n) for n in ns]
    return Lq, Lp, mq, mp


def rounded(B):
    """FP32 records with the FP64 diagonal kept (the mixed format's values)."""
    R = B.astype(np.float32).astype(np.float64)
    if B.shape[0]:
        R[:, 0] = B[:, 0]
    return R


def run_kl(bo, plan, Lq, Lp, mq, mp, prec=0):
    cat = lambda a: np.concatenate([x.ravel() for x in a]) if a else np.zeros(0)
    dt = torch.float64 if prec == 0 else torch.float32
    dev = lambda a: torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")
    Lqf, Lpf = cat(Lq), cat(Lp)
    t = dict(Lq=dev(Lqf), Lp=dev(Lpf), mq=dev(cat(mq)), mp=dev(cat(mp)))
    E, N = Lqf.size, plan.rows
    for nm in ("Sig", "Lqbar", "Lpbar"):
        t[nm] = torch.full((E,), float("nan"), dtype=dt, device="cuda")
    for nm in ("mqbar", "mpbar"):
        t[nm] = torch.full((N,), float("nan"), dtype=dt, device="cuda")
    t["parts"] = torch.full((plan.nprob, 4), float("nan"), dtype=torch.float64, device="cuda")
    if prec == 1:
        diag = lambda arrs: torch.tensor(np.concatenate([a[:, 0] for a in arrs]) if arrs else np.zeros(0),
                                         dtype=torch.float64, device="cuda")
        t["Lqd"], t["Lpd"] = diag(Lq), diag(Lp)
        for nm in ("Sigd", "Lqbard", "Lpbard"):
            t[nm] = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
    plan.vi_kl(prec, plan.kl_io(**t))
    torch.cuda.synchronize()
    res = {k: v.detach().cpu().numpy().astype(np.float64) for k, v in t.items()}
    if prec == 1:   # put the FP64 diagonals into the records
        for nm in ("Sig", "Lqbar", "Lpbar"):
            for p, (n, k) in enumerate(zip(plan.ns, plan.ks)):
                o, v = plan.boff[p], plan.voff[p]
                res[nm][o:o + n * (k + 1):k + 1] = res[nm + "d"][v:v + n]
    return res


def check(bo, plan, Lq, Lp, mq, mp, res, tol):
    for p, (n, k) in enumerate(zip(plan.ns, plan.ks)):
        r = oracle.vi_kl(Lq[p], Lp[p], k, mq[p], mp[p])
        o, v = plan.boff[p], plan.voff[p]
        m = band_mask(n, k)
        # part scales: the log part is a difference of sums that cancel, so it
        # is measured against the sum of the magnitudes of its terms
        lsc = float(np.abs(np.log(Lq[p][:, 0])).sum() + np.abs(np.log(Lp[p][:, 0])).sum()) if n else 0.0
        t, maha = abs(r["parts"][1]), abs(r["parts"][3])
        scales = (0.5 * (t + 2 * lsc + maha + n), t, lsc, maha)
        for i in range(4):
            assert abs(res["parts"][p, i] - r["parts"][i]) <= tol * max(1.0, scales[i]), (p, i)
        for nm, rn in (("Sig", "Sig"), ("Lqbar", "Lqbar"), ("Lpbar", "Lpbar")):
            got = res[nm][o:o + n * (k + 1)].reshape(n, k + 1)
            assert rel_err(got * m, r[rn] * m) <= tol, (p, nm)
            assert np.all(got[m == 0] == 0), (p, nm, "pads")
        assert rel_err(res["mqbar"][v:v + n], r["mqbar"]) <= tol, (p, "mqbar")
        assert rel_err(res["mpbar"][v:v + n], r["mpbar"]) <= tol, (p, "mpbar")


BATCHES = [
    ([3000, 1, 0, 700, 257, 4, 12000, 3], [3, 0, 2, 5, 11, 12, 1, 5]),
    ([20011, 5, 999], [5, 5, 11]),
    ([1, 2, 3], [0, 1, 2]),
]


@pytest.mark.parametrize("ns,ks", BATCHES)
def test_vi_kl_fp64(bo, ns, ks):
    print(f"case vi_kl fp64 ns={ns} ks={ks}", flush=True)
    Lq, Lp, mq, mp = draw(ns, ks, 21 + len(ns))
    plan = bo.Plan(ns, ks, target_chunks=300)
    res = run_kl(bo, plan, Lq, Lp, mq, mp)
    check(bo, plan, Lq, Lp, mq, mp, res, TOL)


@pytest.mark.parametrize("ns,ks", BATCHES[:2])
def test_vi_kl_mixed(bo, ns, ks):
    print(f"case vi_kl mixed ns={ns} ks={ks}", flush=True)
    Lq, Lp, mq, mp = draw(ns, ks, 31 + len(ns))
    plan = bo.Plan(ns, ks, target_chunks=300)
    res = run_kl(bo, plan, Lq, Lp, mq, mp, prec=1)
    Lqr, Lpr = [rounded(a) for a in Lq], [rounded(a) for a in Lp]
    mqr = [a.astype(np.float32).astype(np.float64) for a in mq]
    mpr = [a.astype(np.float32).astype(np.float64) for a in mp]
    check(bo, plan, Lqr, Lpr, mqr, mpr, res, TOL_MIXED)


def test_vi_kl_of_q_with_itself(bo):
    """KL(q || q) = 0 and the gradients with respect to q vanish."""
    ns, ks = [5000, 333], [5, 3]
    Lq, _, mq, _ = draw(ns, ks, 77)
    plan = bo.Plan(ns, ks, target_chunks=200)
    res = run_kl(bo, plan, Lq, Lq, mq, mq)
    for p, (n, k) in enumerate(zip(ns, ks)):
        assert abs(res["parts"][p, 0]) <= 1e-10 * n
        o, v = plan.boff[p], plan.voff[p]
        m = band_mask(n, k)
        assert np.abs(res["Lqbar"][o:o + n * (k + 1)].reshape(n, k + 1) * m).max() <= 1e-9
        assert np.abs(res["mqbar"][v:v + n]).max() <= 1e-12


def test_vi_kl_full_size_rows(bo):
    """Two problems of 3e5 rows (k = 5) in the chunk schedule of the default
    plan: every output against the oracle."""
    ns, ks = [300_000, 300_000], [5, 5]
    print("case vi_kl full size", flush=True)
    Lq, Lp, mq, mp = draw(ns, ks, 5)
    plan = bo.Plan(ns, ks)
    res = run_kl(bo, plan, Lq, Lp, mq, mp)
    check(bo, plan, Lq, Lp, mq, mp, res, TOL)


def test_vi_kl_autograd_vs_dense_and_composed(bo):
    """The autograd Function against dense torch autograd (CPU, FP64) and
    against the same KL composed from the separate operators' Functions."""
    from paper_1902_10078_amd import autograd as ag
    ns, ks = [9, 23, 4], [2, 3, 1]
    Lq, Lp, mq, mp = draw(ns, ks, 61)
    plan = bo.Plan(ns, ks)
    cat = lambda a: np.concatenate([x.ravel() for x in a])
    cu = lambda a: torch.tensor(a, dtype=torch.float64, device="cuda", requires_grad=True)
    tq, tp, tmq, tmp = cu(cat(Lq)), cu(cat(Lp)), cu(cat(mq)), cu(cat(mp))
    g = torch.tensor([1.0, -0.5, 2.0], dtype=torch.float64, device="cuda")
    kl = ag.vi_kl(plan, tq, tp, tmq, tmp)
    (kl * g).sum().backward()
    grads = [t.grad.cpu().numpy() for t in (tq, tp, tmq, tmp)]
    for p, (n, k) in enumerate(zip(ns, ks)):
        o, v = plan.boff[p], plan.voff[p]
        # dense reference: scatter the band parameters into dense factors
        c = [torch.tensor(a, dtype=torch.float64, requires_grad=True) for a in (Lq[p], Lp[p], mq[p], mp[p])]

        def dense(B):
            M = torch.zeros((n, n), dtype=torch.float64)
            for d in range(k + 1):
                idx = torch.arange(n - d)
                M = M.index_put((idx + d, idx), B[: n - d, d])
            return M
        Dq, Dp = dense(c[0]), dense(c[1])
        Qq, Qp = Dq @ Dq.T, Dp @ Dp.T
        dm = c[3] - c[2]
        ref = 0.5 * (torch.trace(torch.linalg.solve(Qq, Qp)) + torch.logdet(Qq) - torch.logdet(Qp)
                     + dm @ Qp @ dm - n)
        assert abs(kl[p].item() - ref.item()) <= 1e-11 * max(1.0, abs(ref.item()))
        (ref * float(g[p])).backward()
        m = band_mask(n, k)
        sz = n * (k + 1)
        for got, rt in ((grads[0][o:o + sz].reshape(n, k + 1), c[0].grad.numpy() * m),
                        (grads[1][o:o + sz].reshape(n, k + 1), c[1].grad.numpy() * m),
                        (grads[2][v:v + n], c[2].grad.numpy()), (grads[3][v:v + n], c[3].grad.numpy())):
            assert np.max(np.abs(got - rt)) <= 1e-10 * max(1.0, np.max(np.abs(rt)))
        # composed from the operators' own Functions
        cq, cp = cu(Lq[p]), cu(Lp[p])
        lc = composed.vi_kl_composed(cq, cp, cu(mq[p]), cu(mp[p]))
        lc.backward()
        assert abs(lc.item() - kl[p].item()) <= 1e-11 * max(1.0, abs(ref.item()))
        refq = grads[0][o:o + sz].reshape(n, k + 1) / float(g[p])
        assert np.max(np.abs(cq.grad.cpu().numpy() * m - refq)) <= 1e-10 * max(1.0, np.max(np.abs(refq)))
