"""GPU parity of Gaussian-process regression with banded natural parameters
(bo_plan_natgp; Appendix C.5, Algorithm 10) against the FP64 oracle, through
the C ABI: seeded batches of random well-conditioned problems over several
bandwidths, chunks and groups with ragged tails and the degenerate sizes n = 0,
n = 1, k = 0, k >= n; CO2-shaped state-space problems (Matérn-3/2 trend plus
quasi-periodic harmonics, k = 7 and k = 11) up to the benchmark's size; the
mixed format; and the info codes.

Tolerances.  Random problems: FP64 1e-12 relative (max-norm per output array;
per part against the sum of the magnitudes of the terms that cancel in it).
CO2-shaped problems are ill-conditioned (condition numbers near 1e8 for the
prior precision), so their floor is measured: the oracle's own change under a
random relative perturbation of its inputs of 2^-52 per entry, times 100 (the
banded Cholesky is backward stable, with a backward error of a small multiple
of (k+1) eps per entry), and at least 1e-12.  Mixed format: against the oracle
on the same FP32-rounded inputs (FP64 diagonals kept) at 1e-6."""
import numpy as np
import pytest
import torch

import oracle
from bandutil import band_mask, rel_err
from paper_1902_10078_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12
TOL_MIXED = 1e-6
OUTS = ("Lprbar", "Llikbar", "etaprbar", "etalikbar")


@pytest.fixture(scope="module")
def bo():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1902_10078_amd import bandops
    bandops.lib()
    return bandops


def random_problems(ns, ks, seed):
    rng = np.random.default_rng(seed)
    out = []
    for n, k in zip(ns, ks):
        if n == 0:
            z = np.zeros((0, k + 1))
            out.append(dict(Lam_pr=z, eta_pr=np.zeros(0), Lam_lik=z.copy(), eta_lik=np.zeros(0), k=k))
            continue
        L0 = inputs.random_lower_band(n, k, rng)
        Lam_pr = oracle.gbmm(L0, k, 0, L0, k, 0, tB=1, lc=k, uc=0)
        kb = min(k, 2)
        B = inputs.random_lower_band(n, kb, rng, diag=(0.0, 1.0), off_sd=0.5)
        B *= (rng.random(n) < 0.7)[:, None]
        Lam_lik = np.zeros((n, k + 1))
        Lam_lik[:, :kb + 1] = oracle.gbmm(B, kb, 0, B, kb, 0, tB=1, lc=kb, uc=0) / 0.3
        out.append(dict(Lam_pr=Lam_pr, eta_pr=rng.normal(size=n) * 0.5, Lam_lik=Lam_lik,
                        eta_lik=rng.normal(size=n), k=k))
    return out


def co2_problems(Ts, Js, seed):
    return [inputs.co2_natgp(T, seed=seed + i, J=J) for i, (T, J) in enumerate(zip(Ts, Js))]


def rounded(B):
    R = B.astype(np.float32).astype(np.float64)
    if B.shape[0]:
        R[:, 0] = B[:, 0]
    return R


def run_ng(bo, plan, probs, prec=0):
    cat = lambda key: np.concatenate([p[key].ravel() for p in probs])
    dt = torch.float64 if prec == 0 else torch.float32
    dev = lambda a, d=dt: torch.tensor(np.ascontiguousarray(a), dtype=d, device="cuda")
    t = dict(Lpr=dev(cat("Lam_pr")), etapr=dev(cat("eta_pr")), Llik=dev(cat("Lam_lik")), etalik=dev(cat("eta_lik")))
    E, N, P = t["Lpr"].numel(), plan.rows, plan.nprob
    for nm in ("L", "Sig", "Lprbar", "Llikbar"):
        t[nm] = torch.full((E,), float("nan"), dtype=dt, device="cuda")
    for nm in ("x", "etaprbar"):
        t[nm] = torch.full((N,), float("nan"), dtype=dt, device="cuda")
    t["parts"] = torch.full((P, 5), float("nan"), dtype=torch.float64, device="cuda")
    t["info"] = torch.full((P,), -7, dtype=torch.int32, device="cuda")
    if prec == 1:
        diag = lambda key: torch.tensor(np.concatenate([p[key][:, 0] for p in probs]), dtype=torch.float64,
                                        device="cuda")
        t["Lprd"], t["Llikd"] = diag("Lam_pr"), diag("Lam_lik")
        for nm in ("Ld", "Sigd", "Lprbard", "Llikbard"):
            t[nm] = torch.full((N,), float("nan"), dtype=torch.float64, device="cuda")
    plan.natgp(prec, plan.ng_io(**t))
    torch.cuda.synchronize()
    res = {k: v.detach().cpu().numpy() for k, v in t.items()}
    res = {k: (v if k == "info" else v.astype(np.float64)) for k, v in res.items()}
    if prec == 1:
        for nm in ("L", "Sig", "Lprbar", "Llikbar"):
            for p, (n, k) in enumerate(zip(plan.ns, plan.ks)):
                o, v = plan.boff[p], plan.voff[p]
                res[nm][o:o + n * (k + 1):k + 1] = res[nm + "d"][v:v + n]
    return res


def oracle_all(p):
    r = oracle.natgp(p["Lam_pr"], p["eta_pr"], p["Lam_lik"], p["eta_lik"], p["k"])
    n, k = p["Lam_pr"].shape[0], p["k"]
    if n and r["info"] == 0:
        C, _ = oracle.chol(p["Lam_pr"] + p["Lam_lik"], k)
        r["L"], r["Sig"] = C, oracle.subset_inv(C, k)
    return r


def perturbation_floor(p, seed):
    """Largest relative change of each oracle output under a random relative
    perturbation of 2^-52 of every input entry."""
    rng = np.random.default_rng(seed)
    q = dict(p)
    for key in ("Lam_pr", "eta_pr", "Lam_lik", "eta_lik"):
        q[key] = p[key] * (1.0 + 2.0 ** -52 * rng.choice([-1.0, 1.0], size=p[key].shape))
    a, b = oracle_all(p), oracle_all(q)
    fl = {nm: rel_err(b[nm], a[nm]) for nm in OUTS + ("L", "Sig")}
    fl["parts"] = np.abs(b["parts"] - a["parts"])
    return fl


def check(plan, probs, res, tol, floors=None):
    for p, pr in enumerate(probs):
        n, k = plan.ns[p], plan.ks[p]
        r = oracle_all(pr)
        assert r["info"] == 0 and res["info"][p] == 0, (p, res["info"][p])
        o, v = plan.boff[p], plan.voff[p]
        m = band_mask(n, k)
        fl = floors[p] if floors else None
        t = lambda nm: max(tol, 100 * fl[nm]) if fl else tol
        parts = r["parts"]
        scales = (abs(parts[1]) + abs(parts[2]) + 0.5 * (parts[3] + parts[4]), abs(parts[1]), abs(parts[2]),
                  parts[3], parts[4])
        for i in range(5):
            lim = tol * max(1.0, scales[i])
            if fl:
                lim = max(lim, 100 * fl["parts"][i])
            assert abs(res["parts"][p, i] - parts[i]) <= lim, (p, i, res["parts"][p, i], parts[i])
        got = lambda nm: res[nm][o:o + n * (k + 1)].reshape(n, k + 1)
        for nm in ("Lprbar", "Llikbar", "L", "Sig"):
            if n == 0:
                continue
            assert rel_err(got(nm) * m, r[nm] * m) <= t(nm), (p, nm, rel_err(got(nm) * m, r[nm] * m))
            if nm in ("Lprbar", "Llikbar"):
                assert np.all(got(nm)[m == 0] == 0), (p, nm, "pads")
        assert rel_err(res["etaprbar"][v:v + n], r["etaprbar"]) <= t("etaprbar"), (p, "etaprbar")
        assert rel_err(res["x"][v:v + n], r["etalikbar"]) <= t("etalikbar"), (p, "x")


BATCHES = [
    ([3000, 1, 0, 700, 257, 4, 12000, 3], [3, 0, 2, 5, 11, 12, 1, 5]),
    ([20011, 5, 999], [5, 5, 11]),
    ([1, 2, 3], [0, 1, 2]),
]


@pytest.mark.parametrize("ns,ks", BATCHES)
def test_natgp_fp64(bo, ns, ks):
    print(f"case natgp fp64 ns={ns} ks={ks}", flush=True)
    probs = random_problems(ns, ks, 13 + len(ns))
    plan = bo.Plan(ns, ks, target_chunks=300)
    res = run_ng(bo, plan, probs)
    check(plan, probs, res, TOL)


@pytest.mark.parametrize("ns,ks", BATCHES[:2])
def test_natgp_mixed(bo, ns, ks):
    print(f"case natgp mixed ns={ns} ks={ks}", flush=True)
    probs = random_problems(ns, ks, 29 + len(ns))
    plan = bo.Plan(ns, ks, target_chunks=300)
    res = run_ng(bo, plan, probs, prec=1)
    rp = [dict(p, Lam_pr=rounded(p["Lam_pr"]), Lam_lik=rounded(p["Lam_lik"]),
               eta_pr=p["eta_pr"].astype(np.float32).astype(np.float64),
               eta_lik=p["eta_lik"].astype(np.float32).astype(np.float64)) for p in probs]
    check(plan, rp, res, TOL_MIXED)


@pytest.mark.parametrize("Ts,Js,chunks", [([500, 77, 1200], [2, 1, 2], 200), ([3082] * 6, [2] * 6, 0)])
def test_natgp_co2_shaped(bo, Ts, Js, chunks):
    """CO2-shaped problems (k = 7 for one harmonic, 11 for two); the second
    case has the benchmark's problem size in the default chunk schedule."""
    print(f"case natgp co2 Ts={Ts} Js={Js}", flush=True)
    probs = co2_problems(Ts, Js, 40)
    ns, ks = [p["Lam_pr"].shape[0] for p in probs], [p["k"] for p in probs]
    plan = bo.Plan(ns, ks, target_chunks=chunks)
    res = run_ng(bo, plan, probs)
    floors = [perturbation_floor(p, 7 + i) for i, p in enumerate(probs)]
    check(plan, probs, res, TOL, floors)


def test_natgp_info_codes(bo):
    """A prior precision that is not positive definite gives its failing row;
    a positive-definite prior whose posterior is not gives n + the
    posterior's failing row; the problems around them are unaffected."""
    print("case natgp info codes", flush=True)
    ns, ks = [300, 400, 500], [3, 2, 4]
    probs = random_problems(ns, ks, 81)
    probs[0]["Lam_pr"][123, 0] = -1.0
    probs[1]["Lam_lik"][77, 0] = -1e4
    plan = bo.Plan(ns, ks, target_chunks=60)
    res = run_ng(bo, plan, probs)
    for p in (0, 1):
        r = oracle_all(probs[p])
        assert r["info"] != 0 and res["info"][p] == r["info"], (p, res["info"][p], r["info"])
        assert np.all(np.isnan(res["parts"][p]))
    assert res["info"][0] == 124 and res["info"][1] == 400 + 78
    r = oracle_all(probs[2])
    assert res["info"][2] == 0
    assert abs(res["parts"][2, 0] - r["parts"][0]) <= 1e-12 * max(1.0, abs(r["parts"][1]) + abs(r["parts"][2]))


def test_natgp_autograd_vs_dense(bo):
    """The autograd Function against dense torch autograd (CPU, FP64) of
    a(eta_pr, Lam_pr) - a(eta_po, Lam_po) in all four inputs, with per-problem
    output weights."""
    from paper_1902_10078_amd import autograd as ag
    ns, ks = [9, 23, 4], [2, 3, 1]
    probs = random_problems(ns, ks, 93)
    plan = bo.Plan(ns, ks)
    cu = lambda key: torch.tensor(np.concatenate([p[key].ravel() for p in probs]), dtype=torch.float64,
                                  device="cuda", requires_grad=True)
    ts = [cu("Lam_pr"), cu("eta_pr"), cu("Lam_lik"), cu("eta_lik")]
    w = torch.tensor([0.5, 2.0, -1.0], dtype=torch.float64, device="cuda")
    val = ag.natgp(plan, *ts)
    (val * w).sum().backward()
    grads = [t.grad.cpu().numpy() for t in ts]
    for p, (n, k) in enumerate(zip(ns, ks)):
        c = [torch.tensor(probs[p][key], requires_grad=True) for key in ("Lam_pr", "eta_pr", "Lam_lik", "eta_lik")]

        def sym(B):
            M = torch.zeros((n, n), dtype=torch.float64)
            for d in range(min(k, n - 1) + 1):
                idx = torch.arange(n - d)
                M = M.index_put((idx + d, idx), B[: n - d, d])
                if d:
                    M = M.index_put((idx, idx + d), B[: n - d, d])
            return M
        a = lambda e, P: 0.5 * torch.logdet(P) - 0.5 * e @ torch.linalg.solve(P, e)
        ref = a(c[1], sym(c[0])) - a(c[1] + c[3], sym(c[0]) + sym(c[2]))
        assert abs(val[p].item() - ref.item()) <= 1e-11 * max(1.0, abs(ref.item()))
        (ref * float(w[p])).backward()
        o, v = plan.boff[p], plan.voff[p]
        m = band_mask(n, k)
        for i, (ct, band) in enumerate(zip(c, (True, False, True, False))):
            if band:
                got, want = grads[i][o:o + n * (k + 1)].reshape(n, k + 1) * m, ct.grad.numpy() * m
            else:
                got, want = grads[i][v:v + n], ct.grad.numpy()
            assert np.max(np.abs(got - want)) <= 1e-10 * max(1.0, np.abs(want).max()), i
