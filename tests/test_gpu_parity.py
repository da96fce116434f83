"""GPU parity: every operator of libbandops.so against the FP64 oracle on the
same seeded inputs, through the C ABI.  Sizes span many chunks and groups of
the chunked scans (chunks of >= 32 rows, 64 chunks per group) and end in a
ragged tail; edge cases cover n = 0, 1, k = 0, k >= n, the widest compiled k,
non-SPD inputs and NaN inputs.

Tolerances: 1e-12 relative (max-norm per output array) in FP64 on the
well-conditioned inputs; the mixed format is compared with the oracle run on
the same FP32-rounded inputs, at 1e-6 (intermediates are stored in FP32:
observed ~1e-8, bound 1e-4)."""
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


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


def problem(n, k, seed):
    rng = np.random.default_rng(seed)
    L0 = inputs.random_lower_band(n, k, rng)
    Q = oracle.gbmm(L0, k, 0, L0, k, 0, tB=1, lc=k, uc=0) if n > 0 else np.zeros((0, k + 1))
    y = rng.normal(size=n)
    S = inputs.random_sym_band_dd(n, k, rng) if n > 0 else np.zeros((0, k + 1))
    return Q, y, S


def band(bo, A, l, u=0, prec=0):
    return bo.band_from(dev(A), l, u, prec)


def bands_close(got, ref, n, k, tol):
    m = band_mask(n, k)
    return rel_err(got * m, ref * m) <= tol


SIZES = [(0, 3), (1, 0), (1, 3), (2, 1), (5, 5), (13, 12), (31, 3), (33, 3), (100, 0), (257, 1),
         (1000, 3), (2049, 5), (5000, 2), (4099, 11), (3001, 12), (20011, 5), (70001, 3)]


@pytest.mark.parametrize("n,k", SIZES)
def test_chol_logdet_solve(bo, n, k):
    print(f"case chol n={n} k={k}", flush=True)
    Q, y, _ = problem(n, k, 1000 + n + k)
    Lref, info = oracle.chol(Q, k)
    assert info == 0
    L, z, logdet, dinfo = bo.bo_chol(band(bo, Q, k), dev(y))
    torch.cuda.synchronize()
    assert int(dinfo.item()) == 0
    assert bands_close(host(L.band), Lref, n, k, TOL)
    if n:
        assert rel_err(host(z), oracle.trsv(Lref, k, y, 0)) <= TOL
        ld = oracle.logdet(Lref, k)
        assert abs(logdet.item() - ld) <= TOL * max(1.0, abs(ld))


@pytest.mark.parametrize("n,k", SIZES)
def test_trsv_and_subset_inverse(bo, n, k):
    print(f"case trsv/subset_inv n={n} k={k}", flush=True)
    Q, y, _ = problem(n, k, 2000 + n + k)
    Lref, _ = oracle.chol(Q, k)
    Lb = band(bo, Lref, k)
    for trans in (0, 1):
        x = bo.bo_trsv(Lb, dev(y), trans)
        torch.cuda.synchronize()
        if n:
            assert rel_err(host(x), oracle.trsv(Lref, k, y, trans)) <= TOL, trans
    S = bo.bo_subset_inv(Lb)
    torch.cuda.synchronize()
    assert bands_close(host(S.band), oracle.subset_inv(Lref, k), n, k, TOL)


@pytest.mark.parametrize("n,k", SIZES)
def test_reverse_modes(bo, n, k):
    print(f"case bwd n={n} k={k}", flush=True)
    Q, y, _ = problem(n, k, 3000 + n + k)
    Lref, _ = oracle.chol(Q, k)
    rng = np.random.default_rng(n * 13 + k)
    m = band_mask(n, k)
    Lbar = rng.normal(size=Lref.shape) * m
    Sbar = rng.normal(size=Lref.shape) * m
    Lb = band(bo, Lref, k)
    # Algorithm 2
    Qbar = bo.bo_chol_bwd(Lb, band(bo, Lbar, k))
    # Algorithm 4
    Sref = oracle.subset_inv(Lref, k)
    Lbar4 = bo.bo_subset_inv_bwd(Lb, band(bo, Sref, k), band(bo, Sbar, k))
    torch.cuda.synchronize()
    assert bands_close(host(Qbar.band), oracle.chol_bwd(Lref, k, Lbar), n, k, TOL)
    assert bands_close(host(Lbar4.band), oracle.subset_inv_bwd(Lref, k, Sref, Sbar), n, k, TOL)
    # Table 1 solve rows, both transposes
    xbar = rng.normal(size=n)
    for trans in (0, 1):
        x = oracle.trsv(Lref, k, y, trans)
        bbar, Lbs = bo.bo_trsv_bwd(Lb, dev(x), dev(xbar), trans)
        torch.cuda.synchronize()
        rb, rL = oracle.trsv_bwd(Lref, k, x, xbar, trans)
        if n:
            assert rel_err(host(bbar), rb) <= TOL
        assert bands_close(host(Lbs.band), rL, n, k, TOL)
    # log-determinant
    g = torch.tensor([0.7], dtype=torch.float64, device="cuda")
    Lg = bo.bo_logdet_bwd(Lb, g, out=band(bo, Lbar, k), accumulate=True)
    torch.cuda.synchronize()
    assert bands_close(host(Lg.band), oracle.logdet_bwd(Lref, k, 0.7, Lbar), n, k, TOL)


@pytest.mark.parametrize("n", [1, 7, 500])
@pytest.mark.parametrize("la,ua,lb,ub,tA,tB", [(3, 0, 3, 0, 0, 1), (2, 1, 1, 3, 0, 0),
                                               (0, 2, 1, 1, 1, 0), (2, 2, 0, 3, 1, 1)])
def test_products_and_outer(bo, n, la, ua, lb, ub, tA, tB):
    rng = np.random.default_rng(n + 10 * la + ub)
    A = rng.normal(size=(n, la + ua + 1))
    B = rng.normal(size=(n, lb + ub + 1))
    C = bo.bo_gbmm(band(bo, A, la, ua), band(bo, B, lb, ub), tA, tB)
    x = rng.normal(size=n)
    yv = bo.bo_gbmv(band(bo, A, la, ua), dev(x), tA)
    mv, vv = rng.normal(size=n), rng.normal(size=n)
    O = bo.bo_outer_band(dev(mv), dev(vv), la, ua)
    torch.cuda.synchronize()
    ref = oracle.gbmm(A, la, ua, B, lb, ub, tA=tA, tB=tB)
    # the oracle writes zeros at out-of-matrix slots of its output; so does the GPU
    assert rel_err(host(C.band), ref) <= 1e-14
    # inputs may hold garbage in their padding: compare against padding-free A
    assert rel_err(host(yv), oracle.gbmv(A, la, ua, x, tA)) <= 1e-14
    assert rel_err(host(O.band), oracle.outer_band(mv, vv, la, ua)) == 0


def test_padding_is_never_read(bo):
    """NaN in every out-of-matrix slot of the inputs changes no output."""
    n, k = 1500, 5
    Q, y, S = problem(n, k, 77)
    Qn = Q.copy()
    Qn[band_mask(n, k) == 0] = np.nan
    L1, z1, ld1, _ = bo.bo_chol(band(bo, Q, k), dev(y))
    L2, z2, ld2, _ = bo.bo_chol(band(bo, Qn, k), dev(y))
    torch.cuda.synchronize()
    assert torch.equal(L1.band, L2.band) and torch.equal(z1, z2) and torch.equal(ld1, ld2)
    Ln = host(L1.band).copy()
    Ln[band_mask(n, k) == 0] = np.nan
    S1 = bo.bo_subset_inv(L1)
    S2 = bo.bo_subset_inv(band(bo, Ln, k))
    torch.cuda.synchronize()
    assert torch.equal(S1.band, S2.band)


@pytest.mark.parametrize("n,k,r", [(5000, 3, 4321), (300, 5, 0), (3000, 11, 64), (900, 1, 899)])
def test_non_spd_info(bo, n, k, r):
    Q, y, _ = problem(n, k, 99 + r)
    Lref, _ = oracle.chol(Q, k)
    Qb = Q.copy()
    Qb[r, 0] -= 1.5 * Lref[r, 0] ** 2
    _, oinfo = oracle.chol(Qb, k)
    assert oinfo == r + 1
    L, z, ld, info = bo.bo_chol(band(bo, Qb, k), dev(y))
    torch.cuda.synchronize()
    assert int(info.item()) == r + 1
    assert np.isnan(ld.item())
    # rows before r are still exact
    m = band_mask(n, k)
    assert rel_err(host(L.band)[:max(r - k, 0)] * m[:max(r - k, 0)], Lref[:max(r - k, 0)]) <= TOL or r <= k
    # NaN input
    Qn = Q.copy()
    Qn[r, 0] = np.nan
    _, _, _, info2 = bo.bo_chol(band(bo, Qn, k), dev(y))
    torch.cuda.synchronize()
    assert int(info2.item()) == r + 1


# --------------------------------------------------------------- mixed format

@pytest.mark.parametrize("n,k", [(1, 0), (999, 3), (6000, 5), (4099, 11)])
def test_mixed_precision_forward_and_backward(bo, n, k):
    Q, y, S = problem(n, k, 4000 + n + k)
    # the oracle runs on exactly the values the mixed format holds
    Qr = Q.astype(np.float32).astype(np.float64)
    Qr[:, 0] = Q[:, 0]
    yr = y.astype(np.float32).astype(np.float64)
    Lref, _ = oracle.chol(Qr, k)
    Qm = bo.band_from(dev(Q), k, 0, bo.MIXED)
    L, z, ld, info = bo.bo_chol(Qm, dev(y, torch.float32))
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    assert bands_close(host(L.dense_slots()), Lref, n, k, TOL_MIXED)
    assert rel_err(host(z), oracle.trsv(Lref, k, yr, 0)) <= TOL_MIXED
    ldr = oracle.logdet(Lref, k)
    assert abs(ld.item() - ldr) <= 1e-10 * max(1, abs(ldr))
    # backward through the mixed format: inputs L (FP32 + FP64 diag) as stored
    Lst = host(L.dense_slots())
    Sig = bo.bo_subset_inv(L)
    torch.cuda.synchronize()
    assert bands_close(host(Sig.dense_slots()), oracle.subset_inv(Lst, k), n, k, TOL_MIXED)


# ------------------------------------------------------------- batched plans

def packed_batch(ns, ks, seed):
    Ls, ys = inputs.config2_factors(seed, ns, ks)
    rng = np.random.default_rng(seed + 1)
    Qs = [oracle.gbmm(L, k, 0, L, k, 0, tB=1, lc=k, uc=0) for L, k in zip(Ls, ks)]
    Ss = [inputs.random_sym_band_dd(n, k, rng) for n, k in zip(ns, ks)]
    return Qs, ys, Ss


def run_plan_loss(bo, plan, Qs, ys, Ss, prec=0):
    cat = lambda arrs: np.concatenate([a.ravel() for a in arrs]) if arrs else np.zeros(0)
    Qf, yf, Sf = cat(Qs), cat(ys), cat(Ss)
    vdt = torch.float64 if prec == 0 else torch.float32
    Qt = dev(Qf, vdt)
    yt = dev(yf, vdt)
    St = dev(Sf, vdt)
    E, N = Qf.size, yf.size
    out = {nm: torch.full((E,), float("nan"), dtype=vdt, device="cuda") for nm in ("L", "Sig", "Lbar", "Qbar")}
    z = torch.zeros(N, dtype=vdt, device="cuda")
    yb = torch.zeros(N, dtype=vdt, device="cuda")
    parts = torch.zeros((len(Qs), 3), dtype=torch.float64, device="cuda")
    info = torch.zeros(len(Qs), dtype=torch.int32, device="cuda")
    kw = dict(Q=Qt, y=yt, S=St, L=out["L"], z=z, x=yb, Sig=out["Sig"], Lbar=out["Lbar"],
              Qbar=out["Qbar"], parts=parts, info=info)
    if prec == 1:
        diag_of = lambda arrs: dev(np.concatenate([a[:, 0] for a in arrs]))
        d = {nm: torch.zeros(N, dtype=torch.float64, device="cuda") for nm in ("Ld", "Sigd", "Lbard", "Qbard")}
        kw.update(Qd=diag_of(Qs), Sd=diag_of(Ss), **d)
    io = plan.io(**kw)
    plan.gauss_loss(prec, io)
    torch.cuda.synchronize()
    res = dict(parts=host(parts), info=info.cpu().numpy(), z=host(z), ybar=host(yb))
    for nm in ("L", "Sig", "Lbar", "Qbar"):
        res[nm] = host(out[nm])
    if prec == 1:
        for nm in ("L", "Sig", "Lbar", "Qbar"):
            res[nm + "d"] = host(kw[nm + "d"])
    return res, io, kw


def test_plan_gauss_loss_uneven_batch(bo):
    ns = [700, 1, 33, 5000, 0, 257, 12000, 64, 3, 2500]
    ks = [3, 0, 1, 5, 2, 11, 3, 12, 1, 5]
    Qs, ys, Ss = packed_batch(ns, ks, 5)
    plan = bo.Plan(ns, ks, target_chunks=600)
    res, _, _ = run_plan_loss(bo, plan, Qs, ys, Ss)
    assert np.all(res["info"] == 0)
    for p, (n, k) in enumerate(zip(ns, ks)):
        r = oracle.gauss_loss(Qs[p], k, ys[p], Ss[p])
        o, v = plan.boff[p], plan.voff[p]
        sz = n * (k + 1)
        for i in range(3):
            assert abs(res["parts"][p, i] - r["parts"][i]) <= TOL * max(1, abs(r["parts"][i])), (p, i)
        m = band_mask(n, k)
        for nm in ("L", "Sig", "Qbar"):
            assert rel_err(res[nm][o:o + sz].reshape(n, k + 1) * m, r[nm] * m) <= TOL, (p, nm)
        assert rel_err(res["ybar"][v:v + n], r["ybar"]) <= TOL
        assert rel_err(res["z"][v:v + n], r["z"]) <= TOL


@pytest.mark.parametrize("ks", [[4, 6, 7], [1, 2, 8, 9, 10]])
def test_plan_gauss_loss_more_bandwidths(bo, ks):
    ns = [3001, 2222, 1777, 999, 1500][: len(ks)]
    Qs, ys, Ss = packed_batch(ns, ks, 11 + len(ks))
    plan = bo.Plan(ns, ks, target_chunks=180)
    res, _, _ = run_plan_loss(bo, plan, Qs, ys, Ss)
    assert np.all(res["info"] == 0)
    for p, (n, k) in enumerate(zip(ns, ks)):
        r = oracle.gauss_loss(Qs[p], k, ys[p], Ss[p])
        o, v = plan.boff[p], plan.voff[p]
        m = band_mask(n, k)
        for i in range(3):
            assert abs(res["parts"][p, i] - r["parts"][i]) <= TOL * max(1, abs(r["parts"][i])), (p, i)
        for nm in ("L", "Sig", "Lbar", "Qbar"):
            if nm == "Lbar":
                continue   # the plan's Lbar is the subset-inverse part only
            assert rel_err(res[nm][o:o + n * (k + 1)].reshape(n, k + 1) * m, r[nm] * m) <= TOL, (p, nm)
        assert rel_err(res["ybar"][v:v + n], r["ybar"]) <= TOL


def test_plan_gauss_loss_mixed(bo):
    ns = [3000, 17, 9000, 400]
    ks = [3, 5, 11, 1]
    Qs, ys, Ss = packed_batch(ns, ks, 6)
    plan = bo.Plan(ns, ks, target_chunks=300)
    res, _, _ = run_plan_loss(bo, plan, Qs, ys, Ss, prec=1)
    for p, (n, k) in enumerate(zip(ns, ks)):
        Qr = Qs[p].astype(np.float32).astype(np.float64)
        Qr[:, 0] = Qs[p][:, 0]
        Sr = Ss[p].astype(np.float32).astype(np.float64)
        Sr[:, 0] = Ss[p][:, 0]
        yr = ys[p].astype(np.float32).astype(np.float64)
        r = oracle.gauss_loss(Qr, k, yr, Sr)
        o, v = plan.boff[p], plan.voff[p]
        sz = n * (k + 1)
        m = band_mask(n, k)
        for i in range(3):
            assert abs(res["parts"][p, i] - r["parts"][i]) <= TOL_MIXED * max(1, abs(r["parts"][i])), (p, i)
        Qb = res["Qbar"][o:o + sz].reshape(n, k + 1).copy()
        Qb[:, 0] = res["Qbard"][v:v + n]
        assert rel_err(Qb * m, r["Qbar"] * m) <= TOL_MIXED, p
        assert rel_err(res["ybar"][v:v + n], r["ybar"]) <= TOL_MIXED


def test_plan_forward(bo):
    ns = [4000, 100, 20000]
    ks = [5, 3, 1]
    Qs, ys, _ = packed_batch(ns, ks, 8)
    plan = bo.Plan(ns, ks, target_chunks=500)
    Qt = dev(np.concatenate([q.ravel() for q in Qs]))
    yt = dev(np.concatenate(ys))
    L = torch.zeros_like(Qt)
    Sig = torch.zeros_like(Qt)
    z, x = torch.zeros_like(yt), torch.zeros_like(yt)
    logdet = torch.zeros(3, dtype=torch.float64, device="cuda")
    info = torch.zeros(3, dtype=torch.int32, device="cuda")
    plan.forward(0, plan.io(Q=Qt, y=yt, L=L, z=z, x=x, Sig=Sig, logdet=logdet, info=info))
    torch.cuda.synchronize()
    Lh, Sh, zh, xh, ldh = host(L), host(Sig), host(z), host(x), host(logdet)
    for p, (n, k) in enumerate(zip(ns, ks)):
        Lr, _ = oracle.chol(Qs[p], k)
        o, v = plan.boff[p], plan.voff[p]
        m = band_mask(n, k)
        assert rel_err(Lh[o:o + n * (k + 1)].reshape(n, k + 1) * m, Lr) <= TOL
        assert rel_err(Sh[o:o + n * (k + 1)].reshape(n, k + 1) * m, oracle.subset_inv(Lr, k)) <= TOL
        zr = oracle.trsv(Lr, k, ys[p], 0)
        assert rel_err(zh[v:v + n], zr) <= TOL
        assert rel_err(xh[v:v + n], oracle.trsv(Lr, k, zr, 1)) <= TOL
        assert abs(ldh[p] - oracle.logdet(Lr, k)) <= TOL * abs(oracle.logdet(Lr, k))


def test_plan_isolation_of_failing_problem(bo):
    ns, ks = [3000, 2000, 1000], [3, 3, 5]
    Qs, ys, Ss = packed_batch(ns, ks, 9)
    Lr, _ = oracle.chol(Qs[1], 3)
    Qbad = [q.copy() for q in Qs]
    Qbad[1][1500, 0] -= 2 * Lr[1500, 0] ** 2
    plan = bo.Plan(ns, ks, target_chunks=200)
    good, _, _ = run_plan_loss(bo, plan, Qs, ys, Ss)
    bad, _, _ = run_plan_loss(bo, plan, Qbad, ys, Ss)
    assert list(bad["info"]) == [0, 1501, 0]
    for p in (0, 2):
        o, sz = plan.boff[p], ns[p] * (ks[p] + 1)
        assert np.array_equal(bad["Qbar"][o:o + sz], good["Qbar"][o:o + sz])
        assert np.array_equal(bad["parts"][p], good["parts"][p])


def test_graph_capture_replays(bo):
    """The batched loss captured into a HIP graph: every replay equals the eager
    result, also after the inputs change in place."""
    ns, ks = [5000, 300, 7000], [5, 3, 1]
    Qs, ys, Ss = packed_batch(ns, ks, 10)
    plan = bo.Plan(ns, ks, target_chunks=400)
    eager, io, kw = run_plan_loss(bo, plan, Qs, ys, Ss)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.gauss_loss(0, io)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        kw["Qbar"].fill_(float("nan"))
        kw["parts"].zero_()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(host(kw["Qbar"]), eager["Qbar"]), rep
        assert np.array_equal(host(kw["parts"]), eager["parts"]), rep
    # change y in place: the replay follows
    y2 = [2.0 * y for y in ys]
    kw["y"].copy_(dev(np.concatenate(y2)))
    g.replay()
    torch.cuda.synchronize()
    for p, (n, k) in enumerate(zip(ns, ks)):
        r = oracle.gauss_loss(Qs[p], k, y2[p], Ss[p])
        assert abs(host(kw["parts"])[p, 1] - r["parts"][1]) <= TOL * abs(r["parts"][1])


@pytest.mark.parametrize("n,k", [(3001, 5), (4099, 2), (257, 1)])
def test_padded_record_stride(bo, n, k):
    """Records with stride ld = k + 3 (two padding slots after the band) go
    through the per-lane work items; the factor, solve and subset inverse must
    equal the oracle's and the padding must stay untouched."""
    import ctypes
    print(f"case padded stride n={n} k={k}", flush=True)
    Q, y, _ = problem(n, k, 5000 + n + k)
    Lref, _ = oracle.chol(Q, k)
    ld = k + 3
    Qp = np.zeros((n, ld))
    Qp[:, :k + 1] = Q
    Qb = bo.Band(dev(Qp), k)
    Lb = bo.Band(torch.full((n, ld), 7.0, dtype=torch.float64, device="cuda"), k)
    Sb = bo.Band(torch.full((n, ld), 7.0, dtype=torch.float64, device="cuda"), k)
    yd, z = dev(y), torch.empty(n, dtype=torch.float64, device="cuda")
    logdet = torch.zeros(1, dtype=torch.float64, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    ws = bo.workspace(n, k)
    qc, lc, sc = Qb.c(), Lb.c(), Sb.c()
    bo._check(bo.lib().bo_chol(0, ctypes.byref(qc), ctypes.byref(lc), bo._ptr(yd), bo._ptr(z),
                               bo._ptr(logdet), bo._ptr(info), bo._ptr(ws), ws.numel(), bo._stream()),
              "bo_chol")
    bo._check(bo.lib().bo_subset_inv(0, ctypes.byref(lc), ctypes.byref(sc), bo._ptr(ws), ws.numel(),
                                     bo._stream()), "bo_subset_inv")
    torch.cuda.synchronize()
    assert int(info.item()) == 0
    Lg, Sg = host(Lb.band), host(Sb.band)
    assert bands_close(Lg[:, :k + 1], Lref, n, k, TOL)
    assert np.all(Lg[:, k + 1:] == 7.0) and np.all(Sg[:, k + 1:] == 7.0)
    assert rel_err(host(z), oracle.trsv(Lref, k, y, 0)) <= TOL
    assert abs(logdet.item() - oracle.logdet(Lref, k)) <= TOL * abs(oracle.logdet(Lref, k))
    assert bands_close(Sg[:, :k + 1], oracle.subset_inv(Lref, k), n, k, TOL)


@pytest.mark.parametrize("n,k,prec", [(100003, 10, 0), (100003, 11, 0), (70001, 12, 0), (100003, 11, 1)])
def test_quad_scans_same_bits_as_items(bo, n, k, prec):
    """From k = 10 the packed path runs the F1 summaries, group composes and
    sweeps on quads of lanes (fixed window slots in the summary); records with
    a padded stride run the one-lane work items on the same schedule.  Both
    compute every entry with the same operands in the same order, so the
    factor, z, log det and subset inverse agree bit for bit (and with the
    oracle)."""
    import ctypes
    print(f"case quad vs items n={n} k={k} prec={prec}", flush=True)
    Q, y, _ = problem(n, k, 7000 + n + k)
    Lref, _ = oracle.chol(Q, k)
    vdt = torch.float64 if prec == 0 else torch.float32
    bdt = vdt

    def run(ld):
        Qp = np.zeros((n, ld))
        Qp[:, :k + 1] = Q
        diag = dev(Q[:, 0]) if prec == 1 else None
        Qb = bo.Band(dev(Qp, bdt), k, 0, diag)
        Lb = bo.Band(torch.zeros((n, ld), dtype=bdt, device="cuda"), k, 0,
                     torch.zeros(n, dtype=torch.float64, device="cuda") if prec == 1 else None)
        Sb = bo.Band(torch.zeros((n, ld), dtype=bdt, device="cuda"), k, 0,
                     torch.zeros(n, dtype=torch.float64, device="cuda") if prec == 1 else None)
        yd, z = dev(y, vdt), torch.empty(n, dtype=vdt, device="cuda")
        logdet = torch.zeros(1, dtype=torch.float64, device="cuda")
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        ws = bo.workspace(n, k)
        qc, lc, sc = Qb.c(), Lb.c(), Sb.c()
        bo._check(bo.lib().bo_chol(prec, ctypes.byref(qc), ctypes.byref(lc), bo._ptr(yd), bo._ptr(z),
                                   bo._ptr(logdet), bo._ptr(info), bo._ptr(ws), ws.numel(),
                                   bo._stream()), "bo_chol")
        bo._check(bo.lib().bo_subset_inv(prec, ctypes.byref(lc), ctypes.byref(sc), bo._ptr(ws),
                                         ws.numel(), bo._stream()), "bo_subset_inv")
        torch.cuda.synchronize()
        assert int(info.item()) == 0
        out = {"L": host(Lb.band)[:, :k + 1], "S": host(Sb.band)[:, :k + 1], "z": host(z),
               "logdet": logdet.item()}
        if prec == 1:
            out["Ld"], out["Sd"] = host(Lb.diag), host(Sb.diag)
        return out

    quad, items = run(k + 1), run(k + 3)
    for nm in quad:
        assert np.array_equal(np.asarray(quad[nm]), np.asarray(items[nm])), nm
    tol = TOL if prec == 0 else TOL_MIXED
    assert abs(quad["logdet"] - oracle.logdet(Lref, k)) <= tol * abs(oracle.logdet(Lref, k))
    if prec == 0:
        assert bands_close(quad["L"], Lref, n, k, tol)


def test_graph_capture_forward_four_ranges_mixed(bo):
    """The forward list over problems of four bandwidths in the mixed format
    (each bandwidth range on its own stream, forked from and joined to the
    caller's stream) captured into a HIP graph: every replay, with eager
    library work on the same buffers in between, equals the eager call bit for
    bit."""
    ns, ks = [4000, 1300, 2500, 3100, 700, 5000], [11, 1, 5, 3, 11, 1]
    Qs, ys, _ = packed_batch(ns, ks, 21)
    plan = bo.Plan(ns, ks, target_chunks=240)
    Qf = np.concatenate([q.ravel() for q in Qs])
    N = sum(ns)
    kw = dict(Q=dev(Qf, torch.float32), Qd=dev(np.concatenate([q[:, 0] for q in Qs])),
              y=dev(np.concatenate(ys), torch.float32))
    for nm in ("L", "Sig"):
        kw[nm] = torch.zeros(Qf.size, dtype=torch.float32, device="cuda")
        kw[nm + "d"] = torch.zeros(N, dtype=torch.float64, device="cuda")
    for nm in ("z", "x"):
        kw[nm] = torch.zeros(N, dtype=torch.float32, device="cuda")
    kw["logdet"] = torch.zeros(len(ns), dtype=torch.float64, device="cuda")
    kw["info"] = torch.zeros(len(ns), dtype=torch.int32, device="cuda")
    io = plan.io(**kw)
    plan.forward(1, io)
    torch.cuda.synchronize()
    eager = {nm: t.clone() for nm, t in kw.items()}
    assert int(eager["info"].abs().max().item()) == 0
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.forward(1, io)
    torch.cuda.current_stream().wait_stream(s)
    for rep in range(3):
        for nm in ("L", "Sig", "Ld", "Sigd", "z", "x", "logdet"):
            kw[nm].fill_(float("nan"))
        plan.forward(1, io)          # eager work between the replays
        for nm in ("L", "Sig", "x"):
            kw[nm].fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        for nm in ("L", "Sig", "Ld", "Sigd", "z", "x", "logdet", "info"):
            assert torch.equal(kw[nm], eager[nm]), (rep, nm)
    # the eager result itself against the oracle on the stored inputs
    Lh = host(eager["L"])
    Ldh = host(eager["Ld"])
    for p, (n, k) in enumerate(zip(ns, ks)):
        Qr = Qs[p].astype(np.float32).astype(np.float64)
        Qr[:, 0] = Qs[p][:, 0]
        Lr, _ = oracle.chol(Qr, k)
        o, v = plan.boff[p], plan.voff[p]
        Lg = Lh[o:o + n * (k + 1)].reshape(n, k + 1).copy()
        Lg[:, 0] = Ldh[v:v + n]
        assert rel_err(Lg * band_mask(n, k), Lr) <= TOL_MIXED, p
