"""The composite plan calls captured into HIP graphs: the marginal likelihood
(bo_plan_marglik), the natural-parameter GP regression (bo_plan_natgp), the
whitened sample and its reverse mode (bo_plan_whiten, bo_plan_whiten_bwd),
the KL term (bo_plan_vi_kl), and the graph GMRF band assembly with its
gradient gather (bo_csr_to_band, bo_band_to_csr_grad).  Each graph is
replayed several times, with the outputs overwritten and other eager work on
the device between replays, and every replay must equal the eager call bit
for bit (the kernels have no floating-point atomics, so a replay repeats the
same arithmetic in the same order)."""
import numpy as np
import pytest
import torch

import oracle
from paper_1902_10078_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bo():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1902_10078_amd import bandops
    bandops.lib()
    return bandops


def dev(a, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def spd_bands(ns, ks, rng):
    out = []
    for n, k in zip(ns, ks):
        L0 = inputs.random_lower_band(n, k, rng)
        out.append(oracle.gbmm(L0, k, 0, L0, k, 0, tB=1, lc=k, uc=0))
    return out


def check_replays(call, outs, reps=3):
    """Eager call, capture, then replays with the outputs poisoned before each
    and unrelated device work in between; every replay equals the eager run."""
    call()
    torch.cuda.synchronize()
    eager = {k: v.clone() for k, v in outs.items()}
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            call()
    torch.cuda.current_stream().wait_stream(s)
    junk = torch.randn(1 << 20, device="cuda", dtype=torch.float64)
    for rep in range(reps):
        for v in outs.values():
            if v.dtype.is_floating_point:
                v.fill_(float("nan"))
            else:
                v.fill_(-9)
        junk.mul_(1.0001).add_(0.5)   # eager work between the replays
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for k, v in outs.items():
            assert torch.equal(v, eager[k]), (rep, k)


def test_marglik_graph_replays(bo):
    print("case graph capture marglik", flush=True)
    rng = np.random.default_rng(1)
    ns, ks = [6000, 333, 2500], [5, 3, 11]
    Q = spd_bands(ns, ks, rng)
    mask = [(rng.random(n) < 0.5).astype(float) for n in ns]
    b = [rng.normal(size=n) * m for n, m in zip(ns, mask)]
    plan = bo.Plan(ns, ks, target_chunks=300)
    cat = lambda a: np.concatenate([x.ravel() for x in a])
    E, N, P = sum(q.size for q in Q), sum(ns), len(ns)
    t = dict(Q=dev(cat(Q)), mask=dev(cat(mask)), b=dev(cat(b)), tau2=dev([0.5, 1.0, 2.0]))
    outs = {nm: torch.zeros(E, dtype=torch.float64, device="cuda") for nm in ("L", "Sig", "Qbar")}
    outs.update({nm: torch.zeros(N, dtype=torch.float64, device="cuda") for nm in ("x", "bbar")})
    outs["tau2bar"] = torch.zeros(P, dtype=torch.float64, device="cuda")
    outs["parts"] = torch.zeros((P, 4), dtype=torch.float64, device="cuda")
    outs["info"] = torch.zeros(P, dtype=torch.int32, device="cuda")
    io = plan.ml_io(**t, **outs)
    check_replays(lambda: plan.marglik(0, io), outs)
    assert int(outs["info"].max()) == 0


def test_natgp_graph_replays(bo):
    print("case graph capture natgp", flush=True)
    rng = np.random.default_rng(2)
    ns, ks = [4000, 777, 1500], [5, 2, 11]
    Lpr = spd_bands(ns, ks, rng)
    Llik = [np.zeros_like(a) for a in Lpr]
    for a in Llik:
        a[:, 0] = rng.uniform(0.0, 2.0, size=a.shape[0])
    plan = bo.Plan(ns, ks, target_chunks=300)
    cat = lambda a: np.concatenate([x.ravel() for x in a])
    E, N, P = sum(q.size for q in Lpr), sum(ns), len(ns)
    t = dict(Lpr=dev(cat(Lpr)), etapr=dev(rng.normal(size=N)), Llik=dev(cat(Llik)), etalik=dev(rng.normal(size=N)))
    outs = {nm: torch.zeros(E, dtype=torch.float64, device="cuda") for nm in ("L", "Sig", "Lprbar", "Llikbar")}
    outs.update({nm: torch.zeros(N, dtype=torch.float64, device="cuda") for nm in ("x", "etaprbar")})
    outs["parts"] = torch.zeros((P, 5), dtype=torch.float64, device="cuda")
    outs["info"] = torch.zeros(P, dtype=torch.int32, device="cuda")
    io = plan.ng_io(**t, **outs)
    check_replays(lambda: plan.natgp(0, io), outs)
    assert int(outs["info"].max()) == 0


def test_whiten_graph_replays(bo):
    print("case graph capture whiten", flush=True)
    rng = np.random.default_rng(3)
    ns, ks = [5000, 1000, 3000], [5, 9, 1]
    Q = spd_bands(ns, ks, rng)
    plan = bo.Plan(ns, ks, target_chunks=300)
    E, N, P = sum(q.size for q in Q), sum(ns), len(ns)
    t = dict(Q=dev(np.concatenate([q.ravel() for q in Q])), v=dev(rng.normal(size=N)),
             Fbar=dev(rng.normal(size=N)))
    outs = dict(L=torch.zeros(E, dtype=torch.float64, device="cuda"),
                Qbar=torch.zeros(E, dtype=torch.float64, device="cuda"),
                F=torch.zeros(N, dtype=torch.float64, device="cuda"),
                vbar=torch.zeros(N, dtype=torch.float64, device="cuda"),
                logdet=torch.zeros(P, dtype=torch.float64, device="cuda"),
                info=torch.zeros(P, dtype=torch.int32, device="cuda"))
    io = plan.wh_io(**t, **outs)

    def call():
        plan.whiten(0, io)
        plan.whiten_bwd(0, io)
    check_replays(call, outs)


def test_vi_kl_graph_replays(bo):
    print("case graph capture vi_kl", flush=True)
    rng = np.random.default_rng(4)
    ns, ks = [3000, 700], [5, 3]
    Lq = [inputs.random_lower_band(n, k, rng) for n, k in zip(ns, ks)]
    Lp = [inputs.random_lower_band(n, k, rng) for n, k in zip(ns, ks)]
    plan = bo.Plan(ns, ks, target_chunks=200)
    E, N = sum(a.size for a in Lq), sum(ns)
    t = dict(Lq=dev(np.concatenate([a.ravel() for a in Lq])), Lp=dev(np.concatenate([a.ravel() for a in Lp])),
             mq=dev(rng.normal(size=N)), mp=dev(rng.normal(size=N)))
    outs = {nm: torch.zeros(E, dtype=torch.float64, device="cuda") for nm in ("Sig", "Lqbar", "Lpbar")}
    outs.update({nm: torch.zeros(N, dtype=torch.float64, device="cuda") for nm in ("mqbar", "mpbar")})
    outs["parts"] = torch.zeros((len(ns), 4), dtype=torch.float64, device="cuda")
    io = plan.kl_io(**t, **outs)
    check_replays(lambda: plan.vi_kl(0, io), outs)


def test_graph_gmrf_assembly_replays(bo):
    print("case graph capture csr_to_band", flush=True)
    n, ip, ix, ln = inputs.road_graph(3, 2000, seed=4)
    qip, qix, vals = inputs.graph_gmrf_csr(n, ip, ix, ln, ell=[2.0, 3.0])
    perm, iperm, bw = bo.rcm(qip, qix)
    pip, pix, mp = bo.csr_permute(qip, qix, perm, iperm)
    d_ip, d_ix = dev(pip, torch.int64), dev(pix, torch.int64)
    v = dev(np.concatenate([x[mp] for x in vals]))
    gband = dev(np.random.default_rng(5).normal(size=2 * n * (bw + 1)))
    outs = dict(band=torch.zeros(2 * n * (bw + 1), dtype=torch.float64, device="cuda"),
                dropped=torch.zeros(1, dtype=torch.int64, device="cuda"),
                gvals=torch.zeros(2 * pix.size, dtype=torch.float64, device="cuda"))

    def call():
        bo.csr_to_band(0, d_ip, d_ix, v, bw, outs["band"], None, outs["dropped"], nsets=2)
        bo.band_to_csr_grad(0, d_ip, d_ix, bw, gband, None, outs["gvals"], nsets=2)
    check_replays(call, outs)
    assert int(outs["dropped"].item()) == 0
