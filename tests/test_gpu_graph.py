"""GPU band assembly of a graph GMRF precision in its reverse Cuthill-McKee
order (bo_csr_to_band) and the gather of band gradients back to the graph's
entries (bo_band_to_csr_grad), through the C ABI, against the oracle: exact
(byte work) in FP64 and in the mixed format's FP32 records with FP64
diagonals, with the dropped-entry count of a band that is too narrow; and end
to end: the whitened sample of the graph GMRF and its reverse mode gathered
to the graph's entries, against dense torch autograd (CPU, FP64) of the same
map."""
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


def graph(W, L, seed):
    n, ip, ix, ln = inputs.road_graph(W, L, seed=seed)
    qip, qix, qv = inputs.graph_gmrf_csr(n, ip, ix, ln)
    return n, qip, qix, qv


def dev(a, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


@pytest.mark.parametrize("W,L,prec", [(4, 3000, 0), (6, 500, 0), (4, 3000, 1), (3, 1, 0)])
def test_csr_to_band_exact(bo, W, L, prec):
    print(f"case csr_to_band W={W} L={L} prec={prec}", flush=True)
    n, ip, ix, v = graph(W, L, 1)
    perm, iperm, bw = bo.rcm(ip, ix)
    for k in (bw, bw + 2, max(bw - 2, 0)):
        ref, dropped = oracle.csr_to_band(n, ip, ix, v, perm, k)
        dt = torch.float64 if prec == 0 else torch.float32
        band = torch.full((n * (k + 1),), float("nan"), dtype=dt, device="cuda")
        diag = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda") if prec else None
        cnt = bo.csr_to_band(prec, dev(ip, torch.int64), dev(ix, torch.int64), dev(v), dev(iperm, torch.int64), k,
                             band, diag)
        got = band.cpu().numpy().astype(np.float64).reshape(n, k + 1)
        want = ref if prec == 0 else ref.astype(np.float32).astype(np.float64)
        assert np.array_equal(got, want), k
        if prec:
            assert np.array_equal(diag.cpu().numpy(), ref[:, 0])
        assert int(cnt.item()) == dropped, (k, int(cnt.item()), dropped)


def test_band_to_csr_grad_exact(bo):
    print("case band_to_csr_grad", flush=True)
    n, ip, ix, v = graph(4, 2000, 2)
    perm, iperm, bw = bo.rcm(ip, ix)
    k = bw - 1   # a narrow band: some entries were dropped and get 0
    rng = np.random.default_rng(4)
    gband = rng.normal(size=(n, k + 1))
    gv = torch.full((ix.size,), float("nan"), dtype=torch.float64, device="cuda")
    bo.band_to_csr_grad(0, dev(ip, torch.int64), dev(ix, torch.int64), dev(iperm, torch.int64), k,
                        dev(gband.ravel()), None, gv)
    rows = np.repeat(np.arange(n), np.diff(ip))
    a, b = iperm[rows], iperm[ix]
    inside = (a >= b) & (a - b <= k)
    want = np.zeros(ix.size)
    want[inside] = gband[b[inside], (a - b)[inside]]
    assert np.array_equal(gv.cpu().numpy(), want)


def test_graph_whiten_end_to_end(bo):
    """RCM, band assembly, the whitened sample and its reverse mode, and the
    gather to the graph's entries: the gradient of sum(F * Fbar) with respect
    to the CSR values against dense autograd of the same map (the band reads
    the entries on or below the diagonal of P Q P^T, mirrored)."""
    print("case graph whiten end to end", flush=True)
    n, ip, ix, v = graph(3, 30, 3)
    perm, iperm, bw = bo.rcm(ip, ix)
    k = bw
    rng = np.random.default_rng(5)
    vv, Fb = rng.normal(size=n), rng.normal(size=n)
    band = torch.zeros(n * (k + 1), dtype=torch.float64, device="cuda")
    d_ip, d_ix, d_ip2 = dev(ip, torch.int64), dev(ix, torch.int64), dev(iperm, torch.int64)
    bo.csr_to_band(0, d_ip, d_ix, dev(v), d_ip2, k, band)
    plan = bo.Plan([n], [k])
    # the plan runs in the new order: v and Fbar are given in that order
    z = lambda: torch.zeros(n, dtype=torch.float64, device="cuda")
    t = dict(Q=band, v=dev(vv[perm]), Fbar=dev(Fb[perm]), L=torch.zeros_like(band), Qbar=torch.zeros_like(band),
             F=z(), vbar=z())
    io = plan.wh_io(**t)
    plan.whiten(0, io)
    plan.whiten_bwd(0, io)
    gv = torch.zeros(ix.size, dtype=torch.float64, device="cuda")
    bo.band_to_csr_grad(0, d_ip, d_ix, d_ip2, k, t["Qbar"], None, gv)
    torch.cuda.synchronize()
    # dense reference in the new order
    vt = torch.tensor(v, requires_grad=True)
    rows = np.repeat(np.arange(n), np.diff(ip))
    a, b = iperm[rows], iperm[ix]
    low = a >= b
    M = torch.zeros((n, n), dtype=torch.float64)
    M = M.index_put((torch.tensor(a[low]), torch.tensor(b[low])), vt[torch.tensor(np.nonzero(low)[0])])
    M = M + torch.tril(M, -1).T
    Lt = torch.linalg.cholesky(M)
    Ft = torch.linalg.solve_triangular(Lt.T.contiguous(), torch.tensor(vv)[perm].reshape(n, 1), upper=True).reshape(n)
    (Ft * torch.tensor(Fb)[perm]).sum().backward()
    assert np.max(np.abs(t["F"].cpu().numpy() - Ft.detach().numpy())) <= 1e-12 * max(1.0, Ft.abs().max().item())
    g = vt.grad.numpy()
    assert np.max(np.abs(gv.cpu().numpy() - g)) <= 1e-11 * max(1.0, np.abs(g).max())
