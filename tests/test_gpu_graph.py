"""GPU band assembly of a graph GMRF precision in its reverse Cuthill-McKee
order (bo_csr_to_band) and the gather of band gradients back to the graph's
entries (bo_band_to_csr_grad), through the C ABI, against the oracle: exact
(byte work) in FP64 and in the mixed format's FP32 records with FP64
diagonals, for one and several value sets on a pattern, with the
dropped-entry count of a band that is too narrow; and end to end: the
whitened sample of the graph GMRF and its reverse mode gathered to the
graph's entries, against dense torch autograd (CPU, FP64) of the same map
(the pattern is permuted once on the host; the assembly reads each row of
P Q P^T from the diagonal rightwards)."""
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


def permuted(bo, n, ip, ix):
    perm, iperm, bw = bo.rcm(ip, ix)
    pip, pix, mp = bo.csr_permute(ip, ix, perm, iperm)
    return perm, bw, pip, pix, mp


@pytest.mark.parametrize("W,L,prec,nsets", [(4, 3000, 0, 1), (6, 500, 0, 3), (4, 3000, 1, 2), (3, 1, 0, 1)])
def test_csr_to_band_exact(bo, W, L, prec, nsets):
    print(f"case csr_to_band W={W} L={L} prec={prec} nsets={nsets}", flush=True)
    n, ip, ix, v = graph(W, L, 1)
    sets = [v * (1.0 + 0.25 * s) for s in range(nsets)]
    perm, bw, pip, pix, mp = permuted(bo, n, ip, ix)
    for k in (bw, bw + 2, max(bw - 2, 0)):
        refs = [oracle.csr_to_band(n, ip, ix, vs, perm, k) for vs in sets]
        dt = torch.float64 if prec == 0 else torch.float32
        band = torch.full((nsets * n * (k + 1),), float("nan"), dtype=dt, device="cuda")
        diag = torch.full((nsets * n,), float("nan"), dtype=torch.float64, device="cuda") if prec else None
        cnt = bo.csr_to_band(prec, dev(pip, torch.int64), dev(pix, torch.int64),
                             dev(np.concatenate([vs[mp] for vs in sets])), k, band, diag, nsets=nsets)
        got = band.cpu().numpy().astype(np.float64).reshape(nsets, n, k + 1)
        for s_, (ref, dropped) in enumerate(refs):
            want = ref if prec == 0 else ref.astype(np.float32).astype(np.float64)
            assert np.array_equal(got[s_], want), (k, s_)
            if prec:
                assert np.array_equal(diag.cpu().numpy()[s_ * n:(s_ + 1) * n], ref[:, 0])
        assert int(cnt.item()) == sum(d for _, d in refs), (k, int(cnt.item()))


def test_band_to_csr_grad_exact(bo):
    print("case band_to_csr_grad", flush=True)
    n, ip, ix, v = graph(4, 2000, 2)
    perm, bw, pip, pix, mp = permuted(bo, n, ip, ix)
    k = bw - 1   # a narrow band: some entries were dropped and get 0
    nsets = 2
    rng = np.random.default_rng(4)
    gband = rng.normal(size=(nsets, n, k + 1))
    gv = torch.full((nsets * pix.size,), float("nan"), dtype=torch.float64, device="cuda")
    bo.band_to_csr_grad(0, dev(pip, torch.int64), dev(pix, torch.int64), k, dev(gband.ravel()), None, gv,
                        nsets=nsets)
    rows = np.repeat(np.arange(n), np.diff(pip))
    inside = (pix >= rows) & (pix - rows <= k)
    got = gv.cpu().numpy().reshape(nsets, pix.size)
    for s_ in range(nsets):
        want = np.zeros(pix.size)
        want[inside] = gband[s_][rows[inside], (pix - rows)[inside]]
        assert np.array_equal(got[s_], want)


def test_graph_whiten_end_to_end(bo):
    """RCM, the permuted pattern, band assembly, the whitened sample and its
    reverse mode, and the gather to the graph's entries: the gradient of
    sum(F * Fbar) with respect to the permuted CSR values against dense
    autograd of the same map."""
    print("case graph whiten end to end", flush=True)
    n, ip, ix, v = graph(3, 30, 3)
    perm, bw, pip, pix, mp = permuted(bo, n, ip, ix)
    k = bw
    vn = v[mp]
    rng = np.random.default_rng(5)
    vv, Fb = rng.normal(size=n), rng.normal(size=n)   # in the new order
    band = torch.zeros(n * (k + 1), dtype=torch.float64, device="cuda")
    d_ip, d_ix = dev(pip, torch.int64), dev(pix, torch.int64)
    bo.csr_to_band(0, d_ip, d_ix, dev(vn), k, band)
    plan = bo.Plan([n], [k])
    z = lambda: torch.zeros(n, dtype=torch.float64, device="cuda")
    t = dict(Q=band, v=dev(vv), Fbar=dev(Fb), L=torch.zeros_like(band), Qbar=torch.zeros_like(band), F=z(), vbar=z())
    io = plan.wh_io(**t)
    plan.whiten(0, io)
    plan.whiten_bwd(0, io)
    gv = torch.zeros(pix.size, dtype=torch.float64, device="cuda")
    bo.band_to_csr_grad(0, d_ip, d_ix, k, t["Qbar"], None, gv)
    torch.cuda.synchronize()
    # dense reference: the entries the assembly reads are (j, c), c >= j, stored at (c, j)
    vt = torch.tensor(vn, requires_grad=True)
    rows = np.repeat(np.arange(n), np.diff(pip))
    up = pix >= rows
    M = torch.zeros((n, n), dtype=torch.float64)
    M = M.index_put((torch.tensor(pix[up]), torch.tensor(rows[up])), vt[torch.tensor(np.nonzero(up)[0])])
    M = M + torch.tril(M, -1).T
    Lt = torch.linalg.cholesky(M)
    Ft = torch.linalg.solve_triangular(Lt.T.contiguous(), torch.tensor(vv).reshape(n, 1), upper=True).reshape(n)
    (Ft * torch.tensor(Fb)).sum().backward()
    assert np.max(np.abs(t["F"].cpu().numpy() - Ft.detach().numpy())) <= 1e-12 * max(1.0, Ft.abs().max().item())
    g = vt.grad.numpy()
    assert np.max(np.abs(gv.cpu().numpy() - g)) <= 1e-11 * max(1.0, np.abs(g).max())
