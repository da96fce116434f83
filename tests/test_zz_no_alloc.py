"""bo_chol_noalloc (the Cholesky entry point whose workspace is the library's
fixed device array) against bo_chol (the same operation with a caller
workspace) through the C ABI: two calls in a row, the second on a smaller
problem, so the second call runs on scratch memory that still holds the first
call's contents.  Same schedule and kernels, so the results must be equal bit
for bit, and within 1e-12 of the FP64 oracle."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from bandutil import band_mask, rel_err
from paper_1902_10078_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def bo():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1902_10078_amd import bandops
    bandops.lib()
    return bandops


def problem(n, k, seed):
    rng = np.random.default_rng(seed)
    L0 = inputs.random_lower_band(n, k, rng)
    return oracle.gbmm(L0, k, 0, L0, k, 0, tB=1, lc=k, uc=0), rng.normal(size=n)


def run_both(bo, Q, y, k, prec):
    Qb = bo.band_from(torch.tensor(Q, device="cuda"), k, 0, prec)
    vdt = torch.float64 if prec == bo.F64 else torch.float32
    yt = torch.tensor(y, dtype=vdt, device="cuda")
    a = bo.bo_chol(Qb, yt)
    n = Q.shape[0]
    out = (bo.new_band(n, k, 0, prec), torch.full((n,), float("nan"), dtype=vdt, device="cuda"),
           torch.full((1,), float("nan"), dtype=torch.float64, device="cuda"),
           torch.full((1,), -7, dtype=torch.int32, device="cuda"))
    out[0].band.fill_(float("nan"))
    b = bo.bo_chol_noalloc(Qb, yt, out=out)
    torch.cuda.synchronize()
    return a, b


@pytest.mark.parametrize("prec", [0, 1])
def test_noalloc_matches_bo_chol_twice(bo, prec):
    assert bo.lib().bo_chol_noalloc_scratch_bytes() == 64 << 20
    for n, k, seed in ((70001, 11, 1), (1000, 3, 2)):   # the second call is smaller
        print(f"case noalloc prec={prec} n={n} k={k}", flush=True)
        Q, y = problem(n, k, seed)
        (La, za, lda, ia), (Lb, zb, ldb, ib) = run_both(bo, Q, y, k, prec)
        assert int(ia.item()) == 0 and int(ib.item()) == 0
        m = band_mask(n, k)
        for x, w in ((La.band, Lb.band), (za, zb), (lda, ldb)):   # pads included: both write them 0
            assert torch.equal(x, w)
        if prec == 1:
            assert torch.equal(La.diag, Lb.diag)
        else:
            Lr, _ = oracle.chol(Q, k)
            assert rel_err(Lb.band.cpu().numpy() * m, Lr) <= 1e-12
            assert rel_err(zb.cpu().numpy(), oracle.trsv(Lr, k, y, 0)) <= 1e-12
            ld = oracle.logdet(Lr, k)
            assert abs(ldb.item() - ld) <= 1e-12 * abs(ld)


def test_noalloc_reports_failure_and_rejects_bad_arguments(bo):
    n, k = 5000, 5
    Q, y = problem(n, k, 3)
    Q = Q.copy()
    Q[1234, 0] = -1.0
    (_, _, _, ia), (_, _, ldb, ib) = run_both(bo, Q, y, k, 0)
    assert int(ia.item()) == 1235 and int(ib.item()) == 1235
    assert np.isnan(ldb.item())
    # argument errors return before any launch
    Qb = bo.band_from(torch.tensor(Q, device="cuda"), k)
    L = bo.new_band(n, k)
    qc, lc = Qb.c(), L.c()
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    lib = bo.lib()
    assert lib.bo_chol_noalloc(0, ctypes.byref(qc), ctypes.byref(lc), None, None, None, None, bo._stream()) == -1
    assert lib.bo_chol_noalloc(0, ctypes.byref(qc), ctypes.byref(lc), bo._ptr(info), None, None, bo._ptr(info),
                               bo._stream()) == -1
    L2 = bo.new_band(n, k - 1)
    l2 = L2.c()
    assert lib.bo_chol_noalloc(0, ctypes.byref(qc), ctypes.byref(l2), None, None, None, bo._ptr(info),
                               bo._stream()) == -1
