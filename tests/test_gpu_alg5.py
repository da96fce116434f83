"""GPU parity of the matrix solve with a banded right-hand side (Algorithm 5,
bo_solve_band_mat) and its reverse mode (Table 1, solve matrix-matrix;
bo_solve_band_mat_bwd) against the FP64 oracle, through the C ABI, on seeded
inputs: n from 1 to 2e5 (many blocks of 256 lanes and a ragged tail), widths
with lr > k, u = 0, k = 0 and k >= n; the mixed format against the oracle on
FP32-rounded inputs.  Tolerances: FP64 1e-12 relative (max-norm per output);
mixed 1e-5 (the outputs are stored in FP32)."""
import numpy as np
import pytest
import torch

import oracle
from bandutil import dense_to_gen, rel_err
from paper_1902_10078_amd import inputs

pytestmark = pytest.mark.gpu

SHAPES = [(1, 2, 1, 1), (9, 4, 0, 0), (12, 0, 1, 3), (300, 3, 2, 2), (1001, 2, 5, 1), (4099, 11, 3, 12),
          (200_000, 5, 2, 5)]


@pytest.fixture(scope="module")
def bo():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_1902_10078_amd import bandops
    bandops.lib()
    return bandops


def gen_mask(n, l, u):
    m = np.zeros((n, l + u + 1))
    for s in range(l + u + 1):
        j = np.arange(n)
        m[(j - u + s >= 0) & (j - u + s < n), s] = 1.0
    return m


def draw(n, k, lr, ur, seed):
    rng = np.random.default_rng(seed)
    L = inputs.random_lower_band(n, k, rng)
    R = rng.normal(size=(n, lr + ur + 1)) * gen_mask(n, lr, ur)
    return L, R, rng


def dev(a, dt=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dt, device="cuda")


def host(t):
    return t.detach().cpu().numpy().astype(np.float64)


@pytest.mark.parametrize("n,k,lr,ur", SHAPES)
def test_alg5_forward_and_reverse_fp64(bo, n, k, lr, ur):
    print(f"case alg5 n={n} k={k} lr={lr} ur={ur}", flush=True)
    L, R, rng = draw(n, k, lr, ur, 7 + n + k)
    O_ref = oracle.solve_band_mat(L, k, R, lr, ur)
    Obar = rng.normal(size=O_ref.shape) * gen_mask(n, k, ur)
    Rbar_ref, Lbar_ref = oracle.solve_band_mat_bwd(L, k, O_ref, Obar, lr, ur)
    Lb, Rb = bo.Band(dev(L), k), bo.Band(dev(R), lr, ur)
    O = bo.bo_solve_band_mat(Lb, Rb)
    Rbar, Lbar = bo.bo_solve_band_mat_bwd(Lb, O, bo.Band(dev(Obar), k, ur), lr)
    torch.cuda.synchronize()
    assert rel_err(host(O.band), O_ref * gen_mask(n, k, ur)) <= 1e-12
    assert rel_err(host(Rbar.band), Rbar_ref * gen_mask(n, lr, ur)) <= 1e-12
    assert rel_err(host(Lbar.band), Lbar_ref * gen_mask(n, k, 0)) <= 1e-12
    # pads are written as zero
    assert np.all(host(O.band)[gen_mask(n, k, ur) == 0] == 0)


@pytest.mark.parametrize("n,k,lr,ur", [(1001, 2, 5, 1), (4099, 11, 3, 12)])
def test_alg5_mixed(bo, n, k, lr, ur):
    print(f"case alg5 mixed n={n} k={k}", flush=True)
    L, R, rng = draw(n, k, lr, ur, 70 + n)
    Lr = L.astype(np.float32).astype(np.float64)
    Lr[:, 0] = L[:, 0]
    Rr = R.astype(np.float32).astype(np.float64)
    Rr[:, ur] = R[:, ur]
    O_ref = oracle.solve_band_mat(Lr, k, Rr, lr, ur)
    Lb = bo.Band(dev(L, torch.float32), k, 0, dev(L[:, 0]))
    Rb = bo.Band(dev(R, torch.float32), lr, ur, dev(R[:, ur]))
    O = bo.bo_solve_band_mat(Lb, Rb)
    torch.cuda.synchronize()
    got = host(O.band)
    got[:, ur] = host(O.diag)
    assert rel_err(got, O_ref * gen_mask(n, k, ur)) <= 1e-5


def test_alg5_argument_errors(bo):
    L = bo.Band(dev(np.ones((10, 3))), 2)
    R = bo.Band(dev(np.ones((10, 2))), 0, 1)
    O = bo.new_band(10, 1, 1)   # wrong lower width
    import ctypes
    lc, rc, oc = L.c(), R.c(), O.c()
    assert bo.lib().bo_solve_band_mat(0, ctypes.byref(lc), ctypes.byref(rc), ctypes.byref(oc), None) == -1
    W = bo.Band(dev(np.ones((10, 14))), 13)
    wc = W.c()
    O2 = bo.new_band(10, 13, 1)
    o2c = O2.c()
    assert bo.lib().bo_solve_band_mat(0, ctypes.byref(wc), ctypes.byref(rc), ctypes.byref(o2c), None) == -4


def test_alg5_autograd_gradcheck(bo):
    from paper_1902_10078_amd import autograd as ag
    n, k, lr, ur = 8, 2, 1, 2
    L, R, _ = draw(n, k, lr, ur, 5)
    Lt = dev(L).requires_grad_(True)
    Rt = dev(R).requires_grad_(True)
    mL, mR = dev(gen_mask(n, k, 0)), dev(gen_mask(n, lr, ur))
    f = lambda Lx, Rx: ag.solve_band_mat(Lx * mL, Rx * mR, lr, ur)
    assert torch.autograd.gradcheck(f, (Lt, Rt), eps=1e-6, atol=1e-7, rtol=1e-5)
