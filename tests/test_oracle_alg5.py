"""Pins for the oracle's matrix solve with a banded right-hand side
(Algorithm 5) and its reverse mode (Table 1, solve matrix-matrix): dense
triangular solves, dense torch autograd (CPU, FP64) through the map
(L, R) -> band of L^{-1} R, and central finite differences."""
import numpy as np
import pytest
import torch

import oracle
from bandutil import dense_to_gen, gen_to_dense, lower_to_dense, rel_err
from paper_1902_10078_amd import inputs

# (n, k, lr, ur): k sub-diagonals of L; R with lr lower and ur upper diagonals
SHAPES = [(25, 3, 2, 2), (17, 2, 5, 1), (12, 0, 1, 3), (9, 4, 0, 0), (1, 2, 1, 1), (3, 5, 2, 4), (30, 1, 1, 0)]


def draw(n, k, lr, ur, seed):
    rng = np.random.default_rng(seed)
    L = inputs.random_lower_band(n, k, rng)
    R = dense_to_gen(rng.normal(size=(n, n)), lr, ur)
    return L, R, rng


def gen_mask(n, l, u):
    m = np.zeros((n, l + u + 1))
    for j in range(n):
        for s in range(l + u + 1):
            if 0 <= j - u + s < n:
                m[j, s] = 1.0
    return m


@pytest.mark.parametrize("n,k,lr,ur", SHAPES)
def test_alg5_forward_matches_dense(n, k, lr, ur):
    L, R, _ = draw(n, k, lr, ur, 3 + n + k)
    O = oracle.solve_band_mat(L, k, R, lr, ur)
    ref = np.linalg.solve(lower_to_dense(L), gen_to_dense(R, lr, ur))
    assert rel_err(O * gen_mask(n, k, ur), dense_to_gen(ref, k, ur)) < 1e-12


def dense_band_map(Lt, Rt, n, k, lr, ur):
    """torch: band (k, ur) of L^{-1} R from the band parameters."""
    Ld = torch.zeros((n, n), dtype=torch.float64)
    for d in range(min(k, n - 1) + 1):
        idx = torch.arange(n - d)
        Ld = Ld.index_put((idx + d, idx), Lt[: n - d, d])
    Rd = torch.zeros((n, n), dtype=torch.float64)
    for s in range(lr + ur + 1):
        dd = s - ur   # row offset i - j
        for j in range(n):
            i = j + dd
            if 0 <= i < n:
                Rd = Rd.index_put((torch.tensor([i]), torch.tensor([j])), Rt[j, s].reshape(1))
    Od = torch.linalg.solve_triangular(Ld, Rd, upper=False)
    rows = []
    for j in range(n):
        rec = [Od[j - ur + s, j] if 0 <= j - ur + s < n else torch.zeros((), dtype=torch.float64)
               for s in range(k + ur + 1)]
        rows.append(torch.stack(rec))
    return torch.stack(rows)


@pytest.mark.parametrize("n,k,lr,ur", SHAPES)
def test_alg5_reverse_matches_dense_autograd(n, k, lr, ur):
    L, R, rng = draw(n, k, lr, ur, 50 + n + k)
    O = oracle.solve_band_mat(L, k, R, lr, ur)
    Obar = rng.normal(size=O.shape) * gen_mask(n, k, ur)
    Rbar, Lbar = oracle.solve_band_mat_bwd(L, k, O, Obar, lr, ur)
    Lt = torch.tensor(L, requires_grad=True)
    Rt = torch.tensor(R, requires_grad=True)
    Ob = dense_band_map(Lt, Rt, n, k, lr, ur)
    (Ob * torch.tensor(Obar)).sum().backward()
    mL = gen_mask(n, k, 0)
    assert rel_err(Lbar * mL, Lt.grad.numpy() * mL) < 1e-11
    mR = gen_mask(n, lr, ur)
    assert rel_err(Rbar * mR, Rt.grad.numpy() * mR) < 1e-11


@pytest.mark.parametrize("n,k,lr,ur", [(11, 2, 3, 1), (8, 3, 1, 2)])
def test_alg5_reverse_finite_differences(n, k, lr, ur):
    L, R, rng = draw(n, k, lr, ur, 90 + n)
    O = oracle.solve_band_mat(L, k, R, lr, ur)
    Obar = rng.normal(size=O.shape) * gen_mask(n, k, ur)
    Rbar, Lbar = oracle.solve_band_mat_bwd(L, k, O, Obar, lr, ur)
    f = lambda Lx, Rx: float(np.sum(oracle.solve_band_mat(Lx, k, Rx, lr, ur) * Obar))
    h = 1e-6
    for _ in range(3):
        dL = rng.normal(size=L.shape) * gen_mask(n, k, 0)
        dR = rng.normal(size=R.shape) * gen_mask(n, lr, ur)
        fdL = (f(L + h * dL, R) - f(L - h * dL, R)) / (2 * h)
        fdR = (f(L, R + h * dR) - f(L, R - h * dR)) / (2 * h)
        assert abs(fdL - np.sum(Lbar * dL)) <= 1e-6 * max(1.0, abs(fdL))
        assert abs(fdR - np.sum(Rbar * dR)) <= 1e-6 * max(1.0, abs(fdR))
