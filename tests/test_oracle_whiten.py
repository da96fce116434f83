"""Pins for the oracle's whitened GMRF sample (Section 3.2, Algorithm 6) and
its reverse mode: F = L^{-T} v with L L^T = Q.

- Whitening: stacking F over v = the unit vectors gives L^{-T}, and
  L^{-T} (L^{-T})^T must be the dense inverse of Q (F has covariance Q^{-1}).
- The forward map against a dense triangular solve (numpy).
- The reverse mode against dense torch autograd (CPU, FP64) through the
  band -> symmetric -> Cholesky -> triangular solve construction, and
  central differences."""
import numpy as np
import pytest
import torch

import oracle
from bandutil import band_mask, lower_to_dense, sym_to_dense
from paper_1902_10078_amd import inputs

SHAPES = [(30, 3), (17, 5), (12, 0), (6, 8), (1, 2), (25, 1)]


def draw(n, k, seed):
    rng = np.random.default_rng(seed)
    L0 = inputs.random_lower_band(n, k, rng)
    Q = oracle.gbmm(L0, k, 0, L0, k, 0, tB=1, lc=k, uc=0)
    return Q, rng


@pytest.mark.parametrize("n,k", SHAPES)
def test_whitened_samples_have_covariance_q_inverse(n, k):
    Q, _ = draw(n, k, 3 + n)
    cols = []
    for i in range(n):
        e = np.zeros(n)
        e[i] = 1.0
        L, F, info = oracle.whiten(Q, k, e)
        assert info == 0
        cols.append(F)
    Minv = np.array(cols).T   # column i = L^{-T} e_i
    Qd = sym_to_dense(Q, k)
    S = np.linalg.inv(Qd)
    assert np.max(np.abs(Minv @ Minv.T - S)) <= 1e-12 * max(1.0, np.abs(S).max())
    # the factor is the Cholesky factor: L L^T = Q
    Ld = lower_to_dense(L, k)
    assert np.max(np.abs(Ld @ Ld.T - Qd)) <= 1e-12 * np.abs(Qd).max()


@pytest.mark.parametrize("n,k", SHAPES)
def test_whiten_forward_matches_dense_solve(n, k):
    Q, rng = draw(n, k, 20 + n)
    v = rng.normal(size=n)
    L, F, info = oracle.whiten(Q, k, v)
    Ld = np.linalg.cholesky(sym_to_dense(Q, k))
    ref = np.linalg.solve(Ld.T, v)
    assert np.max(np.abs(F - ref)) <= 1e-12 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("n,k", SHAPES)
def test_whiten_reverse_matches_dense_autograd(n, k):
    Q, rng = draw(n, k, 40 + n)
    v = rng.normal(size=n)
    Fbar = rng.normal(size=n)
    L, F, _ = oracle.whiten(Q, k, v)
    vbar, Qbar = oracle.whiten_bwd(L, k, F, Fbar)
    Qt = torch.tensor(Q, requires_grad=True)
    vt = torch.tensor(v, requires_grad=True)
    M = torch.zeros((n, n), dtype=torch.float64)
    for d in range(min(k, n - 1) + 1):
        idx = torch.arange(n - d)
        M = M.index_put((idx + d, idx), Qt[: n - d, d])
        if d:
            M = M.index_put((idx, idx + d), Qt[: n - d, d])
    Lt = torch.linalg.cholesky(M)
    Ft = torch.linalg.solve_triangular(Lt.T.contiguous(), vt.reshape(n, 1), upper=True).reshape(n)
    (Ft * torch.tensor(Fbar)).sum().backward()
    m = band_mask(n, k)
    g = Qt.grad.numpy() * m
    assert np.max(np.abs(Qbar * m - g)) <= 1e-11 * max(1.0, np.abs(g).max())
    assert np.max(np.abs(vbar - vt.grad.numpy())) <= 1e-12 * max(1.0, np.abs(vbar).max())


def test_whiten_reverse_finite_differences():
    n, k = 14, 3
    Q, rng = draw(n, k, 77)
    v, Fbar = rng.normal(size=n), rng.normal(size=n)
    L, F, _ = oracle.whiten(Q, k, v)
    vbar, Qbar = oracle.whiten_bwd(L, k, F, Fbar)
    f = lambda Qx, vx: float(oracle.whiten(Qx, k, vx)[1] @ Fbar)
    m = band_mask(n, k)
    h = 1e-6
    for _ in range(3):
        dQ, dv = rng.normal(size=Q.shape) * m * 0.1, rng.normal(size=n)
        fd = (f(Q + h * dQ, v + h * dv) - f(Q - h * dQ, v - h * dv)) / (2 * h)
        an = float(np.sum(Qbar * dQ) + vbar @ dv)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd))


def test_whiten_info():
    Q, rng = draw(20, 2, 5)
    Q[9, 0] = -1.0
    _, F, info = oracle.whiten(Q, 2, rng.normal(size=20))
    assert info == 10 and np.all(np.isnan(F))
