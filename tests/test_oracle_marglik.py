"""Pins for the oracle's log marginal likelihood with partial observations
(Section 3.1, Eq. (marg_lik); Algorithm 8) against the dense definition
log N(Y; 0, E Q^{-1} E^T + tau2 I) (numpy), its gradients against dense torch
autograd (CPU, FP64) through the band -> symmetric construction, and a
central difference in tau2; with every node observed, none, one, and k >= n."""
import numpy as np
import pytest
import torch

import oracle
from bandutil import band_mask, sym_to_dense
from paper_1902_10078_amd import inputs

CASES = [(40, 3, 0.6, 0.7), (25, 0, 1.0, 2.0), (30, 5, 0.0, 0.5), (12, 2, 0.1, 1.3), (6, 8, 0.5, 0.3), (1, 1, 1.0, 0.9)]


def draw(n, k, frac, seed):
    rng = np.random.default_rng(seed)
    L0 = inputs.random_lower_band(n, k, rng)
    Q = oracle.gbmm(L0, k, 0, L0, k, 0, tB=1, lc=k, uc=0)
    mask = (rng.random(n) < frac).astype(float)
    b = rng.normal(size=n) * mask
    return Q, mask, b


def dense_marglik(Qd, mask, b, tau2):
    obs = np.nonzero(mask)[0]
    if len(obs) == 0:
        return 0.0
    E = np.eye(Qd.shape[0])[obs]
    C = E @ np.linalg.inv(Qd) @ E.T + tau2 * np.eye(len(obs))
    Y = b[obs]
    return -0.5 * len(obs) * np.log(2 * np.pi) - 0.5 * np.linalg.slogdet(C)[1] - 0.5 * Y @ np.linalg.solve(C, Y)


@pytest.mark.parametrize("n,k,frac,tau2", CASES)
def test_marglik_matches_dense(n, k, frac, tau2):
    Q, mask, b = draw(n, k, frac, 3 + n + k)
    r = oracle.marglik(Q, k, mask, b, tau2)
    assert r["info"] == 0
    ref = dense_marglik(sym_to_dense(Q, k), mask, b, tau2)
    assert abs(r["parts"][0] - ref) <= 1e-11 * max(1.0, abs(ref))


@pytest.mark.parametrize("n,k,frac,tau2", CASES)
def test_marglik_gradients_match_dense_autograd(n, k, frac, tau2):
    Q, mask, b = draw(n, k, frac, 40 + n + k)
    r = oracle.marglik(Q, k, mask, b, tau2)
    obs = np.nonzero(mask)[0]
    Qt = torch.tensor(Q, requires_grad=True)
    Yt = torch.tensor(b[obs], requires_grad=True)
    tt = torch.tensor(tau2, dtype=torch.float64, requires_grad=True)
    # symmetric dense Q from the stored lower band (differentiable)
    Qd = torch.zeros((n, n), dtype=torch.float64)
    for d in range(min(k, n - 1) + 1):
        idx = torch.arange(n - d)
        Qd = Qd.index_put((idx + d, idx), Qt[: n - d, d])
        if d:
            Qd = Qd.index_put((idx, idx + d), Qt[: n - d, d])
    if len(obs):
        E = torch.eye(n, dtype=torch.float64)[torch.tensor(obs)]
        C = E @ torch.linalg.inv(Qd) @ E.T + tt * torch.eye(len(obs), dtype=torch.float64)
        lp = (-0.5 * len(obs) * np.log(2 * np.pi) - 0.5 * torch.logdet(C)
              - 0.5 * Yt @ torch.linalg.solve(C, Yt))
        lp.backward()
        gQ, gY, gt = Qt.grad.numpy(), Yt.grad.numpy(), tt.grad.item()
    else:
        gQ, gY, gt = np.zeros_like(Q), np.zeros(0), 0.0
    m = band_mask(n, k)
    scale = max(1.0, np.abs(gQ).max())
    assert np.abs(r["Qbar"] * m - gQ * m).max() <= 1e-9 * scale
    assert np.abs(r["bbar"][obs] - gY).max(initial=0.0) <= 1e-9 * max(1.0, np.abs(gY).max(initial=0.0))
    assert np.all(r["bbar"][mask == 0] == 0)
    assert abs(r["tau2bar"] - gt) <= 1e-9 * max(1.0, abs(gt))


def test_marglik_tau2_finite_difference():
    Q, mask, b = draw(30, 3, 0.5, 9)
    h = 1e-6
    f = lambda t: oracle.marglik(Q, 3, mask, b, t)["parts"][0]
    fd = (f(0.8 + h) - f(0.8 - h)) / (2 * h)
    assert abs(oracle.marglik(Q, 3, mask, b, 0.8)["tau2bar"] - fd) <= 1e-6 * max(1.0, abs(fd))
