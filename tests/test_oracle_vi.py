"""Pins for the oracle's variational KL term (Section 3.3, Eq. (KL),
Algorithm 7) against what the mathematics fixes, independently of the banded
recurrences: the dense closed form of the KL divergence between two Gaussians
(numpy inverse and log-determinants), KL(q || q) = 0 with a vanishing gradient
there, KL >= 0, central finite differences of the dense closed form for every
input, the marginal variances as the diagonal of the dense inverse, and the
batch entry point against the single one."""
import numpy as np
import pytest

import oracle
from bandutil import band_mask, lower_to_dense, rel_err
from paper_1902_10078_amd import inputs

SHAPES = [(1, 0), (1, 2), (2, 1), (3, 2), (5, 5), (7, 0), (12, 3), (17, 5), (23, 11), (40, 1)]


def draw(n, k, seed):
    rng = np.random.default_rng(seed)
    Lq = inputs.random_lower_band(n, k, rng) if n else np.zeros((0, k + 1))
    Lp = inputs.random_lower_band(n, k, rng) if n else np.zeros((0, k + 1))
    return Lq, Lp, rng.normal(size=n), rng.normal(size=n)


def dense_kl(Lq, Lp, mq, mp):
    """KL(N(mq, Qq^-1) || N(mp, Qp^-1)) from dense matrices."""
    Dq, Dp = lower_to_dense(Lq), lower_to_dense(Lp)
    Qq, Qp = Dq @ Dq.T, Dp @ Dp.T
    n = Qq.shape[0]
    dm = mp - mq
    return 0.5 * (np.trace(np.linalg.solve(Qq, Qp)) + np.linalg.slogdet(Qq)[1] - np.linalg.slogdet(Qp)[1]
                  + dm @ Qp @ dm - n)


@pytest.mark.parametrize("n,k", SHAPES)
def test_kl_matches_dense_closed_form(n, k):
    Lq, Lp, mq, mp = draw(n, k, 100 + n + 13 * k)
    r = oracle.vi_kl(Lq, Lp, k, mq, mp)
    kl = dense_kl(Lq, Lp, mq, mp)
    assert abs(r["parts"][0] - kl) <= 1e-11 * max(1.0, abs(kl))
    # the parts add up as Eq. (KL) states
    t, ld, maha = r["parts"][1:]
    assert abs(r["parts"][0] - 0.5 * (t + 2 * ld + maha - n)) <= 1e-12 * max(1.0, abs(kl))
    Dq, Dp = lower_to_dense(Lq), lower_to_dense(Lp)
    Sq = np.linalg.inv(Dq @ Dq.T)
    assert abs(t - np.trace(Sq @ (Dp @ Dp.T))) <= 1e-11 * max(1.0, abs(t))
    assert abs(ld - (np.log(np.diag(Dq)).sum() - np.log(np.diag(Dp)).sum())) <= 1e-12 * max(1.0, abs(ld))
    assert abs(maha - np.sum((Dp.T @ (mp - mq)) ** 2)) <= 1e-11 * max(1.0, maha)
    # marginal variances of q: diagonal of the dense inverse
    assert rel_err(r["Sig"][:, 0], np.diag(Sq)) <= 1e-12


@pytest.mark.parametrize("n,k", [(9, 2), (30, 5), (16, 0)])
def test_kl_of_a_distribution_with_itself(n, k):
    Lq, _, mq, _ = draw(n, k, 7 + n)
    r = oracle.vi_kl(Lq, Lq, k, mq, mq)
    assert abs(r["parts"][0]) <= 1e-11 * n
    # q = p is the minimum over q: the gradients in q vanish
    m = band_mask(n, k)
    assert np.abs(r["Lqbar"] * m).max() <= 1e-10
    assert np.abs(r["mqbar"]).max() <= 1e-12


def test_kl_nonnegative():
    for seed in range(20):
        Lq, Lp, mq, mp = draw(25, 3, 500 + seed)
        assert oracle.vi_kl(Lq, Lp, 3, mq, mp)["parts"][0] >= -1e-12


@pytest.mark.parametrize("n,k", [(6, 2), (11, 3), (9, 0), (14, 5)])
def test_kl_gradients_match_finite_differences(n, k):
    """Central differences of the dense closed form along random directions of
    the stored band entries of L_q, L_p and of m_q, m_p."""
    Lq, Lp, mq, mp = draw(n, k, 900 + n + k)
    r = oracle.vi_kl(Lq, Lp, k, mq, mp)
    rng = np.random.default_rng(3 + n)
    m = band_mask(n, k)
    h = 1e-6
    for _ in range(3):
        dLq, dLp = rng.normal(size=Lq.shape) * m, rng.normal(size=Lp.shape) * m
        dmq, dmp = rng.normal(size=n), rng.normal(size=n)
        for name, args_p, args_m, grad, dirn in (
                ("Lq", (Lq + h * dLq, Lp, mq, mp), (Lq - h * dLq, Lp, mq, mp), r["Lqbar"], dLq),
                ("Lp", (Lq, Lp + h * dLp, mq, mp), (Lq, Lp - h * dLp, mq, mp), r["Lpbar"], dLp),
                ("mq", (Lq, Lp, mq + h * dmq, mp), (Lq, Lp, mq - h * dmq, mp), r["mqbar"], dmq),
                ("mp", (Lq, Lp, mq, mp + h * dmp), (Lq, Lp, mq, mp - h * dmp), r["mpbar"], dmp)):
            fd = (dense_kl(*args_p) - dense_kl(*args_m)) / (2 * h)
            an = float(np.sum(grad * dirn))
            assert abs(fd - an) <= 1e-6 * max(1.0, abs(fd)), (name, fd, an)


def test_kl_batch_equals_single():
    ns, ks = [30, 1, 0, 45, 12], [3, 0, 2, 5, 11]
    Lqs, Lps, mqs, mps = zip(*[draw(n, k, 40 + i) for i, (n, k) in enumerate(zip(ns, ks))])
    cat = lambda a: np.concatenate([x.ravel() for x in a])
    parts, Lqbar, Lpbar, mqbar, mpbar, _ = oracle.vi_kl_batch(ns, ks, cat(Lqs), cat(Lps), cat(mqs), cat(mps))
    bo = vo = 0
    for p, (n, k) in enumerate(zip(ns, ks)):
        r = oracle.vi_kl(Lqs[p], Lps[p], k, mqs[p], mps[p])
        sz = n * (k + 1)
        assert np.array_equal(parts[p], r["parts"])
        assert np.array_equal(Lqbar[bo:bo + sz], r["Lqbar"].ravel())
        assert np.array_equal(Lpbar[bo:bo + sz], r["Lpbar"].ravel())
        assert np.array_equal(mqbar[vo:vo + n], r["mqbar"])
        assert np.array_equal(mpbar[vo:vo + n], r["mpbar"])
        bo += sz
        vo += n
