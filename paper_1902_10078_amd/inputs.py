"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers and assembles model matrices (state-space
Matérn precisions, random band factors); it holds none of the banded operators
themselves (no Cholesky, solve, subset inverse, product or their gradients), so
both the oracle-side tests and the GPU path can use it.  numpy only.

Band arrays follow the library's storage: shape (n, k+1), row j = record j =
column j of the lower band, slot d = element (j+d, j).  Slots past the end of the
matrix are 0.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


def _zero_pads(B: np.ndarray) -> np.ndarray:
    n, w = B.shape
    for d in range(1, w):
        B[max(n - d, 0):, d] = 0.0
    return B


def random_lower_band(n: int, k: int, rng: np.random.Generator,
                      diag=(1.0, 2.0), off_sd=0.3) -> np.ndarray:
    """Lower band factor with diagonal U[diag] and off-diagonals N(0, off_sd^2)."""
    L = np.empty((n, k + 1))
    L[:, 0] = rng.uniform(diag[0], diag[1], size=n)
    if k > 0:
        L[:, 1:] = rng.normal(0.0, off_sd, size=(n, k))
    return _zero_pads(L)


def random_sym_band_dd(n: int, k: int, rng: np.random.Generator,
                       off_sd=0.3, diag_extra=(0.5, 1.0)) -> np.ndarray:
    """Symmetric band (stored lower) made positive semi-definite by diagonal
    dominance: S_ij ~ N(0, off_sd^2) for 0 < i-j <= k, and
    S_ii = sum_{j != i} |S_ij| + U[diag_extra] (Gershgorin)."""
    S = np.zeros((n, k + 1))
    if k > 0:
        S[:, 1:] = rng.normal(0.0, off_sd, size=(n, k))
    _zero_pads(S)
    absrow = np.zeros(n)
    for d in range(1, k + 1):
        a = np.abs(S[: n - d, d]) if n > d else np.zeros(0)
        absrow[: n - d] += a          # |S[j+d, j]| counted in row j (upper part)
        absrow[d:] += a               # and in row j+d (lower part)
    S[:, 0] = absrow + rng.uniform(diag_extra[0], diag_extra[1], size=n)
    return S


# ---------------------------------------------------------------------------
# Matérn state-space models (Section 2; appendix "GP regression with banded
# precision"): state s_t = (f, f', ...)(x_t) of dimension d, s_0 ~ N(0, P0),
# s_t | s_{t-1} ~ N(A_t s_{t-1}, Q_t).  Interleaving the states gives a
# block-tridiagonal precision with scalar lower bandwidth 2d - 1.
# ---------------------------------------------------------------------------

@dataclass
class SSM:
    A: np.ndarray    # (T, d, d): A[t] maps s_{t-1} -> s_t for t >= 1 (A[0] unused)
    Qt: np.ndarray   # (T, d, d): Q[t] innovation covariance, Q[0] = P0
    d: int
    Qinv: np.ndarray = None   # set by ssm_precision_band


def _expm1_tail(y: np.ndarray, order: int) -> np.ndarray:
    """sum_{m > order} y^m / m!  without cancellation (series for small y)."""
    y = np.asarray(y, dtype=np.float64)
    out = np.empty_like(y)
    small = y < 1.0
    ys = y[small]
    term = ys ** (order + 1) / math.factorial(order + 1)
    acc = term.copy()
    for m in range(order + 2, order + 40):
        term = term * ys / m
        acc += term
    out[small] = acc
    yl = y[~small]
    poly = np.zeros_like(yl)
    for m in range(order + 1):
        poly += yl ** m / math.factorial(m)
    out[~small] = np.exp(yl) - poly
    return out


def matern32_ssm(x: np.ndarray, ell: float, sigma2: float = 1.0) -> SSM:
    """Matérn-3/2 (d = 2) transition and innovation covariances for sorted
    inputs x, with the innovation covariance written without cancellation
    (y = 2 lambda Delta):
      Q11 = s2 e^-y sum_{m>=3} y^m/m!,  Q12 = 2 lambda^3 Delta^2 s2 e^-y,
      Q22 = lambda^2 s2 e^-y (2y + sum_{m>=3} y^m/m!)."""
    lam = math.sqrt(3.0) / ell
    T = len(x)
    dx = np.diff(x)
    A = np.zeros((T, 2, 2))
    Qt = np.zeros((T, 2, 2))
    Qt[0] = np.diag([sigma2, lam * lam * sigma2])
    e = np.exp(-lam * dx)
    A[1:, 0, 0] = e * (1 + lam * dx)
    A[1:, 0, 1] = e * dx
    A[1:, 1, 0] = -e * lam * lam * dx
    A[1:, 1, 1] = e * (1 - lam * dx)
    y = 2 * lam * dx
    ey = np.exp(-y)
    tail = _expm1_tail(y, 2)
    Qt[1:, 0, 0] = sigma2 * ey * tail
    Qt[1:, 0, 1] = Qt[1:, 1, 0] = 2 * lam ** 3 * dx ** 2 * sigma2 * ey
    Qt[1:, 1, 1] = lam * lam * sigma2 * ey * (2 * y + tail)
    return SSM(A=A, Qt=Qt, d=2)


def quasi_periodic_ssm(x: np.ndarray, ell: float, sigma2: float, f0: float, J: int) -> SSM:
    """k(tau) = sigma2 e^{-|tau|/ell} sum_{j=1..J} cos(2 pi j f0 tau): a
    Matérn-1/2 envelope on J harmonics, two states per harmonic (d = 2J).  Per
    harmonic: A = e^{-Delta/ell} R(2 pi j f0 Delta) (R a rotation), stationary
    covariance sigma2 I, innovation sigma2 (1 - e^{-2 Delta/ell}) I."""
    T = len(x)
    dx = np.diff(x)
    A = np.zeros((T, 2 * J, 2 * J))
    Qt = np.zeros((T, 2 * J, 2 * J))
    e = np.exp(-dx / ell)
    q = -sigma2 * np.expm1(-2.0 * dx / ell)
    for j in range(J):
        w = 2.0 * math.pi * (j + 1) * f0 * dx
        a = 2 * j
        A[1:, a, a] = e * np.cos(w)
        A[1:, a, a + 1] = -e * np.sin(w)
        A[1:, a + 1, a] = e * np.sin(w)
        A[1:, a + 1, a + 1] = e * np.cos(w)
        Qt[0, a, a] = Qt[0, a + 1, a + 1] = sigma2
        Qt[1:, a, a] = Qt[1:, a + 1, a + 1] = q
    return SSM(A=A, Qt=Qt, d=2 * J)


def sum_ssm(*ms: SSM) -> SSM:
    """The state-space model of a sum of kernels: the components' states
    stacked per input (block-diagonal transitions and covariances)."""
    T = ms[0].A.shape[0]
    d = sum(m.d for m in ms)
    A = np.zeros((T, d, d))
    Qt = np.zeros((T, d, d))
    o = 0
    for m in ms:
        A[:, o:o + m.d, o:o + m.d] = m.A
        Qt[:, o:o + m.d, o:o + m.d] = m.Qt
        o += m.d
    return SSM(A=A, Qt=Qt, d=d)


def co2_natgp(T: int, seed: int = 6, J: int = 2, h: float = 1.0 / 52, ell_s: float = 2.0,
              s2_s: float = 1.0, ell_q: float = 1.0, s2_q: float = 0.5, f0: float = 1.0,
              tau2: float = 0.1, p_obs: float = 0.95):
    """A CO2-shaped regression problem in banded natural parameters: weekly
    inputs x_t = t h (years), a Matérn-3/2 trend plus the quasi-periodic kernel
    of J harmonics (d = 2 + 2J states per input, bandwidth 2d - 1 = 4J + 3),
    observation y_t = H s_t + N(0, tau2) with H summing the components' first
    states, each week observed with probability p_obs.
    Returns dict: Lam_pr (lower band of the prior precision), eta_pr (a prior
    natural mean, N(0, 0.1^2) entries), Lam_lik (lower band of H^T H / tau2 per
    observed input), eta_lik (H^T y_t / tau2 per observed input), k, d, H, y,
    obs, tau2."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, T, J]))
    x = np.arange(T) * h
    m = sum_ssm(matern32_ssm(x, ell_s, s2_s), quasi_periodic_ssm(x, ell_q, s2_q, f0, J))
    d = m.d
    k = 2 * d - 1
    Lam_pr = ssm_precision_band(m)
    N = T * d
    H = np.zeros(d)
    H[0] = 1.0
    H[2::2] = 1.0
    obs = rng.random(T) < p_obs
    y = (0.05 * x + np.sin(2 * math.pi * x) + rng.normal(scale=math.sqrt(tau2), size=T)) * obs
    Lam_lik = np.zeros((N, k + 1))
    Bl = Lam_lik.reshape(T, d, k + 1)
    for a in range(d):
        for b in range(a, d):
            Bl[:, a, b - a] = obs * H[a] * H[b] / tau2
    eta_lik = (obs[:, None] * y[:, None] * H[None, :] / tau2).reshape(N)
    eta_pr = rng.normal(scale=0.1, size=N)
    return dict(Lam_pr=Lam_pr, eta_pr=eta_pr, Lam_lik=_zero_pads(Lam_lik), eta_lik=eta_lik, k=k, d=d, H=H,
                y=y, obs=obs, tau2=tau2)


def matern52_stationary(ell: float, sigma2: float = 1.0) -> np.ndarray:
    lam = math.sqrt(5.0) / ell
    k = lam * lam / 3.0
    return sigma2 * np.array([[1.0, 0.0, -k], [0.0, k, 0.0], [-k, 0.0, lam ** 4]])


def matern52_transition_mp(delta: float, ell: float, sigma2: float = 1.0,
                           dps: int = 50):
    """A = expm(F delta) and Q = Pinf - A Pinf A^T for Matérn-5/2 evaluated in
    `dps`-digit arithmetic (mpmath), rounded to float64."""
    import mpmath as mp
    with mp.workdps(dps):
        lam = mp.sqrt(5) / mp.mpf(ell)
        F = mp.matrix([[0, 1, 0], [0, 0, 1], [-lam ** 3, -3 * lam ** 2, -3 * lam]])
        A = mp.expm(F * mp.mpf(delta))
        kk = lam ** 2 / 3
        s2 = mp.mpf(sigma2)
        P = mp.matrix([[s2, 0, -s2 * kk], [0, s2 * kk, 0], [-s2 * kk, 0, s2 * lam ** 4]])
        Q = P - A * P * A.T
        An = np.array([[float(A[i, j]) for j in range(3)] for i in range(3)])
        Qn = np.array([[float(Q[i, j]) for j in range(3)] for i in range(3)])
    Qn = 0.5 * (Qn + Qn.T)
    return An, Qn


def matern52_grid_ssm(T: int, h: float, ell: float, sigma2: float = 1.0) -> SSM:
    """Matérn-5/2 (d = 3) on the regular grid x_t = t h."""
    An, Qn = matern52_transition_mp(h, ell, sigma2)
    A = np.broadcast_to(An, (T, 3, 3)).copy()
    Qt = np.broadcast_to(Qn, (T, 3, 3)).copy()
    Qt[0] = matern52_stationary(ell, sigma2)
    return SSM(A=A, Qt=Qt, d=3)


def ssm_precision_band(m: SSM) -> np.ndarray:
    """Lower band (k = 2d - 1) of the precision of the stacked states
    (s_0, ..., s_{T-1}):  diagonal blocks Q_t^{-1} + A_{t+1}^T Q_{t+1}^{-1}
    A_{t+1}, sub-diagonal blocks -Q_{t+1}^{-1} A_{t+1}."""
    A, Qt, d = m.A, m.Qt, m.d
    T = A.shape[0]
    Qinv = np.linalg.inv(Qt)
    Qinv = 0.5 * (Qinv + np.transpose(Qinv, (0, 2, 1)))
    m.Qinv = Qinv   # the exact blocks the precision is assembled from
    Dg = Qinv.copy()
    # A_{t+1}^T Q_{t+1}^{-1} A_{t+1} added to block t
    Dg[:-1] += np.einsum("tba,tbc,tcd->tad", A[1:], Qinv[1:], A[1:])
    Dg = 0.5 * (Dg + np.transpose(Dg, (0, 2, 1)))
    Off = -np.einsum("tab,tbc->tac", Qinv[1:], A[1:])    # block (t+1, t), t = 0..T-2
    k = 2 * d - 1
    N = T * d
    B = np.zeros((T, d, k + 1))
    for a in range(d):
        for s in range(k + 1):
            b = a + s
            if b < d:
                B[:, a, s] = Dg[:, b, a]
            elif b - d < d:
                B[:-1, a, s] = Off[:, b - d, a]
    B = B.reshape(N, k + 1)
    return _zero_pads(B)


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------

def config0(seed: int = 0, n: int = 1000, k: int = 3):
    """Single SPD band: L0 diag U[1,2], off N(0,0.3^2); y ~ N(0,1).  Q is
    band(L0 L0^T), formed by the caller."""
    rng = np.random.default_rng(seed)
    L0 = random_lower_band(n, k, rng)
    y = rng.normal(size=n)
    return L0, y


def config1_inputs(seed: int = 1, n_in: int = 100_000, ell: float = 10.0,
                   spacing: float = 0.01):
    """Matérn-3/2 on jittered stratified inputs x_i = (i + U[.25,.75]) spacing
    (a sorted U[0, n_in spacing] sample with no near-duplicate inputs)."""
    rng = np.random.default_rng(seed)
    x = (np.arange(n_in) + rng.uniform(0.25, 0.75, size=n_in)) * spacing
    m = matern32_ssm(x, ell)
    Q = ssm_precision_band(m)
    y = rng.normal(size=Q.shape[0])
    return Q, y, m, x


def config2_shapes(seed: int = 2, nprob: int = 4096, nmin: int = 256,
                   nmax: int = 65536, kset=(1, 3, 5, 11)):
    rng = np.random.default_rng(seed)
    ns = np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), size=nprob))).astype(np.int64)
    ks = rng.choice(np.asarray(kset), size=nprob).astype(np.int32)
    return ns, ks


def config2_factors(seed: int, ns, ks):
    """Per-problem substreams: L_b as config 0 and y_b ~ N(0,1), packed."""
    ss = np.random.SeedSequence(seed).spawn(len(ns))
    Ls, ys = [], []
    for p, (n, k) in enumerate(zip(ns, ks)):
        rng = np.random.default_rng(ss[p])
        Ls.append(random_lower_band(int(n), int(k), rng))
        ys.append(rng.normal(size=int(n)))
    return Ls, ys


def grid_precision_band(m: SSM) -> np.ndarray:
    """ssm_precision_band for a time-invariant model (regular grid): the
    interior records repeat, so the band is assembled on five states and the
    middle record block is tiled."""
    T, d = m.A.shape[0], m.d
    if T <= 5:
        return ssm_precision_band(m)
    small = SSM(A=m.A[:5].copy(), Qt=m.Qt[:5].copy(), d=d)
    B5 = ssm_precision_band(small).reshape(5, d, -1)
    m.Qinv = np.concatenate([small.Qinv[:2], np.broadcast_to(small.Qinv[2], (T - 2, d, d))])
    B = np.empty((T, d, B5.shape[2]))
    B[0] = B5[0]
    B[1:T - 1] = B5[1]          # every interior state sees the same blocks
    B[T - 1] = B5[4]
    B[T - 2] = B5[3] if T > 2 else B[T - 2]
    B = B.reshape(T * d, -1)
    return _zero_pads(B)


def config3_problem(b: int, seed: int = 3, n_in: int = 1_000_000, h: float = 0.1,
                    nbatch: int = 16):
    """Problem b of the differentiation workload: Matérn-5/2 on a regular
    grid, lengthscale 1 + b/nbatch, y ~ N(0, I), S a diagonally dominant
    symmetric band (k = 5).  Returns (Q, y, S, ssm)."""
    ell = 1.0 + b / nbatch
    m = matern52_grid_ssm(n_in, h, ell)
    Q = grid_precision_band(m)
    rng = np.random.default_rng(np.random.SeedSequence([seed, b]))
    y = rng.normal(size=Q.shape[0])
    S = random_sym_band_dd(Q.shape[0], 5, rng)
    return Q, y, S, m


def config5_marglik(b: int, seed: int = 5, n_in: int = 1_000_000, h: float = 0.1, nbatch: int = 16,
                    p_obs: float = 0.8, tau2: float = 0.1):
    """Problem b of the marginal-likelihood workload: the Matérn-5/2 prior
    precision of config3_problem (lengthscale 1 + b/nbatch, states (f, f', f'')
    stacked per input); each input's function value observed with probability
    p_obs (the derivative states are never observed), Y_t = sin(2 pi x_t / 5) +
    N(0, tau2).  Returns (Q, mask, b = E^T Y, tau2)."""
    ell = 1.0 + b / nbatch
    m = matern52_grid_ssm(n_in, h, ell)
    Q = grid_precision_band(m)
    rng = np.random.default_rng(np.random.SeedSequence([seed, b]))
    obs = rng.random(n_in) < p_obs
    x = np.arange(n_in) * h
    mask = np.zeros(Q.shape[0])
    mask[0::3] = obs
    y = np.zeros(Q.shape[0])
    y[0::3] = (np.sin(2 * np.pi * x / 5.0) + rng.normal(scale=math.sqrt(tau2), size=n_in)) * obs
    return Q, mask, y, tau2


def road_graph(W: int, L: int, seed: int = 9, p_drop: float = 0.15, p_diag: float = 0.1):
    """A synthetic road network on a long strip: a W x L grid of junctions with
    jittered positions (unit spacing); each link along the strip dropped with
    probability p_drop, except in the strip's first row; every link across
    the strip kept (so every junction connects to the first row and the graph
    is connected); random diagonal shortcuts with probability p_diag; nodes
    are numbered in a random order.  Returns (n, indptr, indices, lengths):
    a symmetric CSR pattern without self-loops and the edge lengths in the
    same layout."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, W, L]))
    n = W * L
    pos = np.stack(np.meshgrid(np.arange(L), np.arange(W), indexing="ij"), -1).reshape(n, 2).astype(float)
    pos += rng.uniform(-0.3, 0.3, size=pos.shape)
    grid = np.arange(n).reshape(L, W)
    # along the strip (x -> x+1): kept unless dropped; row y = 0 is never dropped
    ax, bx = grid[:-1, :].ravel(), grid[1:, :].ravel()
    keep_x = (np.tile(np.arange(W), L - 1) == 0) | (rng.random(ax.size) >= p_drop)
    # across the strip (y -> y+1): always kept
    ay, by = grid[:, :-1].ravel(), grid[:, 1:].ravel()
    keep_y = np.ones(ay.size, dtype=bool)
    # diagonal shortcuts (x, y) -> (x+1, y+1)
    ad, bd = grid[:-1, :-1].ravel(), grid[1:, 1:].ravel()
    keep_d = rng.random(ad.size) < p_diag
    e = np.stack([np.concatenate([ax[keep_x], ay[keep_y], ad[keep_d]]),
                  np.concatenate([bx[keep_x], by[keep_y], bd[keep_d]])], 1).astype(np.int64)
    relabel = rng.permutation(n)
    a, b = relabel[e[:, 0]], relabel[e[:, 1]]
    length = np.linalg.norm(pos[e[:, 0]] - pos[e[:, 1]], axis=1)
    rows = np.concatenate([a, b])
    cols = np.concatenate([b, a])
    lens = np.concatenate([length, length])
    order = np.lexsort((cols, rows))
    rows, cols, lens = rows[order], cols[order], lens[order]
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(indptr, rows + 1, 1)
    return n, np.cumsum(indptr), cols.astype(np.int64), lens


def graph_gmrf_csr(n, indptr, indices, lengths, sigma2: float = 1.0, ell=3.0):
    """Precision of a GMRF on a graph from Matérn-1/2 inner products over the
    edges: each edge (i, j) with correlation lam = exp(-d_ij / ell) adds
    (1/sigma2) [[c, -lam c], [-lam c, c]] - (1/(2 sigma2)) I, c = 1/(1 - lam^2),
    on nodes (i, j); every 2 x 2 term is positive definite.  Returns the CSR
    of Q on the pattern with the diagonal inserted (indptr, indices, vals);
    for a sequence of lengthscales, vals is a list with one array per value."""
    n = int(n)
    rows = np.repeat(np.arange(n), np.diff(indptr))
    all_r = np.concatenate([rows, np.arange(n)])
    all_c = np.concatenate([indices, np.arange(n)])
    order = np.lexsort((all_c, all_r))
    ip = np.zeros(n + 1, dtype=np.int64)
    np.add.at(ip, all_r[order] + 1, 1)

    def vals_for(el):
        lam = np.exp(-lengths / el)
        c = 1.0 / (1.0 - lam * lam)
        diag = np.zeros(n)
        np.add.at(diag, rows, c / sigma2 - 0.5 / sigma2)
        return np.concatenate([-lam * c / sigma2, diag])[order]
    many = isinstance(ell, (list, tuple, np.ndarray))
    vals = [vals_for(el) for el in ell] if many else vals_for(ell)
    return np.cumsum(ip), all_c[order].astype(np.int64), vals


def config4_factors(b: int, seed: int = 4, n: int = 200_000, k: int = 64):
    """Problem b of the wide block-banded workload: B lower-banded with k+1
    diagonals (main included), entries N(0, 1/k); D diagonal U[1, 2].  The
    precision is Q = D + band_k(B B^T), formed by the caller."""
    rng = np.random.default_rng(np.random.SeedSequence([seed, b]))
    B = _zero_pads(rng.normal(scale=1.0 / math.sqrt(k), size=(n, k + 1)))
    D = rng.uniform(1.0, 2.0, size=n)
    return B, D


def to_mixed(B: np.ndarray):
    """Split a band into the mixed-precision storage: FP32 band (diagonal slot
    kept too, as an FP32 copy) plus the FP64 diagonal side array."""
    return B.astype(np.float32), B[:, 0].copy()
