"""FP64 CPU oracle for the banded operator set (Durrande et al., AISTATS 2019).

TEST INFRASTRUCTURE ONLY.  The product library never imports, links or calls
this package; only the tests, the smoke check and the benchmark's CPU-baseline
leg do.  ``liboracle.so`` is compiled from ``oracle.c`` (plain C, FP64) by
``__graft_entry__.build()`` or by :func:`build_oracle`.

Band arrays are numpy float64 arrays of shape ``(n, ld)``: row j is record j, the
column j of the matrix restricted to its band (Section 4.3), slot ``u + i - j``
holding element (i, j).  For lower bands slot d holds element (j+d, j).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle.so")
_SRC = os.path.join(_HERE, "oracle.c")

_lib = None


def build_oracle(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (FP64, OpenMP across problems)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        cmd = ["gcc", "-O3", "-fPIC", "-shared", "-fopenmp", "-std=c99",
               "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.check_call(cmd, cwd=_HERE)
        os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build_oracle(force=True)
    lib = ctypes.CDLL(_SO)
    i64, i32, dbl = ctypes.c_int64, ctypes.c_int, ctypes.c_double
    P = ctypes.c_void_p
    sig = {
        "or_chol": (i32, [i64, i32, i64, P, P]),
        "or_logdet": (dbl, [i64, i32, i64, P]),
        "or_trsv": (None, [i64, i32, i64, P, i32, P, P]),
        "or_subset_inv": (None, [i64, i32, i64, P, i32, i64, P]),
        "or_chol_bwd": (None, [i64, i32, i64, P, P, P]),
        "or_subset_inv_bwd": (None, [i64, i32, i64, P, P, P, P]),
        "or_trsv_bwd": (None, [i64, i32, i64, P, i32, P, P, P, P]),
        "or_logdet_bwd": (None, [i64, i32, i64, P, dbl, P]),
        "or_gbmm": (None, [i64, i32, i32, i64, P, i32, i32, i32, i64, P, i32,
                           i32, i32, i64, P]),
        "or_gbmv": (None, [i64, i32, i32, i64, P, i32, P, P]),
        "or_outer_band": (None, [i64, i32, i32, i64, P, P, P]),
        "or_solve_band_mat": (None, [i64, i32, i64, P, i32, i32, i64, P, i64, P]),
        "or_gauss_loss": (i32, [i64, i32, i64, P, P, P, P, P, P, P, P, P, P]),
        "or_gauss_loss_batch": (i32, [i32, P, P, P, P, P, P, P, P, P, P, P]),
        "or_forward_batch": (i32, [i32, P, P, P, P, P, P, P, P, P, P, P, P]),
        "or_solve_band_mat_bwd": (None, [i64, i32, i64, P, i32, i32, i64, P, P, i64, P, P]),
        "or_marglik": (i32, [i64, i32, i64, P, P, P, dbl, P, P, P, P]),
        "or_natgp": (i32, [i64, i32, i64, P, P, P, P, P, P, P, P, P]),
        "or_whiten": (i32, [i64, i32, i64, P, P, P, P]),
        "or_whiten_bwd": (None, [i64, i32, i64, P, P, P, P, P]),
        "or_vi_kl": (None, [i64, i32, i64, P, P, P, P, P, P, P, P, P, P]),
        "or_vi_kl_batch": (i32, [i32, P, P, P, P, P, P, P, P, P, P, P, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def chol(Q, k):
    """Algorithm 1.  Returns (L, info)."""
    Q = _f64(Q)
    n, ld = Q.shape
    L = np.zeros_like(Q)
    info = _load().or_chol(n, k, ld, _p(Q), _p(L))
    return L, int(info)


def logdet(L, k):
    L = _f64(L)
    return float(_load().or_logdet(L.shape[0], k, L.shape[1], _p(L)))


def trsv(L, k, b, trans=0):
    L, b = _f64(L), _f64(b)
    x = np.zeros_like(b)
    _load().or_trsv(L.shape[0], k, L.shape[1], _p(L), int(trans), _p(b), _p(x))
    return x


def subset_inv(L, k, kout=None):
    """Algorithm 3: lower band (width kout >= k) of (L L^T)^{-1}."""
    L = _f64(L)
    kout = k if kout is None else kout
    n = L.shape[0]
    S = np.zeros((n, kout + 1))
    _load().or_subset_inv(n, k, L.shape[1], _p(L), kout, kout + 1, _p(S))
    return S


def chol_bwd(L, k, Lbar):
    """Algorithm 2."""
    L, Lbar = _f64(L), _f64(Lbar)
    Qbar = np.zeros_like(L)
    _load().or_chol_bwd(L.shape[0], k, L.shape[1], _p(L), _p(Lbar), _p(Qbar))
    return Qbar


def subset_inv_bwd(L, k, S, Sbar):
    """Algorithm 4."""
    L, S, Sbar = _f64(L), _f64(S), _f64(Sbar)
    Lbar = np.zeros_like(L)
    _load().or_subset_inv_bwd(L.shape[0], k, L.shape[1], _p(L), _p(S), _p(Sbar), _p(Lbar))
    return Lbar


def trsv_bwd(L, k, x, xbar, trans=0):
    """Table 1, solve matrix-vector.  Returns (bbar, Lbar)."""
    L, x, xbar = _f64(L), _f64(x), _f64(xbar)
    bbar = np.zeros_like(x)
    Lbar = np.zeros_like(L)
    _load().or_trsv_bwd(L.shape[0], k, L.shape[1], _p(L), int(trans), _p(x), _p(xbar),
                        _p(bbar), _p(Lbar))
    return bbar, Lbar


def logdet_bwd(L, k, gbar, Lbar=None):
    L = _f64(L)
    Lbar = np.zeros_like(L) if Lbar is None else _f64(Lbar).copy()
    _load().or_logdet_bwd(L.shape[0], k, L.shape[1], _p(L), float(gbar), _p(Lbar))
    return Lbar


def gbmm(A, la, ua, B, lb, ub, tA=0, tB=0, lc=None, uc=None):
    """Band of op(A) op(B); default output widths are the full product band."""
    A, B = _f64(A), _f64(B)
    n = A.shape[0]
    lA, uA = (ua, la) if tA else (la, ua)
    lB, uB = (ub, lb) if tB else (lb, ub)
    lc = lA + lB if lc is None else lc
    uc = uA + uB if uc is None else uc
    C = np.zeros((n, lc + uc + 1))
    _load().or_gbmm(n, la, ua, A.shape[1], _p(A), int(tA), lb, ub, B.shape[1], _p(B),
                    int(tB), lc, uc, lc + uc + 1, _p(C))
    return C


def gbmv(A, l, u, x, tA=0):
    A, x = _f64(A), _f64(x)
    y = np.zeros_like(x)
    _load().or_gbmv(A.shape[0], l, u, A.shape[1], _p(A), int(tA), _p(x), _p(y))
    return y


def outer_band(m, v, l, u):
    m, v = _f64(m), _f64(v)
    n = m.shape[0]
    O = np.zeros((n, l + u + 1))
    _load().or_outer_band(n, l, u, l + u + 1, _p(m), _p(v), _p(O))
    return O


def solve_band_mat(L, k, R, lr, ur):
    """Algorithm 5: band (k, ur) of L^{-1} R."""
    L, R = _f64(L), _f64(R)
    n = L.shape[0]
    O = np.zeros((n, k + ur + 1))
    _load().or_solve_band_mat(n, k, L.shape[1], _p(L), lr, ur, R.shape[1], _p(R),
                              k + ur + 1, _p(O))
    return O


def solve_band_mat_bwd(L, k, O, Obar, lr, ur):
    """Reverse mode of Algorithm 5 (Table 1, solve matrix-matrix): returns
    (Rbar on the (lr, ur) band of R, Lbar on the lower band of L)."""
    L, O, Obar = _f64(L), _f64(O), _f64(Obar)
    n = L.shape[0]
    Rbar = np.zeros((n, lr + ur + 1))
    Lbar = np.zeros_like(L)
    _load().or_solve_band_mat_bwd(n, k, L.shape[1], _p(L), lr, ur, O.shape[1], _p(O), _p(Obar),
                                  lr + ur + 1, _p(Rbar), _p(Lbar))
    return Rbar, Lbar


def gauss_loss(Q, k, y, S):
    """loss = logdet Q - y^T Q^{-1} y + tr(Q^{-1} S) and its gradients.

    Returns dict with parts (3,), Qbar, ybar, L, z, Sig, Lbar, info."""
    Q, y, S = _f64(Q), _f64(y), _f64(S)
    n, ld = Q.shape
    parts = np.zeros(3)
    out = {k_: np.zeros_like(Q) for k_ in ("Qbar", "L", "Sig", "Lbar")}
    ybar = np.zeros_like(y)
    z = np.zeros_like(y)
    info = _load().or_gauss_loss(n, k, ld, _p(Q), _p(y), _p(S), _p(parts), _p(out["Qbar"]),
                                 _p(ybar), _p(out["L"]), _p(z), _p(out["Sig"]),
                                 _p(out["Lbar"]))
    out.update(parts=parts, ybar=ybar, z=z, info=int(info))
    return out


def _batch_tables(ns, ks):
    ns = np.ascontiguousarray(ns, dtype=np.int64)
    ks = np.ascontiguousarray(ks, dtype=np.int32)
    voff = np.zeros(len(ns), dtype=np.int64)
    voff[1:] = np.cumsum(ns)[:-1]
    return ns, ks, voff


def gauss_loss_batch(ns, ks, Q, y, S):
    """Packed batch: flat arrays, problem p's records (stride k_p + 1) follow
    problem p-1's.  Returns (parts (nprob,3), Qbar flat, ybar, info, threads)."""
    ns, ks, voff = _batch_tables(ns, ks)
    Q, y, S = _f64(Q), _f64(y), _f64(S)
    boff = np.zeros(len(ns), dtype=np.int64)
    boff[1:] = np.cumsum(ns * (ks.astype(np.int64) + 1))[:-1]
    parts = np.zeros((len(ns), 3))
    Qbar = np.zeros_like(Q)
    ybar = np.zeros_like(y)
    info = np.zeros(len(ns), dtype=np.int32)
    th = _load().or_gauss_loss_batch(len(ns), _p(ns), _p(ks), _p(boff), _p(voff), _p(Q), _p(y),
                                     _p(S), _p(parts), _p(Qbar), _p(ybar), _p(info))
    return parts, Qbar, ybar, info, int(th)


def forward_batch(ns, ks, Q, y):
    """Packed batch forward list (Cholesky, logdet, L^{-1} y, L^{-T} L^{-1} y,
    band of Q^{-1}), OpenMP across problems.  Returns (L, z, x, Sig, logdet,
    info, threads)."""
    ns, ks, voff = _batch_tables(ns, ks)
    Q, y = _f64(Q), _f64(y)
    boff = np.zeros(len(ns), dtype=np.int64)
    boff[1:] = np.cumsum(ns * (ks.astype(np.int64) + 1))[:-1]
    L, Sig = np.zeros_like(Q), np.zeros_like(Q)
    z, x = np.zeros_like(y), np.zeros_like(y)
    logdet = np.zeros(len(ns))
    info = np.zeros(len(ns), dtype=np.int32)
    th = _load().or_forward_batch(len(ns), _p(ns), _p(ks), _p(boff), _p(voff), _p(Q), _p(y), _p(L),
                                  _p(z), _p(x), _p(Sig), _p(logdet), _p(info))
    return L, z, x, Sig, logdet, info, int(th)


def vi_kl(Lq, Lp, k, mq, mp):
    """KL(q || p) of Eq. (KL) / Algorithm 7 and its reverse mode.

    Returns dict with parts (4,) = (KL, trace, sum log-diagonal difference,
    squared norm), Lqbar, Lpbar, mqbar, mpbar, Sig (= I(L_q))."""
    Lq, Lp, mq, mp = _f64(Lq), _f64(Lp), _f64(mq), _f64(mp)
    n, ld = Lq.shape
    parts = np.zeros(4)
    out = {k_: np.zeros_like(Lq) for k_ in ("Lqbar", "Lpbar", "Sig")}
    mqbar, mpbar = np.zeros_like(mq), np.zeros_like(mp)
    _load().or_vi_kl(n, k, ld, _p(Lq), _p(Lp), _p(mq), _p(mp), _p(parts), _p(out["Lqbar"]),
                     _p(out["Lpbar"]), _p(mqbar), _p(mpbar), _p(out["Sig"]))
    out.update(parts=parts, mqbar=mqbar, mpbar=mpbar)
    return out


def vi_kl_batch(ns, ks, Lq, Lp, mq, mp):
    """Packed batch of KL terms (layout as gauss_loss_batch).  Returns (parts
    (nprob, 4), Lqbar, Lpbar, mqbar, mpbar, threads)."""
    ns, ks, voff = _batch_tables(ns, ks)
    Lq, Lp, mq, mp = _f64(Lq), _f64(Lp), _f64(mq), _f64(mp)
    boff = np.zeros(len(ns), dtype=np.int64)
    boff[1:] = np.cumsum(ns * (ks.astype(np.int64) + 1))[:-1]
    parts = np.zeros((len(ns), 4))
    Lqbar, Lpbar = np.zeros_like(Lq), np.zeros_like(Lp)
    mqbar, mpbar = np.zeros_like(mq), np.zeros_like(mp)
    th = _load().or_vi_kl_batch(len(ns), _p(ns), _p(ks), _p(boff), _p(voff), _p(Lq), _p(Lp), _p(mq),
                                _p(mp), _p(parts), _p(Lqbar), _p(Lpbar), _p(mqbar), _p(mpbar))
    return parts, Lqbar, Lpbar, mqbar, mpbar, int(th)


def marglik(Q, k, mask, b, tau2):
    """Log marginal likelihood of Eq. (marg_lik) / Algorithm 8 and its reverse
    mode.  Returns dict with parts (4,) = (log p(Y), log|L|, log|L_Q|,
    ||L^{-1} b||^2), Qbar, bbar, tau2bar, info."""
    Q, mask, b = _f64(Q), _f64(mask), _f64(b)
    n, ld = Q.shape
    parts = np.zeros(4)
    Qbar = np.zeros_like(Q)
    bbar = np.zeros_like(b)
    t2 = ctypes.c_double(0.0)
    info = _load().or_marglik(n, k, ld, _p(Q), _p(mask), _p(b), float(tau2), _p(parts), _p(Qbar), _p(bbar),
                              ctypes.byref(t2))
    return dict(parts=parts, Qbar=Qbar, bbar=bbar, tau2bar=t2.value, info=int(info))


def natgp(Lam_pr, eta_pr, Lam_lik, eta_lik, k):
    """GP regression with banded natural parameters (Appendix C.5, Algorithm
    10): value = a(eta_pr, Lam_pr) - a(eta_po, Lam_po) and its reverse mode.
    Returns dict with parts (5,) = (value, sum log C_pr,ii, sum log C_po,ii,
    ||C_pr^-1 eta_pr||^2, ||C_po^-1 eta_po||^2), Lprbar, Llikbar, etaprbar,
    etalikbar, info."""
    Lam_pr, Lam_lik = _f64(Lam_pr), _f64(Lam_lik)
    eta_pr, eta_lik = _f64(eta_pr), _f64(eta_lik)
    n, ld = Lam_pr.shape
    out = dict(parts=np.zeros(5), Lprbar=np.zeros_like(Lam_pr), Llikbar=np.zeros_like(Lam_pr),
               etaprbar=np.zeros(n), etalikbar=np.zeros(n))
    info = _load().or_natgp(n, k, ld, _p(Lam_pr), _p(eta_pr), _p(Lam_lik), _p(eta_lik), _p(out["parts"]),
                            _p(out["Lprbar"]), _p(out["Llikbar"]), _p(out["etaprbar"]), _p(out["etalikbar"]))
    out["info"] = int(info)
    return out


def whiten(Q, k, v):
    """Whitened sample (Section 3.2, Algorithm 6): (L, F = L^{-T} v, info)."""
    Q, v = _f64(Q), _f64(v)
    n, ld = Q.shape
    L = np.zeros_like(Q)
    F = np.zeros(n)
    info = _load().or_whiten(n, k, ld, _p(Q), _p(v), _p(L), _p(F))
    return L, F, int(info)


def whiten_bwd(L, k, F, Fbar):
    """Reverse mode of the whitened sample: (vbar, Qbar)."""
    L, F, Fbar = _f64(L), _f64(F), _f64(Fbar)
    n, ld = L.shape
    vbar = np.zeros(n)
    Qbar = np.zeros_like(L)
    _load().or_whiten_bwd(n, k, ld, _p(L), _p(F), _p(Fbar), _p(vbar), _p(Qbar))
    return vbar, Qbar


# ---------------------------------------------------------------------------
# Bandwidth-reducing node ordering for GMRFs on graphs (Section 2: the
# ordering heuristics the paper points to for graph precisions; Section 5 uses
# reverse Cuthill-McKee).  Integer work: plain Python loops.

def rcm(n, indptr, indices):
    """Reverse Cuthill-McKee ordering of a symmetric sparsity pattern (CSR,
    self-loops ignored).  Cuthill-McKee: every connected component is
    traversed breadth-first from its node of lowest degree (ties: lowest
    index); the unvisited neighbours of each visited node join the order by
    ascending degree (ties: lowest index).  The reverse of that order is
    returned: perm[new] = old."""
    indptr = [int(v) for v in indptr]
    indices = [int(v) for v in indices]
    adj = [[j for j in indices[indptr[i]:indptr[i + 1]] if j != i] for i in range(n)]
    deg = [len(set(a)) for a in adj]
    seen = [False] * n
    order = []
    by_degree = sorted(range(n), key=lambda i: (deg[i], i))
    for s in by_degree:
        if seen[s]:
            continue
        seen[s] = True
        order.append(s)
        head = len(order) - 1
        while head < len(order):
            i = order[head]
            head += 1
            new = sorted({j for j in adj[i] if not seen[j]}, key=lambda j: (deg[j], j))
            for j in new:
                seen[j] = True
                order.append(j)
    return np.array(order[::-1], dtype=np.int64)


def bandwidth(n, indptr, indices, perm=None):
    """Lower bandwidth max |inv[i] - inv[j]| over the pattern's entries under
    the ordering perm (perm[new] = old; identity when None)."""
    inv = np.arange(n) if perm is None else np.argsort(perm)
    rows = np.repeat(np.arange(n), np.diff(np.asarray(indptr)))
    cols = np.asarray(indices)
    return int(np.max(np.abs(inv[rows] - inv[cols]), initial=0))


def csr_to_band(n, indptr, indices, vals, perm, k):
    """Lower band (k sub-diagonals, n x (k+1) records) of P Q P^T for a
    symmetric CSR matrix Q and the ordering perm (perm[new] = old): entry
    (i, j) of Q lands at (inv[i], inv[j]).  Entries outside the band are
    counted and dropped.  Returns (band, dropped)."""
    inv = np.argsort(perm)
    rows = np.repeat(np.arange(n), np.diff(np.asarray(indptr)))
    a, b = inv[rows], inv[np.asarray(indices)]
    low = a >= b
    inside = low & (a - b <= k)
    B = np.zeros((n, k + 1))
    B[b[inside], (a - b)[inside]] = np.asarray(vals, dtype=np.float64)[inside]
    return B, int(np.sum(low & ~inside))
