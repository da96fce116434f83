"""Dense <-> band conversions used by the tests (record-major band storage:
row j of the band array is column j of the matrix, slot u+i-j = element (i,j))."""
import numpy as np


def lower_to_dense(B, k=None):
    n, w = B.shape
    k = w - 1 if k is None else k
    M = np.zeros((n, n), dtype=np.float64)
    for d in range(min(k, n - 1) + 1):
        idx = np.arange(n - d)
        M[idx + d, idx] = B[: n - d, d]
    return M


def sym_to_dense(B, k=None):
    M = lower_to_dense(B, k)
    return M + np.tril(M, -1).T


def dense_to_lower(M, k):
    n = M.shape[0]
    B = np.zeros((n, k + 1))
    for d in range(k + 1):
        idx = np.arange(max(n - d, 0))
        B[idx, d] = M[idx + d, idx]
    return B


def gen_to_dense(B, l, u):
    n = B.shape[0]
    M = np.zeros((n, n))
    for s in range(l + u + 1):
        d = s - u              # i - j
        j = np.arange(n)
        i = j + d
        ok = (i >= 0) & (i < n)
        M[i[ok], j[ok]] = B[j[ok], s]
    return M


def dense_to_gen(M, l, u):
    n = M.shape[0]
    B = np.zeros((n, l + u + 1))
    for s in range(l + u + 1):
        d = s - u
        j = np.arange(n)
        i = j + d
        ok = (i >= 0) & (i < n)
        B[j[ok], s] = M[i[ok], j[ok]]
    return B


def band_mask(n, k):
    """1 where a lower-band slot is inside the matrix, 0 on padding."""
    m = np.ones((n, k + 1))
    for d in range(1, k + 1):
        m[max(n - d, 0):, d] = 0.0
    return m


def rel_err(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    if a.size == 0:
        return 0.0
    den = max(np.max(np.abs(b)), 1e-300)
    return float(np.max(np.abs(a - b)) / den)
