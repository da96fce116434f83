// bandops_gbk.hpp -- kernels on general bands (l lower, u upper diagonals) of
// one matrix: the products P (Section 4.1; Appendix A.2 and A.4), the band
// outer product O (Appendix A.1), the log-determinant's reverse (Table 1),
// and the matrix solve with a banded right-hand side (Algorithm 5) with its
// reverse mode (Table 1, solve matrix-matrix).  Included by the host library
// inside its file-local namespace.
#pragma once

// ------------------------------------------------- bandwidth-free kernels
template <typename T> struct GB {   // general band view
  T *p;
  double *diag;
  int64_t ld;
  int32_t l, u;
  __device__ __forceinline__ double get(int64_t i, int64_t j) const {
    int64_t d = i - j;
    if (d > l || d < -u) return 0.0;
    if (d == 0 && diag) return diag[j];
    return (double)p[j * ld + u + d];
  }
};

template <typename T> GB<T> gb(const bo_band *b) {
  return GB<T>{(T *)b->band, b->diag64, (int64_t)b->ld, b->l, b->u};
}

// C(i,j) = sum_m op(A)(i,m) op(B)(m,j) over the band overlap, one lane per
// stored entry of C.
template <typename T>
__global__ void k_gbmm(int64_t n, GB<T> A, int tA, GB<T> B, int tB, GB<T> C) {
  int64_t w = C.l + C.u + 1;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * w) return;
  int64_t j = t / w, s = t - j * w;
  int64_t i = j - C.u + s;
  double acc = 0.0;
  if (i >= 0 && i < n) {
    int lA = tA ? A.u : A.l, uA = tA ? A.l : A.u;
    int lB = tB ? B.u : B.l, uB = tB ? B.l : B.u;
    int64_t m0 = i - lA, m1 = i + uA;
    if (j - uB > m0) m0 = j - uB;
    if (j + lB < m1) m1 = j + lB;
    if (m0 < 0) m0 = 0;
    if (m1 > n - 1) m1 = n - 1;
    for (int64_t m = m0; m <= m1; ++m) {
      double a = tA ? A.get(m, i) : A.get(i, m);
      double b = tB ? B.get(j, m) : B.get(m, j);
      acc += a * b;
    }
  }
  C.p[j * C.ld + s] = (T)acc;
  if (s == C.u && C.diag) C.diag[j] = acc;
}

template <typename T>
__global__ void k_gbmv(int64_t n, GB<T> A, int tA, const T *x, T *y) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int64_t m0 = tA ? i - A.u : i - A.l, m1 = tA ? i + A.l : i + A.u;
  if (m0 < 0) m0 = 0;
  if (m1 > n - 1) m1 = n - 1;
  double acc = 0.0;
  for (int64_t m = m0; m <= m1; ++m) acc += (tA ? A.get(m, i) : A.get(i, m)) * (double)x[m];
  y[i] = (T)acc;
}

template <typename T>
__global__ void k_outer(int64_t n, const T *m, const T *v, double alpha, int acc, GB<T> O) {
  int64_t w = O.l + O.u + 1;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * w) return;
  int64_t j = t / w, s = t - j * w;
  int64_t i = j - O.u + s;
  double val = 0.0;
  if (i >= 0 && i < n) {
    val = alpha * (double)m[i] * (double)v[j];
    if (acc) val += O.get(i, j);
  }
  O.p[j * O.ld + s] = (T)val;
  if (s == O.u && O.diag) O.diag[j] = val;
}

template <typename T>
__global__ void k_logdet_bwd(int64_t n, GB<T> L, const double *g, int acc, GB<T> Lb) {
  int64_t w = Lb.l + 1;
  int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * w) return;
  int64_t j = t / w, s = t - j * w;
  double val = (acc && j + s < n) ? Lb.get(j + s, j) : 0.0;
  if (s == 0) val += 2.0 * g[0] / L.get(j, j);
  Lb.p[j * Lb.ld + s] = (T)val;
  if (s == 0 && Lb.diag) Lb.diag[j] = val;
}

// Algorithm 5: O = band (k, u) of L^{-1} R, one lane per column c of O.  The
// column's entries, rows c-u .. c+k, follow by forward substitution down the
// column; each needs only the column's entries above it (the column of L^{-1} R
// is zero above row c-u because R has u upper diagonals).  A workgroup takes
// TC consecutive columns: the L records they reach (columns c0-u .. c1+k-1),
// their R records and the O records being built are staged in LDS as FP64
// (consecutive lanes copy consecutive elements), and O goes back the same way.
// Widths k, u <= 12.
template <typename T>
__device__ __forceinline__ void stage_rec(double *dst, const GB<T> &B, int64_t r0, int64_t r1, int64_t n, int W) {
  const int64_t lo = r0 > 0 ? r0 : 0, hi = r1 < n ? r1 : n;
  for (int64_t e = threadIdx.x; e < (hi - lo) * W; e += blockDim.x) {
    const int64_t r = lo + e / W;
    const int s = (int)(e - (r - lo) * W);
    dst[(r - r0) * W + s] = (s == B.u && B.diag) ? B.diag[r] : (double)B.p[r * B.ld + s];
  }
}
template <typename T>
__device__ __forceinline__ void store_rec(const GB<T> &B, const double *src, int64_t r0, int64_t r1, int W) {
  for (int64_t e = threadIdx.x; e < (r1 - r0) * W; e += blockDim.x) {
    const int64_t r = r0 + e / W;
    const int s = (int)(e - (r - r0) * W);
    B.p[r * B.ld + s] = (T)src[e];
    if (s == B.u && B.diag) B.diag[r] = src[e];
  }
}

// LDS of the two column kernels for TC columns.
__host__ __device__ constexpr size_t solve_mat_lds(int TC, int k, int lr, int u) {
  return (size_t)((TC + u + k) * (k + 1) + TC * (lr + u + 1) + TC * (k + u + 1)) * 8;
}
__host__ __device__ constexpr size_t solve_mat_g_lds(int TC, int k, int u) {
  return (size_t)((TC + u + k) * (k + 1) + TC * (k + u + 1)) * 8;
}

template <typename T> __global__ void __launch_bounds__(256) k_solve_mat(int64_t n, GB<T> L, GB<T> R, GB<T> O) {
  extern __shared__ double dyn[];
  const int k = L.l, u = O.u, WL = k + 1, WR = R.l + R.u + 1, WO = k + u + 1, TC = (int)blockDim.x;
  const int64_t c0 = (int64_t)blockIdx.x * TC, c1 = c0 + TC < n ? c0 + TC : n;
  double *sL = dyn;                       // L records [c0 - u, c1 + k)
  double *sR = sL + (TC + u + k) * WL;    // R records [c0, c1)
  double *sO = sR + TC * WR;              // O records [c0, c1)
  stage_rec(sL, L, c0 - u, c1 + k, n, WL);
  stage_rec(sR, R, c0, c1, n, WR);
  __syncthreads();
  const int64_t c = c0 + threadIdx.x;
  if (c < c1) {
    double *col = sO + threadIdx.x * WO;                          // O(c-u+s, c) at col[s]
    auto lv = [&](int64_t i, int64_t m) { return sL[(m - (c0 - u)) * WL + (i - m)]; };   // L(i, m)
    for (int s = 0; s < WO; ++s) {
      const int64_t i = c - u + s;
      double v = 0.0;
      if (i >= 0 && i < n) {
        double acc = (i - c <= R.l) ? sR[threadIdx.x * WR + s] : 0.0;   // R(i, c): slot u + i - c = s
        int64_t m0 = i - k > c - u ? i - k : c - u;
        if (m0 < 0) m0 = 0;
        for (int64_t m = m0; m < i; ++m) acc -= lv(i, m) * col[m - (c - u)];
        v = acc / lv(i, i);
      }
      col[s] = v;
    }
  }
  __syncthreads();
  store_rec(O, sO, c0, c1, WO);
}

// Reverse mode of Algorithm 5 (Table 1, solve matrix-matrix), first step:
// G = L^{-T} Obar on the band (k, u) (FP64, record c at G + c (k+u+1)), one
// lane per column, rows c+k .. c-u descending (back substitution with L^T).
// Staged like the forward kernel; a column's Obar record is overwritten in
// LDS by G as the substitution goes (slot s is read before it is written, and
// later slots only read G).
template <typename T>
__global__ void __launch_bounds__(256) k_solve_mat_g(int64_t n, GB<T> L, GB<T> Ob, double *G, GB<T> Rb) {
  extern __shared__ double dyn[];
  const int k = L.l, u = Ob.u, WL = k + 1, WO = k + u + 1, TC = (int)blockDim.x;
  const int64_t c0 = (int64_t)blockIdx.x * TC, c1 = c0 + TC < n ? c0 + TC : n;
  double *sL = dyn;                       // L records [c0 - u, c1 + k)
  double *sG = sL + (TC + u + k) * WL;    // Obar, then G, records [c0, c1)
  stage_rec(sL, L, c0 - u, c1 + k, n, WL);
  stage_rec(sG, Ob, c0, c1, n, WO);
  __syncthreads();
  const int64_t c = c0 + threadIdx.x;
  if (c < c1) {
    double *col = sG + threadIdx.x * WO;
    auto lv = [&](int64_t i, int64_t m) { return sL[(m - (c0 - u)) * WL + (i - m)]; };
    for (int s = WO - 1; s >= 0; --s) {
      const int64_t i = c - u + s;
      double v = 0.0;
      if (i >= 0 && i < n) {
        double acc = col[s];
        int64_t m1 = i + k < c + k ? i + k : c + k;
        if (m1 > n - 1) m1 = n - 1;
        for (int64_t m = i + 1; m <= m1; ++m) acc -= lv(m, i) * col[m - (c - u)];
        v = acc / lv(i, i);
      }
      col[s] = v;
    }
  }
  __syncthreads();
  for (int64_t e = threadIdx.x; e < (c1 - c0) * WO; e += blockDim.x) G[c0 * WO + e] = sG[e];
  // Rbar = G on R's band (lr lower, u upper): slot u + (i - c) of both
  const int WR = Rb.l + Rb.u + 1;
  for (int64_t e = threadIdx.x; e < (c1 - c0) * WR; e += blockDim.x) {
    const int64_t cc = e / WR;
    const int sr = (int)(e - cc * WR);
    const int64_t c = c0 + cc, i = c - Rb.u + sr;
    const double v = (i >= 0 && i < n && sr < WO) ? sG[cc * WO + sr] : 0.0;
    Rb.p[c * Rb.ld + sr] = (T)v;
    if (sr == Rb.u && Rb.diag) Rb.diag[c] = v;
  }
}

// Second step, one lane per record m of Lbar: Lbar(i, m) = -sum_c G(i, c)
// O(m, c) over c in [i-k, m+u] (both factors in their bands there), i = m ..
// m+k.  The G and O records of columns m0-k .. m1+u-1 are staged in LDS.
__host__ __device__ constexpr size_t solve_mat_lbar_lds(int TC, int k, int u) {
  return (size_t)(2 * (TC + k + u) * (k + u + 1) + TC * (k + 1)) * 8;
}
template <typename T>
__global__ void __launch_bounds__(256) k_solve_mat_lbar(int64_t n, int k, int u, const double *G, GB<T> O, GB<T> Lb) {
  extern __shared__ double dyn[];
  const int WO = k + u + 1, WL = k + 1, TC = (int)blockDim.x;
  const int64_t m0 = (int64_t)blockIdx.x * TC, m1 = m0 + TC < n ? m0 + TC : n;
  const int64_t r0 = m0 - k, r1 = m1 + u;
  double *sG = dyn;                        // G records [r0, r1)
  double *sO = sG + (TC + k + u) * WO;     // O records [r0, r1)
  double *sOut = sO + (TC + k + u) * WO;   // Lbar records [m0, m1)
  {
    const int64_t lo = r0 > 0 ? r0 : 0, hi = r1 < n ? r1 : n;
    for (int64_t e = threadIdx.x; e < (hi - lo) * WO; e += blockDim.x) sG[(lo - r0) * WO + e] = G[lo * WO + e];
  }
  stage_rec(sO, O, r0, r1, n, WO);
  __syncthreads();
  const int64_t m = m0 + threadIdx.x;
  if (m < m1) {
    for (int d = 0; d < WL; ++d) {
      const int64_t i = m + d;
      double acc = 0.0;
      if (i < n) {
        int64_t ca = i - k > 0 ? i - k : 0, cb = m + u < n - 1 ? m + u : n - 1;
        for (int64_t c = ca; c <= cb; ++c) acc += sG[(c - r0) * WO + u + (i - c)] * sO[(c - r0) * WO + u + (m - c)];
      }
      sOut[threadIdx.x * WL + d] = -acc;
    }
  }
  __syncthreads();
  store_rec(Lb, sOut, m0, m1, WL);
}

unsigned blocks_for(int64_t count, int block) { return (unsigned)((count + block - 1) / block); }

// ------------------------------------------ widened factor (subset inverse)
// dst = src widened from k to K sub-diagonals (K > k), packed (stride K+1):
// slot d of record j is src's slot d for d <= k inside the matrix, else 0.
// Algorithm 3 on the widened factor gives the band of width K of Q^{-1}:
// the sums over m only ever meet L's own k sub-diagonals.  One lane per
// stored element of dst.
template <typename T>
__global__ void k_widen_lower(int64_t n, const T *src, int64_t lds, int k, T *dst, int K) {
  const int64_t w = K + 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n * w) return;
  const int64_t j = t / w;
  const int d = (int)(t - j * w);
  dst[t] = (d <= k && j + d < n) ? src[j * lds + d] : (T)0;
}

// -------------------------------------------- per-problem scaling of a plan
// One workgroup per chunk of the plan's schedule, over that chunk's rows of
// its problem: out = s_p * in (s_p = g[problem] or 1), with the factor 2 off
// the diagonal for BO_SCALE_BAND_SYM; band pads (slots past the matrix end)
// are written 0.  Mixed format: records are float and the diagonal is the
// FP64 side array (ind -> outd).
template <typename T>
__global__ void __launch_bounds__(256) k_plan_scale(const bo::ProbDesc *probs, const int32_t *chunk_prob,
                                                    int kind, const double *g, const T *in, const double *ind,
                                                    T *out, double *outd) {
  const int32_t c = (int32_t)blockIdx.x;
  const bo::ProbDesc &pd = probs[chunk_prob[c]];
  int64_t a, b;
  bo::chunk_rows(pd, c, a, b);
  const double s = g ? g[pd.orig] : 1.0;
  if (kind == BO_SCALE_VEC) {
    for (int64_t j = a + threadIdx.x; j < b; j += blockDim.x) out[pd.voff + j] = (T)(s * (double)in[pd.voff + j]);
    return;
  }
  const int64_t w = pd.ld;
  const T *src = in + pd.boff;
  T *dst = out + pd.boff;
  for (int64_t e = a * w + threadIdx.x; e < b * w; e += blockDim.x) {
    const int64_t j = e / w;
    const int d = (int)(e - j * w);
    double v = (d <= pd.k && j + d < pd.n) ? s * (double)src[e] : 0.0;
    if (kind == BO_SCALE_BAND_SYM && d > 0) v *= 2.0;
    dst[e] = (T)v;
  }
  if (outd)
    for (int64_t j = a + threadIdx.x; j < b; j += blockDim.x) outd[pd.voff + j] = s * ind[pd.voff + j];
}

// out[p] = g[p] * in[p] for the nprob per-problem values (BO_SCALE_PROBLEM).
__global__ void k_problem_scale(int64_t nprob, const double *g, const double *in, double *out) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < nprob) out[p] = (g ? g[p] : 1.0) * in[p];
}
