/*
 * oracle.c -- FP64 CPU reference for the banded operator set (Durrande et al.,
 * AISTATS 2019).  TEST INFRASTRUCTURE ONLY: the product library never links,
 * loads or calls this file; only the tests, the smoke check and the CPU-baseline
 * leg of the benchmark do.  It shares no code with the HIP path.
 *
 * Each routine follows the operator's definition or the paper's algorithm in the
 * paper's order, using dense (i,j) indices mapped onto band storage through the
 * accessors below (the appendix on algorithms writes them the same way).  No
 * blocking, fusion or reordering beyond what the algorithm states.
 *
 * Readings of the paper taken here:
 *  - band storage index: B[i,j] is slot u+i-j of record j (Section 4.3; the
 *    printed index formula has its sign garbled);
 *  - Algorithms 3 and 4 use the band *height* in their ranges; here every range
 *    is written with k = number of sub-diagonals;
 *  - Algorithm 4's local copy of bS holds the user's sensitivities in its lower
 *    triangle and zeros in its strict upper triangle, which gives the gradient
 *    with respect to the stored lower-band entries of S;
 *  - the solve gradient follows Table 1 (the appendix derivation drops a sign);
 *  - Algorithm 1 has no positivity check; a LAPACK-style info is added;
 *  - Algorithm 8's last line lacks the -(m/2) log tau2 term of Eq. (marg_lik);
 *    the equation is followed;
 *  - Appendix C.5's log-likelihood and Algorithm 10's last line are garbled in
 *    their signs; the natural-parameter identity the appendix states,
 *    a(eta_pr, Lam_pr) - a(eta_po, Lam_po) plus the data-space normaliser, is
 *    followed.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static inline int64_t imax64(int64_t a, int64_t b) { return a > b ? a : b; }
static inline int64_t imin64(int64_t a, int64_t b) { return a < b ? a : b; }

/* Lower-band accessor: element (i,j), j <= i <= j+k, of a lower band. */
#define LOW(M, ld, i, j) ((M)[(int64_t)(j) * (ld) + ((i) - (j))])
/* General-band accessor: element (i,j), j-u <= i <= j+l, slot u+i-j. */
#define GEN(M, ld, u, i, j) ((M)[(int64_t)(j) * (ld) + (u) + ((i) - (j))])

/* Read element (i,j) of a symmetric matrix stored as its lower band. */
static inline double sym_get(const double *M, int64_t ld, int k, int64_t i,
                             int64_t j) {
  int64_t a = i > j ? i : j, b = i > j ? j : i;
  if (a - b > k) return 0.0;
  return LOW(M, ld, a, b);
}

/* Element (i,j) of a general (l,u) band, or 0 outside the band. */
static inline double gen_get(const double *M, int64_t ld, int l, int u,
                             int64_t i, int64_t j) {
  int64_t d = i - j;
  if (d > l || d < -u) return 0.0;
  return GEN(M, ld, u, i, j);
}

/* --------------------------------------------------------------------------
 * Algorithm 1: Cholesky of a banded SPD matrix.  Row i, columns
 * j = max(i-k,0) .. i; s = sum_{m=max(i-k,0)}^{j-1} L[i,m] L[j,m];
 * diagonal sqrt(Q_ii - s), off-diagonal (Q_ij - s)/L_jj.
 * ------------------------------------------------------------------------ */
int or_chol(int64_t n, int k, int64_t ld, const double *Q, double *L) {
  for (int64_t j = 0; j < n; ++j)
    for (int d = 0; d <= k; ++d) L[j * ld + d] = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    int64_t jstart = imax64(i - k, 0);
    for (int64_t j = jstart; j <= i; ++j) {
      int64_t m0 = jstart; /* max(i-k, j-k, 0) with j <= i */
      double s = 0.0;
      for (int64_t m = m0; m < j; ++m) s += LOW(L, ld, i, m) * LOW(L, ld, j, m);
      if (i == j) {
        double piv = LOW(Q, ld, i, i) - s;
        if (!(piv > 0.0)) { /* not positive definite, or NaN */
          for (int64_t jj = jstart; jj < i; ++jj) LOW(L, ld, i, jj) = 0.0;
          return (int)(i + 1);
        }
        LOW(L, ld, i, i) = sqrt(piv);
      } else {
        LOW(L, ld, i, j) = (LOW(Q, ld, i, j) - s) / LOW(L, ld, j, j);
      }
    }
  }
  return 0;
}

/* log det(L L^T) = 2 sum log L_ii, Neumaier compensated summation. */
double or_logdet(int64_t n, int k, int64_t ld, const double *L) {
  (void)k;
  double sum = 0.0, c = 0.0;
  for (int64_t i = 0; i < n; ++i) {
    double t = log(LOW(L, ld, i, i));
    double s = sum + t;
    if (fabs(sum) >= fabs(t))
      c += (sum - s) + t;
    else
      c += (t - s) + sum;
    sum = s;
  }
  return 2.0 * (sum + c);
}

/* --------------------------------------------------------------------------
 * Triangular solve restricted to the band (Section 4.1, "Triangular solve").
 * trans = 0: forward substitution x_i = (b_i - sum_{m=i-k}^{i-1} L_im x_m)/L_ii.
 * trans = 1: back substitution with L^T,
 *            x_i = (b_i - sum_{m=i+1}^{i+k} L_mi x_m)/L_ii.
 * ------------------------------------------------------------------------ */
void or_trsv(int64_t n, int k, int64_t ld, const double *L, int trans,
             const double *b, double *x) {
  if (!trans) {
    for (int64_t i = 0; i < n; ++i) {
      double s = b[i];
      for (int64_t m = imax64(i - k, 0); m < i; ++m) s -= LOW(L, ld, i, m) * x[m];
      x[i] = s / LOW(L, ld, i, i);
    }
  } else {
    for (int64_t i = n - 1; i >= 0; --i) {
      double s = b[i];
      for (int64_t m = i + 1; m <= imin64(i + k, n - 1); ++m)
        s -= LOW(L, ld, m, i) * x[m];
      x[i] = s / LOW(L, ld, i, i);
    }
  }
}

/* --------------------------------------------------------------------------
 * Algorithm 3: band of (L L^T)^{-1} (Takahashi).  vec = diag(L),
 * U = (L / vec)^T so U[i,m] = L[m,i]/L[i,i].  Columns j descending; rows
 * i = j down to j-kout:  Sym[i,j] = - sum_{m=i+1}^{i+k} U[i,m] Sym[m,j],
 * Sym[j,i] = Sym[i,j], and Sym[i,i] += 1/vec_i^2.  Sym is a symmetric band of
 * width kout held in full (both halves) as the algorithm describes.
 * ------------------------------------------------------------------------ */
void or_subset_inv(int64_t n, int k, int64_t ld, const double *L, int kout,
                   int64_t lds, double *S) {
  if (kout < k) kout = k;
  int64_t ldsym = 2 * (int64_t)kout + 1;
  double *Sym = (double *)calloc((size_t)(n * ldsym + 1), sizeof(double));
  for (int64_t j = n - 1; j >= 0; --j) {
    for (int64_t i = j; i >= imax64(j - kout, 0); --i) {
      double s = 0.0;
      double vec_i = LOW(L, ld, i, i);
      for (int64_t m = i + 1; m <= imin64(i + k, n - 1); ++m) {
        double U_im = LOW(L, ld, m, i) / vec_i;
        s += U_im * GEN(Sym, ldsym, kout, m, j);
      }
      GEN(Sym, ldsym, kout, i, j) = -s;
      GEN(Sym, ldsym, kout, j, i) = GEN(Sym, ldsym, kout, i, j);
      if (i == j) GEN(Sym, ldsym, kout, i, i) += 1.0 / (vec_i * vec_i);
    }
  }
  for (int64_t j = 0; j < n; ++j)
    for (int d = 0; d <= kout; ++d)
      S[j * lds + d] = (j + d < n) ? GEN(Sym, ldsym, kout, j + d, j) : 0.0;
  free(Sym);
}

/* --------------------------------------------------------------------------
 * Algorithm 2: reverse mode of the banded Cholesky (Giles 2008, banded).
 * Rows i descending, j = i down to jstop = max(i-k,0):
 *   j == i : Qb[i,i] = 1/2 Lb[i,i] / L[i,i]
 *   j <  i : Qb[i,j] = Lb[i,j] / L[j,j];  Lb[j,j] -= Lb[i,j] L[i,j] / L[j,j]
 *   p = j-1 down to jstop : Lb[i,p] -= Qb[i,j] L[j,p]; Lb[j,p] -= Qb[i,j] L[i,p]
 * (the algorithm's inner variable is renamed p; ranges are inclusive).
 * ------------------------------------------------------------------------ */
void or_chol_bwd(int64_t n, int k, int64_t ld, const double *L,
                 const double *Lbar, double *Qbar) {
  double *Lb = (double *)malloc((size_t)(n * ld + 1) * sizeof(double));
  memcpy(Lb, Lbar, (size_t)(n * ld) * sizeof(double));
  for (int64_t j = 0; j < n; ++j)
    for (int d = 0; d <= k; ++d) Qbar[j * ld + d] = 0.0;
  for (int64_t i = n - 1; i >= 0; --i) {
    int64_t jstop = imax64(i - k, 0);
    for (int64_t j = i; j >= jstop; --j) {
      double qb;
      if (j == i) {
        qb = 0.5 * LOW(Lb, ld, i, i) / LOW(L, ld, i, i);
      } else {
        qb = LOW(Lb, ld, i, j) / LOW(L, ld, j, j);
        LOW(Lb, ld, j, j) -= LOW(Lb, ld, i, j) * LOW(L, ld, i, j) / LOW(L, ld, j, j);
      }
      LOW(Qbar, ld, i, j) = qb;
      for (int64_t p = j - 1; p >= jstop; --p) {
        LOW(Lb, ld, i, p) -= qb * LOW(L, ld, j, p);
        LOW(Lb, ld, j, p) -= qb * LOW(L, ld, i, p);
      }
    }
  }
  free(Lb);
}

/* --------------------------------------------------------------------------
 * Algorithm 4: reverse mode of the subset inverse.  The local copy bS is a
 * (k,k) general band: lower triangle = the caller's Sbar, strict upper = 0.
 * Columns j ascending, rows i = max(0,j-k) .. j:
 *   i == j : bvec_inv_2[i] += bS[i,i]
 *   grad of S[j,i] = S[i,j]:  tmp = bS[j,i]; bS[j,i] = 0; bS[i,j] += tmp
 *   grad of S[i,j] = -sum_m U[i,m] S[m,j], m = i+1 .. i+k:
 *       bU[i,m] -= S[m,j] bS[i,j];  bS[m,j] -= U[i,m] bS[i,j];  bS[i,j] = 0
 * then bL = bU^T / vec, bvec = -2 bvec_inv_2 / vec^3
 *      - colsum(bU^T * L) / vec^2, bL += diag(bvec).
 * ------------------------------------------------------------------------ */
void or_subset_inv_bwd(int64_t n, int k, int64_t ld, const double *L,
                       const double *S, const double *Sbar, double *Lbar) {
  int64_t ldb = 2 * (int64_t)k + 1; /* (k,k) general band for bS */
  double *bS = (double *)calloc((size_t)(n * ldb + 1), sizeof(double));
  double *bU = (double *)calloc((size_t)(n * (k + 1) + 1), sizeof(double)); /* bU[i,m] at i*(k+1)+(m-i) */
  double *bvi2 = (double *)calloc((size_t)(n + 1), sizeof(double));
  for (int64_t j = 0; j < n; ++j)
    for (int d = 0; d <= k && j + d < n; ++d)
      GEN(bS, ldb, k, j + d, j) = LOW(Sbar, ld, j + d, j);

  for (int64_t j = 0; j < n; ++j) {
    for (int64_t i = imax64(0, j - k); i <= j; ++i) {
      if (i == j) bvi2[i] += GEN(bS, ldb, k, i, i);
      double tmp = GEN(bS, ldb, k, j, i);
      GEN(bS, ldb, k, j, i) = 0.0;
      GEN(bS, ldb, k, i, j) += tmp;
      double bsij = GEN(bS, ldb, k, i, j);
      double vec_i = LOW(L, ld, i, i);
      for (int64_t m = i + 1; m <= imin64(i + k, n - 1); ++m) {
        double U_im = LOW(L, ld, m, i) / vec_i;
        bU[i * (k + 1) + (m - i)] -= sym_get(S, ld, k, m, j) * bsij;
        GEN(bS, ldb, k, m, j) -= U_im * bsij;
      }
      GEN(bS, ldb, k, i, j) = 0.0;
    }
  }
  for (int64_t i = 0; i < n; ++i) {
    double vec_i = LOW(L, ld, i, i);
    for (int d = 0; d <= k; ++d) Lbar[i * ld + d] = 0.0;
    double colsum = 0.0;
    for (int64_t m = i + 1; m <= imin64(i + k, n - 1); ++m) {
      double bu = bU[i * (k + 1) + (m - i)];
      LOW(Lbar, ld, m, i) = bu / vec_i;
      colsum += bu * LOW(L, ld, m, i);
    }
    double bvec = -2.0 * bvi2[i] / (vec_i * vec_i * vec_i) - colsum / (vec_i * vec_i);
    LOW(Lbar, ld, i, i) += bvec;
  }
  free(bS);
  free(bU);
  free(bvi2);
}

/* --------------------------------------------------------------------------
 * Reverse mode of the solve (Table 1, "solve matrix-vector").
 * trans = 0, s = L^{-1} v :  vbar = L^{-T} sbar,  Lbar_ij = -vbar_i s_j
 * trans = 1, x = L^{-T} b :  bbar = L^{-1} xbar,  Lbar_ij = -x_i bbar_j
 * both restricted to the lower band of L.
 * ------------------------------------------------------------------------ */
void or_trsv_bwd(int64_t n, int k, int64_t ld, const double *L, int trans,
                 const double *x, const double *xbar, double *bbar,
                 double *Lbar) {
  or_trsv(n, k, ld, L, trans ? 0 : 1, xbar, bbar);
  for (int64_t j = 0; j < n; ++j)
    for (int d = 0; d <= k; ++d) {
      int64_t i = j + d;
      double v = 0.0;
      if (i < n) v = trans ? -x[i] * bbar[j] : -bbar[i] * x[j];
      Lbar[j * ld + d] = v;
    }
}

void or_logdet_bwd(int64_t n, int k, int64_t ld, const double *L, double gbar,
                   double *Lbar) {
  (void)k;
  for (int64_t i = 0; i < n; ++i) LOW(Lbar, ld, i, i) += 2.0 * gbar / LOW(L, ld, i, i);
}

/* --------------------------------------------------------------------------
 * Products (Section 4.1): C_ij = sum_m op(A)_im op(B)_mj over the band overlap,
 * for (i,j) in the requested (lc,uc) band of C.
 * ------------------------------------------------------------------------ */
void or_gbmm(int64_t n, int la, int ua, int64_t lda, const double *A, int tA,
             int lb, int ub, int64_t ldb, const double *B, int tB, int lc,
             int uc, int64_t ldc, double *C) {
  /* op(A) has lower width la' and upper width ua' */
  int lA = tA ? ua : la, uA = tA ? la : ua;
  for (int64_t j = 0; j < n; ++j) {
    for (int s = 0; s <= lc + uc; ++s) {
      int64_t i = j - uc + s;
      double acc = 0.0;
      if (i >= 0 && i < n) {
        int64_t m0 = imax64(0, i - lA), m1 = imin64(n - 1, i + uA);
        for (int64_t m = m0; m <= m1; ++m) {
          double a = tA ? gen_get(A, lda, la, ua, m, i) : gen_get(A, lda, la, ua, i, m);
          double b = tB ? gen_get(B, ldb, lb, ub, j, m) : gen_get(B, ldb, lb, ub, m, j);
          acc += a * b;
        }
      }
      C[j * ldc + s] = acc;
    }
  }
}

void or_gbmv(int64_t n, int l, int u, int64_t ld, const double *A, int tA,
             const double *x, double *y) {
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0;
    int64_t m0 = tA ? i - u : i - l, m1 = tA ? i + l : i + u;
    for (int64_t m = imax64(0, m0); m <= imin64(n - 1, m1); ++m)
      acc += (tA ? gen_get(A, ld, l, u, m, i) : gen_get(A, ld, l, u, i, m)) * x[m];
    y[i] = acc;
  }
}

void or_outer_band(int64_t n, int l, int u, int64_t ld, const double *m,
                   const double *v, double *O) {
  for (int64_t j = 0; j < n; ++j)
    for (int s = 0; s <= l + u; ++s) {
      int64_t i = j - u + s;
      O[j * ld + s] = (i >= 0 && i < n) ? m[i] * v[j] : 0.0;
    }
}

/* --------------------------------------------------------------------------
 * Algorithm 5: band (k,u) of L^{-1} R.  Diagonals t = -u .. k in order; on
 * diagonal t, rows i descending: O[i,i-t] = (R[i,i-t] - sum_{m<i} L[i,m]
 * O[m,i-t]) / L[i,i], the sum running over m = max(0,i-k) .. i-1 (entries of
 * O outside its band are zero).
 * ------------------------------------------------------------------------ */
void or_solve_band_mat(int64_t n, int k, int64_t ldl, const double *L, int lr,
                       int ur, int64_t ldr, const double *R, int64_t ldo,
                       double *O) {
  int uo = ur, lo = k;
  for (int64_t j = 0; j < n; ++j)
    for (int s = 0; s <= lo + uo; ++s) O[j * ldo + s] = 0.0;
  for (int t = -uo; t <= lo; ++t) {
    for (int64_t i = imin64(n + t - 1, n - 1); i >= imax64(0, t); --i) {
      int64_t c = i - t;
      double r = gen_get(R, ldr, lr, ur, i, c);
      double dot = 0.0;
      for (int64_t m = imax64(0, i - k); m < i; ++m)
        dot += LOW(L, ldl, i, m) * gen_get(O, ldo, lo, uo, m, c);
      GEN(O, ldo, uo, i, c) = (r - dot) / LOW(L, ldl, i, i);
    }
  }
}

/* --------------------------------------------------------------------------
 * Reverse mode of Algorithm 5 (Table 1, solve matrix-matrix, with B = R and
 * S = O): Rbar = S(L^T, Obar), Lbar^T = -P(O, S(L^T, Obar)^T).
 * G = L^{-T} Obar column by column, rows descending (back substitution with
 * L^T); column c of Obar lives on rows c-ur .. c+k, so G's column c is zero
 * below row c+k and its band entries need only band entries above them.
 * ------------------------------------------------------------------------ */
void or_solve_band_mat_bwd(int64_t n, int k, int64_t ldl, const double *L, int lr,
                           int ur, int64_t ldo, const double *O,
                           const double *Obar, int64_t ldr, double *Rbar,
                           double *Lbar) {
  int lo = k, uo = ur;
  int64_t ldg = lo + uo + 1;
  double *G = (double *)calloc((size_t)(n * ldg + 1), sizeof(double));
  for (int64_t c = 0; c < n; ++c)
    for (int64_t i = imin64(n - 1, c + lo); i >= imax64(0, c - uo); --i) {
      double acc = gen_get(Obar, ldo, lo, uo, i, c);
      for (int64_t m = i + 1; m <= imin64(n - 1, i + k); ++m)
        acc -= LOW(L, ldl, m, i) * gen_get(G, ldg, lo, uo, m, c);
      GEN(G, ldg, uo, i, c) = acc / LOW(L, ldl, i, i);
    }
  for (int64_t c = 0; c < n; ++c)
    for (int s = 0; s <= lr + ur; ++s) {
      int64_t i = c - ur + s;
      Rbar[c * ldr + s] = (i >= 0 && i < n) ? gen_get(G, ldg, lo, uo, i, c) : 0.0;
    }
  for (int64_t m = 0; m < n; ++m)
    for (int d = 0; d <= k; ++d) {
      int64_t i = m + d;
      double acc = 0.0;
      if (i < n)
        for (int64_t c = imax64(0, i - lo); c <= imin64(n - 1, m + uo); ++c)
          acc += gen_get(G, ldg, lo, uo, i, c) * gen_get(O, ldo, lo, uo, m, c);
      Lbar[m * ldl + d] = -acc;
    }
  free(G);
}

/* --------------------------------------------------------------------------
 * loss = log det Q - y^T Q^{-1} y + tr(Q^{-1} S) and its gradients, composed
 * from C, S, I and their reverse modes (Table 1, Algorithms 1-4):
 *   L = C(Q); z = S(L, y); Sig = I(L)
 *   log det Q = 2 sum log L_ii;  y^T Q^{-1} y = z^T z;
 *   tr(Q^{-1} S) = sum_i Sig_ii S_ii + 2 sum_{i>j} Sig_ij S_ij
 * reverse: Sigbar (stored entries) = S_ii on the diagonal, 2 S_ij off it;
 *   Lbar  = subset_inv_bwd(L, Sig, Sigbar)
 *         + solve bwd with zbar = -2 z (ybar and -band(ybar z^T))
 *         + logdet bwd (2 / L_ii);
 *   Qbar  = chol_bwd(L, Lbar).
 * ------------------------------------------------------------------------ */
int or_gauss_loss(int64_t n, int k, int64_t ld, const double *Q,
                  const double *y, const double *S, double *parts,
                  double *Qbar, double *ybar, double *L, double *z,
                  double *Sig, double *Lbar) {
  size_t bsz = (size_t)(n * ld + 1) * sizeof(double);
  size_t vsz = (size_t)(n + 1) * sizeof(double);
  double *Lw = L ? L : (double *)malloc(bsz);
  double *zw = z ? z : (double *)malloc(vsz);
  double *Sw = Sig ? Sig : (double *)malloc(bsz);
  double *Lbw = Lbar ? Lbar : (double *)malloc(bsz);
  double *Sb = (double *)malloc(bsz);
  double *Lb2 = (double *)malloc(bsz);
  double *zb = (double *)malloc(vsz);
  int info = or_chol(n, k, ld, Q, Lw);
  if (info == 0) {
    parts[0] = or_logdet(n, k, ld, Lw);
    or_trsv(n, k, ld, Lw, 0, y, zw);
    double q = 0.0;
    for (int64_t i = 0; i < n; ++i) q += zw[i] * zw[i];
    parts[1] = q;
    or_subset_inv(n, k, ld, Lw, k, ld, Sw);
    double tr = 0.0;
    for (int64_t j = 0; j < n; ++j)
      for (int d = 0; d <= k && j + d < n; ++d) {
        double w = (d == 0) ? 1.0 : 2.0;
        tr += w * Sw[j * ld + d] * S[j * ld + d];
        Sb[j * ld + d] = w * S[j * ld + d];
      }
    parts[2] = tr;
    for (int64_t j = 0; j < n; ++j)
      for (int d = 0; d <= k; ++d)
        if (j + d >= n) Sb[j * ld + d] = 0.0;
    or_subset_inv_bwd(n, k, ld, Lw, Sw, Sb, Lbw);
    for (int64_t i = 0; i < n; ++i) zb[i] = -2.0 * zw[i];
    or_trsv_bwd(n, k, ld, Lw, 0, zw, zb, ybar, Lb2);
    for (int64_t t = 0; t < n * ld; ++t) Lbw[t] += Lb2[t];
    or_logdet_bwd(n, k, ld, Lw, 1.0, Lbw);
    or_chol_bwd(n, k, ld, Lw, Lbw, Qbar);
  } else {
    parts[0] = parts[1] = parts[2] = NAN;
  }
  if (!L) free(Lw);
  if (!z) free(zw);
  if (!Sig) free(Sw);
  if (!Lbar) free(Lbw);
  free(Sb);
  free(Lb2);
  free(zb);
  return info;
}

/* --------------------------------------------------------------------------
 * Marginal likelihood (Eq. (marg_lik), Algorithm 8) in the order of Algorithm
 * 8: L = C(Q + tau^-2 E^T E), L' = C(Q), R = S(L, E^T Y), then the terms of
 * Eq. (marg_lik) (Algorithm 8 as printed omits -(m/2) log tau2; the equation
 * keeps it, and it is kept here).  Reverse mode through Table 1:
 *   -log|L|:            Lbar  = logdet_bwd(L, -1/2)
 *   R^T R / (2 tau^4):  Rbar = R / tau^4; (bbar, Lbar') = solve bwd
 *   Qbar = chol_bwd(L, Lbar + Lbar') + chol_bwd(L', logdet_bwd(L', 1/2))
 * (Q + tau^-2 E^T E and Q share their stored off-diagonal entries, and the
 * diagonal shift is additive, so both factors' sensitivities add onto Q);
 *   bbar += -b / tau2 (the Y^T Y term), restricted to the observed nodes;
 *   tau2bar = -tau^-4 sum_i mask_i Qbar1_ii (Q1's dependence on tau2)
 *             - m / (2 tau2) + Y^T Y / (2 tau2^2) - R^T R / tau2^3.
 * ------------------------------------------------------------------------ */
int or_marglik(int64_t n, int k, int64_t ld, const double *Q, const double *mask,
               const double *b, double tau2, double *parts, double *Qbar,
               double *bbar, double *tau2bar) {
  size_t bsz = (size_t)(n * ld + 1) * sizeof(double);
  size_t vsz = (size_t)(n + 1) * sizeof(double);
  double *Q1 = (double *)malloc(bsz), *L = (double *)malloc(bsz), *Lp = (double *)malloc(bsz);
  double *Lb = (double *)calloc((size_t)(n * ld + 1), sizeof(double));
  double *Lb2 = (double *)calloc((size_t)(n * ld + 1), sizeof(double));
  double *Lpb = (double *)calloc((size_t)(n * ld + 1), sizeof(double));
  double *Qb1 = (double *)calloc((size_t)(n * ld + 1), sizeof(double));
  double *Qb0 = (double *)calloc((size_t)(n * ld + 1), sizeof(double));
  double *R = (double *)malloc(vsz), *Rb = (double *)malloc(vsz);
  double m = 0.0, yy = 0.0;
  for (int64_t t = 0; t < n * ld; ++t) Q1[t] = Q[t];
  for (int64_t i = 0; i < n; ++i) {
    LOW(Q1, ld, i, i) += mask[i] / tau2;
    m += mask[i];
    yy += b[i] * b[i];
  }
  int info = or_chol(n, k, ld, Q1, L);
  int info0 = info ? 0 : or_chol(n, k, ld, Q, Lp);
  if (info || info0) {
    parts[0] = parts[1] = parts[2] = parts[3] = NAN;
    *tau2bar = NAN;
  } else {
    double lL = 0.5 * or_logdet(n, k, ld, L), lLp = 0.5 * or_logdet(n, k, ld, Lp), rr = 0.0;
    or_trsv(n, k, ld, L, 0, b, R);
    for (int64_t i = 0; i < n; ++i) rr += R[i] * R[i];
    parts[1] = lL;
    parts[2] = lLp;
    parts[3] = rr;
    parts[0] = -0.5 * m * log(2.0 * 3.14159265358979323846) - lL + lLp - 0.5 * m * log(tau2) - yy / (2.0 * tau2) +
               rr / (2.0 * tau2 * tau2);
    /* reverse */
    or_logdet_bwd(n, k, ld, L, -0.5, Lb);
    for (int64_t i = 0; i < n; ++i) Rb[i] = R[i] / (tau2 * tau2);
    or_trsv_bwd(n, k, ld, L, 0, R, Rb, bbar, Lb2);
    for (int64_t t = 0; t < n * ld; ++t) Lb[t] += Lb2[t];
    or_chol_bwd(n, k, ld, L, Lb, Qb1);
    or_logdet_bwd(n, k, ld, Lp, 0.5, Lpb);
    or_chol_bwd(n, k, ld, Lp, Lpb, Qb0);
    double dq = 0.0;
    for (int64_t i = 0; i < n; ++i) dq += mask[i] * LOW(Qb1, ld, i, i);
    for (int64_t t = 0; t < n * ld; ++t) Qbar[t] = Qb1[t] + Qb0[t];
    for (int64_t i = 0; i < n; ++i) bbar[i] = mask[i] != 0.0 ? bbar[i] - b[i] / tau2 : 0.0;
    *tau2bar = -dq / (tau2 * tau2) - 0.5 * m / tau2 + yy / (2.0 * tau2 * tau2) - rr / (tau2 * tau2 * tau2);
  }
  free(Q1);
  free(L);
  free(Lp);
  free(Lb);
  free(Lb2);
  free(Lpb);
  free(Qb1);
  free(Qb0);
  free(R);
  free(Rb);
  return info ? info : (info0 ? (int)(info0 + n) : 0);
}

/* --------------------------------------------------------------------------
 * Gaussian-process regression with banded natural parameters (Appendix C.5,
 * Algorithm 10), in the algorithm's order: C of the prior precision, C of the
 * posterior precision (prior + likelihood), then the log-determinants and the
 * two squared norms ||C^{-1} eta||^2.  Reverse mode: each factor's value term
 * s * (sum log C_ii) + t * ||C^{-1} eta||^2 (s = +1, t = -1/2 for the prior;
 * s = -1, t = +1/2 for the posterior) goes back through the log-determinant
 * and solve rows of Table 1 and Algorithm 2; the posterior's precision and
 * natural mean are sums, so their gradients flow to both summands.
 * ------------------------------------------------------------------------ */
static void natgp_term(int64_t n, int k, int64_t ld, const double *L, const double *eta, double s,
                       double t, double *Lambar, double *etabar) {
  size_t bsz = (size_t)(n * ld + 1);
  double *R = (double *)malloc((n + 1) * sizeof(double));
  double *Rb = (double *)malloc((n + 1) * sizeof(double));
  double *Lb = (double *)calloc(bsz, sizeof(double));
  double *Lb2 = (double *)calloc(bsz, sizeof(double));
  or_trsv(n, k, ld, L, 0, eta, R);
  or_logdet_bwd(n, k, ld, L, 0.5 * s, Lb);   /* sum log C_ii = logdet / 2 */
  for (int64_t i = 0; i < n; ++i) Rb[i] = 2.0 * t * R[i];
  or_trsv_bwd(n, k, ld, L, 0, R, Rb, etabar, Lb2);
  for (int64_t e = 0; e < n * ld; ++e) Lb[e] += Lb2[e];
  or_chol_bwd(n, k, ld, L, Lb, Lambar);
  free(R);
  free(Rb);
  free(Lb);
  free(Lb2);
}

static double natgp_sqnorm(int64_t n, int k, int64_t ld, const double *L, const double *eta) {
  double *R = (double *)malloc((n + 1) * sizeof(double)), q = 0.0;
  or_trsv(n, k, ld, L, 0, eta, R);
  for (int64_t i = 0; i < n; ++i) q += R[i] * R[i];
  free(R);
  return q;
}

int or_natgp(int64_t n, int k, int64_t ld, const double *Lam_pr, const double *eta_pr,
             const double *Lam_lik, const double *eta_lik, double *parts, double *Lprbar,
             double *Llikbar, double *etaprbar, double *etalikbar) {
  size_t bsz = (size_t)(n * ld + 1);
  double *Cpr = (double *)malloc(bsz * sizeof(double)), *Cpo = (double *)malloc(bsz * sizeof(double));
  double *Lpo = (double *)malloc(bsz * sizeof(double));
  double *eta_po = (double *)malloc((n + 1) * sizeof(double));
  double *gpr = (double *)calloc(bsz, sizeof(double)), *gpo = (double *)calloc(bsz, sizeof(double));
  double *epr = (double *)calloc(n + 1, sizeof(double)), *epo = (double *)calloc(n + 1, sizeof(double));
  for (int64_t e = 0; e < n * ld; ++e) Lpo[e] = Lam_pr[e] + Lam_lik[e];
  for (int64_t i = 0; i < n; ++i) eta_po[i] = eta_pr[i] + eta_lik[i];
  int info = or_chol(n, k, ld, Lam_pr, Cpr);
  int info1 = info ? 0 : or_chol(n, k, ld, Lpo, Cpo);
  if (info || info1) {
    for (int i = 0; i < 5; ++i) parts[i] = NAN;
  } else {
    double lpr = 0.5 * or_logdet(n, k, ld, Cpr), lpo = 0.5 * or_logdet(n, k, ld, Cpo);
    double qpr = natgp_sqnorm(n, k, ld, Cpr, eta_pr), qpo = natgp_sqnorm(n, k, ld, Cpo, eta_po);
    parts[0] = lpr - 0.5 * qpr - lpo + 0.5 * qpo;
    parts[1] = lpr;
    parts[2] = lpo;
    parts[3] = qpr;
    parts[4] = qpo;
    natgp_term(n, k, ld, Cpr, eta_pr, 1.0, -0.5, gpr, epr);
    natgp_term(n, k, ld, Cpo, eta_po, -1.0, 0.5, gpo, epo);
    for (int64_t e = 0; e < n * ld; ++e) {
      Lprbar[e] = gpr[e] + gpo[e];
      Llikbar[e] = gpo[e];
    }
    for (int64_t i = 0; i < n; ++i) {
      etaprbar[i] = epr[i] + epo[i];
      etalikbar[i] = epo[i];
    }
  }
  free(Cpr);
  free(Cpo);
  free(Lpo);
  free(eta_po);
  free(gpr);
  free(gpo);
  free(epr);
  free(epo);
  return info ? info : (info1 ? (int)(info1 + n) : 0);
}

/* --------------------------------------------------------------------------
 * Whitened GMRF sample (Section 3.2, Algorithm 6): C, then S with the
 * transposed factor; the reverse mode composes the solve row of Table 1 (for
 * the transposed factor) with Algorithm 2.
 * ------------------------------------------------------------------------ */
int or_whiten(int64_t n, int k, int64_t ld, const double *Q, const double *v, double *L, double *F) {
  int info = or_chol(n, k, ld, Q, L);
  if (info) {
    for (int64_t i = 0; i < n; ++i) F[i] = NAN;
    return info;
  }
  or_trsv(n, k, ld, L, 1, v, F);
  return 0;
}

void or_whiten_bwd(int64_t n, int k, int64_t ld, const double *L, const double *F, const double *Fbar,
                   double *vbar, double *Qbar) {
  double *Lb = (double *)calloc((size_t)(n * ld + 1), sizeof(double));
  or_trsv_bwd(n, k, ld, L, 1, F, Fbar, vbar, Lb);
  or_chol_bwd(n, k, ld, L, Lb, Qbar);
  free(Lb);
}

/* --------------------------------------------------------------------------
 * Variational KL term (Section 3.3, Eq. (KL), Algorithm 7), in the order of
 * Algorithm 7: the band of I(L_q), the product P(L_p, L_p^T), the trace as the
 * element-wise product over the band, the log-diagonals, P(L_p^T, m_p - m_q).
 * Reverse mode (Table 1 compositions):
 *   Sigmabar_q = 1/2 w Q_p (w = 1 on the diagonal, 2 off it: a stored
 *     off-diagonal entry of a symmetric band stands for two entries), then
 *     Algorithm 4 gives Lqbar, plus 1/[L_q]_ii from the log term;
 *   Lpbar = band(I(L_q) L_p) from the trace (the symmetric band of I(L_q)
 *     suffices on the band of L_p), + d v^T restricted to the band
 *     (v = L_p^T d, d = m_p - m_q), - 1/[L_p]_ii;
 *   mpbar = L_p v = -mqbar.
 * ------------------------------------------------------------------------ */
void or_vi_kl(int64_t n, int k, int64_t ld, const double *Lq, const double *Lp,
              const double *mq, const double *mp, double *parts, double *Lqbar,
              double *Lpbar, double *mqbar, double *mpbar, double *Sig) {
  size_t bsz = (size_t)(n * ld + 1) * sizeof(double);
  size_t vsz = (size_t)(n + 1) * sizeof(double);
  int64_t lds = 2 * (int64_t)k + 1;
  double *Sw = Sig ? Sig : (double *)malloc(bsz);
  double *Qp = (double *)calloc((size_t)(n * ld + 1), sizeof(double));
  double *Sb = (double *)calloc((size_t)(n * ld + 1), sizeof(double));
  double *Ssym = (double *)calloc((size_t)(n * lds + 1), sizeof(double));
  double *Ob = (double *)calloc((size_t)(n * ld + 1), sizeof(double));
  double *d = (double *)malloc(vsz);
  double *v = (double *)malloc(vsz);
  /* forward */
  or_subset_inv(n, k, ld, Lq, k, ld, Sw);
  or_gbmm(n, k, 0, ld, Lp, 0, k, 0, ld, Lp, 1, k, 0, ld, Qp);
  double tr = 0.0, lq = 0.0, lp = 0.0, maha = 0.0;
  for (int64_t j = 0; j < n; ++j)
    for (int s = 0; s <= k && j + s < n; ++s) tr += (s == 0 ? 1.0 : 2.0) * Sw[j * ld + s] * Qp[j * ld + s];
  /* the log-diagonal sums are compensated, as the log-determinant is */
  lq = 0.5 * or_logdet(n, k, ld, Lq);
  lp = 0.5 * or_logdet(n, k, ld, Lp);
  for (int64_t i = 0; i < n; ++i) d[i] = mp[i] - mq[i];
  or_gbmv(n, k, 0, ld, Lp, 1, d, v);
  for (int64_t i = 0; i < n; ++i) maha += v[i] * v[i];
  parts[0] = 0.5 * (tr + 2.0 * (lq - lp) + maha - (double)n);
  parts[1] = tr;
  parts[2] = lq - lp;
  parts[3] = maha;
  /* reverse: L_q */
  for (int64_t j = 0; j < n; ++j)
    for (int s = 0; s <= k && j + s < n; ++s) Sb[j * ld + s] = 0.5 * (s == 0 ? 1.0 : 2.0) * Qp[j * ld + s];
  or_subset_inv_bwd(n, k, ld, Lq, Sw, Sb, Lqbar);
  or_logdet_bwd(n, k, ld, Lq, 0.5, Lqbar);
  /* reverse: L_p */
  for (int64_t j = 0; j < n; ++j)
    for (int64_t i = imax64(0, j - k); i <= imin64(n - 1, j + k); ++i)
      Ssym[j * lds + k + (i - j)] = i >= j ? LOW(Sw, ld, i, j) : LOW(Sw, ld, j, i);
  or_gbmm(n, k, k, lds, Ssym, 0, k, 0, ld, Lp, 0, k, 0, ld, Lpbar);
  or_outer_band(n, k, 0, ld, d, v, Ob);
  for (int64_t t = 0; t < n * ld; ++t) Lpbar[t] += Ob[t];
  or_logdet_bwd(n, k, ld, Lp, -0.5, Lpbar);
  /* reverse: means */
  or_gbmv(n, k, 0, ld, Lp, 0, v, mpbar);
  for (int64_t i = 0; i < n; ++i) mqbar[i] = -mpbar[i];
  if (!Sig) free(Sw);
  free(Qp);
  free(Sb);
  free(Ssym);
  free(Ob);
  free(d);
  free(v);
}

int or_vi_kl_batch(int nprob, const int64_t *n, const int *k,
                   const int64_t *boff, const int64_t *voff, const double *Lq,
                   const double *Lp, const double *mq, const double *mp,
                   double *parts, double *Lqbar, double *Lpbar, double *mqbar,
                   double *mpbar) {
  int nthreads = 1;
#ifdef _OPENMP
#pragma omp parallel
  {
#pragma omp single
    nthreads = omp_get_num_threads();
  }
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int p = 0; p < nprob; ++p)
    or_vi_kl(n[p], k[p], (int64_t)k[p] + 1, Lq + boff[p], Lp + boff[p], mq + voff[p],
             mp + voff[p], parts + 4 * p, Lqbar + boff[p], Lpbar + boff[p],
             mqbar + voff[p], mpbar + voff[p], NULL);
  return nthreads;
}

int or_gauss_loss_batch(int nprob, const int64_t *n, const int *k,
                        const int64_t *boff, const int64_t *voff,
                        const double *Q, const double *y, const double *S,
                        double *parts, double *Qbar, double *ybar, int *info) {
  int nthreads = 1;
#ifdef _OPENMP
#pragma omp parallel
  {
#pragma omp single
    nthreads = omp_get_num_threads();
  }
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int p = 0; p < nprob; ++p) {
    int64_t ld = k[p] + 1;
    info[p] = or_gauss_loss(n[p], k[p], ld, Q + boff[p], y + voff[p],
                            S + boff[p], parts + 3 * p,
                            Qbar + boff[p], ybar + voff[p], NULL, NULL,
                            NULL, NULL);
  }
  return nthreads;
}

int or_forward_batch(int nprob, const int64_t *n, const int *k,
                     const int64_t *boff, const int64_t *voff, const double *Q,
                     const double *y, double *L, double *z, double *x,
                     double *Sig, double *logdet, int *info) {
  int nthreads = 1;
#ifdef _OPENMP
#pragma omp parallel
  {
#pragma omp single
    nthreads = omp_get_num_threads();
  }
#pragma omp parallel for schedule(dynamic, 1)
#endif
  for (int p = 0; p < nprob; ++p) {
    int64_t ld = k[p] + 1, np = n[p];
    size_t bsz = (size_t)(np * ld + 1) * sizeof(double);
    size_t vsz = (size_t)(np + 1) * sizeof(double);
    double *Lp = L ? L + boff[p] : (double *)malloc(bsz);
    double *zp = z ? z + voff[p] : (double *)malloc(vsz);
    double *xp = x ? x + voff[p] : (double *)malloc(vsz);
    info[p] = or_chol(np, k[p], ld, Q + boff[p], Lp);
    if (info[p] == 0) {
      logdet[p] = or_logdet(np, k[p], ld, Lp);
      or_trsv(np, k[p], ld, Lp, 0, y + voff[p], zp);
      or_trsv(np, k[p], ld, Lp, 1, zp, xp);
      if (Sig) or_subset_inv(np, k[p], ld, Lp, k[p], ld, Sig + boff[p]);
    } else {
      logdet[p] = NAN;
    }
    if (!L) free(Lp);
    if (!z) free(zp);
    if (!x) free(xp);
  }
  return nthreads;
}
