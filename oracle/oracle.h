/*
 * oracle.h -- plain, slow, FP64 CPU reference of the banded operator set of
 * "Banded Matrix Operators for Gaussian Markov Models in the Automatic
 * Differentiation Era" (Durrande et al., AISTATS 2019).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark do.  It shares no source with the HIP path.
 *
 * Storage (Section 4.3, "Storage footprint"): a banded n x n matrix B with lower
 * bandwidth l and upper bandwidth u is kept as n records of l+u+1 values; record
 * j is column j of B restricted to the band, B[j-u .. j+l, j], and the value
 * B[i,j] sits at slot u+i-j of record j.  Records are ld >= l+u+1 doubles apart.
 * For lower-banded / symmetric-stored matrices u = 0 and slot d = i-j holds
 * B[j+d, j].  Slots that fall outside the matrix (i < 0 or i >= n) are never read
 * and are written as 0 in outputs.
 *
 * All pointers are host pointers owned by the caller.  Every routine is a direct
 * transcription of the operator's definition or of the paper's algorithm using
 * dense (i,j) indices mapped onto the band, as the appendix on algorithms does.
 */
#ifndef BANDED_ORACLE_H
#define BANDED_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* C: banded Cholesky Q = L L^T (Algorithm 1; Section 4.1).  Q symmetric, stored
 * as its lower band with k sub-diagonals.  Returns 0, or r > 0 when the leading
 * minor of order r is not positive definite (pivot <= 0 or NaN); rows >= r-1 of
 * L are then zero. */
int or_chol(int64_t n, int k, int64_t ld, const double *Q, double *L);

/* log det(L L^T) = 2 sum_i log L_ii (Eq. (2), Eq. (3)), Neumaier-compensated. */
double or_logdet(int64_t n, int k, int64_t ld, const double *L);

/* S: triangular solve (Section 4.1).  trans = 0: x = L^{-1} b;
 * trans = 1: x = L^{-T} b (the upper-banded variant). */
void or_trsv(int64_t n, int k, int64_t ld, const double *L, int trans,
             const double *b, double *x);

/* I: lower band of width kout >= k of (L L^T)^{-1} (Algorithm 3, Takahashi),
 * output records of stride lds >= kout+1. */
void or_subset_inv(int64_t n, int k, int64_t ld, const double *L, int kout,
                   int64_t lds, double *S);

/* Reverse mode of C (Algorithm 2): Qbar = d c / d Q for the stored lower-band
 * entries of Q, given Lbar = d c / d L.  Lbar is not modified. */
void or_chol_bwd(int64_t n, int k, int64_t ld, const double *L,
                 const double *Lbar, double *Qbar);

/* Reverse mode of I (Algorithm 4): Lbar = d c / d L given S = I(L) and
 * Sbar = d c / d S for the stored lower-band entries of S (width k). */
void or_subset_inv_bwd(int64_t n, int k, int64_t ld, const double *L,
                       const double *S, const double *Sbar, double *Lbar);

/* Reverse mode of S (Table 1, solve matrix-vector).  x is the forward output
 * (L^{-1} b for trans = 0, L^{-T} b for trans = 1), xbar its sensitivity.
 * Writes bbar and Lbar (overwrites both). */
void or_trsv_bwd(int64_t n, int k, int64_t ld, const double *L, int trans,
                 const double *x, const double *xbar, double *bbar,
                 double *Lbar);

/* Reverse mode of the log-determinant: Lbar_ii += 2 gbar / L_ii. */
void or_logdet_bwd(int64_t n, int k, int64_t ld, const double *L, double gbar,
                   double *Lbar);

/* P: band of op(A) op(B) restricted to lower/upper widths (lc, uc); op = ^T
 * when the flag is set (Section 4.1, Products; appendix derivation of P). */
void or_gbmm(int64_t n,
             int la, int ua, int64_t lda, const double *A, int tA,
             int lb, int ub, int64_t ldb, const double *B, int tB,
             int lc, int uc, int64_t ldc, double *C);

/* P: y = op(A) x for a (l,u)-banded A. */
void or_gbmv(int64_t n, int l, int u, int64_t ld, const double *A, int tA,
             const double *x, double *y);

/* O: band (l,u) of the outer product m v^T (Section 4.1). */
void or_outer_band(int64_t n, int l, int u, int64_t ld, const double *m,
                   const double *v, double *O);

/* Solve of a lower-banded L (k sub-diagonals) against a banded right-hand side
 * R with upper width u (Algorithm 5): band (k,u) of L^{-1} R. */
void or_solve_band_mat(int64_t n, int k, int64_t ldl, const double *L, int lr,
                       int ur, int64_t ldr, const double *R, int64_t ldo,
                       double *O);

/* Reverse mode of Algorithm 5 (Table 1, solve matrix-matrix): given the band
 * O (k lower, ur upper) of L^{-1} R and its sensitivity Obar on that band,
 *   G = S(L^T, Obar) = L^{-T} Obar, exact on the band (k, ur),
 *   Rbar = G on the band (lr, ur) of R (zero where that band exceeds G's),
 *   Lbar = -band_k(G O^T), which needs only band entries of O.
 * Writes Rbar (stride ldr) and Lbar (stride ldl). */
void or_solve_band_mat_bwd(int64_t n, int k, int64_t ldl, const double *L, int lr,
                           int ur, int64_t ldo, const double *O,
                           const double *Obar, int64_t ldr, double *Rbar,
                           double *Lbar);

/* The Gaussian loss of a banded precision and its gradients, composed from the
 * operators above (Table 1 and Algorithms 1-4):
 *   loss = log det Q - y^T Q^{-1} y + tr(Q^{-1} S)
 * Q and S are symmetric, stored as lower bands with k sub-diagonals.
 * parts[0] = log det Q, parts[1] = y^T Q^{-1} y, parts[2] = tr(Q^{-1} S).
 * Qbar is the gradient with respect to the stored lower-band entries of Q, ybar
 * the gradient with respect to y.  Any of L, z, Sig, Lbar may be NULL (then
 * scratch memory is used); when given they receive the intermediates
 * L = C(Q), z = L^{-1} y, Sig = I(L), Lbar = d loss / d L.
 * Returns the Cholesky info. */
int or_gauss_loss(int64_t n, int k, int64_t ld, const double *Q,
                  const double *y, const double *S, double *parts,
                  double *Qbar, double *ybar, double *L, double *z,
                  double *Sig, double *Lbar);

/* Log marginal likelihood of a conjugate GMRF with partial observations
 * (Section 3.1, Eq. (marg_lik); Algorithm 8): prior precision Q (lower band,
 * k sub-diagonals, stride ld) over n nodes, observation mask (1 at the
 * observed nodes, 0 elsewhere: the diagonal of E^T E), b = E^T Y (observed
 * values at their nodes, 0 elsewhere) and noise variance tau2:
 *   log p(Y) = -(m/2) log 2 pi - log|L| + log|L_Q| - (m/2) log tau2
 *              - Y^T Y / (2 tau2) + ||L^{-1} b||^2 / (2 tau2^2),
 * L L^T = Q + E^T E / tau2, L_Q L_Q^T = Q, m = number of observed nodes.
 * parts[0] = log p(Y), parts[1] = log|L|, parts[2] = log|L_Q|,
 * parts[3] = ||L^{-1} b||^2.  Reverse mode (Table 1 compositions): Qbar
 * (stored lower-band entries), bbar (d log p / d b at the observed nodes, 0
 * elsewhere) and *tau2bar.  Returns 0, or the Cholesky info of the posterior
 * (as is) or of the prior (+ n). */
int or_marglik(int64_t n, int k, int64_t ld, const double *Q, const double *mask,
               const double *b, double tau2, double *parts, double *Qbar,
               double *bbar, double *tau2bar);

/* Gaussian-process regression with banded natural parameters (Appendix C.5,
 * Algorithm 10).  Prior N(F; eta_pr, Lam_pr) and Gaussian likelihood
 * N(F; eta_lik, Lam_lik) in natural parameters (Lam_pr, Lam_lik symmetric, lower
 * bands of width k, stride ld); posterior Lam_po = Lam_pr + Lam_lik,
 * eta_po = eta_pr + eta_lik; C_pr = C(Lam_pr), C_po = C(Lam_po).  With
 * a(eta, Lam) = 1/2 log|Lam| - 1/2 eta^T Lam^{-1} eta (the 2 pi terms of the
 * prior and posterior cancel):
 *   value = a(eta_pr, Lam_pr) - a(eta_po, Lam_po)
 *         = sum_i log[C_pr]_ii - 1/2 ||C_pr^{-1} eta_pr||^2
 *           - sum_i log[C_po]_ii + 1/2 ||C_po^{-1} eta_po||^2,
 * and log p(Y) = value + the likelihood's own normaliser in data space
 * (-(n_y/2) log 2 pi - 1/2 log|R| - 1/2 sum_t Y_t^T R^{-1} Y_t), which involves no
 * banded matrix and is left to the caller.  parts[0] = value,
 * parts[1] = sum log[C_pr]_ii, parts[2] = sum log[C_po]_ii,
 * parts[3] = ||C_pr^{-1} eta_pr||^2, parts[4] = ||C_po^{-1} eta_po||^2.
 * Reverse mode (Table 1 compositions through both Cholesky factors): Lprbar,
 * Llikbar (stored lower-band entries), etaprbar, etalikbar.  Returns 0, the
 * prior's Cholesky info (as is), or the posterior's (+ n). */
int or_natgp(int64_t n, int k, int64_t ld, const double *Lam_pr, const double *eta_pr,
             const double *Lam_lik, const double *eta_lik, double *parts, double *Lprbar,
             double *Llikbar, double *etaprbar, double *etalikbar);

/* Whitened sample of the GMRF for gradient-based MCMC (Section 3.2,
 * Algorithm 6): L = C(Q) and F = S(L^T, v) = L^{-T} v, so that F ~ N(0, Q^{-1})
 * when v ~ N(0, I).  Returns the Cholesky info (0 when Q is positive
 * definite). */
int or_whiten(int64_t n, int k, int64_t ld, const double *Q, const double *v, double *L, double *F);
/* Its reverse mode (Table 1, solve row with the transposed factor, then
 * Algorithm 2): given Fbar, vbar = L^{-1} Fbar, Lbar = -band(F vbar^T) and Qbar
 * from Algorithm 2 (stored lower-band entries). */
void or_whiten_bwd(int64_t n, int k, int64_t ld, const double *L, const double *F, const double *Fbar,
                   double *vbar, double *Qbar);

/* Kullback-Leibler term of the variational objective (Section 3.3, Eq. (KL);
 * Algorithm 7): q = N(m_q, (L_q L_q^T)^{-1}), p = N(m_p, (L_p L_p^T)^{-1}), with
 * L_q and L_p lower bands of the same width k (stride ld), composed from I, P
 * and the log-determinant:
 *   KL = 1/2 (tr(I(L_q) P(L_p, L_p^T)) + 2 sum_i (log[L_q]_ii - log[L_p]_ii)
 *             + ||P(L_p^T, m_p - m_q)||^2 - n).
 * parts[0] = KL, parts[1] = the trace, parts[2] = sum_i log[L_q]_ii -
 * log[L_p]_ii, parts[3] = the squared norm.  Reverse mode: Lqbar, Lpbar (stored
 * lower-band entries), mqbar, mpbar = d KL / d (L_q, L_p, m_q, m_p); Sig (may
 * be NULL) receives I(L_q), whose diagonal holds the marginal variances of q. */
void or_vi_kl(int64_t n, int k, int64_t ld, const double *Lq, const double *Lp,
              const double *mq, const double *mp, double *parts, double *Lqbar,
              double *Lpbar, double *mqbar, double *mpbar, double *Sig);

/* The KL term over a batch (layout as or_gauss_loss_batch), OpenMP across
 * problems; parts is 4*nprob.  Returns the number of threads used. */
int or_vi_kl_batch(int nprob, const int64_t *n, const int *k,
                   const int64_t *boff, const int64_t *voff, const double *Lq,
                   const double *Lp, const double *mq, const double *mp,
                   double *parts, double *Lqbar, double *Lpbar, double *mqbar,
                   double *mpbar);

/* The same over a batch of independent problems with OpenMP across problems
 * (one problem per thread).  Problem p has n[p] rows, k[p] sub-diagonals,
 * records of stride k[p]+1 starting at element offset boff[p] of the band
 * arrays, and vectors starting at element voff[p].  parts is 3*nprob, info is nprob.  Returns the number of threads
 * used. */
int or_gauss_loss_batch(int nprob, const int64_t *n, const int *k,
                        const int64_t *boff, const int64_t *voff,
                        const double *Q, const double *y, const double *S,
                        double *parts, double *Qbar, double *ybar, int *info);

/* Forward list over a batch (chol, logdet, L^{-1}y, L^{-T}L^{-1}y, band of
 * Q^{-1}), OpenMP across problems.  Outputs may be NULL except logdet/info. */
int or_forward_batch(int nprob, const int64_t *n, const int *k,
                     const int64_t *boff, const int64_t *voff, const double *Q,
                     const double *y, double *L, double *z, double *x,
                     double *Sig, double *logdet, int *info);

#ifdef __cplusplus
}
#endif
#endif
