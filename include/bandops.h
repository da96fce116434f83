/*
 * bandops.h -- C ABI of the MI355X (gfx950) banded-matrix operator library.
 *
 * Operators of "Banded Matrix Operators for Gaussian Markov Models in the
 * Automatic Differentiation Era" (Durrande et al., AISTATS 2019):
 * Cholesky C, triangular solves S, subset inverse I, products P, band-restricted
 * outer product O (Section 4.1) and their reverse-mode sensitivities (Section
 * 4.2, Table 1, Algorithms 2 and 4).
 *
 * Conventions shared by every call
 * --------------------------------
 *  - Storage (Section 4.3): a banded n x n matrix B with lower width l and upper
 *    width u is n records of ld >= l+u+1 elements; record j is column j of B on
 *    its band, B[j-u .. j+l, j], element (i,j) at slot u+i-j.  Lower-triangular
 *    factors use (l,u) = (k,0); symmetric matrices (Q, Sigma and their
 *    sensitivities) are stored as their lower band, (k,0).  Slots that fall
 *    outside the matrix are never read; outputs write them as 0.
 *  - Precision: BO_F64 stores everything as double.  BO_MIXED stores band
 *    records and vectors as float and keeps every diagonal in the FP64 side
 *    array `diag64` (n doubles); slot 0 of a mixed record then holds an FP32
 *    copy that is ignored on input.  All arithmetic is FP64 in both modes, and
 *    log-determinants are accumulated in FP64.
 *  - Memory: every data pointer is a DEVICE pointer owned by the caller.  The
 *    library never allocates inside a call; `ws` is caller-provided device
 *    workspace of at least the size reported by the matching *_workspace_size
 *    query.  Inputs are never modified.  Outputs may not alias inputs.
 *  - Execution: calls are asynchronous and ordered on `stream`; no call
 *    synchronises the host.  They contain no allocation, no host sync and no
 *    memset, so they may be captured into a HIP graph.
 *  - Errors: the return value reports argument and launch errors only
 *    (negative bo_status), detected before any work is queued where possible;
 *    bo_last_error() then gives a thread-local message.  Numerical failure is
 *    reported on the device in `info`: 0, or r > 0 when the leading minor of
 *    order r is not positive definite (pivot <= 0 or NaN; LAPACK convention).
 *    Outputs of such a problem are unspecified from row r-1 on; other problems
 *    of a batch are unaffected.
 *  - Gradients are with respect to the stored band entries: an off-diagonal
 *    stored entry of a symmetric matrix stands for both (i,j) and (j,i).
 */
#ifndef BANDOPS_H
#define BANDOPS_H

#include <hip/hip_runtime_api.h>
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Storage formats.  There is no pure-FP32 format: every pass is bound by HBM
 * traffic (0.1 - 1 flop per byte), so FP32 arithmetic would save no time,
 * while FP32 pivots break down on the paper's state-space precisions (an
 * FP32-rounded Matern-3/2 precision at lengthscale 10 is already
 * indefinite).  BO_MIXED halves the off-diagonal traffic and keeps every
 * pivot, log-determinant and diagonal in FP64. */
typedef enum { BO_F64 = 0, BO_MIXED = 1 } bo_prec;

typedef enum {
  BO_OK = 0,
  BO_EINVAL = -1,        /* bad argument (null pointer, shape, stride, width) */
  BO_EDEVICE = -2,       /* HIP launch or runtime error                       */
  BO_EWORKSPACE = -3,    /* workspace too small                               */
  BO_EUNSUPPORTED = -4   /* bandwidth or variant without compiled kernels     */
} bo_status;

/* Largest lower bandwidth k with compiled kernels. */
#define BO_KMAX 12

typedef struct {
  void *band;       /* n records of ld elements (double, or float for BO_MIXED) */
  double *diag64;   /* BO_MIXED: FP64 diagonal (n); must be NULL for BO_F64    */
  int64_t n;        /* order of the matrix                                     */
  int32_t l;        /* lower width (sub-diagonals)                             */
  int32_t u;        /* upper width (0 for lower / symmetric-stored bands)      */
  int32_t ld;       /* record stride in elements, >= l+u+1                     */
  int32_t reserved;
} bo_band;

/* Workspace (bytes) that any single-problem call below needs for an n x n
 * matrix with k sub-diagonals. */
size_t bo_workspace_size(int64_t n, int32_t k);

/* ------------------------------------------------------------ forward ops */

/* C (Algorithm 1, Section 4.1): L with L L^T = Q; also log det Q =
 * 2 sum log L_ii (Eq. (2) and the KL term of Section 3.3), and optionally
 * z = L^{-1} y (S, Section 4.1) in the same pass.  Q, L: (k,0) bands with the
 * same ld.  y, z: n-vectors or both NULL.  logdet: one device double (may be
 * NULL).  info: one device int32 (required). */
bo_status bo_chol(bo_prec prec, const bo_band *Q, bo_band *L, const void *y, void *z,
                  double *logdet, int32_t *info, void *ws, size_t ws_bytes, hipStream_t stream);

/* bo_chol without a workspace argument, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same operation, arguments and results as
 * bo_chol, with the workspace in a fixed device array of the library of
 * BO_NOALLOC_SCRATCH_MB MiB per GPU (bo_chol_noalloc_scratch_bytes()), held
 * until the process ends.  When bo_chol's schedule would need more, fewer
 * chunks are used (same results up to rounding order); a problem whose
 * smallest schedule still does not fit returns BO_EWORKSPACE.  The call
 * allocates nothing.  Every call on one GPU shares that GPU's array: calls
 * that overlap in time on one GPU (different streams, or host threads
 * without ordering) race and must not be issued. */
#define BO_NOALLOC_SCRATCH_MB 64
size_t bo_chol_noalloc_scratch_bytes(void);
bo_status bo_chol_noalloc(bo_prec prec, const bo_band *Q, bo_band *L, const void *y, void *z, double *logdet,
                          int32_t *info, hipStream_t stream);

/* S (Section 4.1): X = L^{-1} B (trans = 0) or X = L^{-T} B (trans = 1, the
 * upper-banded variant the gradients need, Section 4.1 "transposes") for nrhs
 * right-hand sides: column c of B and of X starts at element c * ldx (ldx >=
 * n; ignored when nrhs = 1), in double (BO_F64) or float (BO_MIXED).  The
 * columns are solved one after another on the stream with the same
 * workspace (bo_workspace_size(n, k)).  nrhs = 0 does nothing; B and X may
 * not overlap. */
bo_status bo_trsv(bo_prec prec, const bo_band *L, int trans, const void *b, void *x, int64_t nrhs,
                  int64_t ldx, void *ws, size_t ws_bytes, hipStream_t stream);

/* I (Algorithm 3, Takahashi): Sigma = lower band of (L L^T)^{-1} of width
 * kout = Sigma->l >= L->l (Algorithm 3's recursion read on kout sub-diagonals;
 * the entries beyond L's band follow from the same sums).  With kout = L->l,
 * Sigma has L's stride.  With kout > L->l (kout <= BO_KMAX), Sigma must be
 * packed (ld = kout + 1), and ws holds a copy of L widened to kout with zero
 * slots: at least bo_subset_inv_workspace_size(n, L->l, kout) bytes. */
size_t bo_subset_inv_workspace_size(int64_t n, int32_t k, int32_t kout);
bo_status bo_subset_inv(bo_prec prec, const bo_band *L, bo_band *Sigma, void *ws, size_t ws_bytes,
                        hipStream_t stream);

/* P (Section 4.1, "Products"): C = band of op(A) op(B) on C's (l,u), op = ^T
 * when the flag is set.  A, B, C are general bands. */
bo_status bo_gbmm(bo_prec prec, const bo_band *A, int tA, const bo_band *B, int tB, bo_band *C,
                  hipStream_t stream);

/* P: y = op(A) x. */
bo_status bo_gbmv(bo_prec prec, const bo_band *A, int tA, const void *x, void *y,
                  hipStream_t stream);

/* O (Section 4.1, outer product restricted to a band): O = alpha m v^T on O's
 * (l,u) band, or O += alpha m v^T when accumulate is set. */
bo_status bo_outer_band(bo_prec prec, const void *m, const void *v, double alpha, int accumulate,
                        bo_band *O, hipStream_t stream);

/* S with a banded right-hand side (Algorithm 5): O = the band (k lower, u
 * upper) of L^{-1} R for L lower-banded with k sub-diagonals and R a general
 * band with u upper diagonals (and any lower width).  O must have l = k and
 * u = R's u; its entries are exact (a column of L^{-1} R is zero above row
 * c - u, and the entries in the band need only band entries above them).
 * k, u <= 12; returns BO_EUNSUPPORTED above.  One lane per column. */
bo_status bo_solve_band_mat(bo_prec prec, const bo_band *L, const bo_band *R, bo_band *O,
                            hipStream_t stream);

/* ---------------------------------------------------------- reverse mode */

/* Reverse mode of C (Algorithm 2): Qbar = d c/d Q (stored lower entries) from
 * L and Lbar = d c/d L. */
bo_status bo_chol_bwd(bo_prec prec, const bo_band *L, const bo_band *Lbar, bo_band *Qbar,
                      void *ws, size_t ws_bytes, hipStream_t stream);

/* Reverse mode of I (Algorithm 4): Lbar (=, or += when accumulate) from L,
 * Sigma = I(L) and Sigmabar = d c/d Sigma (stored lower entries; the strict
 * upper triangle of Algorithm 4's local copy of the sensitivity is zero). */
bo_status bo_subset_inv_bwd(bo_prec prec, const bo_band *L, const bo_band *Sigma,
                            const bo_band *Sigmabar, bo_band *Lbar, int accumulate, void *ws,
                            size_t ws_bytes, hipStream_t stream);

/* Reverse mode of S (Table 1, solve matrix-vector).  x is the forward output
 * (L^{-1} b, or L^{-T} b for trans = 1) and xbar its sensitivity.  Writes
 * bbar = L^{-T} xbar (L^{-1} xbar for trans = 1) and the band of
 * Lbar = -bbar x^T (trans = 0) or -x bbar^T (trans = 1), assigned or added. */
bo_status bo_trsv_bwd(bo_prec prec, const bo_band *L, int trans, const void *x, const void *xbar,
                      void *bbar, bo_band *Lbar, int accumulate, void *ws, size_t ws_bytes,
                      hipStream_t stream);

/* Reverse mode of Algorithm 5 (Table 1, solve matrix-matrix): from O (the
 * forward output, band (k, u)) and its sensitivity Obar on that band,
 * Rbar = L^{-T} Obar on Rbar's band (Rbar has R's widths; u must equal O's)
 * and Lbar = -band_k((L^{-T} Obar) O^T), both overwritten.  ws holds
 * L^{-T} Obar on the band (k, u) in FP64: at least
 * bo_solve_band_mat_workspace(n, k, u) bytes (BO_EWORKSPACE otherwise). */
size_t bo_solve_band_mat_workspace(int64_t n, int32_t k, int32_t u);
bo_status bo_solve_band_mat_bwd(bo_prec prec, const bo_band *L, const bo_band *O, const bo_band *Obar,
                                bo_band *Rbar, bo_band *Lbar, void *ws, size_t ws_bytes,
                                hipStream_t stream);

/* Reverse mode of log det: Lbar_ii (=, +=) 2 gbar / L_ii; gbar is one device
 * double. */
bo_status bo_logdet_bwd(bo_prec prec, const bo_band *L, const double *gbar, bo_band *Lbar,
                        int accumulate, hipStream_t stream);

/* ------------------------------------------------ batched, uneven problems */

/* Problem p of a batch: n rows, k sub-diagonals; its band records (stride k+1)
 * start at element boff of every band array of the call, its vector entries at
 * element voff of every vector (and of every diag64 array). */
typedef struct {
  int64_t n;
  int32_t k;
  int32_t reserved;
  int64_t boff;
  int64_t voff;
} bo_problem;

typedef struct bo_plan bo_plan;

/* Arrays of one batched call (device pointers).  diag arrays are used in
 * BO_MIXED only.  Outputs that a call does not produce may be NULL. */
typedef struct {
  const void *Q;   const double *Qd;     /* precision, lower band              */
  const void *y;                          /* right-hand sides                  */
  const void *S;   const double *Sd;     /* S of tr(Q^{-1} S) (gauss_loss)     */
  void *L;         double *Ld;           /* Cholesky factor                    */
  void *z;                                /* L^{-1} y                          */
  void *x;                                /* forward: Q^{-1} y; loss: ybar     */
  void *Sig;       double *Sigd;         /* band of Q^{-1}                     */
  void *Lbar;      double *Lbard;        /* loss: subset-inverse part of Lbar  */
  void *Qbar;      double *Qbard;        /* loss: d loss / d Q (stored)        */
  double *logdet;                         /* per problem                       */
  double *parts;                          /* per problem: logdet, yQ^-1y, trace */
  int32_t *info;                          /* per problem                       */
  double *loss;                           /* loss: per problem (may be NULL)   */
  void *Sbar;      double *Sbard;         /* loss: d loss / d S (may be NULL)  */
} bo_batch_io;

/* Build a plan (host object): chunking of every problem into about
 * target_chunks lanes (0: library default), bandwidth ranges, workspace
 * layout.  Problems may have any n >= 0 and k in [0, BO_KMAX].  A plan with
 * problems of several bandwidths also creates one HIP stream per extra
 * bandwidth range (default priority) and the events that fork them from the
 * caller's stream and join them back within bo_plan_forward and
 * bo_plan_gauss_loss, so create it with the device current that runs it; one
 * plan serves one call at a time. */
bo_status bo_plan_create(const bo_problem *probs, int32_t nprob, int64_t target_chunks,
                         bo_plan **out);
bo_status bo_plan_workspace_size(const bo_plan *plan, size_t *bytes);
/* Workspace bytes for bo_plan_gauss_loss when it keeps L, Sig and Lbar in the
 * workspace (io->L, io->Sig and io->Lbar all NULL, BO_F64): the workspace
 * proper followed by three FP64 band arrays and two FP64 vectors (z and a
 * copy of ybar) in which the chunks of every wavefront lie interleaved row by
 * row, so that the passes read and write them in whole contiguous blocks. */
bo_status bo_plan_loss_workspace_size(const bo_plan *plan, size_t *bytes);
/* Copy the plan's device tables into ws (stream-ordered; do this once, before
 * capture, and again whenever ws is a new buffer). */
bo_status bo_plan_upload(const bo_plan *plan, void *ws, hipStream_t stream);
/* Forward list (Section 3 operations): L = C(Q), log det Q, z = L^{-1} y,
 * x = L^{-T} z = Q^{-1} y, Sig = I(L).  Any of z, x, Sig may be NULL. */
bo_status bo_plan_forward(const bo_plan *plan, bo_prec prec, const bo_batch_io *io, void *ws,
                          hipStream_t stream);
/* loss = log det Q - y^T Q^{-1} y + tr(Q^{-1} S) per problem and its reverse
 * mode: forward (C, log det, S, I), then Algorithm 4 with Sigmabar = S, the
 * solve sensitivity of Table 1 with zbar = -2z, the log-determinant
 * sensitivity and Algorithm 2.  Writes L, z, Sig, Lbar, x (= ybar), Qbar,
 * parts and info; when given, loss[p] (the sum of the parts) and Sbar =
 * d loss / d S on S's stored entries (Sigma_ii on the diagonal, 2 Sigma_ij off
 * it: an off-diagonal stored entry of S stands for S_ij and S_ji).  With L,
 * Sig and Lbar all NULL (BO_F64 only) the intermediates L, Sig, Lbar and z
 * are kept in ws, which must then hold bo_plan_loss_workspace_size bytes; z
 * may then be NULL (written when given), and the other outputs are the same,
 * bit for bit. */
bo_status bo_plan_gauss_loss(const bo_plan *plan, bo_prec prec, const bo_batch_io *io, void *ws,
                             hipStream_t stream);
/* Kullback-Leibler term of the variational objective (Section 3.3, Eq. (KL);
 * Algorithm 7) for every problem of the plan: q = N(m_q, (L_q L_q^T)^{-1}),
 * p = N(m_p, (L_p L_p^T)^{-1}), L_q and L_p lower bands of the plan's widths
 * (records at boff, vectors at voff as for the other plan calls):
 *   KL = 1/2 (tr(I(L_q) P(L_p, L_p^T)) + 2 sum_i (log[L_q]_ii - log[L_p]_ii)
 *             + ||P(L_p^T, m_p - m_q)||^2 - n),
 * and its reverse mode (Algorithm 4 on L_q with Sigmabar = P(L_p, L_p^T)/2,
 * Table 1 for the products and the log-determinants).  Every array is
 * required (the diagonals only in BO_MIXED); all are device arrays of the
 * caller.  Outputs: Sig = I(L_q) (its diagonal holds the marginal variances of
 * q), Lqbar, Lpbar (stored lower-band entries; Lpbar also serves as scratch
 * during the call), mqbar, mpbar, parts[4 p .. 4 p + 3] = (KL, the trace, sum
 * of log-diagonal differences, the squared norm).  The diagonals of L_q and
 * L_p must be positive (else the parts are NaN); the workspace is the plan's. */
typedef struct {
  const void *Lq;  const double *Lqd;    /* variational factor L_q              */
  const void *Lp;  const double *Lpd;    /* prior factor L_p                    */
  const void *mq;  const void *mp;       /* means of q and p                    */
  void *Sig;       double *Sigd;         /* out: I(L_q)                         */
  void *Lqbar;     double *Lqbard;       /* out: d KL / d L_q                   */
  void *Lpbar;     double *Lpbard;       /* out: d KL / d L_p                   */
  void *mqbar;     void *mpbar;          /* out: d KL / d m_q, d KL / d m_p     */
  double *parts;                          /* out: 4 per problem                  */
} bo_kl_io;
bo_status bo_plan_vi_kl(const bo_plan *plan, bo_prec prec, const bo_kl_io *io, void *ws,
                        hipStream_t stream);
/* Log marginal likelihood of a conjugate Gaussian Markov model with partial
 * observations (Section 3.1, Eq. (marg_lik); Algorithm 8) for every problem of
 * the plan: prior x ~ N(0, Q^{-1}), Y = E x + noise of variance tau2, m observed
 * nodes, mask = diag(E^T E) (1 at an observed node, 0 elsewhere), b = E^T Y
 * (the observed values at their nodes, 0 elsewhere), Q1 = Q + E^T E / tau2:
 *   log p(Y) = -(m/2) log 2 pi - log|L| + log|L_Q| - (m/2) log tau2
 *              - b^T b / (2 tau2) + ||L^{-1} b||^2 / (2 tau2^2),
 * L = C(Q1), L_Q = C(Q), with its reverse mode with respect to the stored
 * band of Q, b and tau2 (from forward quantities: I(L), I(L_Q), Q1^{-1} b).
 * Records of Q, L, Sig, Qbar at boff and vectors at voff as for the other plan
 * calls; every array is required (the diagonals only in BO_MIXED), all device
 * arrays of the caller.  Outputs: L (posterior factor), Sig = I(L) (the
 * posterior covariances on the band), x = Q1^{-1} b (the posterior mean is
 * x / tau2), Qbar (stored lower entries; it also holds I(L_Q) during the call),
 * bbar (0 at unobserved nodes; it holds L^{-1} b during the call), tau2bar[p],
 * parts[4 p .. 4 p + 3] = (log p(Y), log|L|, log|L_Q|, ||L^{-1} b||^2) and
 * info[p]: 0, else the first row at which C(Q1) fails (1-based), else n + the
 * row at which C(Q) fails; then the parts and tau2bar are NaN and the other
 * outputs unspecified.  tau2 must be positive (not checked on the device).
 * No output array may overlap an input or another output (intermediates are
 * kept in the outputs during the call).  The workspace is the plan's. */
typedef struct {
  const void *Q;   const double *Qd;     /* prior precision Q (lower band)       */
  const void *mask;                       /* observation mask (vector)            */
  const void *b;                          /* E^T Y (vector)                       */
  const double *tau2;                     /* noise variance, one per problem      */
  void *L;         double *Ld;           /* out: C(Q1)                           */
  void *Sig;       double *Sigd;         /* out: I(C(Q1))                        */
  void *x;                                /* out: Q1^{-1} b                       */
  void *Qbar;      double *Qbard;        /* out: d log p / d Q                   */
  void *bbar;                             /* out: d log p / d b                   */
  double *tau2bar;                        /* out: d log p / d tau2, per problem   */
  double *parts;                          /* out: 4 per problem                   */
  int32_t *info;                          /* out: per problem                     */
} bo_ml_io;
bo_status bo_plan_marglik(const bo_plan *plan, bo_prec prec, const bo_ml_io *io, void *ws,
                          hipStream_t stream);
/* Gaussian-process regression with banded natural parameters (Appendix C.5,
 * Algorithm 10) for every problem of the plan: prior N(F; eta_pr, Lam_pr) and
 * likelihood N(F; eta_lik, Lam_lik) in natural parameters (Lam_pr, Lam_lik
 * symmetric, stored as lower bands of the plan's widths), posterior
 * Lam_po = Lam_pr + Lam_lik, eta_po = eta_pr + eta_lik, C_pr = C(Lam_pr),
 * C_po = C(Lam_po):
 *   value = sum_i log[C_pr]_ii - 1/2 ||C_pr^{-1} eta_pr||^2
 *           - sum_i log[C_po]_ii + 1/2 ||C_po^{-1} eta_po||^2,
 * which is log p(Y) up to the likelihood's normaliser in data space
 * (-(n_y/2) log 2 pi - 1/2 log|R| - 1/2 sum_t Y_t^T R^{-1} Y_t, no banded matrix
 * in it: the caller's).  Reverse mode from forward quantities (the posterior
 * mean mu = Lam^{-1} eta and I(C) of both factors).  Records at boff, vectors at
 * voff as for the other plan calls; every array is required (the diagonals only
 * in BO_MIXED), all device arrays of the caller.  Outputs: L = C_po, Sig =
 * I(C_po) (posterior covariances on the band), x = the posterior mean
 * Lam_po^{-1} eta_po, which is also d value / d eta_lik, Lprbar, Llikbar (stored
 * lower entries), etaprbar, parts[5 p .. 5 p + 4] = (value, sum log[C_pr]_ii,
 * sum log[C_po]_ii, ||C_pr^{-1} eta_pr||^2, ||C_po^{-1} eta_po||^2) and info[p]:
 * 0, else the first row at which C(Lam_pr) fails (1-based), else n + the row at
 * which C(Lam_po) fails; then the parts are NaN and the other outputs
 * unspecified.  During the call L, x, Lprbar, Llikbar and etaprbar also hold
 * intermediates, so no output array may overlap an input or another output.
 * The workspace is the plan's. */
typedef struct {
  const void *Lpr;   const double *Lprd;   /* prior precision Lam_pr             */
  const void *etapr;                        /* prior natural mean eta_pr          */
  const void *Llik;  const double *Llikd;  /* likelihood precision Lam_lik       */
  const void *etalik;                       /* likelihood natural mean eta_lik    */
  void *L;           double *Ld;           /* out: C(Lam_po)                     */
  void *Sig;         double *Sigd;         /* out: I(C(Lam_po))                  */
  void *x;                                  /* out: Lam_po^{-1} eta_po            */
  void *Lprbar;      double *Lprbard;      /* out: d value / d Lam_pr            */
  void *Llikbar;     double *Llikbard;     /* out: d value / d Lam_lik           */
  void *etaprbar;                           /* out: d value / d eta_pr            */
  double *parts;                            /* out: 5 per problem                 */
  int32_t *info;                            /* out: per problem                   */
} bo_natgp_io;
bo_status bo_plan_natgp(const bo_plan *plan, bo_prec prec, const bo_natgp_io *io, void *ws,
                        hipStream_t stream);
/* Whitened GMRF sample for gradient-based MCMC (Section 3.2, Algorithm 6) for
 * every problem of the plan: L = C(Q) and F = S(L^T, v) = L^{-T} v, so that
 * F ~ N(0, Q^{-1}) when v ~ N(0, I).  bo_plan_whiten reads Q (Qd), v and writes
 * L (Ld), F, logdet[p] = log det Q (may be NULL) and info[p] (may be NULL: 0,
 * or the first failing row of C(Q), 1-based; F is then unspecified).
 * bo_plan_whiten_bwd is its reverse mode (Table 1, solve row; Algorithm 2): it
 * reads L (Ld), F and Fbar = d f / d F for a scalar f (the likelihood's
 * gradient: model-specific, the caller's) and writes vbar = L^{-1} Fbar and
 * Qbar (stored lower-band entries, Qbard in BO_MIXED).  The log density of v
 * itself, -1/2 v^T v - n/2 log 2 pi, holds no banded matrix and is the caller's
 * too.  Records at boff and vectors at voff as for the other plan calls; all
 * arrays are device arrays of the caller; the workspace is the plan's. */
typedef struct {
  const void *Q;     const double *Qd;     /* in (forward): precision Q         */
  const void *v;                            /* in (forward): white noise v       */
  void *L;           double *Ld;           /* out (forward), in (backward)      */
  void *F;                                  /* out (forward), in (backward)      */
  const void *Fbar;                         /* in (backward)                     */
  void *vbar;                               /* out (backward)                    */
  void *Qbar;        double *Qbard;        /* out (backward)                    */
  double *logdet;                           /* out (forward), per problem        */
  int32_t *info;                            /* out (forward), per problem        */
  int32_t reuse;   /* backward: nonzero reuses the chunk products of L that the
                      preceding bo_plan_whiten on this plan left in ws (L and ws
                      unchanged since, no other call on ws in between); 0
                      recomputes them */
} bo_whiten_io;
bo_status bo_plan_whiten(const bo_plan *plan, bo_prec prec, const bo_whiten_io *io, void *ws,
                         hipStream_t stream);
bo_status bo_plan_whiten_bwd(const bo_plan *plan, bo_prec prec, const bo_whiten_io *io, void *ws,
                             hipStream_t stream);
/* ------------------------------------------------- GMRF precisions on graphs */
/* A GMRF on a graph has Q_ij = 0 off the edges, and the bandwidth of Q
 * depends on the node ordering (Section 2); Section 5 orders a road network
 * with reverse Cuthill-McKee before using the banded operators.
 *
 * bo_rcm (host; every pointer is a host pointer): the reverse Cuthill-McKee
 * ordering of the symmetric pattern (indptr[n+1], indices[indptr[n]], CSR,
 * self-loops and repeated entries ignored).  Cuthill-McKee traverses every
 * connected component breadth-first from its node of lowest degree (ties: lower
 * index) and appends a visited node's unvisited neighbours by ascending degree
 * (ties: lower index); the reverse of that order is returned as perm[new] =
 * old, with iperm[old] = new (iperm may be NULL) and *bandwidth =
 * max |iperm[i] - iperm[j]| over the entries (may be NULL).  Malformed CSR
 * (indptr[0] != 0, decreasing indptr, an index outside [0, n)) is BO_EINVAL. */
bo_status bo_rcm(int64_t n, const int64_t *indptr, const int64_t *indices, int64_t *perm, int64_t *iperm,
                 int64_t *bandwidth);
/* bo_csr_permute (host): the pattern of P Q P^T for the ordering perm[new] =
 * old, iperm[old] = new: row j is row perm[j] of Q with its columns renamed
 * by iperm and sorted; map[e'] is the position in Q's CSR of the new entry e'
 * (so a value set in Q's layout goes to the new layout as vals[map]).
 * out_indptr has n+1 entries, out_indices and map indptr[n].  BO_EINVAL for
 * malformed CSR or when perm and iperm are not inverse permutations. */
bo_status bo_csr_permute(int64_t n, const int64_t *indptr, const int64_t *indices, const int64_t *perm,
                         const int64_t *iperm, int64_t *out_indptr, int64_t *out_indices, int64_t *map);
/* bo_csr_to_band (device arrays, stream-ordered): for nsets value sets on one
 * symmetric CSR pattern whose rows are in band order (indptr[n+1],
 * indices[nnz], sorted or not; set s's values at vals + s nnz, FP64), the
 * lower band (k <= 64 sub-diagonals, records of ld >= k+1 elements, pads 0;
 * set s's records at band + s n ld).  Record j, column j of the matrix, is
 * read as row j from the diagonal rightwards: the entries (j, c), c >= j, at
 * slot c - j (the matrix is symmetric); entries past slot k are dropped and
 * counted in *dropped (a device int64, cleared by the call).  band is FP64
 * (BO_F64) or FP32 with the FP64 diagonal in diag (at diag + s n; BO_MIXED;
 * diag must be NULL in BO_F64).  Repeated CSR entries are not allowed. */
bo_status bo_csr_to_band(bo_prec prec, int64_t n, int32_t nsets, const int64_t *indptr, const int64_t *indices,
                         int64_t nnz, const double *vals, int32_t k, int64_t ld, void *band, double *diag,
                         int64_t *dropped, hipStream_t stream);
/* bo_band_to_csr_grad: the reverse of bo_csr_to_band: gvals[s nnz + e] = the
 * band gradient of set s at the slot entry e was read into, 0 for the entries
 * the assembly did not read (left of the diagonal, or past the band).  Device
 * arrays, stream-ordered; gdiag is the FP64 diagonal in BO_MIXED (NULL in
 * BO_F64). */
bo_status bo_band_to_csr_grad(bo_prec prec, int64_t n, int32_t nsets, const int64_t *indptr,
                              const int64_t *indices, int64_t nnz, int32_t k, int64_t ld, const void *gband,
                              const double *gdiag, double *gvals, hipStream_t stream);

/* The chain rule over a plan's batch (the step a reverse-mode caller takes
 * with the upstream sensitivity g of each problem's scalar output):
 *   kind BO_SCALE_BAND:      out = g[p] * in on every stored entry of problem
 *                            p's records (boff, stride k+1);
 *   kind BO_SCALE_BAND_SYM:  as BO_SCALE_BAND with an extra factor 2 off the
 *                            diagonal (the stored-entry gradient of a trace
 *                            tr(Sigma S) with respect to a symmetric S);
 *   kind BO_SCALE_VEC:       out = g[p] * in on problem p's n entries (voff);
 *   kind BO_SCALE_PROBLEM:   out[p] = g[p] * in[p], one FP64 value per problem
 *                            (a per-problem scalar input such as tau2).
 * g: nprob device doubles in the caller's problem order, or NULL for 1.
 * BO_MIXED: records and vectors are float and the band diagonals are the FP64
 * arrays ind / outd (used for the band kinds only).  out may equal in.  The
 * workspace is the plan's (its problem tables).  Slots past a matrix's end
 * are written 0. */
enum { BO_SCALE_BAND = 0, BO_SCALE_BAND_SYM = 1, BO_SCALE_VEC = 2, BO_SCALE_PROBLEM = 3 };
bo_status bo_plan_scale(const bo_plan *plan, bo_prec prec, int32_t kind, const double *g, const void *in,
                        const double *ind, void *out, double *outd, void *ws, hipStream_t stream);

/* Plan statistics: out[0] problems, out[1] chunks, out[2] groups, out[3] rows,
 * out[4] largest k. */
bo_status bo_plan_stats(const bo_plan *plan, int64_t out[5]);
bo_status bo_plan_destroy(bo_plan *plan);

/* ------------------------------------ wide block-banded problems (k = 64) */
/* A lower bandwidth equal to the block size 64 is also handled as a
 * block-tridiagonal matrix of 64 x 64 blocks: Algorithms 1-4 written by blocks
 * (the O(N l^2) recurrences of Section 4.1 with the band cut into dense
 * tiles).  Dense block products run on the matrix cores in FP32 (MFMA); the
 * diagonal-block Cholesky, its inverse, the pivots and the log-determinant
 * are FP64.  Storage is BO_MIXED only: FP32 records of 65 elements (ld = 65)
 * plus FP64 diagonals.  probs[p].k must be 64; boff / voff as for plans.
 * Each problem's blocks are cut into chunks spread over the compute units and
 * every pass is an exact chunked scan (chunk maps, an in-order combination per
 * problem, replays from the exact entering states).  The workspace holds the
 * problem and chunk tables, two FP32 64 x 64 blocks per block row and eleven
 * per chunk; every call takes the same probs. */
bo_status bo_wide_workspace_size(const bo_problem *probs, int32_t nprob, size_t *bytes);
/* Copy the problem and chunk tables into ws (synchronous).  Call it before
 * any call that uses ws, and before graph capture. */
bo_status bo_wide_upload(const bo_problem *probs, int32_t nprob, void *ws, size_t ws_bytes);
/* Forward: L (with Ld), Sig (with Sigd), parts[3p] = log det Q_p (parts may
 * be NULL) and info; io->Q and io->Qd are the input. */
bo_status bo_wide_forward(const bo_problem *probs, int32_t nprob, const bo_batch_io *io, void *ws, size_t ws_bytes,
                          hipStream_t stream);
/* loss_p = log det Q_p + tr(Q_p^{-1} W_p), W_p given in io->S / io->Sd, and
 * its reverse mode: Algorithm 4 by blocks with Sigmabar = (W_ii, 2 W_ij), the
 * log-determinant sensitivity and Algorithm 2 by blocks.  Writes L, Sig,
 * Lbar (the subset-inverse part), Qbar (stored entries), parts (log det, 0,
 * trace) and info; a problem whose factorisation fails gets info > 0 and NaN
 * parts, its other outputs unspecified. */
bo_status bo_wide_gauss_loss(const bo_problem *probs, int32_t nprob, const bo_batch_io *io, void *ws,
                             size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------- profiling */
/* Kernel timing on the launch stream (a tracing aid).  While enabled, every
 * launch issued by this process is bracketed by two HIP events; do not enable
 * it around graph capture.  bo_profile_read waits for the recorded events and
 * returns, per step kind (slot), the summed duration in ms and the number of
 * launches since the last read, then resets.  Slot names come from
 * bo_profile_slot_name; bo_profile_slots gives their number. */
bo_status bo_profile_enable(int on);
bo_status bo_profile_read(double *ms, int64_t *launches, int nslots);
int bo_profile_slots(void);
const char *bo_profile_slot_name(int slot);

const char *bo_status_string(int status);
const char *bo_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* BANDOPS_H */
