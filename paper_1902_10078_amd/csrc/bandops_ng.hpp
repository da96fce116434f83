// bandops_ng.hpp -- Gaussian-process regression with banded natural parameters
// (Appendix C.5, Algorithm 10) over a batch.  Prior N(F; eta_pr, Lam_pr),
// likelihood N(F; eta_lik, Lam_lik) in natural parameters, posterior
// Lam_po = Lam_pr + Lam_lik, eta_po = eta_pr + eta_lik, and
//
//   value = a(eta_pr, Lam_pr) - a(eta_po, Lam_po),
//   a(eta, Lam) = 1/2 log|Lam| - 1/2 eta^T Lam^{-1} eta = sum_i log C_ii - 1/2 ||C^{-1} eta||^2
//
// (C = C(Lam); log p(Y) is value plus the likelihood's own normaliser in data
// space, which holds no banded matrix).  With mu = Lam^{-1} eta and
// Sigma = I(C), d a / d Lam = 1/2 (Sigma + mu mu^T) and d a / d eta = -mu, so
// on the stored lower band (w = 1 on the diagonal, 2 off it):
//   Lam_pr bar  = w/2 (Sigma_pr + mu_pr mu_pr^T - Sigma_po - mu_po mu_po^T),
//   Lam_lik bar = -w/2 (Sigma_po + mu_po mu_po^T),
//   eta_pr bar  = mu_po - mu_pr,   eta_lik bar = mu_po.
// A call is the library's forward list twice, with row kernels around them:
//   1. on Lam_pr with right-hand side eta_pr: C_pr into the L arrays (later
//      overwritten), z_pr in the x array, mu_pr into etaprbar, Sigma_pr into
//      the Lprbar arrays;
//   pre:  Lam_po into the Sigma arrays, eta_po into x;
//   2. on Lam_po with right-hand side eta_po: C_po, z_po (kept in the first
//      entries of the Llikbar records' storage), Sigma_po, mu_po over eta_po in x;
//   post: both band gradients element by element (Sigma_pr read and replaced
//      by the same thread);
//   neg:  etaprbar = mu_po - mu_pr (after post: post reads mu_pr in a halo of
//      neighbouring rows);
//   finalize: the value and its parts from the forward lists'
//      log-determinants and squared norms, and the info code.
// Included by the host library after the backend definition.
#pragma once
#include "bandops_vi.hpp"

namespace bo_ng {

using bo_vi::ChunkRows;
using bo_vi::chunk_of_block;
using bo_vi::kRowBlock;

struct NGP {
  const void *Lpr;        // prior precision (lower band records)
  const double *Lprd;
  const void *etapr;
  const void *Llik;       // likelihood precision
  const double *Llikd;
  const void *etalik;
  void *Lpo;              // Lam_po, written by pre (the Sigma arrays)
  double *Lpod;
  void *x;                // eta_po after pre, mu_po after the second forward list
  const void *Sig;        // Sigma_po after the second forward list
  const double *Sigd;
  void *Lprbar;           // Sigma_pr until post replaces it
  double *Lprbard;
  void *Llikbar;
  double *Llikbard;
  void *etaprbar;         // mu_pr until neg replaces it
  double *parts;          // 5 per problem
  int32_t *info;          // the first forward list's info on entry to finalize
  const double *prior_parts, *post_parts;   // the forward lists' finalize parts (3 per problem)
  const int32_t *post_info;
};

template <typename T> __global__ void __launch_bounds__(kRowBlock) k_ng_pre(const bo::Args A, const NGP P) {
  const ChunkRows C = chunk_of_block(A);
  const bo::ProbDesc &pd = *C.pd;
  const int64_t ld = pd.ld;
  const T *pr = (const T *)P.Lpr + pd.boff, *lk = (const T *)P.Llik + pd.boff;
  const double *prd = P.Lprd ? P.Lprd + pd.voff : nullptr, *lkd = P.Llikd ? P.Llikd + pd.voff : nullptr;
  T *po = (T *)P.Lpo + pd.boff;
  double *pod = P.Lpod ? P.Lpod + pd.voff : nullptr;
  // element e = j * ld + s: (j, s) advance with e, so no element is divided by ld
  const int ldi = (int)ld, dj = kRowBlock / ldi, ds = kRowBlock % ldi;
  int64_t j = C.a + (int)threadIdx.x / ldi;
  int s = (int)threadIdx.x % ldi;
  for (int64_t e = C.a * ld + threadIdx.x; e < C.b * ld; e += kRowBlock) {
    if (s != 0 || !pod) {
      po[e] = (T)((double)pr[e] + (double)lk[e]);
    } else {
      const double d = prd[j] + lkd[j];
      po[e] = (T)d;
      pod[j] = d;
    }
    j += dj;
    s += ds;
    if (s >= ldi) { s -= ldi; ++j; }
  }
  const T *ep = (const T *)P.etapr + pd.voff, *el = (const T *)P.etalik + pd.voff;
  T *eo = (T *)P.x + pd.voff;
  for (int64_t j = C.a + threadIdx.x; j < C.b; j += kRowBlock) eo[j] = (T)((double)ep[j] + (double)el[j]);
}

template <typename T> __global__ void __launch_bounds__(kRowBlock) k_ng_post(const bo::Args A, const NGP P) {
  const ChunkRows C = chunk_of_block(A);
  const bo::ProbDesc &pd = *C.pd;
  const int K = pd.k;
  const int64_t ld = pd.ld, n = pd.n;
  const T *so = (const T *)P.Sig + pd.boff;
  const double *sod = P.Sigd ? P.Sigd + pd.voff : nullptr;
  const T *mo = (const T *)P.x + pd.voff, *mp = (const T *)P.etaprbar + pd.voff;
  T *gp = (T *)P.Lprbar + pd.boff, *gl = (T *)P.Llikbar + pd.boff;
  double *gpd = P.Lprbard ? P.Lprbard + pd.voff : nullptr, *gld = P.Llikbard ? P.Llikbard + pd.voff : nullptr;
  // element e = j * ld + s: (j, s) advance with e, so no element is divided by ld
  const int ldi = (int)ld, dj = kRowBlock / ldi, ds = kRowBlock % ldi;
  int64_t j = C.a + (int)threadIdx.x / ldi;
  int s = (int)threadIdx.x % ldi;
  for (int64_t e = C.a * ld + threadIdx.x; e < C.b * ld; e += kRowBlock, j += dj, s += ds) {
    if (s >= ldi) { s -= ldi; ++j; }
    const int64_t i = j + s;
    double g_pr = 0.0, g_lk = 0.0;
    if (s <= K && i < n) {
      const double spo = (s == 0 && sod) ? sod[j] : (double)so[e];
      const double spr = (s == 0 && gpd) ? gpd[j] : (double)gp[e];
      const double w = s == 0 ? 0.5 : 1.0;
      const double opo = spo + (double)mo[i] * (double)mo[j];
      g_pr = w * (spr + (double)mp[i] * (double)mp[j] - opo);
      g_lk = -w * opo;
    }
    gp[e] = (T)g_pr;
    gl[e] = (T)g_lk;
    if (s == 0 && gpd) gpd[j] = g_pr;
    if (s == 0 && gld) gld[j] = g_lk;
  }
}

template <typename T> __global__ void __launch_bounds__(kRowBlock) k_ng_neg(const bo::Args A, const NGP P) {
  const ChunkRows C = chunk_of_block(A);
  const bo::ProbDesc &pd = *C.pd;
  const T *mo = (const T *)P.x + pd.voff;
  T *g = (T *)P.etaprbar + pd.voff;
  for (int64_t j = C.a + threadIdx.x; j < C.b; j += kRowBlock) g[j] = (T)((double)mo[j] - (double)g[j]);
}

// One thread per problem.
__global__ void __launch_bounds__(64) k_ng_finalize(const bo::Args A, const NGP P, int32_t nprob) {
  const int32_t p = (int32_t)(blockIdx.x * 64 + threadIdx.x);
  if (p >= nprob) return;
  const bo::ProbDesc &pd = bo::prob_at(A, p);
  const int32_t o = pd.orig;
  const int32_t info0 = P.info[o], info1 = P.post_info[o];
  double *out = P.parts + 5 * (int64_t)o;
  if (info0 || info1) {
    for (int i = 0; i < 5; ++i) out[i] = NAN;
    P.info[o] = info0 ? info0 : (int32_t)(info1 + pd.n);
    return;
  }
  const double lpr = 0.5 * P.prior_parts[3 * (int64_t)o], qpr = P.prior_parts[3 * (int64_t)o + 1];
  const double lpo = 0.5 * P.post_parts[3 * (int64_t)o], qpo = P.post_parts[3 * (int64_t)o + 1];
  out[0] = lpr - 0.5 * qpr - lpo + 0.5 * qpo;
  out[1] = lpr;
  out[2] = lpo;
  out[3] = qpr;
  out[4] = qpo;
}

// The call's sequence.  `prior` and `post` are the two forward lists'
// arguments; `launch(which, count, args)` runs 0 = pre, 1 = post, 2 = neg (per
// chunk) and 3 = finalize (count = problems).
template <class BE, class Launch>
int pipe_natgp(BE &be, const bo::Sched &s, const bo::Args &prior, const bo::Args &post, int prec,
               Launch &&launch) {
  if (int e = bo::pipe_forward(be, s, prior, prec)) return e;
  bo::Args A = post;
  for (const bo::KRange &r : s.ranges) {
    bo::set_range(A, r);
    if (int e = launch(0, r.c_cnt, A)) return e;
  }
  if (int e = bo::pipe_forward(be, s, post, prec)) return e;
  for (int which = 1; which <= 2; ++which)
    for (const bo::KRange &r : s.ranges) {
      bo::set_range(A, r);
      if (int e = launch(which, r.c_cnt, A)) return e;
    }
  A.p_beg = 0;
  return launch(3, s.nprob, A);
}

}  // namespace bo_ng
