// bandops_ml.hpp -- log marginal likelihood of a conjugate GMRF with partial
// observations (Section 3.1, Eq. (marg_lik); Algorithm 8) over a batch:
//
//   log p(Y) = -(m/2) log 2 pi - log|L| + log|L_Q| - (m/2) log tau2
//              - Y^T Y / (2 tau2) + ||L^{-1} E^T Y||^2 / (2 tau2^2),
//
// L L^T = Q1 = Q + E^T E / tau2, L_Q L_Q^T = Q, m observed nodes.  E^T E is the
// diagonal observation mask and b = E^T Y puts the observed values at their
// nodes.  The reverse mode needs forward quantities only: with Sigma1 = I(L),
// x = Q1^{-1} b and Sigma0 = I(L_Q), on the stored lower band (w = 1 on the
// diagonal, 2 off it: a stored entry stands for two),
//   Qbar    = w (-Sigma1/2 - x x^T / (2 tau2^2) + Sigma0/2),
//   bbar_i  = x_i / tau2^2 - b_i / tau2 at the observed nodes (0 elsewhere),
//   tau2bar = -tau2^-2 sum_i mask_i Q1bar_ii - m / (2 tau2) + Y^T Y / (2 tau2^2)
//             - ||L^{-1} b||^2 / tau2^3,  Q1bar_ii = -Sigma1_ii/2 - x_i^2/(2 tau2^2)
// (tau2 enters log p through Q1 and through the explicit terms).  A call runs
// the library's forward list twice, each ending in the per-problem finalize:
//   1. on Q: L_Q into the L arrays, Sigma0 into the Qbar arrays;
//   2. on Q1 with the right-hand side b: L, z = L^{-1} b (kept in the bbar
//         arrays), Sigma1, x = L^{-T} z.  Q1 is never stored: the F1 pass reads
//         Q and adds mask_j / tau2 to each diagonal entry as it reads it;
//   post: Qbar (over Sigma0, element by element), bbar, and per chunk the sums
//         of mask_i Q1bar_ii, mask_i and b_i^2;
//   finalize: per problem, log p(Y), its parts and tau2bar from the two forward
//         lists' log-determinants, ||z||^2 and the chunk sums.
// One workgroup of kRowBlock threads per chunk for the row kernels.  Included by
// the host library after the backend definition.
#pragma once
#include "bandops_vi.hpp"

namespace bo_ml {

using bo_vi::ChunkRows;
using bo_vi::chunk_of_block;
using bo_vi::kRowBlock;

struct MLP {
  const void *Q;          // prior precision (lower band records)
  const double *Qd;
  const void *mask, *b;   // observation mask and E^T Y (vectors)
  const double *tau2;     // per problem
  const void *Sig1;       // I(L) after the second forward list
  const double *Sig1d;
  const void *x;          // Q1^{-1} b
  void *Qbar;             // holds I(L_Q) until post overwrites it
  double *Qbard;
  void *bbar;
  double *tau2bar, *parts;
  int32_t *info;          // the second forward list's info on entry to finalize
  const double *prior_parts, *post_parts;   // the forward lists' finalize parts (3 per problem)
  const int32_t *prior_info;
};

template <typename T> __global__ void __launch_bounds__(kRowBlock) k_ml_post(const bo::Args A, const MLP P) {
  __shared__ double sh[kRowBlock];
  const ChunkRows C = chunk_of_block(A);
  const bo::ProbDesc &pd = *C.pd;
  const int K = pd.k;
  const int64_t ld = pd.ld, n = pd.n;
  const T *s1 = (const T *)P.Sig1 + pd.boff;
  const double *s1d = P.Sig1d ? P.Sig1d + pd.voff : nullptr;
  const T *x = (const T *)P.x + pd.voff;
  const T *mask = (const T *)P.mask + pd.voff, *b = (const T *)P.b + pd.voff;
  T *qb = (T *)P.Qbar + pd.boff;   // I(L_Q) on entry
  double *qbd = P.Qbard ? P.Qbard + pd.voff : nullptr;
  T *bb = (T *)P.bbar + pd.voff;
  const double it2 = 1.0 / P.tau2[pd.orig], it4 = it2 * it2;
  // Qbar record entries: consecutive threads take consecutive entries; each
  // entry of I(L_Q) is read and replaced by the same thread
  // element e = j * ld + s: (j, s) advance with e, so no element is divided by ld
  const int ldi = (int)ld, dj = kRowBlock / ldi, ds = kRowBlock % ldi;
  int64_t j = C.a + (int)threadIdx.x / ldi;
  int s = (int)threadIdx.x % ldi;
  for (int64_t e = C.a * ld + threadIdx.x; e < C.b * ld; e += kRowBlock, j += dj, s += ds) {
    if (s >= ldi) { s -= ldi; ++j; }
    const int64_t i = j + s;
    double g = 0.0;
    if (s <= K && i < n) {
      const double sg1 = (s == 0 && s1d) ? s1d[j] : (double)s1[e];
      const double sg0 = (s == 0 && qbd) ? qbd[j] : (double)qb[e];
      g = (s == 0 ? 0.5 : 1.0) * (sg0 - sg1 - it4 * (double)x[i] * (double)x[j]);
    }
    qb[e] = (T)g;
    if (s == 0 && qbd) qbd[j] = g;
  }
  double p1 = 0.0, pm = 0.0, pyy = 0.0;
  for (int64_t j = C.a + threadIdx.x; j < C.b; j += kRowBlock) {
    const double mj = (double)mask[j], bj = (double)b[j], xj = (double)x[j];
    const double sg1 = s1d ? s1d[j] : (double)s1[j * ld];
    bb[j] = (T)(mj != 0.0 ? xj * it4 - bj * it2 : 0.0);
    p1 += mj * (-0.5 * sg1 - 0.5 * it4 * xj * xj);
    pm += mj;
    pyy += bj * bj;
  }
  p1 = bo_vi::block_sum(p1, sh);
  pm = bo_vi::block_sum(pm, sh);
  pyy = bo_vi::block_sum(pyy, sh);
  if (threadIdx.x == 0) {
    double *pt = A.part + 4 * (int64_t)C.c;
    pt[0] = p1;
    pt[1] = pm;
    pt[2] = pyy;
  }
}

// One workgroup of 64 threads per problem.
__global__ void __launch_bounds__(64) k_ml_finalize(const bo::Args A, const MLP P) {
  __shared__ double sh[3][64];
  const int32_t p = A.p_beg + (int32_t)blockIdx.x;
  const bo::ProbDesc &pd = bo::prob_at(A, p);
  double a = 0.0, m = 0.0, yy = 0.0;
  for (int32_t c = pd.chunk0 + (int32_t)threadIdx.x; c < pd.chunk0 + pd.nchunk; c += 64) {
    const double *pt = A.part + 4 * (int64_t)c;
    a += pt[0];
    m += pt[1];
    yy += pt[2];
  }
  sh[0][threadIdx.x] = a;
  sh[1][threadIdx.x] = m;
  sh[2][threadIdx.x] = yy;
  __syncthreads();
  if (threadIdx.x != 0) return;
  a = m = yy = 0.0;
  for (int i = 0; i < 64; ++i) {
    a += sh[0][i];
    m += sh[1][i];
    yy += sh[2][i];
  }
  const int32_t o = pd.orig;
  const double ld0 = P.prior_parts[3 * (int64_t)o + 0];
  const double ld1 = P.post_parts[3 * (int64_t)o + 0], rr = P.post_parts[3 * (int64_t)o + 1];
  const int32_t info1 = P.info[o], info0 = P.prior_info[o];
  const double t2 = P.tau2[o];
  double *out = P.parts + 4 * (int64_t)o;
  if (info1 || info0) {
    out[0] = out[1] = out[2] = out[3] = NAN;
    P.tau2bar[o] = NAN;
    P.info[o] = info1 ? info1 : (int32_t)(info0 + pd.n);
    return;
  }
  out[0] = -0.5 * m * log(2.0 * 3.14159265358979323846) - 0.5 * ld1 + 0.5 * ld0 - 0.5 * m * log(t2) -
           yy / (2.0 * t2) + rr / (2.0 * t2 * t2);
  out[1] = 0.5 * ld1;
  out[2] = 0.5 * ld0;
  out[3] = rr;
  P.tau2bar[o] = -a / (t2 * t2) - 0.5 * m / t2 + yy / (2.0 * t2 * t2) - rr / (t2 * t2 * t2);
}

// The call's sequence.  `prior` and `post` are the two forward lists' arguments
// (their parts / info pointing at the plan's per-problem scratch and at the
// caller's info; post carries the diagonal addend mask / tau2);
// `launch(which, count, args, K)` runs 1 = post, 2 = finalize.
template <class BE, class Launch>
int pipe_marglik(BE &be, const bo::Sched &s, const bo::Args &prior, const bo::Args &post, int prec,
                 Launch &&launch) {
  if (int e = bo::pipe_forward(be, s, prior, prec)) return e;
  if (int e = bo::pipe_forward(be, s, post, prec)) return e;
  bo::Args A = post;
  for (const bo::KRange &r : s.ranges) {
    bo::set_range(A, r);
    if (int e = launch(1, r.c_cnt, A, r.K)) return e;
  }
  A.p_beg = 0;
  return launch(2, s.nprob, A, 0);
}

}  // namespace bo_ml
