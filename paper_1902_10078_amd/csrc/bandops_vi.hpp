// bandops_vi.hpp -- the Kullback-Leibler term of the variational objective
// (Section 3.3, Eq. (KL); Algorithm 7) over a batch of banded problems.
//
//   KL = 1/2 (tr(I(L_q) P(L_p, L_p^T)) + 2 sum_i (log[L_q]_ii - log[L_p]_ii)
//             + ||P(L_p^T, m_p - m_q)||^2 - n)
//
// with L_q and L_p lower bands of the same width k.  The subset inverse and
// its reverse mode (Algorithms 3 and 4) are the chunked F2 and B1 passes of
// the library, run on L_q; around them, one workgroup per chunk with one
// thread per row:
//   pre:  Sigmabar = Q_p / 2 on the band of L_q (stored lower entries; the
//         B1 pass weighs a stored off-diagonal entry twice, as it stands for
//         two entries), v = L_p^T (m_p - m_q), and per chunk the sums of
//         log[L_q]_jj - log[L_p]_jj and of v_j^2;
//   post: Lqbar_jj += 1/[L_q]_jj (log term); Lpbar = band(I(L_q) L_p) (the
//         trace term: the symmetric band of I(L_q) suffices on the band of
//         L_p) + d v^T on the band (d = m_p - m_q) - 1/[L_p]_jj on the
//         diagonal; mpbar = L_p v;
//   neg:  mqbar = -mpbar;
//   finalize: per problem, KL and its parts from the chunk partials (the B1
//         pass leaves tr(I(L_q) Q_p / 2) in the third partial).
// Q_p / 2 is kept in the Lpbar arrays and v in mqbar until post overwrites
// them.  Included by the host library after the backend definition.
#pragma once
#include "bandops_driver.hpp"

namespace bo_vi {

constexpr int kRowBlock = 256;

// Element (i, j), 0 <= i - j <= k, of a lower band of one problem (mixed
// format: FP64 diagonal).
template <typename T> struct LB {
  const T *p;
  const double *d;
  int64_t ld;
  __device__ __forceinline__ double at(int64_t i, int64_t j) const {
    return (i == j && d) ? d[j] : (double)p[j * ld + (i - j)];
  }
};

// The KL term's own arrays (element type T of the band records and vectors).
struct KLP {
  const void *Lp;
  const double *Lpd;
  const void *mq, *mp;
  void *Lpbar;
  double *Lpbard;
  void *mqbar, *mpbar;
  double *parts;
};

__device__ __forceinline__ double block_sum(double v, double *sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int s = kRowBlock / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

struct ChunkRows {
  const bo::ProbDesc *pd;
  int32_t c;
  int64_t a, b;
};
__device__ __forceinline__ ChunkRows chunk_of_block(const bo::Args &A) {
  ChunkRows r;
  r.c = A.c_beg + (int32_t)blockIdx.x;
  r.pd = &bo::prob_at(A, bo::prob_of_chunk(A, r.c));
  bo::chunk_rows(*r.pd, r.c, r.a, r.b);
  return r;
}

template <typename T> __global__ void __launch_bounds__(kRowBlock) k_kl_pre(const bo::Args A, const KLP P) {
  __shared__ double sh[kRowBlock];
  const ChunkRows C = chunk_of_block(A);
  const bo::ProbDesc &pd = *C.pd;
  const int K = pd.k;
  const int64_t n = pd.n, ld = pd.ld;
  const LB<T> Lq{(const T *)A.L + pd.boff, A.Ld ? A.Ld + pd.voff : nullptr, ld};
  const LB<T> Lp{(const T *)P.Lp + pd.boff, P.Lpd ? P.Lpd + pd.voff : nullptr, ld};
  const T *mq = (const T *)P.mq + pd.voff, *mp = (const T *)P.mp + pd.voff;
  T *sb = (T *)P.Lpbar + pd.boff;
  double *sbd = P.Lpbard ? P.Lpbard + pd.voff : nullptr;
  T *v = (T *)P.mqbar + pd.voff;
  double lsum = 0.0, vsum = 0.0;
  for (int64_t j = C.a + threadIdx.x; j < C.b; j += kRowBlock) {
    for (int s = 0; s <= K; ++s) {
      const int64_t i = j + s;
      double q = 0.0;   // (L_p L_p^T)_ij over the columns m both rows reach
      if (i < n)
        for (int64_t m = (i - K > 0 ? i - K : 0); m <= j; ++m) q += Lp.at(i, m) * Lp.at(j, m);
      sb[j * ld + s] = (T)(0.5 * q);
      if (s == 0 && sbd) sbd[j] = 0.5 * q;
    }
    double vj = 0.0;
    for (int s = 0; s <= K && j + s < n; ++s) vj += Lp.at(j + s, j) * ((double)mp[j + s] - (double)mq[j + s]);
    v[j] = (T)vj;
    vsum += vj * vj;
    lsum += log(Lq.at(j, j)) - log(Lp.at(j, j));
  }
  lsum = block_sum(lsum, sh);
  vsum = block_sum(vsum, sh);
  if (threadIdx.x == 0) {
    A.part[4 * (int64_t)C.c + 0] = lsum;
    A.part[4 * (int64_t)C.c + 1] = vsum;
  }
}

template <typename T> __global__ void __launch_bounds__(kRowBlock) k_kl_post(const bo::Args A, const KLP P) {
  const ChunkRows C = chunk_of_block(A);
  const bo::ProbDesc &pd = *C.pd;
  const int K = pd.k;
  const int64_t n = pd.n, ld = pd.ld;
  const LB<T> Lq{(const T *)A.L + pd.boff, A.Ld ? A.Ld + pd.voff : nullptr, ld};
  const LB<T> Lp{(const T *)P.Lp + pd.boff, P.Lpd ? P.Lpd + pd.voff : nullptr, ld};
  const LB<T> Sg{(const T *)A.S + pd.boff, A.Sd ? A.Sd + pd.voff : nullptr, ld};
  const T *mq = (const T *)P.mq + pd.voff, *mp = (const T *)P.mp + pd.voff;
  const T *v = (const T *)P.mqbar + pd.voff;
  T *lqb = (T *)A.Lb + pd.boff;
  double *lqbd = A.Lbd ? A.Lbd + pd.voff : nullptr;
  T *lpb = (T *)P.Lpbar + pd.boff;
  double *lpbd = P.Lpbard ? P.Lpbard + pd.voff : nullptr;
  T *mpb = (T *)P.mpbar + pd.voff;
  for (int64_t j = C.a + threadIdx.x; j < C.b; j += kRowBlock) {
    // log-determinant term of L_q
    const double g0 = (lqbd ? lqbd[j] : (double)lqb[j * ld]) + 1.0 / Lq.at(j, j);
    lqb[j * ld] = (T)g0;
    if (lqbd) lqbd[j] = g0;
    // L_p: trace, squared-norm and log terms
    const double vj = (double)v[j];
    const int64_t m1 = (j + K < n - 1) ? j + K : n - 1;
    for (int s = 0; s <= K; ++s) {
      const int64_t i = j + s;
      double g = 0.0;
      if (i < n) {
        for (int64_t m = j; m <= m1; ++m) g += (i >= m ? Sg.at(i, m) : Sg.at(m, i)) * Lp.at(m, j);
        g += ((double)mp[i] - (double)mq[i]) * vj;
        if (s == 0) g -= 1.0 / Lp.at(j, j);
      }
      lpb[j * ld + s] = (T)g;
      if (s == 0 && lpbd) lpbd[j] = g;
    }
    // means: L_p v
    double mb = 0.0;
    for (int64_t m = (j - K > 0 ? j - K : 0); m <= j; ++m) mb += Lp.at(j, m) * (double)v[m];
    mpb[j] = (T)mb;
  }
}

template <typename T> __global__ void __launch_bounds__(kRowBlock) k_kl_neg(const bo::Args A, const KLP P) {
  const ChunkRows C = chunk_of_block(A);
  T *mqb = (T *)P.mqbar + C.pd->voff;
  const T *mpb = (const T *)P.mpbar + C.pd->voff;
  for (int64_t j = C.a + threadIdx.x; j < C.b; j += kRowBlock) mqb[j] = (T)(-(double)mpb[j]);
}

// Per problem: KL and its parts from the chunk partials (one workgroup of 64
// per problem; Neumaier-compensated sum of the log terms).
__global__ void __launch_bounds__(64) k_kl_finalize(const bo::Args A, double *parts) {
  __shared__ double sh_s[64], sh_c[64], sh_q[64], sh_t[64];
  const int32_t p = A.p_beg + (int32_t)blockIdx.x;
  const bo::ProbDesc &pd = bo::prob_at(A, p);
  double s = 0.0, comp = 0.0, q = 0.0, tr = 0.0;
  for (int32_t c = pd.chunk0 + (int32_t)threadIdx.x; c < pd.chunk0 + pd.nchunk; c += 64) {
    const double *pt = A.part + 4 * (int64_t)c;
    const double t = pt[0], u = s + t;
    comp += (fabs(s) >= fabs(t)) ? (s - u) + t : (t - u) + s;
    s = u;
    q += pt[1];
    tr += pt[2];
  }
  sh_s[threadIdx.x] = s;
  sh_c[threadIdx.x] = comp;
  sh_q[threadIdx.x] = q;
  sh_t[threadIdx.x] = tr;
  __syncthreads();
  if (threadIdx.x != 0) return;
  s = comp = q = tr = 0.0;
  for (int i = 0; i < 64; ++i) {
    const double t = sh_s[i], u = s + t;
    comp += (fabs(s) >= fabs(t)) ? (s - u) + t : (t - u) + s;
    s = u;
    comp += sh_c[i];
    q += sh_q[i];
    tr += sh_t[i];
  }
  const double ldiff = s + comp, trace = 2.0 * tr;
  double *o = parts + 4 * (int64_t)pd.orig;
  o[0] = 0.5 * (trace + 2.0 * ldiff + q - (double)pd.n);
  o[1] = trace;
  o[2] = ldiff;
  o[3] = q;
}

// The whole term: clear, pre, chunk products of L_q, F2 (I(L_q), with the B1
// chunk maps fused in for k <= KMAX_FUSED), B1 (Algorithm 4 with Sigmabar =
// Q_p / 2 and its trace), post, neg, finalize.  A carries the schedule, L =
// L_q, S = Sig, Sb = Lpbar (Q_p / 2), Lb = Lqbar; `launch(which, grid,
// range)` runs pre (0), post (1), neg (2) or finalize (3).
template <class BE, class Launch>
int pipe_vi_kl(BE &be, const bo::Sched &s, bo::Args A, int prec, Launch &&launch) {
  A.sb_is_S = 1;
  A.accumulate = 0;
  A.bx = nullptr;
  A.x = nullptr;
  A.yb = nullptr;
  A.zf = nullptr;
  if (int e = bo::seq_clear(be, s, A)) return e;
  for (const bo::KRange &r : s.ranges) {
    bo::set_range(A, r);
    if (int e = launch(0, r.c_cnt, A)) return e;
  }
  if (int e = bo::seq_pc(be, s, A, prec)) return e;
  bo::Args F2 = A;
  F2.lmap_out = A.lmap2;
  if (int e = bo::seq_lin(be, s, F2, prec, bo::PASS_F2, false)) return e;
  bo::Args B1 = A;
  B1.lmap = A.lmap2;
  B1.lmap_out = nullptr;
  if (int e = bo::seq_lin(be, s, B1, prec, bo::PASS_B1, true)) return e;
  for (int which = 1; which <= 2; ++which)
    for (const bo::KRange &r : s.ranges) {
      bo::set_range(A, r);
      if (int e = launch(which, r.c_cnt, A)) return e;
    }
  A.p_beg = 0;
  return launch(3, s.nprob, A);
}

}  // namespace bo_vi
