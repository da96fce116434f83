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
//   (B1 adds the log term 1/[L_q]_jj to each Lqbar_jj as it writes it)
//   post: Lpbar = band(I(L_q) L_p) (the
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

// LDS staging.  A workgroup takes its chunk's rows in tiles of kRowBlock
// (one thread per row); the records a tile needs, with a halo of up to k
// records on either side, are copied into LDS as FP64 by consecutive threads
// reading consecutive elements (records of a problem are contiguous), and
// output records go back the same way.  Slots past the matrix end are never
// read by the row formulas, so pads in the inputs are harmless.
constexpr int kMaxW = 13;   // record length at the widest compiled k

// Records [r0, r1) of a band (clipped to [0, n)) into dst[(r - r0) * W + s].
// A tile spans at most kRowBlock + k records, so offsets inside it are 32-bit.
template <typename T>
__device__ __forceinline__ void stage_band(double *dst, const T *rec, const double *diag, int64_t r0, int64_t r1,
                                           int64_t n, int W) {
  const int64_t lo = r0 > 0 ? r0 : 0, hi = r1 < n ? r1 : n;
  if (hi <= lo) return;
  const int skip = (int)(lo - r0), rows = (int)(hi - lo), cnt = rows * W;
  const T *src = rec + lo * W;
  double *d = dst + skip * W;
  for (int e = threadIdx.x; e < cnt; e += kRowBlock)
    if (!(diag && e % W == 0)) d[e] = (double)src[e];
  if (diag)
    for (int r = threadIdx.x; r < rows; r += kRowBlock) d[r * W] = diag[lo + r];
}
// src[(r - r0) * W + s] into records [r0, r1) of a band (and its FP64 diagonal).
template <typename T>
__device__ __forceinline__ void store_band(T *rec, double *diag, const double *src, int64_t r0, int64_t r1, int W) {
  const int rows = (int)(r1 - r0), cnt = rows * W;
  T *dst = rec + r0 * W;
  for (int e = threadIdx.x; e < cnt; e += kRowBlock) dst[e] = (T)src[e];
  if (diag)
    for (int r = threadIdx.x; r < rows; r += kRowBlock) diag[r0 + r] = src[r * W];
}

// LDS of the row kernels for records of W elements (launch size, bytes).
__host__ __device__ constexpr int pre_lds_bytes(int W) {
  return (kRowBlock + (kRowBlock + W - 1) * W + kRowBlock * W + (kRowBlock + W - 1)) * 8;
}
__host__ __device__ constexpr int post_lds_bytes(int W) { return (2 * (kRowBlock + W - 1) * (W + 1)) * 8; }

template <typename T> __global__ void __launch_bounds__(kRowBlock) k_kl_pre(const bo::Args A, const KLP P) {
  extern __shared__ double dyn[];
  const ChunkRows C = chunk_of_block(A);
  const bo::ProbDesc &pd = *C.pd;
  const int K = pd.k, W = K + 1, TL = kRowBlock + K;
  double *sh = dyn;                    // block sums
  double *sLp = sh + kRowBlock;        // L_p records [t0 - k, t1)
  double *sQ = sLp + TL * W;           // Q_p / 2 records [t0, t1)
  double *sd = sQ + kRowBlock * W;     // d = m_p - m_q on [t0, t1 + k)
  const int64_t n = pd.n;
  const LB<T> Lq{(const T *)A.L + pd.boff, A.Ld ? A.Ld + pd.voff : nullptr, pd.ld};
  const T *Lp = (const T *)P.Lp + pd.boff;
  const double *Lpd = P.Lpd ? P.Lpd + pd.voff : nullptr;
  const T *mq = (const T *)P.mq + pd.voff, *mp = (const T *)P.mp + pd.voff;
  T *sb = (T *)P.Lpbar + pd.boff;
  double *sbd = P.Lpbard ? P.Lpbard + pd.voff : nullptr;
  T *v = (T *)P.mqbar + pd.voff;
  double lsum = 0.0, vsum = 0.0;
  for (int64_t t0 = C.a; t0 < C.b; t0 += kRowBlock) {
    const int64_t t1 = (t0 + kRowBlock < C.b) ? t0 + kRowBlock : C.b;
    __syncthreads();   // the previous tile's reads of LDS are done
    stage_band(sLp, Lp, Lpd, t0 - K, t1, n, W);
    for (int64_t r = t0 + threadIdx.x; r < t1 + K; r += kRowBlock)
      sd[r - t0] = r < n ? (double)mp[r] - (double)mq[r] : 0.0;
    __syncthreads();
    const int jl = threadIdx.x;   // rows and columns below are offsets from t0
    const int64_t j = t0 + jl;
    if (j < t1) {
      const int nl = (int)(n - t0 < 2 * kRowBlock ? n - t0 : 2 * kRowBlock);   // rows at or past nl are beyond n
      const int ml0 = -(int)(t0 < K ? t0 : K);                                // first column offset >= row 0
      // element (r, m) of L_p, m - t0 in [-k, t1 - t0)
      auto lp = [&](int r, int m) { return sLp[(m + K) * W + (r - m)]; };
      for (int s = 0; s < W; ++s) {
        const int il = jl + s;
        double q = 0.0;   // (L_p L_p^T)_ij over the columns both rows reach
        if (il < nl)
          for (int m = (il - K > ml0 ? il - K : ml0); m <= jl; ++m) q += lp(il, m) * lp(jl, m);
        sQ[jl * W + s] = 0.5 * q;
      }
      double vj = 0.0;
      for (int s = 0; s < W && jl + s < nl; ++s) vj += lp(jl + s, jl) * sd[jl + s];
      v[j] = (T)vj;
      vsum += vj * vj;
      lsum += log(Lq.at(j, j)) - log(lp(jl, jl));
    }
    __syncthreads();
    store_band(sb, sbd, sQ, t0, t1, W);
  }
  lsum = block_sum(lsum, sh);
  vsum = block_sum(vsum, sh);
  if (threadIdx.x == 0) {
    A.part[4 * (int64_t)C.c + 0] = lsum;
    A.part[4 * (int64_t)C.c + 1] = vsum;
  }
}

template <typename T> __global__ void __launch_bounds__(kRowBlock) k_kl_post(const bo::Args A, const KLP P) {
  extern __shared__ double dyn[];
  const ChunkRows C = chunk_of_block(A);
  const bo::ProbDesc &pd = *C.pd;
  const int K = pd.k, W = K + 1, TL = kRowBlock + K;
  double *sLp = dyn;                   // L_p records [t0 - k, t1)
  double *sS = sLp + TL * W;           // Sigma records [t0, t1 + k); reused for the Lpbar output
  double *sd = sS + TL * W;            // d on [t0, t1 + k)
  double *sv = sd + TL;                // v on [t0 - k, t1)
  const int64_t n = pd.n;
  const T *Lp = (const T *)P.Lp + pd.boff;
  const double *Lpd = P.Lpd ? P.Lpd + pd.voff : nullptr;
  const T *Sg = (const T *)A.S + pd.boff;
  const double *Sgd = A.Sd ? A.Sd + pd.voff : nullptr;
  const T *mq = (const T *)P.mq + pd.voff, *mp = (const T *)P.mp + pd.voff;
  const T *v = (const T *)P.mqbar + pd.voff;
  T *lpb = (T *)P.Lpbar + pd.boff;
  double *lpbd = P.Lpbard ? P.Lpbard + pd.voff : nullptr;
  T *mpb = (T *)P.mpbar + pd.voff;
  for (int64_t t0 = C.a; t0 < C.b; t0 += kRowBlock) {
    const int64_t t1 = (t0 + kRowBlock < C.b) ? t0 + kRowBlock : C.b;
    __syncthreads();
    stage_band(sLp, Lp, Lpd, t0 - K, t1, n, W);
    stage_band(sS, Sg, Sgd, t0, t1 + K, n, W);
    for (int64_t r = t0 + threadIdx.x; r < t1 + K; r += kRowBlock)
      sd[r - t0] = r < n ? (double)mp[r] - (double)mq[r] : 0.0;
    for (int64_t r = t0 - K + threadIdx.x; r < t1; r += kRowBlock) sv[r - (t0 - K)] = r >= 0 ? (double)v[r] : 0.0;
    __syncthreads();
    const int jl = threadIdx.x;   // rows and columns below are offsets from t0
    const int64_t j = t0 + jl;
    double g[kMaxW];
    if (j < t1) {
      const int nl = (int)(n - t0 < 2 * kRowBlock ? n - t0 : 2 * kRowBlock);   // rows at or past nl are beyond n
      const int ml0 = -(int)(t0 < K ? t0 : K);                                // first column offset >= row 0
      auto lp = [&](int r, int m) { return sLp[(m + K) * W + (r - m)]; };
      auto sg = [&](int r, int m) {   // symmetric: element (r, m) from the stored lower band
        return r >= m ? sS[m * W + (r - m)] : sS[r * W + (m - r)];
      };
      // L_p: trace, squared-norm and log terms
      const double vj = sv[jl + K];
      const int m1 = (jl + K < nl - 1) ? jl + K : nl - 1;
      for (int s = 0; s < W; ++s) {
        const int il = jl + s;
        double a = 0.0;
        if (il < nl) {
          for (int m = jl; m <= m1; ++m) a += sg(il, m) * lp(m, jl);
          a += sd[il] * vj;
          if (s == 0) a -= 1.0 / lp(jl, jl);
        }
        g[s] = a;
      }
      // means: L_p v
      double mb = 0.0;
      for (int m = (jl - K > ml0 ? jl - K : ml0); m <= jl; ++m) mb += lp(jl, m) * sv[m + K];
      mpb[j] = (T)mb;
    }
    __syncthreads();   // every read of sS is done: reuse it for the output records
    if (j < t1)
      for (int s = 0; s < W; ++s) sS[jl * W + s] = g[s];
    __syncthreads();
    store_band(lpb, lpbd, sS, t0, t1, W);
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
// Q_p / 2 and its trace, plus the log term of L_q), post, neg, finalize.  A carries the schedule, L =
// L_q, S = Sig, Sb = Lpbar (Q_p / 2), Lb = Lqbar; `launch(which, grid,
// range, k)` runs pre (0), post (1), neg (2) or finalize (3).
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
    if (int e = launch(0, r.c_cnt, A, r.K)) return e;
  }
  if (int e = bo::seq_pc(be, s, A, prec)) return e;
  bo::Args F2 = A;
  F2.lmap_out = A.lmap2;
  if (int e = bo::seq_lin(be, s, F2, prec, bo::PASS_F2, false)) return e;
  bo::Args B1 = A;
  B1.lmap = A.lmap2;
  B1.lmap_out = nullptr;
  B1.gl1 = 1.0;   // the log term of L_q, added as B1 writes Lqbar
  if (int e = bo::seq_lin(be, s, B1, prec, bo::PASS_B1, true)) return e;
  for (int which = 1; which <= 2; ++which)
    for (const bo::KRange &r : s.ranges) {
      bo::set_range(A, r);
      if (int e = launch(which, r.c_cnt, A, r.K)) return e;
    }
  A.p_beg = 0;
  return launch(3, s.nprob, A, 0);
}

}  // namespace bo_vi
