// bandops_wide.hip -- the wide block-banded case: lower bandwidth k = 64,
// handled as a block-tridiagonal matrix of 64 x 64 blocks.
//
// Record j = 64b + c of a band (65 slots) holds, for slots d <= 63 - c, the
// diagonal block Q_bb[c+d, c], and for slots d >= 64 - c the coupling block
// C_b = Q[b+1, b] at [d - 64 + c, c]; C_b is upper triangular because the band
// ends 64 rows below the diagonal.  The banded operators then become block
// recurrences on dense 64 x 64 tiles (the complexity argument of Section 4.1
// with the band in blocks):
//
//   Cholesky (Algorithm 1 by blocks), ascending:
//     S_0 = Q_00,  L_bb = chol(S_b),  X_b = L_bb^{-1},  M_b = C_b X_b^T,
//     S_{b+1} = Q_{b+1,b+1} - M_b M_b^T;           M_b is L's block (b+1, b)
//   subset inverse (Algorithm 3 by blocks), descending, P_b = M_b X_b:
//     Sigma_{b+1,b} = -Sigma_{b+1,b+1} P_b,
//     Sigma_bb = X_b^T X_b + P_b^T Sigma_{b+1,b+1} P_b
//   their reverse modes (Algorithm 4 and Algorithm 2 by blocks) are the
//   adjoints of these block steps, run in the opposite directions.
//
// Precision: blocks are stored in the mixed format (FP32 records, FP64
// diagonal).  The diagonal-block Cholesky and triangular inverse run in FP64
// (FP64 pivots and log-determinant); every dense block product runs on the
// matrix cores as FP32 MFMA (v_mfma_f32_16x16x4_f32).
//
// Parallelism: one workgroup (four wavefronts) per problem walks its blocks in
// order; each block step is a handful of 64 x 64 MFMA products plus the FP64
// factorisation of one diagonal block.  The factor's inverse X_b and P_b are
// kept in the workspace between passes.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <functional>
#include <string>
#include <vector>

#include "bandops.h"

namespace wide {

constexpr int NB = 64;         // block size = bandwidth
constexpr int W = NB + 1;      // record width
constexpr int NT = 256;        // threads per workgroup
constexpr int LDF = 65;        // LDS row stride (floats)
constexpr int LDD = 65;        // LDS row stride (doubles)
constexpr int64_t kBlockWs = 2 * NB * NB;   // floats of workspace per block (X, P)

typedef float MatF[NB][LDF];
typedef double MatD[NB][LDD];
typedef float float4_ __attribute__((ext_vector_type(4)));

struct Prob {
  int64_t n, boff, voff, wsoff;   // wsoff: first block of this problem in the workspace
};

struct Args {
  const Prob *probs;
  const float *Q; const double *Qd;     // precision (input)
  const float *Wm; const double *Wmd;   // W of tr(Q^{-1} W) (loss only)
  float *L; double *Ld;
  float *Sig; double *Sigd;
  float *Lb; double *Lbd;
  float *Qb; double *Qbd;
  float *ws;                            // X_b, P_b per block
  double *parts;                        // per problem: logdet, 0, trace
  int32_t *info;
};

__device__ __forceinline__ int64_t nblocks(int64_t n) { return (n + NB - 1) / NB; }

// ----------------------------------------------------------- block I/O
constexpr int kSlotIters = (NB * W + NT - 1) / NT;   // slots of a block per thread

// Visit the 64 records of block b (all 65 slots): f(it, c, d, j, valid) with
// j = 64 b + c; valid when the slot lies inside the matrix.
template <class F> __device__ __forceinline__ void for_block_slots(int64_t b, int64_t n, F &&f) {
#pragma unroll
  for (int it = 0; it < kSlotIters; ++it) {
    const int idx = threadIdx.x + it * NT;
    if (idx < NB * W) {
      const int c = idx / W, d = idx - c * W;
      const int64_t j = NB * b + c;
      f(it, c, d, j, j < n && j + d < n);
    }
  }
}

// Every slot of block b of band Bp/Bd into registers (all loads issued before
// any is used); slots past the matrix end read 1 on the diagonal, else 0.
__device__ __forceinline__ void read_block(const float *Bp, const double *Bd, const Prob &p, int64_t b,
                                           double (&v)[kSlotIters]) {
#pragma unroll
  for (int it = 0; it < kSlotIters; ++it) v[it] = 0.0;
  for_block_slots(b, p.n, [&](int it, int c, int d, int64_t j, bool valid) {
    if (valid) v[it] = d == 0 ? Bd[p.voff + j] : (double)Bp[(p.boff + j * W) + d];
    else if (d == 0) v[it] = 1.0;   // identity past the matrix end
  });
}

// Diagonal block (symmetric, full; E = double or float) and coupling block
// (upper triangular, FP32) of band Bp/Bd at block b; rows past n read as the
// identity on the diagonal and zero elsewhere.
template <typename E>
__device__ void load_blocks(const float *Bp, const double *Bd, const Prob &p, int64_t b, E (&S)[NB][LDF],
                            MatF *Cf) {
  double v[kSlotIters];
  read_block(Bp, Bd, p, b, v);
  if (Cf)
    for (int e = threadIdx.x; e < NB * NB; e += NT) (*Cf)[e / NB][e % NB] = 0.f;
  __syncthreads();
  for_block_slots(b, p.n, [&](int it, int c, int d, int64_t, bool) {
    if (d <= NB - 1 - c) {
      S[c + d][c] = (E)v[it];
      S[c][c + d] = (E)v[it];
    } else if (Cf) {
      (*Cf)[d - NB + c][c] = (float)v[it];
    }
  });
  __syncthreads();
}

// The coupling block alone (upper triangular, zero below).
__device__ void load_coupling(const float *Bp, const double *Bd, const Prob &p, int64_t b, MatF &Cf) {
  double v[kSlotIters];
  read_block(Bp, Bd, p, b, v);
  for (int e = threadIdx.x; e < NB * NB; e += NT) Cf[e / NB][e % NB] = 0.f;
  __syncthreads();
  for_block_slots(b, p.n, [&](int it, int c, int d, int64_t, bool) {
    if (d > NB - 1 - c) Cf[d - NB + c][c] = (float)v[it];
  });
  __syncthreads();
}

// Store a block pair into band Bp/Bd: the lower triangle of Dg (diagonal
// values from dg when given, else Dg's own) and the upper triangle of Cf
// (when given; the coupling slots are written 0 when it is not).
template <class DiagF, class LowF, class CoupF>
__device__ void store_blocks(float *Bp, double *Bd, const Prob &p, int64_t b, DiagF &&diag, LowF &&low,
                             CoupF &&coup) {
  for_block_slots(b, p.n, [&](int, int c, int d, int64_t j, bool valid) {
    if (j >= p.n) return;
    double v = 0.0;
    if (valid) v = d == 0 ? diag(c) : (d <= NB - 1 - c ? low(c + d, c) : coup(d - NB + c, c));
    Bp[p.boff + j * W + d] = (float)v;
    if (d == 0) Bd[p.voff + j] = v;
  });
}

// --------------------------------------------------------- dense blocks
// Out(i, j, v) receives alpha * op(A) op(B) for every element (i, j) of the
// 64 x 64 product (op = transpose when TA / TB).  Four wavefronts; wavefront w
// owns output columns [16w, 16w + 16) as four 16 x 16 MFMA tiles.  A 16x16x4
// FP32 MFMA takes lane l's A value at row l % 16, column l / 16 of the 16 x 4
// slice, its B value at row l / 16, column l % 16 of the 4 x 16 slice, and
// returns rows 4 (l / 16) + r, column l % 16 of the 16 x 16 tile in
// component r.
template <bool TA, bool TB, class Out>
__device__ __forceinline__ void gemm64(const MatF &A, const MatF &B, float alpha, Out &&out) {
  __syncthreads();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int jl = 16 * w + (l & 15), kq = l >> 4;
  float4_ acc[4];
#pragma unroll
  for (int t = 0; t < 4; ++t) acc[t] = float4_{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < NB / 4; ++s) {
    const int k = 4 * s + kq;
    const float bv = TB ? B[jl][k] : B[k][jl];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int il = 16 * t + (l & 15);
      const float av = TA ? A[k][il] : A[il][k];
      acc[t] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[t], 0, 0, 0);
    }
  }
  __syncthreads();   // every read of A and B is done before any output is written
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) out(16 * t + 4 * kq + r, jl, alpha * acc[t][r]);
  __syncthreads();
}


// FP64 Cholesky of the symmetric block S in place: the strict lower triangle
// of S becomes L's, the diagonal goes to dg and its reciprocal to rdg (S's
// diagonal is left as is).  Returns 0, or 1 + the first column whose pivot is
// not positive.  Thread 0 adds the log-determinant of L to lsum.
__device__ int potrf64(MatD &S, double *dg, double *rdg, double &lsum) {
  const int tid = threadIdx.x;
  for (int j = 0; j < NB; ++j) {
    const double piv = S[j][j];
    if (!(piv > 0.0)) return j + 1;
    const double d = sqrt(piv), r = 1.0 / d;
    if (tid == 0) { dg[j] = d; rdg[j] = r; }
    if (tid > j && tid < NB) S[tid][j] *= r;
    __syncthreads();
    const int c = tid & 63, q = tid >> 6;
    const int k = j + 1 + c;
    if (k < NB) {
      const double lk = S[k][j];
      for (int i = k + q; i < NB; i += 4) S[i][k] -= S[i][j] * lk;
    }
    __syncthreads();
  }
  if (tid < NB) {
    double lg = log(dg[tid]);
    for (int off = 32; off >= 1; off >>= 1) lg += __shfl_xor(lg, off, 64);
    if (tid == 0) lsum += lg;
  }
  __syncthreads();
  return 0;
}

// X = L^{-1} for L = (strict lower triangle of S, reciprocal diagonal rdg),
// in FP64.  Four lanes per column j: lane q sums the terms k = j + q (mod 4)
// and keeps (writes, then reads back) exactly those entries of column j.
__device__ void trtri64(const MatD &S, const double *rdg, MatD &X) {
  const int tid = threadIdx.x, j = tid >> 2, q = tid & 3;
  for (int i = q; i < j; i += 4) X[i][j] = 0.0;
  for (int i = j; i < NB; ++i) {
    double s = 0.0;
    for (int k = j + q; k < i; k += 4) s += S[i][k] * X[k][j];
    s += __shfl_xor(s, 1, 64);
    s += __shfl_xor(s, 2, 64);
    const double x = ((i == j ? 1.0 : 0.0) - s) * rdg[i];
    if (((i - j) & 3) == q) X[i][j] = x;
  }
  __syncthreads();
}

__device__ __forceinline__ void ws_load(const float *src, MatF &M) {
  float4 v[NB * NB / (4 * NT)];
#pragma unroll
  for (int it = 0; it < NB * NB / (4 * NT); ++it) v[it] = reinterpret_cast<const float4 *>(src)[threadIdx.x + it * NT];
#pragma unroll
  for (int it = 0; it < NB * NB / (4 * NT); ++it) {
    const int e = 4 * (threadIdx.x + it * NT), r = e / NB, c = e % NB;
    M[r][c] = v[it].x;
    M[r][c + 1] = v[it].y;
    M[r][c + 2] = v[it].z;
    M[r][c + 3] = v[it].w;
  }
  __syncthreads();
}
__device__ __forceinline__ void ws_store(float *dst, const MatF &M) {
  __syncthreads();
  for (int e = threadIdx.x; e < NB * NB; e += NT) dst[e] = M[e / NB][e % NB];
}

__device__ double block_sum(double v, double *red) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// ============================================================= F1 (forward)
// Cholesky by blocks: L, log det, X_b and P_b = M_b X_b for the later passes.
__global__ void __launch_bounds__(NT) k_wide_f1(const Args A) {
  __shared__ MatD S, X;
  __shared__ MatF Cf, Mf, Xf;
  __shared__ double dg[NB], rdg[NB];
  __shared__ int fail_s;
  const Prob p = A.probs[blockIdx.x];
  const int64_t nb = nblocks(p.n);
  double lsum = 0.0;
  int fail = 0;
  for (int64_t b = 0; b < nb && !fail; ++b) {
    load_blocks(A.Q, A.Qd, p, b, S, &Cf);
    if (b > 0)   // S_b = Q_bb - M_{b-1} M_{b-1}^T
      gemm64<false, true>(Mf, Mf, 1.f, [&](int i, int j, float v) { S[i][j] -= (double)v; });
    const int r = potrf64(S, dg, rdg, lsum);
    if (r) {
      fail = (int)(NB * b + r);
      break;
    }
    trtri64(S, rdg, X);
    for (int e = threadIdx.x; e < NB * NB; e += NT) Xf[e / NB][e % NB] = (float)X[e / NB][e % NB];
    // M_b = C_b X_b^T (upper triangular)
    gemm64<false, true>(Cf, Xf, 1.f, [&](int i, int j, float v) { Mf[i][j] = v; });
    store_blocks(A.L, A.Ld, p, b, [&](int c) { return dg[c]; }, [&](int i, int c) { return S[i][c]; },
                 [&](int rr, int c) { return (double)Mf[rr][c]; });
    float *wsb = A.ws + (p.wsoff + b) * kBlockWs;
    ws_store(wsb, Xf);
    // P_b = M_b X_b (into Cf, which is free now)
    gemm64<false, false>(Mf, Xf, 1.f, [&](int i, int j, float v) { Cf[i][j] = v; });
    ws_store(wsb + NB * NB, Cf);
  }
  if (threadIdx.x == 0) fail_s = fail;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int64_t o = blockIdx.x;
    if (A.parts) {
      A.parts[3 * o + 0] = fail_s ? NAN : 2.0 * lsum;
      A.parts[3 * o + 1] = fail_s ? NAN : 0.0;
      A.parts[3 * o + 2] = NAN;   // the trace, written by the F2 pass when it runs
    }
    A.info[o] = fail_s;
  }
}

// ========================================================== F2 (forward)
// Subset inverse by blocks, descending; with Wm given, also tr(Q^{-1} W).
__global__ void __launch_bounds__(NT) k_wide_f2(const Args A) {
  __shared__ MatF Xf, Pf, Wf, Ef, Tf;
  __shared__ double red[4];
  const Prob p = A.probs[blockIdx.x];
  if (A.info[blockIdx.x] != 0) {   // a failed factorisation: every part is NaN
    if (threadIdx.x == 0 && A.parts) A.parts[3 * blockIdx.x + 2] = NAN;
    return;
  }
  const int64_t nb = nblocks(p.n);
  double tr = 0.0;
  for (int64_t b = nb - 1; b >= 0; --b) {
    const float *wsb = A.ws + (p.wsoff + b) * kBlockWs;
    ws_load(wsb, Xf);
    ws_load(wsb + NB * NB, Pf);
    const bool last = b == nb - 1;
    if (!last)   // E = Sigma_{b+1,b} = -W P
      gemm64<false, false>(Wf, Pf, -1.f, [&](int i, int j, float v) { Ef[i][j] = v; });
    // Sigma_bb = X^T X - P^T E
    gemm64<true, false>(Xf, Xf, 1.f, [&](int i, int j, float v) { Tf[i][j] = v; });
    if (!last) gemm64<true, false>(Pf, Ef, -1.f, [&](int i, int j, float v) { Tf[i][j] += v; });
    // FP64 diagonal: sum_k X_ki^2 - sum_k P_ki E_ki
    __shared__ double sdg[NB];
    if (threadIdx.x < NB) {
      const int i = threadIdx.x;
      double s = 0.0;
      for (int k = 0; k < NB; ++k) s += (double)Xf[k][i] * (double)Xf[k][i];
      if (!last)
        for (int k = 0; k < NB; ++k) s -= (double)Pf[k][i] * (double)Ef[k][i];
      sdg[i] = s;
    }
    __syncthreads();
    store_blocks(A.Sig, A.Sigd, p, b, [&](int c) { return sdg[c]; },
                 [&](int i, int c) { return (double)Tf[i][c]; },
                 [&](int rr, int c) { return last ? 0.0 : (double)Ef[rr][c]; });
    if (A.Wm) {   // tr(Sigma W) over the stored entries (off-diagonal ones twice)
      double wv[kSlotIters];
      read_block(A.Wm, A.Wmd, p, b, wv);
      for_block_slots(b, p.n, [&](int it, int c, int d, int64_t, bool valid) {
        if (!valid) return;
        const double sv = d == 0 ? sdg[c] : (d <= NB - 1 - c ? (double)Tf[c + d][c] : (double)Ef[d - NB + c][c]);
        tr += (d == 0 ? 1.0 : 2.0) * wv[it] * sv;
      });
    }
    __syncthreads();
    // carry Sigma_bb (full, symmetric) to the block above
    for (int e = threadIdx.x; e < NB * NB; e += NT) {
      const int i = e / NB, j = e % NB;
      Wf[i][j] = i == j ? (float)sdg[i] : (i > j ? Tf[i][j] : Tf[j][i]);
    }
    __syncthreads();
  }
  const double t = block_sum(tr, red);
  if (threadIdx.x == 0 && A.parts) A.parts[3 * blockIdx.x + 2] = t;
}

// =================================================== B1 (Algorithm 4, blocks)
// Ascending reverse of F2 with Sigmabar from W (S_ii on the diagonal, 2 S_ij
// off it, on the stored entries): writes Lbar (diagonal-block lower triangle
// and coupling-block upper triangle).  Carried: the adjoint of Sigma_bb.
__global__ void __launch_bounds__(NT) k_wide_b1(const Args A) {
  __shared__ MatF Xf, Pf, Wf, EMf, Sf, Cf, A1, A2;
  const Prob p = A.probs[blockIdx.x];
  if (A.info[blockIdx.x] != 0) return;
  const int64_t nb = nblocks(p.n);
  for (int e = threadIdx.x; e < NB * NB; e += NT) Cf[e / NB][e % NB] = 0.f;
  for (int64_t b = 0; b < nb; ++b) {
    const float *wsb = A.ws + (p.wsoff + b) * kBlockWs;
    ws_load(wsb, Xf);
    ws_load(wsb + NB * NB, Pf);
    const bool last = b == nb - 1;
    // Sbar = sym(user's adjoint of Sigma_bb) + sym(carry) = W_bb + sym(C);
    // Ebar = user's adjoint of Sigma_{b+1,b} = 2 W_{b+1,b} (upper triangle)
    load_blocks(A.Wm, A.Wmd, p, b, Sf, &EMf);
    for (int e = threadIdx.x; e < NB * NB; e += NT) {
      const int i = e / NB, j = e % NB;
      const bool pad = NB * b + i >= p.n || NB * b + j >= p.n;
      Sf[i][j] = pad ? 0.f : Sf[i][j] + 0.5f * (Cf[i][j] + Cf[j][i]);
      EMf[i][j] *= 2.f;
    }
    __syncthreads();
    if (!last) {
      // W = Sigma_{b+1,b+1} from the Sigma band
      load_blocks(A.Sig, A.Sigd, p, b + 1, Wf, nullptr);
      // Pbar = 2 W P Sbar - W Ebar   (A2)
      gemm64<false, false>(Wf, Pf, 1.f, [&](int i, int j, float v) { A1[i][j] = v; });
      gemm64<false, false>(A1, Sf, 2.f, [&](int i, int j, float v) { A2[i][j] = v; });
      gemm64<false, false>(Wf, EMf, -1.f, [&](int i, int j, float v) { A2[i][j] += v; });
      // carry to block b+1: P Sbar P^T - Ebar P^T   (Cf)
      gemm64<false, false>(Pf, Sf, 1.f, [&](int i, int j, float v) { A1[i][j] = v; });
      gemm64<false, true>(A1, Pf, 1.f, [&](int i, int j, float v) { Cf[i][j] = v; });
      gemm64<false, true>(EMf, Pf, -1.f, [&](int i, int j, float v) { Cf[i][j] += v; });
      // Mbar = Pbar X^T: Lbar's coupling block (upper triangle kept), in A1
      gemm64<false, true>(A2, Xf, 1.f, [&](int i, int j, float v) { A1[i][j] = v; });
      // M_b from L's coupling slots (into EMf, free now)
      load_coupling(A.L, A.Ld, p, b, EMf);
      // Xbar = 2 X Sbar + M^T Pbar   (Wf)
      gemm64<false, false>(Xf, Sf, 2.f, [&](int i, int j, float v) { Wf[i][j] = v; });
      gemm64<true, false>(EMf, A2, 1.f, [&](int i, int j, float v) { Wf[i][j] += v; });
    } else {
      gemm64<false, false>(Xf, Sf, 2.f, [&](int i, int j, float v) { Wf[i][j] = v; });
    }
    // Lbar_bb = -X^T Xbar X^T (lower triangle kept)
    gemm64<true, false>(Xf, Wf, 1.f, [&](int i, int j, float v) { Sf[i][j] = v; });
    gemm64<false, true>(Sf, Xf, -1.f, [&](int i, int j, float v) { A2[i][j] = v; });
    store_blocks(A.Lb, A.Lbd, p, b, [&](int c) { return (double)A2[c][c]; },
                 [&](int i, int c) { return (double)A2[i][c]; },
                 [&](int rr, int c) { return last ? 0.0 : (double)A1[rr][c]; });
    __syncthreads();
  }
}

// =================================================== B2 (Algorithm 2, blocks)
// Descending reverse of F1: Qbar from L, Lbar and the log-determinant
// sensitivity gl (per unit loss weight).  Carried: the adjoint of S_{b+1}.
__global__ void __launch_bounds__(NT) k_wide_b2(const Args A, double gl) {
  __shared__ MatF Lf, Xf, Mf, MBf, LBf, Sc, A1, A2;
  __shared__ double dg[NB], lbd[NB];
  const Prob p = A.probs[blockIdx.x];
  if (A.info[blockIdx.x] != 0) return;
  const int64_t nb = nblocks(p.n);
  for (int e = threadIdx.x; e < NB * NB; e += NT) Sc[e / NB][e % NB] = 0.f;
  __syncthreads();
  for (int64_t b = nb - 1; b >= 0; --b) {
    const bool last = b == nb - 1;
    ws_load(A.ws + (p.wsoff + b) * kBlockWs, Xf);
    // L_bb (lower) and M_b (upper) from L, the FP64 pivots from Ld
    load_blocks(A.L, A.Ld, p, b, Lf, &Mf);
    for (int e = threadIdx.x; e < NB * NB; e += NT) {
      const int i = e / NB, j = e % NB;
      if (i < j) Lf[i][j] = 0.f;
    }
    if (threadIdx.x < NB) {
      const int64_t j = NB * b + threadIdx.x;
      dg[threadIdx.x] = j < p.n ? A.Ld[p.voff + j] : 1.0;
    }
    __syncthreads();
    // Lbar_bb (lower, with the log-determinant term) and Mbar_b (upper)
    if (threadIdx.x < NB) {
      const int64_t j = NB * b + threadIdx.x;
      lbd[threadIdx.x] = j < p.n ? A.Lbd[p.voff + j] + 2.0 * gl / dg[threadIdx.x] : 0.0;
    }
    load_blocks(A.Lb, A.Lbd, p, b, LBf, &MBf);
    for (int e = threadIdx.x; e < NB * NB; e += NT) {
      const int i = e / NB, j = e % NB;
      const bool pad = NB * b + i >= p.n;
      LBf[i][j] = i == j ? (float)lbd[i] : (i > j && !pad ? LBf[i][j] : 0.f);
    }
    __syncthreads();
    if (!last) {
      // Mbar -= 2 Sc M   (Sc: adjoint of S_{b+1}, symmetric)
      gemm64<false, false>(Sc, Mf, -2.f, [&](int i, int j, float v) { MBf[i][j] += v; });
      // Cbar = Mbar X (upper triangle kept) -> Qbar's coupling block (A2)
      gemm64<false, false>(MBf, Xf, 1.f, [&](int i, int j, float v) { A2[i][j] = v; });
      // Lbar_bb -= X^T (Mbar^T M)
      gemm64<true, false>(MBf, Mf, 1.f, [&](int i, int j, float v) { A1[i][j] = v; });
      gemm64<true, false>(Xf, A1, -1.f, [&](int i, int j, float v) { LBf[i][j] += v; });
    }
    // Phi(L^T Lbar) with Lbar's lower triangle: lower part, halved diagonal
    for (int e = threadIdx.x; e < NB * NB; e += NT) {
      const int i = e / NB, j = e % NB;
      if (i < j) LBf[i][j] = 0.f;
    }
    gemm64<true, false>(Lf, LBf, 1.f, [&](int i, int j, float v) { A1[i][j] = v; });
    for (int e = threadIdx.x; e < NB * NB; e += NT) {
      const int i = e / NB, j = e % NB;
      // Phi + Phi^T: off-diagonal A1[max][min], diagonal A1[i][i]
      Mf[i][j] = i == j ? A1[i][i] : (i > j ? A1[i][j] : A1[j][i]);
    }
    // Sbar = 1/2 X^T (Phi + Phi^T) X   (new carry)
    gemm64<true, false>(Xf, Mf, 1.f, [&](int i, int j, float v) { A1[i][j] = v; });
    gemm64<false, false>(A1, Xf, 0.5f, [&](int i, int j, float v) { Sc[i][j] = v; });
    // Qbar: diagonal block from Sbar (stored entries: S_ii, 2 S_ij), coupling from Cbar
    store_blocks(A.Qb, A.Qbd, p, b, [&](int c) { return (double)Sc[c][c]; },
                 [&](int i, int c) { return (double)(Sc[i][c] + Sc[c][i]); },
                 [&](int rr, int c) { return last ? 0.0 : (double)A2[rr][c]; });
    __syncthreads();
  }
}

}  // namespace wide

// ====================================================================== C ABI
// The library's thread-local error message (defined with the other entry points).
bo_status bo_set_error(bo_status s, const std::string &msg);
// Launch timing hook of the library (slot per wide pass, which = 0..3).
int bo_profile_wide(int which, hipStream_t s, const std::function<int()> &launch);

namespace {
bo_status wfail(bo_status s, const std::string &m) { return bo_set_error(s, m); }
size_t table_bytes(int32_t nprob) { return ((size_t)nprob * sizeof(wide::Prob) + 255) / 256 * 256; }
}  // namespace

static bo_status wide_table(const bo_problem *probs, int32_t nprob, std::vector<wide::Prob> &t,
                            size_t &bytes) {
  if (!probs || nprob <= 0) return wfail(BO_EINVAL, "bo_wide: no problems");
  t.resize(nprob);
  int64_t blocks = 0;
  for (int32_t i = 0; i < nprob; ++i) {
    if (probs[i].k != wide::NB) return wfail(BO_EUNSUPPORTED, "bo_wide: every problem must have k = 64");
    if (probs[i].n < 0 || probs[i].boff < 0 || probs[i].voff < 0) return wfail(BO_EINVAL, "bo_wide: bad problem");
    t[i] = wide::Prob{probs[i].n, probs[i].boff, probs[i].voff, blocks};
    blocks += (probs[i].n + wide::NB - 1) / wide::NB;
  }
  bytes = table_bytes(nprob) + (size_t)blocks * wide::kBlockWs * sizeof(float);
  return BO_OK;
}

extern "C" bo_status bo_wide_workspace_size(const bo_problem *probs, int32_t nprob, size_t *bytes) {
  std::vector<wide::Prob> t;
  if (!bytes) return wfail(BO_EINVAL, "bo_wide_workspace_size: null bytes");
  return wide_table(probs, nprob, t, *bytes);
}

extern "C" bo_status bo_wide_upload(const bo_problem *probs, int32_t nprob, void *ws, size_t ws_bytes) {
  std::vector<wide::Prob> t;
  size_t need = 0;
  if (bo_status e = wide_table(probs, nprob, t, need)) return e;
  if (!ws || ws_bytes < need) return wfail(BO_EWORKSPACE, "bo_wide_upload: workspace too small");
  if (hipMemcpy(ws, t.data(), t.size() * sizeof(wide::Prob), hipMemcpyHostToDevice) != hipSuccess)
    return wfail(BO_EDEVICE, "bo_wide_upload: copy failed");
  return BO_OK;
}

static bo_status wide_args(int32_t nprob, const bo_batch_io *io, void *ws, wide::Args &A) {
  if (nprob <= 0 || !io || !ws) return wfail(BO_EINVAL, "bo_wide: null argument");
  if (!io->Q || !io->Qd || !io->L || !io->Ld || !io->info)
    return wfail(BO_EINVAL, "bo_wide: Q, Qd, L, Ld and info are required");
  A = wide::Args{};
  A.probs = (const wide::Prob *)ws;
  A.ws = (float *)((char *)ws + table_bytes(nprob));
  A.Q = (const float *)io->Q; A.Qd = io->Qd;
  A.Wm = (const float *)io->S; A.Wmd = io->Sd;
  A.L = (float *)io->L; A.Ld = io->Ld;
  A.Sig = (float *)io->Sig; A.Sigd = io->Sigd;
  A.Lb = (float *)io->Lbar; A.Lbd = io->Lbard;
  A.Qb = (float *)io->Qbar; A.Qbd = io->Qbard;
  A.parts = io->parts;
  A.info = io->info;
  return BO_OK;
}

static void launch_f1_f2(int32_t nprob, const wide::Args &A, hipStream_t stream) {
  bo_profile_wide(0, stream, [&] {
    hipLaunchKernelGGL(wide::k_wide_f1, dim3(nprob), dim3(wide::NT), 0, stream, A);
    return 0;
  });
  bo_profile_wide(1, stream, [&] {
    hipLaunchKernelGGL(wide::k_wide_f2, dim3(nprob), dim3(wide::NT), 0, stream, A);
    return 0;
  });
}

static bo_status wide_launch_status(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return wfail(BO_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return BO_OK;
}

extern "C" bo_status bo_wide_forward(int32_t nprob, const bo_batch_io *io, void *ws, hipStream_t stream) {
  wide::Args A;
  if (bo_status e = wide_args(nprob, io, ws, A)) return e;
  if (!io->Sig || !io->Sigd) return wfail(BO_EINVAL, "bo_wide_forward: Sig and Sigd are required");
  A.Wm = nullptr;
  A.Wmd = nullptr;
  launch_f1_f2(nprob, A, stream);
  return wide_launch_status("bo_wide_forward");
}

extern "C" bo_status bo_wide_gauss_loss(int32_t nprob, const bo_batch_io *io, void *ws, hipStream_t stream) {
  wide::Args A;
  if (bo_status e = wide_args(nprob, io, ws, A)) return e;
  if (!io->S || !io->Sd || !io->Sig || !io->Sigd || !io->Lbar || !io->Lbard || !io->Qbar || !io->Qbard ||
      !io->parts)
    return wfail(BO_EINVAL, "bo_wide_gauss_loss: S, Sig, Lbar, Qbar (with diagonals) and parts are required");
  launch_f1_f2(nprob, A, stream);
  bo_profile_wide(2, stream, [&] {
    hipLaunchKernelGGL(wide::k_wide_b1, dim3(nprob), dim3(wide::NT), 0, stream, A);
    return 0;
  });
  bo_profile_wide(3, stream, [&] {
    hipLaunchKernelGGL(wide::k_wide_b2, dim3(nprob), dim3(wide::NT), 0, stream, A, 1.0);
    return 0;
  });
  return wide_launch_status("bo_wide_gauss_loss");
}
