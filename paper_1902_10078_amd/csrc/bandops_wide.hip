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
// (FP64 pivots and log-determinant; one wavefront with the block in
// registers); every dense block product runs on the matrix cores as FP32 MFMA
// (v_mfma_f32_16x16x4_f32).
//
// Parallelism: each problem's blocks are cut into chunks of consecutive
// blocks, one workgroup (four wavefronts) per chunk, and every pass is an exact
// chunked scan:
//   * the subset inverse and both reverse passes are block congruences with
//     the same P_b: Sigma_bb = P_b^T Sigma_{b+1,b+1} P_b + X_b^T X_b, the
//     adjoint of Sigma_bb carried upwards as C_{b+1} = P_b sym(C_b) P_b^T + ...,
//     and the adjoint of S_b (dS_{b+1} = P_b dS_b P_b^T, as S_{b+1} = Q -
//     C_b S_b^{-1} C_b^T) carried downwards as Sbar_b = P_b^T Sbar_{b+1} P_b
//     + ...; a chunk [a, e) maps its entering state affinely through
//     R = P_{e-1} ... P_a and its zero-state run M;
//   * the Cholesky's Schur-complement recurrence is not linear: a chunk maps
//     the correction E_a subtracted from its first diagonal block to the one
//     it leaves on the next block, E_e = D + B (A - E_a)^{-1} B^T, where
//     eliminating the chunk's interior blocks gives A (the Schur complement on
//     its first block), B (the coupling of the next block to the first) and D
//     (the correction on the next block) -- Algorithm 1's elimination order
//     within the chunk, the block form of the scalar passes' chunk maps.
// Per pass: zero-state summaries of every chunk, one workgroup per problem
// applying the chunk maps in order (a few 64 x 64 products per chunk), and a
// replay of every chunk from its exact entering state that writes the outputs.
// Nothing is reordered, so the results are the sequential block recurrences'
// up to rounding.  X_b and P_b are kept in the workspace between passes.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <cstdlib>
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
  int32_t chunk0, nchunk;         // its chunks: consecutive ids [chunk0, chunk0 + nchunk)
};
struct Chunk {
  int32_t prob, pad;
  int64_t b0, b1;                 // blocks [b0, b1) of its problem
};
// Per-chunk workspace, in 64 x 64 FP32 matrices: the Cholesky map (A, B, D),
// the entering states of the four passes, the block product R of the linear
// passes and their zero-state maps.
enum CwSlot { CW_A = 0, CW_B, CW_D, CW_E, CW_R, CW_MF2, CW_MB1, CW_MB2, CW_SF2, CW_SB1, CW_SB2, CW_N };
constexpr int64_t kMat = (int64_t)NB * NB;

struct Args {
  const Prob *probs;
  const float *Q; const double *Qd;     // precision (input)
  const float *Wm; const double *Wmd;   // W of tr(Q^{-1} W) (loss only)
  float *L; double *Ld;
  float *Sig; double *Sigd;
  float *Lb; double *Lbd;
  float *Qb; double *Qbd;
  float *ws;                            // X_b, P_b per block
  const Chunk *chunks;
  float *cws;                           // CW_N matrices per chunk
  double *cpart;                        // per chunk: log-sum, failing row (1-based, 0: none), trace
  double *parts;                        // per problem: logdet, 0, trace
  int32_t *info;
};

__device__ __forceinline__ int64_t nblocks(int64_t n) { return (n + NB - 1) / NB; }

// Workgroup barrier for LDS traffic: waits for this wavefront's LDS accesses
// only (lgkmcnt(0); its global loads may stay in flight across it, so the next
// block's loads overlap the current block's work) and joins the workgroup.
// The empty asm statements keep the compiler from moving memory accesses
// across it.  Threads of a workgroup here exchange data only through LDS.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xc07f);
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// The thread index passed through an empty asm statement: address arithmetic
// derived from it is then recomputed where it is used, instead of being
// hoisted out of the block loops and held (spilled) across them.
__device__ __forceinline__ int opaque_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

// ----------------------------------------------------------- block I/O
constexpr int kSlotIters = (NB * W + NT - 1) / NT;   // slots of a block per thread

// Visit the 64 records of block b (all 65 slots): f(it, c, d, j, valid) with
// j = 64 b + c; valid when the slot lies inside the matrix.
template <class F> __device__ __forceinline__ void for_block_slots(int64_t b, int64_t n, F &&f) {
#pragma unroll
  for (int it = 0; it < kSlotIters; ++it) {
    const int idx = opaque_tid() + it * NT;
    if (idx < NB * W) {
      const int c = idx / W, d = idx - c * W;
      const int64_t j = NB * b + c;
      f(it, c, d, j, j < n && j + d < n);
    }
  }
}

// The raw slots of one block in registers: the FP32 record values and the
// thread's one FP64 diagonal value (a thread's slots idx = tid + 256 it hold
// the diagonal, idx = 0 mod 65, for at most one it).  read_block issues every
// load from an in-bounds address (a slot past the matrix end reads the
// problem's first record) and converts nothing, so that no wait for the loads
// comes before the values are put into LDS; put_blocks then applies the
// identity past the matrix end (1 on the diagonal, else 0).
struct BlockRegs {
  float v[kSlotIters];
  double dv;
};
__device__ __forceinline__ void read_block(const float *Bp, const double *Bd, const Prob &p, int64_t b,
                                           BlockRegs &r) {
  int64_t dj = 0;   // the diagonal slot's row: one load after the loop, not one per slot
  for_block_slots(b, p.n, [&](int it, int c, int d, int64_t j, bool valid) {
    const int64_t jj = valid ? j : 0;
    if (d == 0) dj = jj;
    r.v[it] = Bp[(p.boff + jj * W) + (valid ? d : 0)];
  });
  r.dv = Bd[p.voff + dj];
}
__device__ __forceinline__ double slot_value(const BlockRegs &r, int it, int d, bool valid) {
  return valid ? (d == 0 ? r.dv : (double)r.v[it]) : (d == 0 ? 1.0 : 0.0);
}

// Diagonal block (symmetric, full; E = double or float) and coupling block
// (upper triangular, FP32) of band Bp/Bd at block b, from the registers
// read_block filled (so that the loads of the next block can be issued while
// the current one is worked on); rows past n read as the identity on the
// diagonal and zero elsewhere.
template <typename E>
__device__ __forceinline__ void put_blocks(const BlockRegs &r, const Prob &p, int64_t b, E (&S)[NB][LDF],
                                           MatF *Cf) {
  if (Cf)
    for (int e = threadIdx.x; e < NB * NB; e += NT) (*Cf)[e / NB][e % NB] = 0.f;
  lds_barrier();
  for_block_slots(b, p.n, [&](int it, int c, int d, int64_t, bool valid) {
    const double x = slot_value(r, it, d, valid);
    if (d <= NB - 1 - c) {
      S[c + d][c] = (E)x;
      S[c][c + d] = (E)x;
    } else if (Cf) {
      (*Cf)[d - NB + c][c] = (float)x;
    }
  });
  lds_barrier();
}
template <typename E>
__device__ __forceinline__ void load_blocks(const float *Bp, const double *Bd, const Prob &p, int64_t b,
                                            E (&S)[NB][LDF], MatF *Cf) {
  BlockRegs r;
  read_block(Bp, Bd, p, b, r);
  put_blocks(r, p, b, S, Cf);
}

// The coupling block alone (upper triangular, zero below), from registers.
__device__ __forceinline__ void put_coupling(const BlockRegs &r, const Prob &p, int64_t b, MatF &Cf) {
  for (int e = threadIdx.x; e < NB * NB; e += NT) Cf[e / NB][e % NB] = 0.f;
  lds_barrier();
  for_block_slots(b, p.n, [&](int it, int c, int d, int64_t, bool valid) {
    if (d > NB - 1 - c) Cf[d - NB + c][c] = (float)slot_value(r, it, d, valid);
  });
  lds_barrier();
}

// Store a block pair into band Bp/Bd: the lower triangle of Dg (diagonal
// values from dg when given, else Dg's own) and the upper triangle of Cf
// (when given; the coupling slots are written 0 when it is not).
template <class DiagF, class LowF, class CoupF>
__device__ __forceinline__ void store_blocks(float *Bp, double *Bd, const Prob &p, int64_t b, DiagF &&diag, LowF &&low,
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
  lds_barrier();
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
  lds_barrier();   // every read of A and B is done before any output is written
#pragma unroll
  for (int t = 0; t < 4; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) out(16 * t + 4 * kq + r, jl, alpha * acc[t][r]);
  lds_barrier();
}


// Value of v in lane src of the wavefront (src a compile-time constant after
// unrolling), for every lane.
__device__ __forceinline__ double bcast_lane(double v, int src) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), src);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), src);
  return __hiloint2double(hi, lo);
}

// Reciprocal square root of x > 0 in FP64: the hardware estimate refined by
// two Newton steps y <- y + y (1/2 - (x/2) y^2), each of which roughly doubles
// the number of correct bits.
__device__ __forceinline__ double rsqrt64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
#pragma unroll
  for (int it = 0; it < 2; ++it) {
    const double e = fma(-h * y, y, 0.5);
    y = fma(y, e, y);
  }
  return y;
}

// FP64 Cholesky S = L L^T of the symmetric block S (held full) and X = L^{-1}
// by the workgroup's four wavefronts, wavefront w holding rows [16w, 16w + 16)
// of every column in registers (lane j = column j).
//
// Cholesky, right-looking: at column c the wavefront owning row c takes
// l_j = L[j, c] = S[c, j] / sqrt(S[c, c]) (the trailing update keeps both
// triangles, so row c holds column c), publishes the l_j in LDS (two buffers
// alternate, so one barrier per column suffices), and every wavefront applies
// S[i, j] -= l_i l_j to its rows (l_i = 0 for i <= c leaves those as they
// are).  Lane c's column is never touched after step c, so L[i, c] is that
// column over the pivot's square root.  L's strict lower triangle goes to S.
//
// Inverse by row blocks of 16, L_qq X_q = E_q - sum_{m<q} L_qm X_m (E the
// identity's rows): in round m wavefront m solves its rows with L_mm and
// publishes them (transposed into S's upper triangle, which the Cholesky no
// longer needs, and in FP32 to Xf); after the round's barrier every later
// wavefront subtracts L_qm X_m from its rows.  X is exactly zero above the
// diagonal.  dg / rdg receive L's diagonal and its reciprocal; lsum gains
// log det L.  Returns 0, or 1 + the first column whose pivot is not positive
// (then S, Xf, dg are unspecified).  Every thread of the workgroup calls it.
__device__ int potrf_inv64(MatD &S, double *dg, double *rdg, MatF &Xf, double &lsum) {
  __shared__ int fail_s;
  __shared__ double lb[2][NB];
  const int tid = threadIdx.x, j = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);   // wavefront index (uniform)
  const int r0 = 16 * w;
  double a[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) a[t] = S[r0 + t][j];
  if (tid == 0) fail_s = 0;
#pragma unroll 1
  for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
    for (int tc = 0; tc < 16; ++tc) {
      const int c = 16 * cb + tc;
      if (w == cb) {
        const double piv = bcast_lane(a[tc], c);
        const bool ok = piv > 0.0;
        const double r = rsqrt64(ok ? piv : 1.0);
        lb[tc & 1][j] = j > c ? a[tc] * r : 0.0;
        if (j == c) {
          dg[c] = piv * r;
          rdg[c] = r;
          if (!ok && fail_s == 0) fail_s = c + 1;
        }
      }
      lds_barrier();
      const double lj = lb[tc & 1][j];
      double li[16];
#pragma unroll
      for (int t = 0; t < 16; ++t) li[t] = lb[tc & 1][r0 + t];
#pragma unroll
      for (int t = 0; t < 16; ++t) a[t] = fma(-li[t], lj, a[t]);
      // the update is applied here, not deferred to the end of the loop with
      // every step's l values held in registers meanwhile
#pragma unroll
      for (int t = 0; t < 16; ++t) asm volatile("" : "+v"(a[t]));
    }
  }
  lds_barrier();
  const int fail = fail_s;
  if (fail) return fail;
  {
    const double rj = rdg[j];
#pragma unroll
    for (int t = 0; t < 16; ++t)
      if (r0 + t > j) S[r0 + t][j] = a[t] * rj;
  }
  if (w == 0) {
    double lg = log(dg[j]);
    for (int off = 32; off >= 1; off >>= 1) lg += __shfl_xor(lg, off, 64);
    if (j == 0) lsum += lg;
  }
  lds_barrier();
  double x[16];
#pragma unroll
  for (int t = 0; t < 16; ++t) x[t] = r0 + t == j ? 1.0 : 0.0;
#pragma unroll 1
  for (int m = 0; m < 4; ++m) {
    // L's entries are read a column ahead of their use; the empty asm
    // statements with a memory clobber keep the compiler from hoisting every
    // column's loads to the top (rows and columns are indexed through m, not
    // r0, so that nothing is invariant across the rounds either)
    const int m0 = 16 * m;
    if (w == m) {   // forward substitution with L_mm, then publish X_m
      double cur[16], nxt[16], rd = rdg[m0], rdn = 0.0;
#pragma unroll
      for (int t = 1; t < 16; ++t) cur[t] = S[m0 + t][m0];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        if (k < 15) {
#pragma unroll
          for (int t = k + 2; t < 16; ++t) nxt[t] = S[m0 + t][m0 + k + 1];
          rdn = rdg[m0 + k + 1];
        }
        asm volatile("" ::: "memory");
        x[k] *= rd;
#pragma unroll
        for (int t = k + 1; t < 16; ++t) x[t] = fma(-cur[t], x[k], x[t]);
#pragma unroll
        for (int t = k + 2; t < 16; ++t) cur[t] = nxt[t];
        rd = rdn;
      }
#pragma unroll
      for (int t = 0; t < 16; ++t) {
        if (m0 + t >= j) S[j][m0 + t] = x[t];
        Xf[m0 + t][j] = (float)x[t];
      }
    }
    lds_barrier();
    if (w > m) {   // subtract L_wm X_m (X_m read back from S's upper triangle)
      double lc[16], ln[16], xc = S[j][m0], xn = 0.0;
#pragma unroll
      for (int t = 0; t < 16; ++t) lc[t] = S[r0 + t][m0];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        if (k < 15) {
#pragma unroll
          for (int t = 0; t < 16; ++t) ln[t] = S[r0 + t][m0 + k + 1];
          xn = S[j][m0 + k + 1];
        }
        asm volatile("" ::: "memory");
        const double xm = m0 + k >= j ? xc : 0.0;   // X is zero above the diagonal
#pragma unroll
        for (int t = 0; t < 16; ++t) {
          x[t] = fma(-lc[t], xm, x[t]);
          lc[t] = ln[t];
        }
        xc = xn;
      }
    }
  }
  return 0;
}

// A 64 x 64 FP32 workspace matrix (row-major) into registers, and from them
// into LDS; ws_load does both.
constexpr int kWsIters = NB * NB / (4 * NT);
typedef float4 WsReg[kWsIters];
__device__ __forceinline__ void ws_read(const float *src, WsReg &v) {
#pragma unroll
  for (int it = 0; it < kWsIters; ++it) v[it] = reinterpret_cast<const float4 *>(src)[threadIdx.x + it * NT];
}
__device__ __forceinline__ void ws_put(const WsReg &v, MatF &M) {
#pragma unroll
  for (int it = 0; it < kWsIters; ++it) {
    const int e = 4 * (threadIdx.x + it * NT), r = e / NB, c = e % NB;
    M[r][c] = v[it].x;
    M[r][c + 1] = v[it].y;
    M[r][c + 2] = v[it].z;
    M[r][c + 3] = v[it].w;
  }
  lds_barrier();
}
__device__ __forceinline__ void ws_load(const float *src, MatF &M) {
  WsReg v;
  ws_read(src, v);
  ws_put(v, M);
}
__device__ __forceinline__ void ws_store(float *dst, const MatF &M) {
  lds_barrier();
  for (int e = threadIdx.x; e < NB * NB; e += NT) dst[e] = M[e / NB][e % NB];
}

__device__ double block_sum(double v, double *red) {
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  lds_barrier();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  lds_barrier();
  return red[0] + red[1] + red[2] + red[3];
}

// ------------------------------------------------------ chunk workspace
__device__ __forceinline__ float *cw(const Args &A, int32_t c, int slot) {
  return A.cws + ((int64_t)c * CW_N + slot) * kMat;
}
__device__ __forceinline__ void set_zero(MatF &M) {
  for (int e = threadIdx.x; e < NB * NB; e += NT) M[e / NB][e % NB] = 0.f;
}
__device__ __forceinline__ void set_identity(MatF &M) {
  for (int e = threadIdx.x; e < NB * NB; e += NT) M[e / NB][e % NB] = (e / NB == e % NB) ? 1.f : 0.f;
}
__device__ __forceinline__ void set_nan(MatF &M) {
  for (int e = threadIdx.x; e < NB * NB; e += NT) M[e / NB][e % NB] = NAN;
}

// ============================================== F1 (Algorithm 1 by blocks)
// Chunk summary: eliminate the chunk's interior blocks a+1 .. e-1 with
// Algorithm 1's block steps, carrying V (the coupling of the next block to
// the first block a), Z (the correction on block a) and Pc (the correction on
// the next diagonal block):
//   S_i = Q_ii - Pc,  X = chol(S_i)^{-1},  Y = X V,  Z += Y^T Y,
//   W = X C_i^T,  Pc = W^T W,  V = -W^T Y        (V starts as C_a)
// giving the map A = Q_aa - Z, B = V, D = Pc of E_a -> E_e.  A problem's last
// chunk has no successor and no map.
__global__ void __launch_bounds__(NT) k_wf1_sum(const Args A) {
  __shared__ MatD S, X;   // X: the factor transposed, then Y and W
  __shared__ MatF Xf, V, Z, Pc, Cf;
  __shared__ double dg[NB], rdg[NB];
  const int32_t c = blockIdx.x;
  const Chunk ch = A.chunks[c];
  const Prob p = A.probs[ch.prob];
  if (ch.b1 >= nblocks(p.n)) return;
  MatF &Y = *reinterpret_cast<MatF *>(&X[0][0]);
  MatF &Wt = *reinterpret_cast<MatF *>(reinterpret_cast<char *>(&X[0][0]) + sizeof(MatF));
  float *Am = cw(A, c, CW_A), *Bm = cw(A, c, CW_B), *Dm = cw(A, c, CW_D);
  load_blocks(A.Q, A.Qd, p, ch.b0, S, &V);
  for (int e = threadIdx.x; e < NB * NB; e += NT) {
    Am[e] = (float)S[e / NB][e % NB];
    Z[e / NB][e % NB] = 0.f;
    Pc[e / NB][e % NB] = 0.f;
  }
  lds_barrier();
  double unused = 0.0;
  bool bad = false;
  // each block's loads are issued while the block before it is worked on
  BlockRegs q;
  if (ch.b0 + 1 < ch.b1) read_block(A.Q, A.Qd, p, ch.b0 + 1, q);
  for (int64_t i = ch.b0 + 1; i < ch.b1; ++i) {
    put_blocks(q, p, i, S, &Cf);
    if (i + 1 < ch.b1) read_block(A.Q, A.Qd, p, i + 1, q);
    for (int e = threadIdx.x; e < NB * NB; e += NT) S[e / NB][e % NB] -= (double)Pc[e / NB][e % NB];
    lds_barrier();
    if (potrf_inv64(S, dg, rdg, Xf, unused)) {
      bad = true;
      break;
    }
    gemm64<false, false>(Xf, V, 1.f, [&](int r, int q, float v) { Y[r][q] = v; });
    gemm64<true, false>(Y, Y, 1.f, [&](int r, int q, float v) { Z[r][q] += v; });
    gemm64<false, true>(Xf, Cf, 1.f, [&](int r, int q, float v) { Wt[r][q] = v; });
    gemm64<true, false>(Wt, Wt, 1.f, [&](int r, int q, float v) { Pc[r][q] = v; });
    gemm64<true, false>(Wt, Y, -1.f, [&](int r, int q, float v) { V[r][q] = v; });
  }
  lds_barrier();
  // an interior block that is not positive definite: the leading part of Q is
  // not either, and the replay of this chunk reports where; the map is NaN
  for (int e = threadIdx.x; e < NB * NB; e += NT) {
    const int r = e / NB, q = e % NB;
    Am[e] = bad ? NAN : Am[e] - Z[r][q];
    Bm[e] = bad ? NAN : V[r][q];
    Dm[e] = bad ? NAN : Pc[r][q];
  }
}

// The chunk maps of each problem in order, one workgroup per problem: the
// correction entering chunk c+1 is E_{c+1} = D_c + (X B_c^T)^T (X B_c^T),
// X = chol(A_c - E_c)^{-1}; E_0 = 0.
__global__ void __launch_bounds__(NT) k_wf1_scan(const Args A) {
  __shared__ MatD S, X;
  __shared__ MatF Xf, Bf, Ef, Y;
  __shared__ double dg[NB], rdg[NB];
  const Prob p = A.probs[blockIdx.x];
  set_zero(Ef);
  double unused = 0.0;
  for (int32_t c = p.chunk0; c < p.chunk0 + p.nchunk; ++c) {
    ws_store(cw(A, c, CW_E), Ef);
    if (c == p.chunk0 + p.nchunk - 1) break;
    const float *Am = cw(A, c, CW_A);
    lds_barrier();
    for (int e = threadIdx.x; e < NB * NB; e += NT) S[e / NB][e % NB] = (double)Am[e] - (double)Ef[e / NB][e % NB];
    ws_load(cw(A, c, CW_B), Bf);
    if (potrf_inv64(S, dg, rdg, Xf, unused)) {   // reported by this chunk's replay
      set_nan(Ef);
      lds_barrier();
      continue;
    }
    gemm64<false, true>(Xf, Bf, 1.f, [&](int r, int q, float v) { Y[r][q] = v; });
    ws_load(cw(A, c, CW_D), Ef);
    gemm64<true, false>(Y, Y, 1.f, [&](int r, int q, float v) { Ef[r][q] += v; });
  }
}

// Chunk replay: Algorithm 1 by blocks from the exact correction entering the
// chunk: L, the log-determinant partial, X_b and P_b = M_b X_b for the later
// passes; the first failing row (1-based) of the chunk, if any.
__global__ void __launch_bounds__(NT) k_wf1_rep(const Args A) {
  __shared__ MatD S, X;
  __shared__ MatF Cf, Mf, Xf;
  __shared__ double dg[NB], rdg[NB];
  const int32_t c = blockIdx.x;
  const Chunk ch = A.chunks[c];
  const Prob p = A.probs[ch.prob];
  double lsum = 0.0;
  int64_t fail = 0;
  BlockRegs q;   // the next block's records, loaded behind this block's work
  read_block(A.Q, A.Qd, p, ch.b0, q);
  for (int64_t b = ch.b0; b < ch.b1; ++b) {
    put_blocks(q, p, b, S, &Cf);
    if (b + 1 < ch.b1) read_block(A.Q, A.Qd, p, b + 1, q);
    if (b > ch.b0) {   // S_b = Q_bb - M_{b-1} M_{b-1}^T
      gemm64<false, true>(Mf, Mf, 1.f, [&](int i, int j, float v) { S[i][j] -= (double)v; });
    } else if (b > 0) {   // the correction entering the chunk
      const float *E = cw(A, c, CW_E);
      for (int e = threadIdx.x; e < NB * NB; e += NT) S[e / NB][e % NB] -= (double)E[e];
      lds_barrier();
    }
    const int r = potrf_inv64(S, dg, rdg, Xf, lsum);
    if (r) {
      fail = NB * b + r;
      break;
    }
    // M_b = C_b X_b^T (upper triangular)
    gemm64<false, true>(Cf, Xf, 1.f, [&](int i, int j, float v) { Mf[i][j] = v; });
    store_blocks(A.L, A.Ld, p, b, [&](int cc) { return dg[cc]; }, [&](int i, int cc) { return S[i][cc]; },
                 [&](int rr, int cc) { return (double)Mf[rr][cc]; });
    float *wsb = A.ws + (p.wsoff + b) * kBlockWs;
    ws_store(wsb, Xf);
    // P_b = M_b X_b (into Cf, which is free now)
    gemm64<false, false>(Mf, Xf, 1.f, [&](int i, int j, float v) { Cf[i][j] = v; });
    ws_store(wsb + NB * NB, Cf);
  }
  if (threadIdx.x == 0) {
    A.cpart[3 * (int64_t)c + 0] = lsum;
    A.cpart[3 * (int64_t)c + 1] = (double)fail;
  }
}

// Per problem: log det Q from the chunks' log-sums, info = the first failing
// row over the chunks in order.
__global__ void k_wfin1(const Args A, int32_t nprob) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nprob) return;
  const Prob p = A.probs[q];
  double ls = 0.0;
  int64_t fail = 0;
  for (int32_t c = p.chunk0; c < p.chunk0 + p.nchunk; ++c) {
    ls += A.cpart[3 * (int64_t)c];
    const int64_t f = (int64_t)A.cpart[3 * (int64_t)c + 1];
    if (f > 0 && fail == 0) fail = f;
  }
  if (A.parts) {
    A.parts[3 * (int64_t)q + 0] = fail ? NAN : 2.0 * ls;
    A.parts[3 * (int64_t)q + 1] = fail ? NAN : 0.0;
    A.parts[3 * (int64_t)q + 2] = NAN;   // the trace, written after the F2 pass
  }
  A.info[q] = (int32_t)fail;
}

// ======================================== linear passes: chunk summaries
// One ascending walk over the chunk's blocks gives
//   R = P_{e-1} ... P_a,
//   the subset inverse's zero-state map (descending, written ascending):
//     M_F2 = sum_i R_i^T X_i^T X_i R_i,   R_i = P_{i-1} ... P_a,
//   and, with B1, the zero-state carry of Algorithm 4 by blocks over the chunk
//   (ascending): C <- P (W_ii + sym C) P^T - 2 W_{i+1,i} P^T.
// A problem's first chunk needs no F2 map and its last chunk no B1 map.
__global__ void __launch_bounds__(NT) k_wlin_sum(const Args A, int32_t want_b1) {
  __shared__ MatF Xf, Pf, Rf, Mf2, Cb, Sf, EMf, Tf;
  const int32_t c = blockIdx.x;
  const Chunk ch = A.chunks[c];
  const Prob p = A.probs[ch.prob];
  if (A.info[ch.prob] != 0) return;
  const bool f2 = c != p.chunk0;
  const bool b1 = want_b1 && ch.b1 < nblocks(p.n);
  set_identity(Rf);
  set_zero(Mf2);
  set_zero(Cb);
  WsReg px, pp;   // the next block's X, P and W, loaded behind this block's work
  BlockRegs pw;
  auto fetch = [&](int64_t b) __attribute__((always_inline)) {
    const float *wsb = A.ws + (p.wsoff + b) * kBlockWs;
    ws_read(wsb, px);
    ws_read(wsb + NB * NB, pp);
    if (b1) read_block(A.Wm, A.Wmd, p, b, pw);
  };
  fetch(ch.b0);
  for (int64_t b = ch.b0; b < ch.b1; ++b) {
    ws_put(px, Xf);
    ws_put(pp, Pf);
    if (b1) put_blocks(pw, p, b, Sf, &EMf);
    if (b + 1 < ch.b1) fetch(b + 1);
    if (f2) {
      gemm64<false, false>(Xf, Rf, 1.f, [&](int i, int j, float v) { Tf[i][j] = v; });
      gemm64<true, false>(Tf, Tf, 1.f, [&](int i, int j, float v) { Mf2[i][j] += v; });
    }
    if (b1) {
      for (int e = threadIdx.x; e < NB * NB; e += NT) {
        const int i = e / NB, j = e % NB;
        Sf[i][j] += 0.5f * (Cb[i][j] + Cb[j][i]);
        EMf[i][j] *= 2.f;
      }
      gemm64<false, false>(Pf, Sf, 1.f, [&](int i, int j, float v) { Tf[i][j] = v; });
      gemm64<false, true>(Tf, Pf, 1.f, [&](int i, int j, float v) { Cb[i][j] = v; });
      gemm64<false, true>(EMf, Pf, -1.f, [&](int i, int j, float v) { Cb[i][j] += v; });
    }
    gemm64<false, false>(Pf, Rf, 1.f, [&](int i, int j, float v) { Rf[i][j] = v; });
  }
  ws_store(cw(A, c, CW_R), Rf);
  if (f2) ws_store(cw(A, c, CW_MF2), Mf2);
  if (b1) ws_store(cw(A, c, CW_MB1), Cb);
}

// The linear passes' chunk maps of each problem in order (one workgroup per
// problem):  PASS 0, the subset inverse (descending): S <- R^T S R + M_F2;
// PASS 1, Algorithm 4 (ascending): S <- R sym(S) R^T + M_B1;  PASS 2,
// Algorithm 2 (descending): S <- R^T S R + M_B2.  Zero state at the start;
// every chunk's entering state is stored.
template <int PASS> __global__ void __launch_bounds__(NT) k_wlin_scan(const Args A) {
  __shared__ MatF Sf, Rf, Mf, Tf;
  const Prob p = A.probs[blockIdx.x];
  if (A.info[blockIdx.x] != 0) return;
  constexpr bool DESC = PASS != 1;
  constexpr int MSLOT = PASS == 0 ? CW_MF2 : PASS == 1 ? CW_MB1 : CW_MB2;
  constexpr int SSLOT = PASS == 0 ? CW_SF2 : PASS == 1 ? CW_SB1 : CW_SB2;
  set_zero(Sf);
  for (int32_t t = 0; t < p.nchunk; ++t) {
    const int32_t c = DESC ? p.chunk0 + p.nchunk - 1 - t : p.chunk0 + t;
    ws_store(cw(A, c, SSLOT), Sf);
    if (t == p.nchunk - 1) break;
    ws_load(cw(A, c, CW_R), Rf);
    ws_load(cw(A, c, MSLOT), Mf);
    if (DESC) {
      gemm64<false, false>(Sf, Rf, 1.f, [&](int i, int j, float v) { Tf[i][j] = v; });
      gemm64<true, false>(Rf, Tf, 1.f, [&](int i, int j, float v) { Sf[i][j] = v + Mf[i][j]; });
    } else {
      for (int e = threadIdx.x; e < NB * NB; e += NT) {
        const int i = e / NB, j = e % NB;
        Tf[i][j] = 0.5f * (Sf[i][j] + Sf[j][i]);
      }
      gemm64<false, false>(Rf, Tf, 1.f, [&](int i, int j, float v) { Sf[i][j] = v; });
      gemm64<false, true>(Sf, Rf, 1.f, [&](int i, int j, float v) { Tf[i][j] = v; });
      for (int e = threadIdx.x; e < NB * NB; e += NT) {
        const int i = e / NB, j = e % NB;
        Sf[i][j] = Tf[i][j] + Mf[i][j];
      }
      lds_barrier();
    }
  }
}

// ========================================================== F2 (forward)
// Chunk replay of the subset inverse by blocks (descending) from Sigma of the
// block above the chunk; with Wm given, the chunk's part of tr(Q^{-1} W).
__global__ void __launch_bounds__(NT) k_wf2_rep(const Args A) {
  __shared__ MatF Xf, Pf, Wf, Ef, Tf;
  __shared__ double red[4];
  __shared__ double sdg[NB], red4[4][NB];
  const int32_t c = blockIdx.x;
  const Chunk ch = A.chunks[c];
  const Prob p = A.probs[ch.prob];
  if (A.info[ch.prob] != 0) return;
  const int64_t nb = nblocks(p.n);
  ws_load(cw(A, c, CW_SF2), Wf);
  double tr = 0.0;
  WsReg px, pp;   // the next block's X, P and W, loaded behind this block's work
  BlockRegs pw;
  auto fetch = [&](int64_t b) __attribute__((always_inline)) {
    const float *wsb = A.ws + (p.wsoff + b) * kBlockWs;
    ws_read(wsb, px);
    ws_read(wsb + NB * NB, pp);
    if (A.Wm) read_block(A.Wm, A.Wmd, p, b, pw);
  };
  fetch(ch.b1 - 1);
  for (int64_t b = ch.b1 - 1; b >= ch.b0; --b) {
    ws_put(px, Xf);
    ws_put(pp, Pf);
    const bool last = b == nb - 1;
    const BlockRegs wv = pw;   // W's block for the trace
    if (b - 1 >= ch.b0) fetch(b - 1);
    if (!last)   // E = Sigma_{b+1,b} = -W P
      gemm64<false, false>(Wf, Pf, -1.f, [&](int i, int j, float v) { Ef[i][j] = v; });
    // Sigma_bb = X^T X - P^T E
    gemm64<true, false>(Xf, Xf, 1.f, [&](int i, int j, float v) { Tf[i][j] = v; });
    if (!last) gemm64<true, false>(Pf, Ef, -1.f, [&](int i, int j, float v) { Tf[i][j] += v; });
    // FP64 diagonal: sum_k X_ki^2 - sum_k P_ki E_ki, four threads per entry
    {
      const int i = threadIdx.x & 63, q = threadIdx.x >> 6;
      double s = 0.0;
#pragma unroll
      for (int k = 16 * q; k < 16 * q + 16; ++k) {
        s += (double)Xf[k][i] * (double)Xf[k][i];
        if (!last) s -= (double)Pf[k][i] * (double)Ef[k][i];
      }
      red4[q][i] = s;
    }
    lds_barrier();
    if (threadIdx.x < NB) {
      const int i = threadIdx.x;
      sdg[i] = (red4[0][i] + red4[1][i]) + (red4[2][i] + red4[3][i]);
    }
    lds_barrier();
    store_blocks(A.Sig, A.Sigd, p, b, [&](int cc) { return sdg[cc]; },
                 [&](int i, int cc) { return (double)Tf[i][cc]; },
                 [&](int rr, int cc) { return last ? 0.0 : (double)Ef[rr][cc]; });
    if (A.Wm) {   // tr(Sigma W) over the stored entries (off-diagonal ones twice)
      for_block_slots(b, p.n, [&](int it, int cc, int d, int64_t, bool valid) {
        if (!valid) return;
        const double sv = d == 0 ? sdg[cc] : (d <= NB - 1 - cc ? (double)Tf[cc + d][cc] : (double)Ef[d - NB + cc][cc]);
        tr += (d == 0 ? 1.0 : 2.0) * slot_value(wv, it, d, true) * sv;
      });
    }
    lds_barrier();
    // carry Sigma_bb (full, symmetric) to the block above
    for (int e = threadIdx.x; e < NB * NB; e += NT) {
      const int i = e / NB, j = e % NB;
      Wf[i][j] = i == j ? (float)sdg[i] : (i > j ? Tf[i][j] : Tf[j][i]);
    }
    lds_barrier();
  }
  const double t = block_sum(tr, red);
  if (threadIdx.x == 0) A.cpart[3 * (int64_t)c + 2] = t;
}

// Per problem: tr(Q^{-1} W) from the chunks (NaN for a failed factorisation).
__global__ void k_wfin2(const Args A, int32_t nprob) {
  const int32_t q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= nprob || !A.parts) return;
  const Prob p = A.probs[q];
  if (A.info[q] != 0) {
    A.parts[3 * (int64_t)q + 2] = NAN;
    return;
  }
  double t = 0.0;
  for (int32_t c = p.chunk0; c < p.chunk0 + p.nchunk; ++c) t += A.cpart[3 * (int64_t)c + 2];
  A.parts[3 * (int64_t)q + 2] = A.Wm ? t : 0.0;
}

// =================================================== B1 (Algorithm 4, blocks)
// Chunk replay, ascending, from the carry entering the chunk, with Sigmabar
// from W (S_ii on the diagonal, 2 S_ij off it, on the stored entries): writes
// Lbar (diagonal-block lower triangle and coupling-block upper triangle).
// Carried: the adjoint of Sigma_bb (only its symmetric part is used).
__global__ void __launch_bounds__(NT) k_wb1_rep(const Args A) {
  __shared__ MatF Xf, Pf, Wf, EMf, Sf, Cf, A1, A2, Mc;
  const int32_t c = blockIdx.x;
  const Chunk ch = A.chunks[c];
  const Prob p = A.probs[ch.prob];
  if (A.info[ch.prob] != 0) return;
  const int64_t nb = nblocks(p.n);
  ws_load(cw(A, c, CW_SB1), Cf);
  // The next block's X, P, W, Sigma_{b+2,b+2} and L coupling block are
  // loaded behind this block's products (every wait for them comes at the
  // top of the next iteration).
  WsReg px, pp;
  BlockRegs pw, ps, pl;
  auto fetch = [&](int64_t b) __attribute__((always_inline)) {
    const float *wsb = A.ws + (p.wsoff + b) * kBlockWs;
    ws_read(wsb, px);
    ws_read(wsb + NB * NB, pp);
    read_block(A.Wm, A.Wmd, p, b, pw);
    if (b != nb - 1) {
      read_block(A.Sig, A.Sigd, p, b + 1, ps);
      read_block(A.L, A.Ld, p, b, pl);
    }
  };
  fetch(ch.b0);
  for (int64_t b = ch.b0; b < ch.b1; ++b) {
    ws_put(px, Xf);
    ws_put(pp, Pf);
    const bool last = b == nb - 1;
    // Sbar = sym(user's adjoint of Sigma_bb) + sym(carry) = W_bb + sym(C);
    // Ebar = user's adjoint of Sigma_{b+1,b} = 2 W_{b+1,b} (upper triangle)
    put_blocks(pw, p, b, Sf, &EMf);
    if (!last) {
      put_blocks(ps, p, b + 1, Wf, nullptr);   // W = Sigma_{b+1,b+1}
      put_coupling(pl, p, b, Mc);              // M_b from L's coupling slots
    }
    if (b + 1 < ch.b1) fetch(b + 1);
    for (int e = threadIdx.x; e < NB * NB; e += NT) {
      const int i = e / NB, j = e % NB;
      const bool pad = NB * b + i >= p.n || NB * b + j >= p.n;
      Sf[i][j] = pad ? 0.f : Sf[i][j] + 0.5f * (Cf[i][j] + Cf[j][i]);
      EMf[i][j] *= 2.f;
    }
    lds_barrier();
    if (!last) {
      // U = P Sbar once: Pbar = W (2 U - Ebar) (A2) and the carry to block
      // b+1, (U - Ebar) P^T (Cf, whose incoming value is consumed above)
      gemm64<false, false>(Pf, Sf, 1.f, [&](int i, int j, float v) {
        A1[i][j] = 2.f * v - EMf[i][j];
        Cf[i][j] = v - EMf[i][j];
      });
      gemm64<false, false>(Wf, A1, 1.f, [&](int i, int j, float v) { A2[i][j] = v; });
      gemm64<false, true>(Cf, Pf, 1.f, [&](int i, int j, float v) { Cf[i][j] = v; });
      // Mbar = Pbar X^T: Lbar's coupling block (upper triangle kept), in A1
      gemm64<false, true>(A2, Xf, 1.f, [&](int i, int j, float v) { A1[i][j] = v; });
      // Xbar = 2 X Sbar + M^T Pbar   (Wf)
      gemm64<false, false>(Xf, Sf, 2.f, [&](int i, int j, float v) { Wf[i][j] = v; });
      gemm64<true, false>(Mc, A2, 1.f, [&](int i, int j, float v) { Wf[i][j] += v; });
    } else {
      gemm64<false, false>(Xf, Sf, 2.f, [&](int i, int j, float v) { Wf[i][j] = v; });
    }
    // Lbar_bb = -X^T Xbar X^T (lower triangle kept)
    gemm64<true, false>(Xf, Wf, 1.f, [&](int i, int j, float v) { Sf[i][j] = v; });
    gemm64<false, true>(Sf, Xf, -1.f, [&](int i, int j, float v) { A2[i][j] = v; });
    store_blocks(A.Lb, A.Lbd, p, b, [&](int cc) { return (double)A2[cc][cc]; },
                 [&](int i, int cc) { return (double)A2[i][cc]; },
                 [&](int rr, int cc) { return last ? 0.0 : (double)A1[rr][cc]; });
    lds_barrier();
  }
}

// =================================================== B2 (Algorithm 2, blocks)
// Descending reverse of F1 over a chunk: Qbar from L, Lbar and the
// log-determinant sensitivity gl.  Carried: the adjoint of S_{b+1}.  REPLAY:
// from the carry entering the chunk, writing Qbar; otherwise the zero-state
// run of a chunk, whose final carry is its map M_B2 (a problem's first chunk
// needs none).
template <bool REPLAY> __global__ void __launch_bounds__(NT) k_wb2(const Args A, double gl) {
  __shared__ MatF Lf, Xf, Mf, MBf, LBf, Sc, A1, A2;
  __shared__ double dg[NB], lbd[NB];
  const int32_t c = blockIdx.x;
  const Chunk ch = A.chunks[c];
  const Prob p = A.probs[ch.prob];
  if (A.info[ch.prob] != 0) return;
  if (!REPLAY && c == p.chunk0) return;
  const int64_t nb = nblocks(p.n);
  if (REPLAY) ws_load(cw(A, c, CW_SB2), Sc);
  else set_zero(Sc);
  lds_barrier();
  // the next block's X, L and Lbar (and the pivots and Lbar's diagonal) are
  // loaded behind this block's products
  WsReg px;
  BlockRegs pl, plb;
  double pdg = 1.0, plbd = 0.0;   // (read in bounds; rows past n are masked where used)
  auto fetch = [&](int64_t b) __attribute__((always_inline)) {
    ws_read(A.ws + (p.wsoff + b) * kBlockWs, px);
    read_block(A.L, A.Ld, p, b, pl);
    read_block(A.Lb, A.Lbd, p, b, plb);
    if (threadIdx.x < NB) {
      const int64_t j = NB * b + threadIdx.x;
      pdg = A.Ld[p.voff + (j < p.n ? j : 0)];
      plbd = A.Lbd[p.voff + (j < p.n ? j : 0)];
    }
  };
  fetch(ch.b1 - 1);
  for (int64_t b = ch.b1 - 1; b >= ch.b0; --b) {
    const bool last = b == nb - 1;
    ws_put(px, Xf);
    // L_bb (lower) and M_b (upper) from L, the FP64 pivots from Ld
    put_blocks(pl, p, b, Lf, &Mf);
    for (int e = threadIdx.x; e < NB * NB; e += NT) {
      const int i = e / NB, j = e % NB;
      if (i < j) Lf[i][j] = 0.f;
    }
    if (threadIdx.x < NB) {
      const int64_t j = NB * b + threadIdx.x;
      const double d = j < p.n ? pdg : 1.0;
      dg[threadIdx.x] = d;
      // Lbar_bb's diagonal with the log-determinant term
      lbd[threadIdx.x] = j < p.n ? plbd + 2.0 * gl / d : 0.0;
    }
    // Lbar_bb (lower) and Mbar_b (upper)
    put_blocks(plb, p, b, LBf, &MBf);
    if (b - 1 >= ch.b0) fetch(b - 1);
    for (int e = threadIdx.x; e < NB * NB; e += NT) {
      const int i = e / NB, j = e % NB;
      const bool pad = NB * b + i >= p.n;
      LBf[i][j] = i == j ? (float)lbd[i] : (i > j && !pad ? LBf[i][j] : 0.f);
    }
    lds_barrier();
    if (!last) {
      // Mbar -= 2 Sc M   (Sc: adjoint of S_{b+1}, symmetric)
      gemm64<false, false>(Sc, Mf, -2.f, [&](int i, int j, float v) { MBf[i][j] += v; });
      // Cbar = Mbar X (its upper triangle is Qbar's coupling block, A2)
      gemm64<false, false>(MBf, Xf, 1.f, [&](int i, int j, float v) { A2[i][j] = v; });
      // Lbar_bb -= X^T Mbar^T M = Cbar^T M
      gemm64<true, false>(A2, Mf, -1.f, [&](int i, int j, float v) { LBf[i][j] += v; });
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
    if (REPLAY)
      store_blocks(A.Qb, A.Qbd, p, b, [&](int cc) { return (double)Sc[cc][cc]; },
                   [&](int i, int cc) { return (double)(Sc[i][cc] + Sc[cc][i]); },
                   [&](int rr, int cc) { return last ? 0.0 : (double)A2[rr][cc]; });
    lds_barrier();
  }
  if (!REPLAY) ws_store(cw(A, c, CW_MB2), Sc);
}

}  // namespace wide

// ====================================================================== C ABI
// The library's thread-local error message (defined with the other entry points).
bo_status bo_set_error(bo_status s, const std::string &msg);
// Launch timing hook of the library (slot per wide kernel kind, which = 0..9).
int bo_profile_wide(int which, hipStream_t s, const std::function<int()> &launch);

namespace {
bo_status wfail(bo_status s, const std::string &m) { return bo_set_error(s, m); }
size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Chunks per call: about one workgroup per compute unit (the passes' LDS use,
// up to ~150 KB, allows one per CU), spread over the problems by their block
// counts.  BANDOPS_WIDE_CHUNKS overrides the target.
int64_t wide_target_chunks() {
  static int64_t v = [] {
    const char *e = std::getenv("BANDOPS_WIDE_CHUNKS");
    long long t = e ? std::atoll(e) : 0;
    return (int64_t)(t > 0 ? t : 256);
  }();
  return v;
}

// Host image of a call's tables and its workspace layout.
struct WideLayout {
  std::vector<wide::Prob> probs;
  std::vector<wide::Chunk> chunks;
  size_t off_chunks = 0, off_blockws = 0, off_cws = 0, off_cpart = 0, bytes = 0;
  int64_t blocks = 0;
};
}  // namespace

static bo_status wide_layout(const bo_problem *probs, int32_t nprob, WideLayout &L) {
  if (!probs || nprob <= 0) return wfail(BO_EINVAL, "bo_wide: no problems");
  L = WideLayout{};
  L.probs.resize(nprob);
  int64_t blocks = 0;
  for (int32_t i = 0; i < nprob; ++i) {
    if (probs[i].k != wide::NB) return wfail(BO_EUNSUPPORTED, "bo_wide: every problem must have k = 64");
    if (probs[i].n < 0 || probs[i].boff < 0 || probs[i].voff < 0) return wfail(BO_EINVAL, "bo_wide: bad problem");
    blocks += (probs[i].n + wide::NB - 1) / wide::NB;
  }
  const int64_t target = wide_target_chunks();
  int64_t wsoff = 0;
  for (int32_t i = 0; i < nprob; ++i) {
    const int64_t nb = (probs[i].n + wide::NB - 1) / wide::NB;
    wide::Prob p{probs[i].n, probs[i].boff, probs[i].voff, wsoff, (int32_t)L.chunks.size(), 0};
    if (nb > 0) {
      int64_t nc = blocks > 0 ? (target * nb + blocks / 2) / blocks : 1;
      nc = std::max<int64_t>(1, std::min<int64_t>(nc, nb));
      const int64_t cb = (nb + nc - 1) / nc;
      for (int64_t b0 = 0; b0 < nb; b0 += cb) L.chunks.push_back(wide::Chunk{i, 0, b0, std::min(nb, b0 + cb)});
      p.nchunk = (int32_t)L.chunks.size() - p.chunk0;
    }
    L.probs[i] = p;
    wsoff += nb;
  }
  L.blocks = blocks;
  const size_t nch = L.chunks.size();
  L.off_chunks = align256((size_t)nprob * sizeof(wide::Prob));
  L.off_blockws = L.off_chunks + align256(nch * sizeof(wide::Chunk));
  L.off_cws = L.off_blockws + align256((size_t)blocks * wide::kBlockWs * sizeof(float));
  L.off_cpart = L.off_cws + align256(nch * wide::CW_N * wide::kMat * sizeof(float));
  L.bytes = L.off_cpart + align256(nch * 3 * sizeof(double));
  return BO_OK;
}

extern "C" bo_status bo_wide_workspace_size(const bo_problem *probs, int32_t nprob, size_t *bytes) {
  if (!bytes) return wfail(BO_EINVAL, "bo_wide_workspace_size: null bytes");
  WideLayout L;
  if (bo_status e = wide_layout(probs, nprob, L)) return e;
  *bytes = L.bytes;
  return BO_OK;
}

extern "C" bo_status bo_wide_upload(const bo_problem *probs, int32_t nprob, void *ws, size_t ws_bytes) {
  WideLayout L;
  if (bo_status e = wide_layout(probs, nprob, L)) return e;
  if (!ws || ws_bytes < L.bytes) return wfail(BO_EWORKSPACE, "bo_wide_upload: workspace too small");
  if (hipMemcpy(ws, L.probs.data(), L.probs.size() * sizeof(wide::Prob), hipMemcpyHostToDevice) != hipSuccess ||
      (!L.chunks.empty() && hipMemcpy((char *)ws + L.off_chunks, L.chunks.data(), L.chunks.size() * sizeof(wide::Chunk),
                                      hipMemcpyHostToDevice) != hipSuccess))
    return wfail(BO_EDEVICE, "bo_wide_upload: copy failed");
  return BO_OK;
}

static bo_status wide_args(const bo_problem *probs, int32_t nprob, const bo_batch_io *io, void *ws, size_t ws_bytes,
                           WideLayout &L, wide::Args &A) {
  if (nprob <= 0 || !io || !ws) return wfail(BO_EINVAL, "bo_wide: null argument");
  if (!io->Q || !io->Qd || !io->L || !io->Ld || !io->info)
    return wfail(BO_EINVAL, "bo_wide: Q, Qd, L, Ld and info are required");
  if (bo_status e = wide_layout(probs, nprob, L)) return e;
  if (ws_bytes < L.bytes)
    return wfail(BO_EWORKSPACE, "bo_wide: workspace needs " + std::to_string(L.bytes) + " bytes");
  A = wide::Args{};
  char *w = (char *)ws;
  A.probs = (const wide::Prob *)w;
  A.chunks = (const wide::Chunk *)(w + L.off_chunks);
  A.ws = (float *)(w + L.off_blockws);
  A.cws = (float *)(w + L.off_cws);
  A.cpart = (double *)(w + L.off_cpart);
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

namespace {
// One launch on the stream, timed under the given slot when profiling is on.
template <class K, class... Ts> void wlaunch(int which, K kern, unsigned grid, hipStream_t s, Ts... args) {
  if (grid == 0) return;
  bo_profile_wide(which, s, [&] {
    hipLaunchKernelGGL(kern, dim3(grid), dim3(wide::NT), 0, s, args...);
    return 0;
  });
}
enum { WS_F1 = 0, WS_F2, WS_B1, WS_B2, WS_F1SUM, WS_F1SCAN, WS_LINSUM, WS_LINSCAN, WS_B2SUM, WS_FIN };

// Cholesky, log det, subset inverse (and the trace when W is given), and with
// want_b1 the linear-pass maps Algorithm 4 needs.
void launch_forward(const WideLayout &L, int32_t nprob, const wide::Args &A, bool want_b1, hipStream_t s) {
  const unsigned nch = (unsigned)L.chunks.size(), np = (unsigned)nprob, npb = (unsigned)((nprob + 63) / 64);
  wlaunch(WS_F1SUM, wide::k_wf1_sum, nch, s, A);
  wlaunch(WS_F1SCAN, wide::k_wf1_scan, np, s, A);
  wlaunch(WS_F1, wide::k_wf1_rep, nch, s, A);
  bo_profile_wide(WS_FIN, s, [&] {
    hipLaunchKernelGGL(wide::k_wfin1, dim3(npb), dim3(64), 0, s, A, nprob);
    return 0;
  });
  wlaunch(WS_LINSUM, wide::k_wlin_sum, nch, s, A, (int32_t)(want_b1 ? 1 : 0));
  wlaunch(WS_LINSCAN, wide::k_wlin_scan<0>, np, s, A);
  wlaunch(WS_F2, wide::k_wf2_rep, nch, s, A);
  bo_profile_wide(WS_FIN, s, [&] {
    hipLaunchKernelGGL(wide::k_wfin2, dim3(npb), dim3(64), 0, s, A, nprob);
    return 0;
  });
}
}  // namespace

static bo_status wide_launch_status(const char *what) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return wfail(BO_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  return BO_OK;
}

extern "C" bo_status bo_wide_forward(const bo_problem *probs, int32_t nprob, const bo_batch_io *io, void *ws,
                                     size_t ws_bytes, hipStream_t stream) {
  WideLayout L;
  wide::Args A;
  if (bo_status e = wide_args(probs, nprob, io, ws, ws_bytes, L, A)) return e;
  if (!io->Sig || !io->Sigd) return wfail(BO_EINVAL, "bo_wide_forward: Sig and Sigd are required");
  A.Wm = nullptr;
  A.Wmd = nullptr;
  launch_forward(L, nprob, A, false, stream);
  return wide_launch_status("bo_wide_forward");
}

extern "C" bo_status bo_wide_gauss_loss(const bo_problem *probs, int32_t nprob, const bo_batch_io *io, void *ws,
                                        size_t ws_bytes, hipStream_t stream) {
  WideLayout L;
  wide::Args A;
  if (bo_status e = wide_args(probs, nprob, io, ws, ws_bytes, L, A)) return e;
  if (!io->S || !io->Sd || !io->Sig || !io->Sigd || !io->Lbar || !io->Lbard || !io->Qbar || !io->Qbard ||
      !io->parts)
    return wfail(BO_EINVAL, "bo_wide_gauss_loss: S, Sig, Lbar, Qbar (with diagonals) and parts are required");
  launch_forward(L, nprob, A, true, stream);
  const unsigned nch = (unsigned)L.chunks.size(), np = (unsigned)nprob;
  wlaunch(WS_LINSCAN, wide::k_wlin_scan<1>, np, stream, A);
  wlaunch(WS_B1, wide::k_wb1_rep, nch, stream, A);
  wlaunch(WS_B2SUM, wide::k_wb2<false>, nch, stream, A, 1.0);
  wlaunch(WS_LINSCAN, wide::k_wlin_scan<2>, np, stream, A);
  wlaunch(WS_B2, wide::k_wb2<true>, nch, stream, A, 1.0);
  return wide_launch_status("bo_wide_gauss_loss");
}
