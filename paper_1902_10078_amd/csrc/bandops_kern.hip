// bandops_kern.hip -- kernels of one bandwidth K (compiled once per K with
// -DBO_K=<k>).
//
// The row-streaming steps (summaries, replays, chunk products) run one chunk
// per lane with LDS-tiled input streaming (bandops_tile.hpp); the scan steps
// (group composition and sweeps) run one work item per lane straight from
// bandops_items.hpp.
#include "bandops_steps.hpp"
#include "bandops_tile.hpp"

#ifndef BO_K
#error "compile with -DBO_K=<bandwidth>"
#endif

#define BO_CAT2(a, b) a##b
#define BO_CAT(a, b) BO_CAT2(a, b)

namespace {

using namespace bo;
using tile::BandIn;
using tile::VecIn;
using tile::stream_rows;

constexpr int kBlock = 64;   // one wavefront per workgroup

template <class Item>
__global__ void __launch_bounds__(kBlock) k_item(const Args a, int64_t count) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) Item::run(a, i);
}

// Chunk of this lane (inactive lanes borrow the launch's last chunk so that
// every lane reads a valid problem descriptor; they stream no rows).
struct LaneChunk {
  bool active;
  int32_t c;
  ProbDesc pd;
  int64_t a, b;
};
__device__ __forceinline__ LaneChunk lane_chunk(const Args &A, int64_t count) {
  LaneChunk L;
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  L.active = i < count;
  L.c = A.c_beg + (int32_t)(L.active ? i : count - 1);
  L.pd = prob_at(A, prob_of_chunk(A, L.c));
  chunk_rows(L.pd, L.c, L.a, L.b);
  return L;
}

// Interleaved intermediates (Args::il, FP64): the block of wavefront w of an
// array, and a lane's view of its chunk as a band of stride 64 (K + 1) whose
// record j is row j - a of the lane's slot (only records of the chunk and its
// halo are ever addressed through it; the base is formed in unsigned
// arithmetic and may lie before the array).
template <int K, typename T> __device__ __forceinline__ T *il_wave(void *base, const Args &A, int64_t w) {
  return (T *)base + A.il_off + w * (int64_t)A.il_rows * kBlock * (K + 1);
}
template <int K, typename T>
__device__ __forceinline__ BandP<T> il_view(void *base, const Args &A, int64_t w, int l, int64_t a) {
  constexpr int64_t W = K + 1;
  const uint64_t p = (uint64_t)(il_wave<K, T>(base, A, w) + l * W) - (uint64_t)(a * kBlock * W * (int64_t)sizeof(T));
  return BandP<T>{(T *)p, nullptr, kBlock * W};
}
template <int K, typename T> __device__ __forceinline__ BandP<T> lane_view(void *base, const Args &A, const LaneChunk &C) {
  return il_view<K, T>(base, A, blockIdx.x, threadIdx.x, C.a);
}
// Interleaved vectors (one element per record): the same rows and lanes.
template <typename T> __device__ __forceinline__ T *il_vwave(const void *base, const Args &A, int64_t w) {
  return (T *)base + A.il_voff + w * (int64_t)A.il_rows * kBlock;
}
template <typename T>
__device__ __forceinline__ VecP<T, kBlock> il_vview(const void *base, const Args &A, int64_t w, int l, int64_t a) {
  const uint64_t p = (uint64_t)(il_vwave<T>(base, A, w) + l) - (uint64_t)(a * kBlock * (int64_t)sizeof(T));
  return VecP<T, kBlock>((T *)p);
}
template <typename T>
__device__ __forceinline__ VecP<T, kBlock> lane_vview(const void *base, const Args &A, const LaneChunk &C) {
  return il_vview<T>(base, A, blockIdx.x, threadIdx.x, C.a);
}
// The same view of the previous chunk of the lane's problem (its halo rows
// follow its own rows).
template <typename T>
__device__ __forceinline__ VecP<T, kBlock> prev_vview(const void *base, const Args &A, const LaneChunk &C) {
  const int l = threadIdx.x;
  return il_vview<T>(base, A, l > 0 ? (int64_t)blockIdx.x : (int64_t)blockIdx.x - 1, l > 0 ? l - 1 : kBlock - 1,
                     C.a - C.pd.clen);
}
// A staged vector input: the wave's interleaved block, or the lane's values.
template <bool IL, typename T>
__device__ __forceinline__ VecIn<T> vstaged(const void *base, const Args &A, const T *rm, bool on, int shift = 0) {
  if constexpr (IL) return VecIn<T>{il_vwave<T>(base, A, blockIdx.x), shift};
  else return VecIn<T>{on ? rm : nullptr, shift};
}
template <typename T> __device__ __forceinline__ BandP<const T> const_view(BandP<T> b) {
  return BandP<const T>{b.p, b.diag, b.ld};
}
// A staged band input: the wave's interleaved block, or the lane's records.
template <bool IL, int K, typename T>
__device__ __forceinline__ BandIn<T> staged(void *base, const Args &A, BandP<const T> b, bool on, int shift = 0) {
  if constexpr (IL) return BandIn<T>{il_wave<K, T>(base, A, blockIdx.x), nullptr, shift};
  else return BandIn<T>{on ? b.p : nullptr, on ? b.diag : nullptr, shift};
}
// Kernels with IL = true read and write L, S (Sigma), Lb, z (bx, zf) and the
// copy of ybar (xil) interleaved (Args::il); FP64 only.

// ------------------------------------------------------------------- F1
// DIAG: the factored matrix is Q + diag(qdn / qdd[problem]); the addend is
// staged as a second vector (val[1]) and added to each diagonal entry as it is
// read.
template <int K>
__device__ __forceinline__ void with_diag(const double (&rec)[K + 1], const double (&val)[2], double ds,
                                          double (&q)[K + 1]) {
#pragma unroll
  for (int d = 0; d <= K; ++d) q[d] = rec[d];
  q[0] += val[1] * ds;
}

template <int K, typename T, bool DIAG>
__global__ void __launch_bounds__(kBlock) k_f1_sum(const Args A, int64_t count) {
  constexpr int NV = DIAG ? 2 : 1;
  const LaneChunk C = lane_chunk(A, count);
  const ProbDesc &pd = C.pd;
  const bool on = C.active && C.c != pd.chunk0 + pd.nchunk - 1;
  BandP<const T> Q = cband<T>(A.Q, A.Qd, pd);
  const T *y = cvec<T>(A.y, pd);
  const T *dn = DIAG ? cvec<T>(A.qdn, pd) : nullptr;
  const double ds = DIAG ? qdiag_scale(A, pd) : 0.0;
  F1SumStep<K, T> st;
  double *mw = A.f1map + (int64_t)C.c * A.sw_f1map;   // the map is completed in place
  if (on) st.begin_w(C.a, pd.n, Q, y, mw, dn, ds);
  BandIn<T> bands[1] = {{on ? Q.p : nullptr, on ? Q.diag : nullptr, 0}};
  VecIn<T> vecs[NV];
  vecs[0] = {on ? y : nullptr, 0};
  if constexpr (DIAG) vecs[NV - 1] = {on ? dn : nullptr, 0};
  stream_rows<K, T, 1, NV, false>(bands, vecs, on ? C.a + K : 0, on ? C.b : 0, pd.n, pd.ld,
                                  [&](int64_t, const double (&rec)[1][K + 1], const double (&val)[NV]) {
                                    if constexpr (DIAG) {
                                      double q[K + 1];
                                      with_diag<K>(rec[0], val, ds, q);
                                      st.row(q, val[0]);
                                    } else {
                                      st.row(rec[0], val[0]);
                                    }
                                  });
  if (on) st.end_w(mw);
}

// ------------------------------------------- F1 summary, a quad per chunk
// From K = 10 the summary's state (window correction C, coupling X of the
// window to the boundary rows, boundary correction Z: three K x K blocks)
// does not fit one lane's registers.  Here the four lanes of a quad share one
// chunk, and the window's rows live in fixed slots: row u of the chunk's
// sweep sits in slot (u - a - K) mod K, so advancing by a row rewrites the
// leaving row's slot for the entering one and no register moves.  The row
// loop is unrolled K times so every slot index is a constant.  Lane t keeps
// the C rows and g entries of slots t, t + 4, t + 8 (C stored whole, both
// triangles), columns f = t, t + 4, t + 8 of X for every slot, and rows f of
// Z (in LDS) and e.  The pivot row's C and g come from their owner by DPP broadcasts,
// as do the row's coupling values xf.  Each entry is computed as in
// F1SumStep (same operands and order; a product of two l values in either
// order is the same number), so the maps are the same bits.
constexpr int kQuad = 4;

template <int S> __device__ __forceinline__ double quad_bcast(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), S * 0x55, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), S * 0x55, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}

template <int I, int N, class F> __device__ __forceinline__ void unroll_each(F &&f) {
  if constexpr (I < N) {
    f(std::integral_constant<int, I>{});
    unroll_each<I + 1, N>(f);
  }
}

template <int K, typename T, bool DIAG>
__global__ void __launch_bounds__(kBlock, 2) k_f1_sum_q(const Args A, int64_t count) {
  constexpr int K1 = Dim<K>::K1, NF = (K + kQuad - 1) / kQuad, KK = K1 * K1;
  static_assert(K >= kQuad, "the quad summary needs a column per lane");
  const int t = threadIdx.x & (kQuad - 1);
  const int64_t ci = (int64_t)blockIdx.x * (kBlock / kQuad) + (threadIdx.x / kQuad);
  const bool active = ci < count;
  const int32_t c = A.c_beg + (int32_t)(active ? ci : count - 1);
  const ProbDesc pd = prob_at(A, prob_of_chunk(A, c));
  int64_t a, b;
  chunk_rows(pd, c, a, b);
  const bool on = active && c != pd.chunk0 + pd.nchunk - 1;   // quad-uniform
  const int64_t n = pd.n;
  BandP<const T> Q = cband<T>(A.Q, A.Qd, pd);
  const T *y = cvec<T>(A.y, pd);
  const T *dn = DIAG ? cvec<T>(A.qdn, pd) : nullptr;
  const double ds = DIAG ? qdiag_scale(A, pd) : 0.0;
  double *w = A.f1map + (int64_t)c * A.sw_f1map;
  // Cs[i][v]: C(slot t + 4i, slot v); gs[i]: g of slot t + 4i; X[s][i]:
  // X(slot s, column t + 4i)
  // Z(t + 4i, h) in LDS (only accumulated, so it leaves the registers to the
  // window state), lane-interleaved
  __shared__ double sZ[NF * K1][kBlock];
  double Cs[NF][K1], gs[NF], X[K1][NF], e[NF];
  const int lane = threadIdx.x;
#pragma unroll
  for (int i = 0; i < NF; ++i) {
    gs[i] = e[i] = 0.0;
#pragma unroll
    for (int v = 0; v < K1; ++v) {
      Cs[i][v] = X[v][i] = 0.0;
      sZ[i * K1 + v][lane] = 0.0;
    }
  }
  auto rec_at = [&](int64_t j, double (&r)[K + 1]) {
    load_rec<K, T>(Q.p, Q.diag, Q.ld, j, n, r);
    if (DIAG) r[0] += (double)dn[j] * ds;
  };
  if (on) {
    // boundary rows a .. a+K-1: lane t writes A = Q_FF and r = y_F for its
    // columns f, and takes its columns of X = Q[a+K+p, a+f] (slot p)
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const int f = t + kQuad * i;
      if (f < K) {
        double rec[K + 1];
        rec_at(a + f, rec);
#pragma unroll
        for (int p = 0; p < K; ++p)
          if (p >= f) w[p * K1 + f] = w[f * K1 + p] = rec[p >= f ? p - f : 0];
#pragma unroll
        for (int p = 0; p < K; ++p) X[p][i] = p <= f ? rec[K + (p <= f ? p - f : 0)] : 0.0;
        w[3 * KK + f] = y ? (double)y[a + f] : 0.0;
      }
    }
  }
  const int64_t len = on ? b - a - K : 0;
  const int64_t maxlen = tile::wave_max(len);
  // a row's record as load_rec reads it (entries past the problem's end are
  // zero), with the entry test in 32 bits on the stored values
  // (the off-diagonal entries stay in the stored type until the row is used)
  auto rec_next = [&](int64_t j, double &r0, T (&r)[K + 1]) {
    const T *rp = Q.p + j * Q.ld;
    const int lim = (int)(n - j < K + 1 ? n - j : K + 1);
#pragma unroll
    for (int d = 1; d <= K; ++d) r[d] = d < lim ? rp[d] : T(0);
    r0 = Q.diag ? Q.diag[j] : (double)rp[0];
    if (DIAG) r0 += (double)dn[j] * ds;
  };
  T qn[K + 1];
  double qn0 = 0.0, yn = 0.0;
  if (len > 0) {
    rec_next(a + K, qn0, qn);
    yn = y ? (double)y[a + K] : 0.0;
  }
  // one row with the window's first row in slot PH
  auto row = [&](auto phc, int64_t r) {
    constexpr int PH = decltype(phc)::value;
    if (r >= len) return;   // uniform over the quad
    double q[K + 1];
    q[0] = qn0;
#pragma unroll
    for (int d = 1; d <= K; ++d) q[d] = (double)qn[d];
    const double yi = yn;
    if (r + 1 < len) {   // the next row's loads, behind this row's work
      rec_next(a + K + r + 1, qn0, qn);
      yn = y ? (double)y[a + K + r + 1] : 0.0;
    }
    double cp[K1];   // C(slot PH, slot v): the leaving row's C, from its owner
#pragma unroll
    for (int v = 0; v < K; ++v) cp[v] = quad_bcast<PH % kQuad>(Cs[PH / kQuad][v]);
    const double gp = quad_bcast<PH % kQuad>(gs[PH / kQuad]);
    const double s0 = q[0] - cp[PH];
    const double lii = s0 > 0.0 ? sqrt(s0) : NAN;
    const double inv = 1.0 / lii;
    // ls[v]: l of the row in slot v (window row p = (v - PH - 1) mod K after
    // the step; slot PH takes the entering row, p = K - 1)
    double ls[K1];
#pragma unroll
    for (int v = 0; v < K; ++v) {
      const int p = (v - PH - 1 + 2 * K) % K;
      ls[v] = ((p + 1 < K) ? q[p + 1] - cp[v] : q[K]) * inv;   // slot v holds window row p
    }
    double lo[NF];   // l of the lane's own slots t + 4i
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const int v0 = kQuad * i;
      const double l0 = ls[v0 < K ? v0 : 0], l1 = ls[v0 + 1 < K ? v0 + 1 : 0];
      const double l2 = ls[v0 + 2 < K ? v0 + 2 : 0], l3 = ls[v0 + 3 < K ? v0 + 3 : 0];
      lo[i] = t == 0 ? l0 : t == 1 ? l1 : t == 2 ? l2 : l3;
    }
    double xo[NF], xf[K1];
#pragma unroll
    for (int i = 0; i < NF; ++i) xo[i] = X[PH][i] * inv;
    const double zt = (yi - gp) * inv;
#pragma unroll
    for (int h = 0; h < K; ++h) {   // xf[h] from the lane that owns column h
      const double v = xo[h / kQuad];
      switch (h % kQuad) {
        case 0: xf[h] = quad_bcast<0>(v); break;
        case 1: xf[h] = quad_bcast<1>(v); break;
        case 2: xf[h] = quad_bcast<2>(v); break;
        default: xf[h] = quad_bcast<3>(v); break;
      }
    }
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      e[i] += xo[i] * zt;
#pragma unroll
      for (int h = 0; h < K; ++h) sZ[i * K1 + h][lane] += xo[i] * xf[h];
    }
#pragma unroll
    for (int v = 0; v < K; ++v)
#pragma unroll
      for (int i = 0; i < NF; ++i) X[v][i] = (v == PH ? 0.0 : X[v][i]) - ls[v] * xo[i];
    const bool own_ph = t == PH % kQuad;   // the lane whose slot PH / 4 is the leaving row's
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const bool fresh = i == PH / kQuad && own_ph;
      gs[i] = (fresh ? 0.0 : gs[i]) + lo[i] * zt;
#pragma unroll
      for (int v = 0; v < K; ++v) {
        if (i == PH / kQuad)
          Cs[i][v] = ((fresh || v == PH) ? 0.0 : Cs[i][v]) + lo[i] * ls[v];
        else
          Cs[i][v] = (v == PH ? 0.0 : Cs[i][v]) + lo[i] * ls[v];
      }
    }
  };
#pragma unroll 1
  for (int64_t r0 = 0; r0 < maxlen; r0 += K)
    unroll_each<0, K>([&](auto phc) { row(phc, r0 + decltype(phc)::value); });
  if (on) {
    const int ph = (int)(len % K);   // the window's first row is in slot ph
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const int f = t + kQuad * i;
      if (f < K) {
#pragma unroll
        for (int p = 0; p < K; ++p) w[p * K1 + f] -= sZ[i * K1 + p][lane];   // A = Q_FF - Z (Z symmetric)
#pragma unroll
        for (int v = 0; v < K; ++v) {
          const int p = v >= ph ? v - ph : v - ph + K;
          w[KK + p * K1 + f] = -X[v][i];
        }
        w[3 * KK + f] -= e[i];
      }
    }
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const int s = t + kQuad * i;
      if (s < K) {
        const int p = s >= ph ? s - ph : s - ph + K;
#pragma unroll
        for (int v = 0; v < K; ++v) {
          const int h = v >= ph ? v - ph : v - ph + K;
          w[2 * KK + p * K1 + h] = Cs[i][v];
        }
        w[3 * KK + K1 + p] = gs[i];
      }
    }
  }
}

// PC: accumulates the chunk products (A.Pc); launched without it when A.Pc
// is null.
template <int K, typename T, bool DIAG, bool PC, bool IL>
__global__ void __launch_bounds__(kBlock) k_f1_rep(const Args A, int64_t count) {
  constexpr int NV = DIAG ? 2 : 1;
  const LaneChunk C = lane_chunk(A, count);
  const ProbDesc &pd = C.pd;
  const bool on = C.active;
  BandP<const T> Q = cband<T>(A.Q, A.Qd, pd);
  const T *y = cvec<T>(A.y, pd);
  const T *dn = DIAG ? cvec<T>(A.qdn, pd) : nullptr;
  const double ds = DIAG ? qdiag_scale(A, pd) : 0.0;
  F1State<K> s0;
  if (on && pd.nchunk > 1)
    f1_load_state<K>(A.f1st + (int64_t)C.c * A.sw_f1st, s0);
  else
    f1_zero_state<K>(s0);
  F1RepStep<K, T, PC, IL ? kBlock : 1> st;
  const bool fuse = K <= KMAX_FUSED && A.lmap_out && A.Pc;
  if constexpr (IL) {
    st.begin(s0, lane_view<K, T>(A.L, A, C), y ? lane_vview<T>(A.z, A, C) : VecP<T, kBlock>(), A.Pc != nullptr, fuse);
    if (y && A.zcopy) st.z2 = VecP<T>(vec<T>(A.zcopy, pd));
  } else {
    st.begin(s0, band<T>(A.L, A.Ld, pd), y ? vec<T>(A.z, pd) : nullptr, A.Pc != nullptr, fuse);
  }
  BandIn<T> bands[1] = {{on ? Q.p : nullptr, on ? Q.diag : nullptr, 0}};
  VecIn<T> vecs[NV];
  vecs[0] = {on ? y : nullptr, 0};
  if constexpr (DIAG) vecs[NV - 1] = {on ? dn : nullptr, 0};
  stream_rows<K, T, 1, NV, false>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
                                  [&](int64_t j, const double (&rec)[1][K + 1], const double (&val)[NV]) {
                                    if constexpr (DIAG) {
                                      double q[K + 1];
                                      with_diag<K>(rec[0], val, ds, q);
                                      st.row(j, q, val[0]);
                                    } else {
                                      st.row(j, rec[0], val[0]);
                                    }
                                  });
  if (on) {
    st.end(A.Pc ? A.Pc + (int64_t)C.c * A.sw_mat : nullptr);
    if (fuse) {
      LinMap<K> m;
      st.end_f2(m);
      lin_store<K>(A.lmap_out + (int64_t)C.c * A.sw_lin, m);
    }
    double *pt = A.part + 4 * (int64_t)C.c;
    pt[0] = st.ls;
    pt[1] = st.qs;
    pt[3] = (double)st.fail;
  }
}

template <int K, typename T, bool IL>
__global__ void __launch_bounds__(kBlock) k_pc(const Args A, int64_t count) {
  const LaneChunk C = lane_chunk(A, count);
  const ProbDesc &pd = C.pd;
  const bool on = C.active;
  BandP<const T> L = cband<T>(A.L, A.Ld, pd);
  PcStep<K> st;
  st.begin();
  BandIn<T> bands[1] = {staged<IL, K, T>(A.L, A, L, on)};
  VecIn<T> vecs[1] = {{nullptr, 0}};
  stream_rows<K, T, 1, 0, false, IL ? 1u : 0u>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
                                 [&](int64_t, const double (&rec)[1][K + 1], const double (&)[1]) {
                                   st.row(rec[0]);
                                 });
  if (on) st.end(A.Pc + (int64_t)C.c * A.sw_mat);
}

// ------------------------------------------------------- linear passes
template <int K> __device__ __forceinline__ void lin_in(const Args &A, const LaneChunk &C, bool replay,
                                                        LinMap<K> &st) {
  if (replay && C.active && C.pd.nchunk > 1)
    lin_load<K>(A.lst + (int64_t)C.c * A.sw_lin, st);
  else
    lin_zero<K>(st);
}

// FUSE (replay only): the forward solve also accumulates the chunk maps of a
// B2 pass whose z is this solve's output and which has no Lbar record (needs
// ybar, staged K+1 rows ahead).
template <int K, typename T, bool REPLAY, bool FUSE>
__global__ void __launch_bounds__(kBlock) k_fs(const Args A, int64_t count) {
  const LaneChunk C = lane_chunk(A, count);
  const ProbDesc &pd = C.pd;
  const bool on = C.active && (REPLAY || pd.nchunk > 1);
  BandP<const T> L = cband<T>(A.L, A.Ld, pd);
  LinMap<K> st;
  lin_in<K>(A, C, REPLAY, st);
  FsStep<K, T, REPLAY> s;
  s.begin(st, vec<T>(A.x, pd), A.xscale);
  BandIn<T> bands[1] = {{on ? L.p : nullptr, on ? L.diag : nullptr, 0}};
  if constexpr (FUSE) {
    const T *yb = cvec<T>(A.yb, pd);
    B2MapAcc<K> m2;
    if (on) m2.begin(C.a, pd.n, yb, A.gl);
    const double zero[K + 1] = {};
    VecIn<T> vecs[2] = {{on ? cvec<T>(A.bx, pd) : nullptr, 0}, {on ? yb : nullptr, K + 1}};
    stream_rows<K, T, 1, 2, false>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
                                   [&](int64_t j, const double (&rec)[1][K + 1], const double (&val)[2]) {
                                     const double xj = s.row(j, rec[0], val[0]);
                                     m2.row(rec[0], 1.0 / rec[0][0], zero, xj, val[1]);
                                   });
    if (on) {
      LinMap<K> m;
      m2.end(m);
      lin_store<K>(A.lmap_out + (int64_t)C.c * A.sw_lin, m);
    }
  } else {
    VecIn<T> vecs[1] = {{on ? cvec<T>(A.bx, pd) : nullptr, 0}};
    stream_rows<K, T, 1, 1, false>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
                                   [&](int64_t j, const double (&rec)[1][K + 1], const double (&val)[1]) {
                                     s.row(j, rec[0], val[0]);
                                   });
  }
  if (on && !REPLAY) {
    s.end(st);
    lin_store<K>(A.lmap + (int64_t)C.c * A.sw_lin, st);
  }
}

// FUSE: the replay also accumulates the B1 pass's chunk maps (needs the
// Sigmabar / S band as a second staged input).
template <int K, typename T, bool REPLAY, bool FUSE, bool IL>
__global__ void __launch_bounds__(kBlock) k_f2(const Args A, int64_t count) {
  const LaneChunk C = lane_chunk(A, count);
  const ProbDesc &pd = C.pd;
  const bool on = C.active && (REPLAY || pd.nchunk > 1);
  BandP<const T> L = cband<T>(A.L, A.Ld, pd);
  const T *bx = cvec<T>(A.bx, pd);
  LinMap<K> st;
  lin_in<K>(A, C, REPLAY, st);
  F2Step<K, T, REPLAY, IL> s;
  s.begin(st, IL ? lane_view<K, T>(A.S, A, C) : band<T>(A.S, A.Sd, pd), vec<T>(A.x, pd), A.xscale,
          A.S != nullptr, bx != nullptr, FUSE, A.sb_is_S != 0);
  if constexpr (IL && REPLAY) {
    if (on && C.c > pd.chunk0) {
      // rows a .. a+K are also the halo of the previous chunk of the problem
      const int l = threadIdx.x;
      s.set_halo(il_view<K, T>(A.S, A, l > 0 ? (int64_t)blockIdx.x : (int64_t)blockIdx.x - 1,
                               l > 0 ? l - 1 : kBlock - 1, C.a - pd.clen),
                 C.a + K + 1);
    }
    if (A.sbar_out) s.set_sym_out(band<T>(A.sbar_out, nullptr, pd));
    if (A.xil && on)
      s.set_x_copy(lane_vview<T>(A.xil, A, C), C.c > pd.chunk0 ? prev_vview<T>(A.xil, A, C) : VecP<T, kBlock>(),
                   C.a + K + 1);
  }
  VecIn<T> vecs[1] = {vstaged<IL>(A.bx, A, bx, on)};
  if constexpr (FUSE) {
    BandP<const T> Sb = cband<T>(A.Sb, A.Sbd, pd);
    BandIn<T> bands[2] = {staged<IL, K, T>(A.L, A, L, on),
                          {on ? Sb.p : nullptr, on ? Sb.diag : nullptr, 0}};
    stream_rows<K, T, 2, 1, true, IL ? 1u : 0u, IL ? 1u : 0u>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
                                  [&](int64_t j, const double (&rec)[2][K + 1], const double (&val)[1]) {
                                    s.row(j, rec[0], val[0]);
                                    s.row_b1(rec[0], rec[1]);
                                  });
    if (on) {
      LinMap<K> m;
      s.end_b1(m);
      lin_store<K>(A.lmap_out + (int64_t)C.c * A.sw_lin, m);
    }
  } else {
    BandIn<T> bands[1] = {staged<IL, K, T>(A.L, A, L, on)};
    stream_rows<K, T, 1, 1, true, IL ? 1u : 0u, IL ? 1u : 0u>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
                                  [&](int64_t j, const double (&rec)[1][K + 1], const double (&val)[1]) {
                                    s.row(j, rec[0], val[0]);
                                  });
  }
  if (on && !REPLAY) {
    s.end(st);
    lin_store<K>(A.lmap + (int64_t)C.c * A.sw_lin, st);
  }
}

// FUSE: the replay also accumulates the B2 pass's chunk maps (needs ybar,
// staged K+1 rows ahead, and z).
template <int K, typename T, bool REPLAY, bool FUSE, bool IL>
__global__ void __launch_bounds__(kBlock) k_b1(const Args A, int64_t count) {
  const LaneChunk C = lane_chunk(A, count);
  const ProbDesc &pd = C.pd;
  const bool on = C.active && (REPLAY || pd.nchunk > 1);
  BandP<const T> L = cband<T>(A.L, A.Ld, pd);
  BandP<const T> Sig = cband<T>(A.S, A.Sd, pd);
  BandP<const T> Sb = cband<T>(A.Sb, A.Sbd, pd);
  LinMap<K> st;
  lin_in<K>(A, C, REPLAY, st);
  B1Step<K, T, REPLAY, FUSE> s;
  if (on)
    s.begin(st, C.a, pd.n, IL ? const_view(lane_view<K, T>(A.S, A, C)) : Sig, A.sb_is_S != 0,
            IL ? lane_view<K, T>(A.Lb, A, C) : band<T>(A.Lb, A.Lbd, pd), A.accumulate != 0, A.gl1);
  if constexpr (REPLAY) {
    BandIn<T> bands[3] = {staged<IL, K, T>(A.L, A, L, on),
                          {on ? Sb.p : nullptr, on ? Sb.diag : nullptr, 0},
                          staged<IL, K, T>(A.S, A, Sig, on, K + 1)};
    if constexpr (FUSE) {
      const T *yb = cvec<T>(A.yb, pd);
      if constexpr (IL) {
        if (on) s.begin_b2(C.a, pd.n, lane_vview<const T>(A.xil, A, C), A.gl);
      } else {
        if (on) s.begin_b2(C.a, pd.n, yb, A.gl);
      }
      VecIn<T> vecs[2] = {vstaged<IL>(A.xil, A, yb, on, K + 1), vstaged<IL>(A.zf, A, cvec<T>(A.zf, pd), on)};
      stream_rows<K, T, 3, 2, false, IL ? 5u : 0u, IL ? 3u : 0u>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
                                     [&](int64_t j, const double (&rec)[3][K + 1], const double (&val)[2]) {
                                       s.row(j, pd.n, rec[0], rec[1], rec[2], val[1], val[0]);
                                     });
      if (on) {
        LinMap<K> m;
        s.end_b2(m);
        lin_store<K>(A.lmap_out + (int64_t)C.c * A.sw_lin, m);
      }
    } else {
      VecIn<T> vecs[1] = {{nullptr, 0}};
      stream_rows<K, T, 3, 0, false, IL ? 5u : 0u>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
                                     [&](int64_t j, const double (&rec)[3][K + 1], const double (&)[1]) {
                                       s.row(j, pd.n, rec[0], rec[1], rec[2]);
                                     });
    }
    if (on) A.part[4 * (int64_t)C.c + 2] = s.tr;
  } else {
    BandIn<T> bands[2] = {staged<IL, K, T>(A.L, A, L, on),
                          {on ? Sb.p : nullptr, on ? Sb.diag : nullptr, 0}};
    VecIn<T> vecs[1] = {{nullptr, 0}};
    stream_rows<K, T, 2, 0, false, IL ? 1u : 0u>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
                                   [&](int64_t j, const double (&rec)[2][K + 1], const double (&)[1]) {
                                     s.row(j, pd.n, rec[0], rec[1], rec[1]);
                                   });
    if (on) {
      s.end(st);
      lin_store<K>(A.lmap + (int64_t)C.c * A.sw_lin, st);
    }
  }
}

// WITH_LB: an incoming Lbar band is staged next to L.  Without one (the
// whitened sample's reverse mode) only L is staged, so its tiles hold twice
// the rows.
template <int K, typename T, bool REPLAY, bool WITH_LB, bool IL>
__global__ void __launch_bounds__(kBlock) k_b2(const Args A, int64_t count) {
  constexpr int NB = WITH_LB ? 2 : 1;
  const LaneChunk C = lane_chunk(A, count);
  const ProbDesc &pd = C.pd;
  const bool on = C.active && (REPLAY || pd.nchunk > 1);
  BandP<const T> L = cband<T>(A.L, A.Ld, pd);
  BandP<const T> Lb = cband<T>(A.Lb, A.Lbd, pd);
  const T *yb = cvec<T>(A.yb, pd);
  const T *zf = cvec<T>(A.zf, pd);
  LinMap<K> st;
  lin_in<K>(A, C, REPLAY, st);
  B2Step<K, T, REPLAY> s;
  if constexpr (IL) s.begin_v(st, C.b, pd.n, on ? lane_vview<const T>(A.xil, A, C) : VecP<const T, kBlock>(), A.gl,
                              band<T>(A.Qb, A.Qbd, pd));
  else s.begin(st, C.b, pd.n, on ? yb : nullptr, A.gl, band<T>(A.Qb, A.Qbd, pd));
  BandIn<T> bands[NB];
  bands[0] = staged<IL, K, T>(A.L, A, L, on);
  if constexpr (WITH_LB) bands[NB - 1] = staged<IL, K, T>(A.Lb, A, Lb, on);
  VecIn<T> vecs[2] = {vstaged<IL>(A.xil, A, yb, on), vstaged<IL>(A.zf, A, zf, on)};
  stream_rows<K, T, NB, 2, true, IL ? (WITH_LB ? 3u : 1u) : 0u, IL ? 3u : 0u>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
                                 [&](int64_t j, const double (&rec)[NB][K + 1], const double (&val)[2]) {
                                   if constexpr (WITH_LB) {
                                     s.row(j, pd.n, rec[0], rec[NB - 1], val[0], val[1]);
                                   } else {
                                     const double none[K + 1] = {};
                                     s.row(j, pd.n, rec[0], none, val[0], val[1]);
                                   }
                                 });
  if (on && !REPLAY) {
    s.end(st);
    lin_store<K>(A.lmap + (int64_t)C.c * A.sw_lin, st);
  }
}

// ------------------------------------------------------------ scans
// The chunk summaries of a pass are combined by parallel prefix scans of
// depth log2(64): one wavefront per group scans its chunks' maps, one per
// problem scans the group totals, and every chunk then applies its exclusive
// prefix to its group's entering state.  (The serial work items and, from
// K = 10, the quad kernels do the same with one step per chunk or group.)  A
// map travels between lanes through LDS, 64 doubles per lane at a time.
constexpr int kXch = 64;

template <int N>
__device__ __forceinline__ void wave_xch(const double (&own)[N], double (&got)[N], int src, double *buf) {
  const int lane = threadIdx.x;
#pragma unroll
  for (int b = 0; b < N; b += kXch) {
#pragma unroll
    for (int e = 0; e < kXch; ++e)
      if (b + e < N) buf[e * kBlock + lane] = own[b + e];
    __syncthreads();
#pragma unroll
    for (int e = 0; e < kXch; ++e)
      if (b + e < N) got[b + e] = buf[e * kBlock + src];
    __syncthreads();
  }
}

template <int K> struct LinPair {   // a linear map: product P and (M, v)
  double P[Dim<K>::K1][Dim<K>::K1];
  LinMap<K> m;
};
template <class M> struct Flat {
  static constexpr int N = sizeof(M) / sizeof(double);
  static __device__ __forceinline__ double (&of(M &x))[N] { return *reinterpret_cast<double(*)[N]>(&x); }
};

// Inclusive scan of `cur` over lanes [0, n) with compose(earlier, later).
template <class M, class Compose>
__device__ __forceinline__ void wave_scan(M &cur, int n, double *buf, Compose &&compose) {
  const int q = threadIdx.x;
  M got;
  for (int off = 1; off < n; off <<= 1) {
    wave_xch(Flat<M>::of(cur), Flat<M>::of(got), q >= off ? q - off : 0, buf);
    if (q >= off && q < n) {
      compose(got, cur);   // got <- got then cur
      cur = got;
    }
  }
}

template <int K, bool DESC> __global__ void __launch_bounds__(kBlock) k_lin_gscan(const Args A, int64_t) {
  __shared__ double buf[kXch * kBlock];
  const int32_t g = A.g_beg + (int32_t)blockIdx.x;
  const ProbDesc &pd = prob_at(A, prob_of_group(A, g));
  int32_t c0, c1;
  group_chunks(pd, g, c0, c1);
  const int n = c1 - c0, q = threadIdx.x;
  const int32_t c = DESC ? c1 - 1 - q : c0 + q;
  LinPair<K> cur;
  if (q < n) {
    mat_load<K>(A.Pc + (int64_t)c * A.sw_mat, cur.P);
    lin_load<K>(A.lmap + (int64_t)c * A.sw_lin, cur.m);
  }
  auto comp = [](LinPair<K> &a, const LinPair<K> &b) { lin_compose<K, DESC>(a.P, a.m, b.P, b.m); };
  wave_scan(cur, n, buf, comp);
  LinPair<K> prev;
  wave_xch(Flat<LinPair<K>>::of(cur), Flat<LinPair<K>>::of(prev), q >= 1 ? q - 1 : 0, buf);
  if (q >= 1 && q < n) {   // the exclusive prefix replaces the chunk's own map
    mat_store<K>(A.Pex + (int64_t)c * A.sw_mat, prev.P);
    lin_store<K>(A.lmap + (int64_t)c * A.sw_lin, prev.m);
  }
  if (q == n - 1) {
    mat_store<K>(A.Pg + (int64_t)g * A.sw_mat, cur.P);
    lin_store<K>(A.lgmap + (int64_t)g * A.sw_lin, cur.m);
  }
}

template <int K, bool DESC> __global__ void __launch_bounds__(kBlock) k_lin_pscan(const Args A, int64_t) {
  __shared__ double buf[kXch * kBlock];
  const ProbDesc &pd = prob_at(A, A.p_beg + (int32_t)blockIdx.x);
  const int n = pd.ngroup, q = threadIdx.x;
  const int32_t g = DESC ? pd.group0 + n - 1 - q : pd.group0 + q;
  LinPair<K> cur;
  if (q < n) {
    mat_load<K>(A.Pg + (int64_t)g * A.sw_mat, cur.P);
    lin_load<K>(A.lgmap + (int64_t)g * A.sw_lin, cur.m);
  }
  auto comp = [](LinPair<K> &a, const LinPair<K> &b) { lin_compose<K, DESC>(a.P, a.m, b.P, b.m); };
  wave_scan(cur, n, buf, comp);
  LinPair<K> prev;
  wave_xch(Flat<LinPair<K>>::of(cur), Flat<LinPair<K>>::of(prev), q >= 1 ? q - 1 : 0, buf);
  if (q < n) {   // entering state of a group: the groups before it applied to the zero state
    LinMap<K> st;
    if (q == 0) lin_zero<K>(st);
    else st = prev.m;
    lin_store<K>(A.lgst + (int64_t)g * A.sw_lin, st);
  }
}

template <int K, bool DESC> __global__ void __launch_bounds__(kBlock) k_lin_capply(const Args A, int64_t) {
  constexpr int K1 = Dim<K>::K1;
  const int32_t g = A.g_beg + (int32_t)blockIdx.x;
  const ProbDesc &pd = prob_at(A, prob_of_group(A, g));
  int32_t c0, c1;
  group_chunks(pd, g, c0, c1);
  const int n = c1 - c0, q = threadIdx.x;
  if (q >= n) return;
  const int32_t c = DESC ? c1 - 1 - q : c0 + q;
  LinMap<K> st;
  lin_load<K>(A.lgst + (int64_t)g * A.sw_lin, st);
  if (q >= 1) {
    double P[K1][K1];
    LinMap<K> m;
    mat_load<K>(A.Pex + (int64_t)c * A.sw_mat, P);
    lin_load<K>(A.lmap + (int64_t)c * A.sw_lin, m);
    lin_apply<K, DESC>(P, m, st);
  }
  lin_store<K>(A.lst + (int64_t)c * A.sw_lin, st);
}

// F1 group maps from K = 10, a quad per group: the group's chunk maps are
// composed in order as in F1GroupCompose (f1_compose, same operations per
// entry, so the same bits), with the accumulated map's A, B, D columns and r,
// d rows q = t, t + 4, t + 8 in lane t of the quad.  Each step every lane
// factors the shared block R = A2 - D1 (D1 gathered through LDS), solves for
// its own columns of Y1 = R^{-1} B1 and Y2 = R^{-1} B2^T, and publishes them in
// LDS for the products of its own output columns.  Inactive quads still take
// every barrier.
template <int K> __global__ void __launch_bounds__(kBlock) k_f1_gcomp_q(const Args A, int64_t count) {
  constexpr int K1 = Dim<K>::K1, NF = (K + kQuad - 1) / kQuad, KK = K1 * K1;
  constexpr int NQ = kBlock / kQuad;
  // the quad's accumulated B and D, d (column q written by its owner) and
  // this step's Y1, Y2
  __shared__ double sB[NQ][K1][K1], sD[NQ][K1][K1], sd[NQ][K1], sY1[NQ][K1][K1], sY2[NQ][K1][K1];
  const int t = threadIdx.x & (kQuad - 1), qi = threadIdx.x / kQuad;
  const int64_t gi = (int64_t)blockIdx.x * NQ + qi;
  const int32_t g = A.g_beg + (int32_t)(gi < count ? gi : count - 1);
  const ProbDesc pd = prob_at(A, prob_of_group(A, g));
  int32_t c0, c1;
  group_chunks(pd, g, c0, c1);
  const bool on = gi < count && g != pd.group0 + pd.ngroup - 1;   // the last group's map is never applied
  const int nsteps = on ? c1 - c0 - 1 : 0;
  int maxsteps = nsteps;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const int o = __shfl_xor(maxsteps, off, kBlock);
    maxsteps = o > maxsteps ? o : maxsteps;
  }
  auto col = [&](int i) { return t + kQuad * i; };
  // the accumulated map: A and r in registers (own columns / rows), B, D, d
  // in LDS
  double aA[K1][NF], ar[NF];
  {
    const double *w = A.f1map + (int64_t)c0 * A.sw_f1map;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const int q = col(i) < K ? col(i) : 0;
#pragma unroll
      for (int p = 0; p < K1; ++p) aA[p][i] = on ? w[p * K1 + q] : 0.0;
      ar[i] = on ? w[3 * KK + q] : 0.0;
      if (col(i) < K) {
#pragma unroll
        for (int p = 0; p < K1; ++p) {
          sB[qi][p][q] = on ? w[KK + p * K1 + q] : 0.0;
          sD[qi][p][q] = on ? w[2 * KK + p * K1 + q] : 0.0;
        }
        sd[qi][q] = on ? w[3 * KK + K1 + q] : 0.0;
      }
    }
  }
#pragma unroll 1
  for (int st = 0; st < maxsteps; ++st) {
    const bool act = st < nsteps;   // uniform over the quad
    const double *w2 = A.f1map + (int64_t)(c0 + 1 + (act ? st : 0)) * A.sw_f1map;
    __syncthreads();   // the accumulated B, D, d of every lane are in LDS
    double R[K1][K1], tv[K1][1];
#pragma unroll
    for (int p = 0; p < K1; ++p) {
#pragma unroll
      for (int q = 0; q < K1; ++q) R[p][q] = act ? w2[p * K1 + q] - sD[qi][p][q] : (p == q ? 1.0 : 0.0);
      tv[p][0] = act ? w2[3 * KK + p] - sd[qi][p] : 0.0;
    }
    chol_small<K>(R);
    trsm_small<K, 1>(R, tv);
    double Y1[K1][NF], Y2[K1][NF];
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const int q = col(i) < K ? col(i) : 0;
      double y1[K1][1], y2[K1][1];
#pragma unroll
      for (int p = 0; p < K1; ++p) {
        y1[p][0] = sB[qi][p][q];
        y2[p][0] = act ? w2[KK + q * K1 + p] : 0.0;   // B2^T, column q
      }
      trsm_small<K, 1>(R, y1);
      trsm_small<K, 1>(R, y2);
#pragma unroll
      for (int p = 0; p < K1; ++p) {
        Y1[p][i] = y1[p][0];
        Y2[p][i] = y2[p][0];
      }
    }
#pragma unroll
    for (int i = 0; i < NF; ++i)
      if (col(i) < K) {
#pragma unroll
        for (int p = 0; p < K1; ++p) {
          sY1[qi][p][col(i)] = Y1[p][i];
          sY2[qi][p][col(i)] = Y2[p][i];
        }
      }
    __syncthreads();   // Y1, Y2 complete; the reads of B, D, d are done
    if (act) {
#pragma unroll
      for (int i = 0; i < NF; ++i) {
        if (col(i) >= K) continue;
        const int q = col(i);
        // rows p = q of r and d use this lane's own columns of Y1, Y2
        double rr = ar[i], dd = w2[3 * KK + K1 + q];
#pragma unroll
        for (int f = 0; f < K; ++f) {
          rr += Y1[f][i] * tv[f][0];
          dd -= Y2[f][i] * tv[f][0];
        }
        ar[i] = rr;
        sd[qi][q] = dd;
      }
      // row p of the new A, B, D for every own column: each shared Y entry is
      // read once per row; per entry the sums run over f in order
#pragma unroll
      for (int p = 0; p < K; ++p) {
        double a[NF], bb[NF], dm[NF];
#pragma unroll
        for (int i = 0; i < NF; ++i) {
          a[i] = aA[p][i];
          bb[i] = 0.0;
          dm[i] = w2[2 * KK + p * K1 + (col(i) < K ? col(i) : 0)];
        }
#pragma unroll
        for (int f = 0; f < K; ++f) {
          const double y1p = sY1[qi][f][p], y2p = sY2[qi][f][p];
#pragma unroll
          for (int i = 0; i < NF; ++i) {
            a[i] -= y1p * Y1[f][i];
            bb[i] += y2p * Y1[f][i];
            dm[i] += y2p * Y2[f][i];
          }
        }
#pragma unroll
        for (int i = 0; i < NF; ++i)
          if (col(i) < K) {
            aA[p][i] = a[i];
            sB[qi][p][col(i)] = bb[i];
            sD[qi][p][col(i)] = dm[i];
          }
      }
    }
  }
  __syncthreads();
  if (on) {
    double *w = A.f1gmap + (int64_t)g * A.sw_f1map;
#pragma unroll
    for (int i = 0; i < NF; ++i)
      if (col(i) < K) {
        const int q = col(i);
#pragma unroll
        for (int p = 0; p < K1; ++p) {
          w[p * K1 + q] = aA[p][i];
          w[KK + p * K1 + q] = sB[qi][p][q];
          w[2 * KK + p * K1 + q] = sD[qi][p][q];
        }
        w[3 * KK + q] = ar[i];
        w[3 * KK + K1 + q] = sd[qi][q];
      }
  }
}

// Linear group maps from K = 10, a quad per group: the group's chunk maps
// applied in order as in LinGroupCompose (lin_apply and mat_mul_acc, same
// operations per entry, so the same bits).  The accumulated M and the group
// product G live in LDS (column q written by lane q % 4), with the step's
// chunk product P; every lane keeps the vector v.
template <int K, bool DESC> __global__ void __launch_bounds__(kBlock) k_lin_gcomp_q(const Args A, int64_t count) {
  constexpr int K1 = Dim<K>::K1, NF = (K + kQuad - 1) / kQuad;
  constexpr int NQ = kBlock / kQuad;
  __shared__ double sS[NQ][K1][K1], sG[NQ][K1][K1], sP[NQ][K1][K1];
  const int t = threadIdx.x & (kQuad - 1), qi = threadIdx.x / kQuad;
  const int64_t gi = (int64_t)blockIdx.x * NQ + qi;
  const int32_t g = A.g_beg + (int32_t)(gi < count ? gi : count - 1);
  const ProbDesc pd = prob_at(A, prob_of_group(A, g));
  int32_t c0, c1;
  group_chunks(pd, g, c0, c1);
  const bool on = gi < count;
  const int nsteps = on ? c1 - c0 : 0;
  int maxsteps = nsteps;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const int o = __shfl_xor(maxsteps, off, kBlock);
    maxsteps = o > maxsteps ? o : maxsteps;
  }
  auto col = [&](int i) { return t + kQuad * i; };
  double v[K1];
#pragma unroll
  for (int p = 0; p < K1; ++p) v[p] = 0.0;
#pragma unroll
  for (int i = 0; i < NF; ++i)
    if (col(i) < K)
#pragma unroll
      for (int p = 0; p < K1; ++p) {
        sS[qi][p][col(i)] = 0.0;
        sG[qi][p][col(i)] = p == col(i) ? 1.0 : 0.0;
      }
#pragma unroll 1
  for (int st = 0; st < maxsteps; ++st) {
    const bool act = st < nsteps;   // uniform over the quad
    const int32_t c = act ? (DESC ? c1 - 1 - st : c0 + st) : c0;
    const double *Pw = A.Pc + (int64_t)c * A.sw_mat;
    const double *mw = A.lmap + (int64_t)c * A.sw_lin;
#pragma unroll
    for (int i = 0; i < NF; ++i)
      if (col(i) < K)
#pragma unroll
        for (int p = 0; p < K1; ++p) sP[qi][p][col(i)] = Pw[p * K1 + col(i)];
    __syncthreads();   // P complete (and the previous step's M, G)
    double vn[K1], W[K1][NF], Gn[K1][NF];
    if (act) {
#pragma unroll
      for (int p = 0; p < K; ++p) {
        double acc = mw[K1 * K1 + p];
#pragma unroll
        for (int q = 0; q < K; ++q) acc += (DESC ? sP[qi][q][p] : sP[qi][p][q]) * v[q];
        vn[p] = acc;
      }
      // row p of W and of the new G for every own column: each shared entry
      // of row p is read once; per entry the sums run over r in order
#pragma unroll
      for (int p = 0; p < K; ++p) {
        double w[NF], gg[NF];
#pragma unroll
        for (int i = 0; i < NF; ++i) w[i] = gg[i] = 0.0;
#pragma unroll
        for (int r = 0; r < K; ++r) {
          const double s_pr = sS[qi][p][r];
          const double g_pr = DESC ? sG[qi][p][r] : sP[qi][p][r];
#pragma unroll
          for (int i = 0; i < NF; ++i) {
            const int q = col(i) < K ? col(i) : 0;
            w[i] += s_pr * (DESC ? sP[qi][r][q] : sP[qi][q][r]);
            gg[i] += DESC ? g_pr * sP[qi][r][q] : g_pr * sG[qi][r][q];
          }
        }
#pragma unroll
        for (int i = 0; i < NF; ++i) {
          W[p][i] = w[i];
          Gn[p][i] = gg[i];
        }
      }
    }
    __syncthreads();   // every read of M and G is done
    if (act) {
#pragma unroll
      for (int p = 0; p < K; ++p) v[p] = vn[p];
#pragma unroll
      for (int p = 0; p < K; ++p) {
        double acc[NF];
#pragma unroll
        for (int i = 0; i < NF; ++i) acc[i] = mw[p * K1 + (col(i) < K ? col(i) : 0)];
#pragma unroll
        for (int r = 0; r < K; ++r) {
          const double pr = DESC ? sP[qi][r][p] : sP[qi][p][r];
#pragma unroll
          for (int i = 0; i < NF; ++i) acc[i] += pr * W[r][i];
        }
#pragma unroll
        for (int i = 0; i < NF; ++i)
          if (col(i) < K) {
            sS[qi][p][col(i)] = acc[i];
            sG[qi][p][col(i)] = Gn[p][i];
          }
      }
    }
    __syncthreads();   // every read of P is done
  }
  if (on) {
    double *Gw = A.Pg + (int64_t)g * A.sw_mat;
    double *lw = A.lgmap + (int64_t)g * A.sw_lin;
#pragma unroll
    for (int i = 0; i < NF; ++i)
      if (col(i) < K) {
        const int q = col(i);
#pragma unroll
        for (int p = 0; p < K1; ++p) {
          Gw[p * K1 + q] = sG[qi][p][q];
          lw[p * K1 + q] = sS[qi][p][q];
        }
      }
    if (t == 0)
#pragma unroll
      for (int p = 0; p < K1; ++p) lw[K1 * K1 + p] = v[p];
  }
}

// The sweeps from K = 10, a quad per unit (GROUPS: a problem walking its
// groups, as F1GroupSweep / LinGroupSweep; else a group walking its chunks,
// as F1ChunkSweep / LinChunkSweep): each unit's state is stored, then the
// unit's map applied to it (f1_apply / lin_apply, same operations per entry,
// so the same bits).  The state lives in LDS, column q written by lane q % 4.
template <int K, bool GROUPS> __global__ void __launch_bounds__(kBlock) k_f1_sweep_q(const Args A, int64_t count) {
  constexpr int K1 = Dim<K>::K1, NF = (K + kQuad - 1) / kQuad, KK = K1 * K1;
  constexpr int NQ = kBlock / kQuad;
  __shared__ double sC[NQ][K1][K1], sg[NQ][K1], sY[NQ][K1][K1];
  const int t = threadIdx.x & (kQuad - 1), qi = threadIdx.x / kQuad;
  const int64_t ui = (int64_t)blockIdx.x * NQ + qi;
  const bool on = ui < count;
  const int64_t uu = on ? ui : count - 1;
  ProbDesc pd;
  int32_t first, nunits, last_map;   // items [first, first + nunits); items < last_map have a map
  const double *maps;
  double *states;
  int32_t g = 0;
  if (GROUPS) {
    pd = prob_at(A, A.p_beg + (int32_t)uu);
    first = pd.group0;
    nunits = pd.ngroup;
    last_map = pd.group0 + pd.ngroup - 1;
    maps = A.f1gmap;
    states = A.f1gst;
  } else {
    g = A.g_beg + (int32_t)uu;
    pd = prob_at(A, prob_of_group(A, g));
    int32_t c0, c1;
    group_chunks(pd, g, c0, c1);
    first = c0;
    nunits = c1 - c0;
    last_map = pd.chunk0 + pd.nchunk - 1;
    maps = A.f1map;
    states = A.f1st;
  }
  const int nsteps = on ? nunits : 0;
  int maxsteps = nsteps;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const int o = __shfl_xor(maxsteps, off, kBlock);
    maxsteps = o > maxsteps ? o : maxsteps;
  }
  auto col = [&](int i) { return t + kQuad * i; };
  {
    const double *w0 = A.f1gst + (int64_t)g * A.sw_f1st;   // the group's entering state (chunk sweep)
#pragma unroll
    for (int i = 0; i < NF; ++i)
      if (col(i) < K) {
        const int q = col(i);
#pragma unroll
        for (int p = 0; p < K1; ++p) sC[qi][p][q] = (!GROUPS && on) ? w0[p * K1 + q] : 0.0;
        sg[qi][q] = (!GROUPS && on) ? w0[KK + q] : 0.0;
      }
  }
#pragma unroll 1
  for (int st = 0; st < maxsteps; ++st) {
    const bool act = st < nsteps;   // uniform over the quad
    const int32_t u = first + (act ? st : 0);
    __syncthreads();   // the state of every lane is in LDS
    if (act) {   // store the state entering item u
      double *w = states + (int64_t)u * A.sw_f1st;
#pragma unroll
      for (int i = 0; i < NF; ++i)
        if (col(i) < K) {
          const int q = col(i);
#pragma unroll
          for (int p = 0; p < K1; ++p) w[p * K1 + q] = sC[qi][p][q];
          w[KK + q] = sg[qi][q];
        }
    }
    const bool app = act && u < last_map;
    const double *m = maps + (int64_t)(app ? u : first) * A.sw_f1map;
    double R[K1][K1], tv[K1][1], Y[K1][NF];
#pragma unroll
    for (int p = 0; p < K1; ++p) {
#pragma unroll
      for (int q = 0; q < K1; ++q) R[p][q] = app ? m[p * K1 + q] - sC[qi][p][q] : (p == q ? 1.0 : 0.0);
      tv[p][0] = app ? m[3 * KK + p] - sg[qi][p] : 0.0;
    }
    chol_small<K>(R);
    trsm_small<K, 1>(R, tv);
#pragma unroll
    for (int i = 0; i < NF; ++i) {
      const int q = col(i) < K ? col(i) : 0;
      double y[K1][1];
#pragma unroll
      for (int p = 0; p < K1; ++p) y[p][0] = app ? m[KK + q * K1 + p] : 0.0;   // B^T, column q
      trsm_small<K, 1>(R, y);
#pragma unroll
      for (int p = 0; p < K1; ++p) Y[p][i] = y[p][0];
    }
#pragma unroll
    for (int i = 0; i < NF; ++i)
      if (col(i) < K)
#pragma unroll
        for (int p = 0; p < K1; ++p) sY[qi][p][col(i)] = Y[p][i];
    __syncthreads();   // Y complete; every read of the state is done
    if (app) {
#pragma unroll
      for (int i = 0; i < NF; ++i)
        if (col(i) < K) {
          double acc = m[3 * KK + K1 + col(i)];
#pragma unroll
          for (int f = 0; f < K; ++f) acc -= Y[f][i] * tv[f][0];
          sg[qi][col(i)] = acc;
        }
#pragma unroll
      for (int p = 0; p < K; ++p) {
        double c[NF];
#pragma unroll
        for (int i = 0; i < NF; ++i) c[i] = m[2 * KK + p * K1 + (col(i) < K ? col(i) : 0)];
#pragma unroll
        for (int f = 0; f < K; ++f) {
          const double yfp = sY[qi][f][p];
#pragma unroll
          for (int i = 0; i < NF; ++i) c[i] += yfp * Y[f][i];
        }
#pragma unroll
        for (int i = 0; i < NF; ++i)
          if (col(i) < K) sC[qi][p][col(i)] = c[i];
      }
    }
    __syncthreads();   // every read of Y is done
  }
}

template <int K, bool DESC, bool GROUPS>
__global__ void __launch_bounds__(kBlock) k_lin_sweep_q(const Args A, int64_t count) {
  constexpr int K1 = Dim<K>::K1, NF = (K + kQuad - 1) / kQuad;
  constexpr int NQ = kBlock / kQuad;
  __shared__ double sS[NQ][K1][K1], sP[NQ][K1][K1];
  const int t = threadIdx.x & (kQuad - 1), qi = threadIdx.x / kQuad;
  const int64_t ui = (int64_t)blockIdx.x * NQ + qi;
  const bool on = ui < count;
  const int64_t uu = on ? ui : count - 1;
  ProbDesc pd;
  int32_t first, nunits;
  int32_t g = 0;
  if (GROUPS) {
    pd = prob_at(A, A.p_beg + (int32_t)uu);
    first = pd.group0;
    nunits = pd.ngroup;
  } else {
    g = A.g_beg + (int32_t)uu;
    pd = prob_at(A, prob_of_group(A, g));
    int32_t c0, c1;
    group_chunks(pd, g, c0, c1);
    first = c0;
    nunits = c1 - c0;
  }
  const int nsteps = on ? nunits : 0;
  int maxsteps = nsteps;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const int o = __shfl_xor(maxsteps, off, kBlock);
    maxsteps = o > maxsteps ? o : maxsteps;
  }
  auto col = [&](int i) { return t + kQuad * i; };
  double v[K1];
  {
    const double *w0 = A.lgst + (int64_t)g * A.sw_lin;   // the group's entering state (chunk sweep)
#pragma unroll
    for (int p = 0; p < K1; ++p) v[p] = (!GROUPS && on) ? w0[K1 * K1 + p] : 0.0;
#pragma unroll
    for (int i = 0; i < NF; ++i)
      if (col(i) < K)
#pragma unroll
        for (int p = 0; p < K1; ++p) sS[qi][p][col(i)] = (!GROUPS && on) ? w0[p * K1 + col(i)] : 0.0;
  }
#pragma unroll 1
  for (int st = 0; st < maxsteps; ++st) {
    const bool act = st < nsteps;   // uniform over the quad
    const int32_t u = act ? (DESC ? first + nunits - 1 - st : first + st) : first;
    const bool app = act && (!GROUPS || st + 1 < nunits);
    const double *Pw = (GROUPS ? A.Pg : A.Pc) + (int64_t)u * A.sw_mat;
    const double *mw = (GROUPS ? A.lgmap : A.lmap) + (int64_t)u * A.sw_lin;
    double *sw = (GROUPS ? A.lgst : A.lst) + (int64_t)u * A.sw_lin;
#pragma unroll
    for (int i = 0; i < NF; ++i)
      if (col(i) < K)
#pragma unroll
        for (int p = 0; p < K1; ++p) sP[qi][p][col(i)] = app ? Pw[p * K1 + col(i)] : 0.0;
    __syncthreads();   // P and the state of every lane are in LDS
    if (act) {   // store the state entering item u
#pragma unroll
      for (int i = 0; i < NF; ++i)
        if (col(i) < K)
#pragma unroll
          for (int p = 0; p < K1; ++p) sw[p * K1 + col(i)] = sS[qi][p][col(i)];
      if (t == 0)
#pragma unroll
        for (int p = 0; p < K1; ++p) sw[K1 * K1 + p] = v[p];
    }
    double vn[K1], W[K1][NF];
    if (app) {
#pragma unroll
      for (int p = 0; p < K; ++p) {
        double acc = mw[K1 * K1 + p];
#pragma unroll
        for (int q = 0; q < K; ++q) acc += (DESC ? sP[qi][q][p] : sP[qi][p][q]) * v[q];
        vn[p] = acc;
      }
#pragma unroll
      for (int p = 0; p < K; ++p) {
        double w[NF];
#pragma unroll
        for (int i = 0; i < NF; ++i) w[i] = 0.0;
#pragma unroll
        for (int r = 0; r < K; ++r) {
          const double s_pr = sS[qi][p][r];
#pragma unroll
          for (int i = 0; i < NF; ++i) {
            const int q = col(i) < K ? col(i) : 0;
            w[i] += s_pr * (DESC ? sP[qi][r][q] : sP[qi][q][r]);
          }
        }
#pragma unroll
        for (int i = 0; i < NF; ++i) W[p][i] = w[i];
      }
    }
    __syncthreads();   // every read of the state is done
    if (app) {
#pragma unroll
      for (int p = 0; p < K; ++p) v[p] = vn[p];
#pragma unroll
      for (int p = 0; p < K; ++p) {
        double acc[NF];
#pragma unroll
        for (int i = 0; i < NF; ++i) acc[i] = mw[p * K1 + (col(i) < K ? col(i) : 0)];
#pragma unroll
        for (int r = 0; r < K; ++r) {
          const double pr = DESC ? sP[qi][r][p] : sP[qi][p][r];
#pragma unroll
          for (int i = 0; i < NF; ++i) acc[i] += pr * W[r][i];
        }
#pragma unroll
        for (int i = 0; i < NF; ++i)
          if (col(i) < K) sS[qi][p][col(i)] = acc[i];
      }
    }
    __syncthreads();   // every read of P is done
  }
}

// F1: the last chunk of a problem has no map (nothing follows it), so neither
// does the last group; they are never read.
template <int K> __global__ void __launch_bounds__(kBlock) k_f1_gscan(const Args A, int64_t) {
  __shared__ double buf[kXch * kBlock];
  const int32_t g = A.g_beg + (int32_t)blockIdx.x;
  const ProbDesc &pd = prob_at(A, prob_of_group(A, g));
  int32_t c0, c1;
  group_chunks(pd, g, c0, c1);
  const int32_t cend = pd.chunk0 + pd.nchunk;
  const int n = (c1 == cend ? c1 - 1 : c1) - c0;   // chunks with a map
  const int q = threadIdx.x;
  const int32_t c = c0 + q;
  F1Map<K> cur;
  if (q < n) f1_load_map<K>(A.f1map + (int64_t)c * A.sw_f1map, cur);
  auto comp = [](F1Map<K> &a, const F1Map<K> &b) {
    F1Map<K> o;
    f1_compose<K>(a, b, o);
    a = o;
  };
  wave_scan(cur, n, buf, comp);
  F1Map<K> prev;
  wave_xch(Flat<F1Map<K>>::of(cur), Flat<F1Map<K>>::of(prev), q >= 1 ? q - 1 : 0, buf);
  if (q >= 1 && q < c1 - c0) f1_store_map<K>(A.f1map + (int64_t)c * A.sw_f1map, prev);
  if (q == n - 1 && c1 < cend) f1_store_map<K>(A.f1gmap + (int64_t)g * A.sw_f1map, cur);
}

template <int K> __global__ void __launch_bounds__(kBlock) k_f1_pscan(const Args A, int64_t) {
  __shared__ double buf[kXch * kBlock];
  const ProbDesc &pd = prob_at(A, A.p_beg + (int32_t)blockIdx.x);
  const int ng = pd.ngroup, n = ng - 1, q = threadIdx.x;   // the last group has no map
  const int32_t g = pd.group0 + q;
  F1Map<K> cur;
  if (q < n) f1_load_map<K>(A.f1gmap + (int64_t)g * A.sw_f1map, cur);
  auto comp = [](F1Map<K> &a, const F1Map<K> &b) {
    F1Map<K> o;
    f1_compose<K>(a, b, o);
    a = o;
  };
  wave_scan(cur, n, buf, comp);
  F1Map<K> prev;
  wave_xch(Flat<F1Map<K>>::of(cur), Flat<F1Map<K>>::of(prev), q >= 1 ? q - 1 : 0, buf);
  if (q < ng) {
    F1State<K> z, st;
    f1_zero_state<K>(z);
    if (q == 0) st = z;
    else f1_apply<K>(prev, z, st);
    f1_store_state<K>(A.f1gst + (int64_t)g * A.sw_f1st, st);
  }
}

template <int K> __global__ void __launch_bounds__(kBlock) k_f1_capply(const Args A, int64_t) {
  const int32_t g = A.g_beg + (int32_t)blockIdx.x;
  const ProbDesc &pd = prob_at(A, prob_of_group(A, g));
  int32_t c0, c1;
  group_chunks(pd, g, c0, c1);
  const int q = threadIdx.x;
  if (q >= c1 - c0) return;
  const int32_t c = c0 + q;
  F1State<K> st, t;
  f1_load_state<K>(A.f1gst + (int64_t)g * A.sw_f1st, st);
  if (q >= 1) {
    F1Map<K> m;
    f1_load_map<K>(A.f1map + (int64_t)c * A.sw_f1map, m);
    f1_apply<K>(m, st, t);
    st = t;
  }
  f1_store_state<K>(A.f1st + (int64_t)c * A.sw_f1st, st);
}

template <typename T> struct Launch {
  const Args &a;
  int64_t count;
  hipStream_t s;
  template <class Item> int go() {
    if (count <= 0) return 0;
    int64_t grid = (count + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_item<Item>, dim3((unsigned)grid), dim3(kBlock), 0, s, a, count);
    return hipGetLastError() == hipSuccess ? 0 : -2;
  }
};

inline int hip_ok() { return hipGetLastError() == hipSuccess ? 0 : -2; }

// The LDS-tiled kernels of one step; IL: the variants that keep L, Sigma,
// Lbar, z and the copy of ybar interleaved (Args::il, FP64).
template <typename T, bool IL>
int run_tiled(int step, const Args &a, int64_t count, hipStream_t s, dim3 grid, dim3 block) {
  constexpr int K = BO_K;
  switch (step) {
    case ST_F1_GSWEEP:
    case ST_F1_CSWEEP:
    case ST_ASC_GSWEEP:
    case ST_ASC_CSWEEP:
    case ST_DESC_GSWEEP:
    case ST_DESC_CSWEEP:
      if constexpr (K >= 10) {   // a quad per problem or group
        const dim3 qgrid((unsigned)((count * kQuad + kBlock - 1) / kBlock));
        switch (step) {
          case ST_F1_GSWEEP: hipLaunchKernelGGL((k_f1_sweep_q<K, true>), qgrid, block, 0, s, a, count); break;
          case ST_F1_CSWEEP: hipLaunchKernelGGL((k_f1_sweep_q<K, false>), qgrid, block, 0, s, a, count); break;
          case ST_ASC_GSWEEP: hipLaunchKernelGGL((k_lin_sweep_q<K, false, true>), qgrid, block, 0, s, a, count); break;
          case ST_ASC_CSWEEP: hipLaunchKernelGGL((k_lin_sweep_q<K, false, false>), qgrid, block, 0, s, a, count); break;
          case ST_DESC_GSWEEP: hipLaunchKernelGGL((k_lin_sweep_q<K, true, true>), qgrid, block, 0, s, a, count); break;
          default: hipLaunchKernelGGL((k_lin_sweep_q<K, true, false>), qgrid, block, 0, s, a, count); break;
        }
      } else {
        Launch<T> l{a, count, s};
        return with_item<K, T>(step, l);
      }
      break;
    case ST_ASC_GCOMP:
    case ST_DESC_GCOMP:
      if constexpr (K >= 10) {   // a quad per group (the maps spill from one lane)
        const dim3 qgrid((unsigned)((count * kQuad + kBlock - 1) / kBlock));
        if (step == ST_DESC_GCOMP) hipLaunchKernelGGL((k_lin_gcomp_q<K, true>), qgrid, block, 0, s, a, count);
        else hipLaunchKernelGGL((k_lin_gcomp_q<K, false>), qgrid, block, 0, s, a, count);
      } else {
        Launch<T> l{a, count, s};
        return with_item<K, T>(step, l);
      }
      break;
    case ST_F1_GCOMP:
      if constexpr (K >= 10) {   // a quad per group (the maps spill from one lane)
        const dim3 qgrid((unsigned)((count * kQuad + kBlock - 1) / kBlock));
        hipLaunchKernelGGL((k_f1_gcomp_q<K>), qgrid, block, 0, s, a, count);
      } else {
        Launch<T> l{a, count, s};
        return with_item<K, T>(step, l);
      }
      break;
    case ST_F1_SUM:
      if constexpr (K >= 10) {   // a quad per chunk (the state spills from one lane)
        const dim3 qgrid((unsigned)((count * kQuad + kBlock - 1) / kBlock));
        if (a.qdn) hipLaunchKernelGGL((k_f1_sum_q<K, T, true>), qgrid, block, 0, s, a, count);
        else hipLaunchKernelGGL((k_f1_sum_q<K, T, false>), qgrid, block, 0, s, a, count);
      } else {
        if (a.qdn) hipLaunchKernelGGL((k_f1_sum<K, T, true>), grid, block, 0, s, a, count);
        else hipLaunchKernelGGL((k_f1_sum<K, T, false>), grid, block, 0, s, a, count);
      }
      break;
    case ST_F1_REP:
      if (a.qdn) {
        if constexpr (IL) return -4;   // kept intermediates come with no diagonal addend
        else if (a.Pc) hipLaunchKernelGGL((k_f1_rep<K, T, true, true, false>), grid, block, 0, s, a, count);
        else hipLaunchKernelGGL((k_f1_rep<K, T, true, false, false>), grid, block, 0, s, a, count);
      } else {
        if (a.Pc) hipLaunchKernelGGL((k_f1_rep<K, T, false, true, IL>), grid, block, 0, s, a, count);
        else hipLaunchKernelGGL((k_f1_rep<K, T, false, false, IL>), grid, block, 0, s, a, count);
      }
      break;
    case ST_PC: hipLaunchKernelGGL((k_pc<K, T, IL>), grid, block, 0, s, a, count); break;
    case ST_FS_SUM:
      if constexpr (IL) return -4;
      else hipLaunchKernelGGL((k_fs<K, T, false, false>), grid, block, 0, s, a, count);
      break;
    case ST_FS_REP:
      if constexpr (IL) {
        return -4;
      } else {
        if constexpr (K <= KMAX_FUSED)
          if (a.lmap_out) {
            hipLaunchKernelGGL((k_fs<K, T, true, true>), grid, block, 0, s, a, count);
            break;
          }
        hipLaunchKernelGGL((k_fs<K, T, true, false>), grid, block, 0, s, a, count);
      }
      break;
    case ST_F2_SUM: hipLaunchKernelGGL((k_f2<K, T, false, false, IL>), grid, block, 0, s, a, count); break;
    case ST_F2_REP:
      if constexpr (K <= KMAX_FUSED)
        if (a.lmap_out && a.Sb) {
          hipLaunchKernelGGL((k_f2<K, T, true, true, IL>), grid, block, 0, s, a, count);
          break;
        }
      hipLaunchKernelGGL((k_f2<K, T, true, false, IL>), grid, block, 0, s, a, count);
      break;
    case ST_B1_SUM: hipLaunchKernelGGL((k_b1<K, T, false, false, IL>), grid, block, 0, s, a, count); break;
    case ST_B1_REP:
      if constexpr (K <= KMAX_FUSED)
        if (a.lmap_out) {
          hipLaunchKernelGGL((k_b1<K, T, true, true, IL>), grid, block, 0, s, a, count);
          break;
        }
      hipLaunchKernelGGL((k_b1<K, T, true, false, IL>), grid, block, 0, s, a, count);
      break;
    case ST_B2_SUM:
      if (a.Lb)
        hipLaunchKernelGGL((k_b2<K, T, false, true, IL>), grid, block, 0, s, a, count);
      else
        hipLaunchKernelGGL((k_b2<K, T, false, false, IL>), grid, block, 0, s, a, count);
      break;
    case ST_B2_REP:
      if (a.Lb)
        hipLaunchKernelGGL((k_b2<K, T, true, true, IL>), grid, block, 0, s, a, count);
      else
        hipLaunchKernelGGL((k_b2<K, T, true, false, IL>), grid, block, 0, s, a, count);
      break;
    default: {   // the serial scan items (they read no band or vector)
      Launch<T> l{a, count, s};
      return with_item<K, T>(step, l);
    }
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T> int run_step(int step, const Args &a, int64_t count, hipStream_t s) {
  if (count <= 0) return 0;
  const dim3 grid((unsigned)((count + kBlock - 1) / kBlock)), block(kBlock);
  constexpr int K = BO_K;
  // LDS-tiled streaming needs packed records (plans always are); other
  // strides run the per-lane items.
  const bool packed = a.probs != nullptr || a.one.ld == K + 1;
  // Scans: one wavefront per group or problem (groups hold at most 64 chunks,
  // problems at most 64 groups, when the plan's group size is at most 64).
  // Above K = 6 the maps spill in both forms; measured on gfx950 the
  // wavefront scans still win at K = 9 (a 16-problem batch of 10^6 rows:
  // 12 ms of scans down to 4.5) and lose at K = 11 (5 KB of scratch per
  // lane), so K = 10 and up run on quads of lanes (run_tiled), or as serial
  // work items for records with a padded stride.
  if (K <= 9 && a.G <= kBlock) {
    const dim3 wg((unsigned)count);
    switch (step) {
      case ST_F1_GCOMP: hipLaunchKernelGGL((k_f1_gscan<K>), wg, block, 0, s, a, count); return hip_ok();
      case ST_F1_GSWEEP: hipLaunchKernelGGL((k_f1_pscan<K>), wg, block, 0, s, a, count); return hip_ok();
      case ST_F1_CSWEEP: hipLaunchKernelGGL((k_f1_capply<K>), wg, block, 0, s, a, count); return hip_ok();
      case ST_ASC_GCOMP: hipLaunchKernelGGL((k_lin_gscan<K, false>), wg, block, 0, s, a, count); return hip_ok();
      case ST_ASC_GSWEEP: hipLaunchKernelGGL((k_lin_pscan<K, false>), wg, block, 0, s, a, count); return hip_ok();
      case ST_ASC_CSWEEP: hipLaunchKernelGGL((k_lin_capply<K, false>), wg, block, 0, s, a, count); return hip_ok();
      case ST_DESC_GCOMP: hipLaunchKernelGGL((k_lin_gscan<K, true>), wg, block, 0, s, a, count); return hip_ok();
      case ST_DESC_GSWEEP: hipLaunchKernelGGL((k_lin_pscan<K, true>), wg, block, 0, s, a, count); return hip_ok();
      case ST_DESC_CSWEEP: hipLaunchKernelGGL((k_lin_capply<K, true>), wg, block, 0, s, a, count); return hip_ok();
      default: break;
    }
  }
  if (!packed) {
    Launch<T> l{a, count, s};
    return with_item<K, T>(step, l);
  }
  if constexpr (sizeof(T) == 8)
    if (a.il) return run_tiled<T, true>(step, a, count, s, grid, block);
  return run_tiled<T, false>(step, a, count, s, grid, block);
}

}  // namespace

// Runs `count` items of `step` for bandwidth BO_K; prec 0 = FP64 storage,
// 1 = FP32 storage with FP64 diagonals.
extern "C" int BO_CAT(bo_step_k, BO_K)(int step, int prec, const bo::Args *a, int64_t count,
                                        hipStream_t s) {
  if (prec == 0) return run_step<double>(step, *a, count, s);
  return run_step<float>(step, *a, count, s);
}
