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

// ------------------------------------------------------------------- F1
template <int K, typename T>
__global__ void __launch_bounds__(kBlock) k_f1_sum(const Args A, int64_t count) {
  const LaneChunk C = lane_chunk(A, count);
  const ProbDesc &pd = C.pd;
  const bool on = C.active && C.c != pd.chunk0 + pd.nchunk - 1;
  BandP<const T> Q = cband<T>(A.Q, A.Qd, pd);
  const T *y = cvec<T>(A.y, pd);
  F1Map<K> m;
  F1SumStep<K, T> st;
  if (on) st.begin(C.a, pd.n, Q, y, m);
  BandIn<T> bands[1] = {{on ? Q.p : nullptr, on ? Q.diag : nullptr, 0}};
  VecIn<T> vecs[1] = {{on ? y : nullptr, 0}};
  stream_rows<K, T, 1, 1, false>(bands, vecs, on ? C.a + K : 0, on ? C.b : 0, pd.n, pd.ld,
                                 [&](int64_t, const double (&rec)[1][K + 1], const double (&val)[1]) {
                                   st.row(rec[0], val[0]);
                                 });
  if (on) {
    st.end(m);
    f1_store_map<K>(A.f1map + (int64_t)C.c * A.sw_f1map, m);
  }
}

template <int K, typename T>
__global__ void __launch_bounds__(kBlock) k_f1_rep(const Args A, int64_t count) {
  const LaneChunk C = lane_chunk(A, count);
  const ProbDesc &pd = C.pd;
  const bool on = C.active;
  BandP<const T> Q = cband<T>(A.Q, A.Qd, pd);
  const T *y = cvec<T>(A.y, pd);
  F1State<K> s0;
  if (on && pd.nchunk > 1)
    f1_load_state<K>(A.f1st + (int64_t)C.c * A.sw_f1st, s0);
  else
    f1_zero_state<K>(s0);
  F1RepStep<K, T> st;
  const bool fuse = A.lmap_out && A.Pc;
  st.begin(s0, band<T>(A.L, A.Ld, pd), y ? vec<T>(A.z, pd) : nullptr, A.Pc != nullptr, fuse);
  BandIn<T> bands[1] = {{on ? Q.p : nullptr, on ? Q.diag : nullptr, 0}};
  VecIn<T> vecs[1] = {{on ? y : nullptr, 0}};
  stream_rows<K, T, 1, 1, false>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
                                 [&](int64_t j, const double (&rec)[1][K + 1], const double (&val)[1]) {
                                   st.row(j, rec[0], val[0]);
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

template <int K, typename T>
__global__ void __launch_bounds__(kBlock) k_pc(const Args A, int64_t count) {
  const LaneChunk C = lane_chunk(A, count);
  const ProbDesc &pd = C.pd;
  const bool on = C.active;
  BandP<const T> L = cband<T>(A.L, A.Ld, pd);
  PcStep<K> st;
  st.begin();
  BandIn<T> bands[1] = {{on ? L.p : nullptr, on ? L.diag : nullptr, 0}};
  VecIn<T> vecs[1] = {{nullptr, 0}};
  stream_rows<K, T, 1, 0, false>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
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

template <int K, typename T, bool REPLAY>
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
  VecIn<T> vecs[1] = {{on ? cvec<T>(A.bx, pd) : nullptr, 0}};
  stream_rows<K, T, 1, 1, false>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
                                 [&](int64_t j, const double (&rec)[1][K + 1], const double (&val)[1]) {
                                   s.row(j, rec[0], val[0]);
                                 });
  if (on && !REPLAY) {
    s.end(st);
    lin_store<K>(A.lmap + (int64_t)C.c * A.sw_lin, st);
  }
}

// FUSE: the replay also accumulates the B1 pass's chunk maps (needs the
// Sigmabar / S band as a second staged input).
template <int K, typename T, bool REPLAY, bool FUSE>
__global__ void __launch_bounds__(kBlock) k_f2(const Args A, int64_t count) {
  const LaneChunk C = lane_chunk(A, count);
  const ProbDesc &pd = C.pd;
  const bool on = C.active && (REPLAY || pd.nchunk > 1);
  BandP<const T> L = cband<T>(A.L, A.Ld, pd);
  const T *bx = cvec<T>(A.bx, pd);
  LinMap<K> st;
  lin_in<K>(A, C, REPLAY, st);
  F2Step<K, T, REPLAY> s;
  s.begin(st, band<T>(A.S, A.Sd, pd), vec<T>(A.x, pd), A.xscale, A.S != nullptr, bx != nullptr, FUSE,
          A.sb_is_S != 0);
  VecIn<T> vecs[1] = {{on ? bx : nullptr, 0}};
  if constexpr (FUSE) {
    BandP<const T> Sb = cband<T>(A.Sb, A.Sbd, pd);
    BandIn<T> bands[2] = {{on ? L.p : nullptr, on ? L.diag : nullptr, 0},
                          {on ? Sb.p : nullptr, on ? Sb.diag : nullptr, 0}};
    stream_rows<K, T, 2, 1, true>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
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
    BandIn<T> bands[1] = {{on ? L.p : nullptr, on ? L.diag : nullptr, 0}};
    stream_rows<K, T, 1, 1, true>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
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
template <int K, typename T, bool REPLAY, bool FUSE>
__global__ void __launch_bounds__(kBlock) k_b1(const Args A, int64_t count) {
  const LaneChunk C = lane_chunk(A, count);
  const ProbDesc &pd = C.pd;
  const bool on = C.active && (REPLAY || pd.nchunk > 1);
  BandP<const T> L = cband<T>(A.L, A.Ld, pd);
  BandP<const T> Sig = cband<T>(A.S, A.Sd, pd);
  BandP<const T> Sb = cband<T>(A.Sb, A.Sbd, pd);
  LinMap<K> st;
  lin_in<K>(A, C, REPLAY, st);
  B1Step<K, T, REPLAY> s;
  if (on) s.begin(st, C.a, pd.n, Sig, A.sb_is_S != 0, band<T>(A.Lb, A.Lbd, pd), A.accumulate != 0);
  if constexpr (REPLAY) {
    BandIn<T> bands[3] = {{on ? L.p : nullptr, on ? L.diag : nullptr, 0},
                          {on ? Sb.p : nullptr, on ? Sb.diag : nullptr, 0},
                          {on ? Sig.p : nullptr, on ? Sig.diag : nullptr, K + 1}};
    if constexpr (FUSE) {
      const T *yb = cvec<T>(A.yb, pd);
      if (on) s.begin_b2(C.a, pd.n, yb, A.gl);
      VecIn<T> vecs[2] = {{on ? yb : nullptr, K + 1}, {on ? cvec<T>(A.zf, pd) : nullptr, 0}};
      stream_rows<K, T, 3, 2, false>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
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
      stream_rows<K, T, 3, 0, false>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
                                     [&](int64_t j, const double (&rec)[3][K + 1], const double (&)[1]) {
                                       s.row(j, pd.n, rec[0], rec[1], rec[2]);
                                     });
    }
    if (on) A.part[4 * (int64_t)C.c + 2] = s.tr;
  } else {
    BandIn<T> bands[2] = {{on ? L.p : nullptr, on ? L.diag : nullptr, 0},
                          {on ? Sb.p : nullptr, on ? Sb.diag : nullptr, 0}};
    VecIn<T> vecs[1] = {{nullptr, 0}};
    stream_rows<K, T, 2, 0, false>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
                                   [&](int64_t j, const double (&rec)[2][K + 1], const double (&)[1]) {
                                     s.row(j, pd.n, rec[0], rec[1], rec[1]);
                                   });
    if (on) {
      s.end(st);
      lin_store<K>(A.lmap + (int64_t)C.c * A.sw_lin, st);
    }
  }
}

template <int K, typename T, bool REPLAY>
__global__ void __launch_bounds__(kBlock) k_b2(const Args A, int64_t count) {
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
  s.begin(st, C.b, pd.n, on ? yb : nullptr, A.gl, band<T>(A.Qb, A.Qbd, pd));
  BandIn<T> bands[2] = {{on ? L.p : nullptr, on ? L.diag : nullptr, 0},
                        {on ? Lb.p : nullptr, on ? Lb.diag : nullptr, 0}};
  VecIn<T> vecs[2] = {{on ? yb : nullptr, 0}, {on ? zf : nullptr, 0}};
  stream_rows<K, T, 2, 2, true>(bands, vecs, on ? C.a : 0, on ? C.b : 0, pd.n, pd.ld,
                                [&](int64_t j, const double (&rec)[2][K + 1], const double (&val)[2]) {
                                  s.row(j, pd.n, rec[0], rec[1], val[0], val[1]);
                                });
  if (on && !REPLAY) {
    s.end(st);
    lin_store<K>(A.lmap + (int64_t)C.c * A.sw_lin, st);
  }
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

template <typename T> int run_step(int step, const Args &a, int64_t count, hipStream_t s) {
  if (count <= 0) return 0;
  const dim3 grid((unsigned)((count + kBlock - 1) / kBlock)), block(kBlock);
  constexpr int K = BO_K;
  // LDS-tiled streaming needs packed records (plans always are); other
  // strides run the per-lane items.
  const bool packed = a.probs != nullptr || a.one.ld == K + 1;
  switch (packed ? step : -1) {
    case ST_F1_SUM: hipLaunchKernelGGL((k_f1_sum<K, T>), grid, block, 0, s, a, count); break;
    case ST_F1_REP: hipLaunchKernelGGL((k_f1_rep<K, T>), grid, block, 0, s, a, count); break;
    case ST_PC: hipLaunchKernelGGL((k_pc<K, T>), grid, block, 0, s, a, count); break;
    case ST_FS_SUM: hipLaunchKernelGGL((k_fs<K, T, false>), grid, block, 0, s, a, count); break;
    case ST_FS_REP: hipLaunchKernelGGL((k_fs<K, T, true>), grid, block, 0, s, a, count); break;
    case ST_F2_SUM: hipLaunchKernelGGL((k_f2<K, T, false, false>), grid, block, 0, s, a, count); break;
    case ST_F2_REP:
      if (a.lmap_out && a.Sb)
        hipLaunchKernelGGL((k_f2<K, T, true, true>), grid, block, 0, s, a, count);
      else
        hipLaunchKernelGGL((k_f2<K, T, true, false>), grid, block, 0, s, a, count);
      break;
    case ST_B1_SUM: hipLaunchKernelGGL((k_b1<K, T, false, false>), grid, block, 0, s, a, count); break;
    case ST_B1_REP:
      if (a.lmap_out)
        hipLaunchKernelGGL((k_b1<K, T, true, true>), grid, block, 0, s, a, count);
      else
        hipLaunchKernelGGL((k_b1<K, T, true, false>), grid, block, 0, s, a, count);
      break;
    case ST_B2_SUM: hipLaunchKernelGGL((k_b2<K, T, false>), grid, block, 0, s, a, count); break;
    case ST_B2_REP: hipLaunchKernelGGL((k_b2<K, T, true>), grid, block, 0, s, a, count); break;
    default: {
      Launch<T> l{a, count, s};
      return with_item<K, T>(step, l);
    }
    case -1: break;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace

// Runs `count` items of `step` for bandwidth BO_K; prec 0 = FP64 storage,
// 1 = FP32 storage with FP64 diagonals.
extern "C" int BO_CAT(bo_step_k, BO_K)(int step, int prec, const bo::Args *a, int64_t count,
                                        hipStream_t s) {
  if (prec == 0) return run_step<double>(step, *a, count, s);
  return run_step<float>(step, *a, count, s);
}
