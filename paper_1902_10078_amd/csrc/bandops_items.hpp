// bandops_items.hpp -- work items of the banded-operator kernels.
//
// A work item is what one GPU lane does: one chunk of rows of one problem, one
// group of consecutive chunks, or one problem.  Items decode the schedule
// tables (which problem, which rows), call the per-chunk recurrences of
// bandops_algo.hpp and move summaries and states through the workspace.
// Every kernel of the library is `one lane = one item`.
#pragma once
#include "bandops_step.hpp"

namespace bo {

// One banded problem of a batch.  Chunks of a problem are consecutive global
// chunk ids [chunk0, chunk0 + nchunk); chunk c covers rows
// [(c - chunk0) * clen, min(... + clen, n)).  Groups of G consecutive chunks
// are consecutive global group ids [group0, group0 + ngroup); G = gsize is
// chosen per problem.
struct ProbDesc {
  int64_t n;
  int64_t boff;   // element offset of record 0 in every band array
  int64_t voff;   // element offset of row 0 in every vector
  int64_t clen;   // rows per chunk (the last chunk may be shorter)
  int32_t k, ld;
  int32_t chunk0, nchunk;
  int32_t group0, ngroup;
  int32_t orig;   // index of the problem in the caller's order
  int32_t gsize;  // chunks per group of this problem
};

// Kernel arguments (passed by value to every kernel).
struct Args {
  // ---- schedule
  const ProbDesc *probs;      // device table, or null: single problem `one`
  const int32_t *chunk_prob;  // chunk id -> problem id (batched)
  const int32_t *group_prob;  // group id -> problem id (batched)
  ProbDesc one;
  int32_t c_beg, g_beg, p_beg;  // first chunk / group / problem of this launch
  int32_t G;                    // largest chunks per group (each problem has its own, gsize)
  // workspace slot strides (words)
  int32_t sw_f1map, sw_f1st, sw_mat, sw_lin;
  // ---- data (typed by the item's storage type T)
  const void *Q;  const double *Qd;   // input precision (lower band)
  const void *qdn; const double *qdd; // F1 only: Q_jj + qdn[j] / qdd[problem] (qdn null: none)
  void *L;        double *Ld;         // Cholesky factor (output of F1, input after)
  const void *y;  void *z;            // rhs, forward solve
  const void *bx; void *x;            // back-solve rhs and result
  void *S;        double *Sd;         // subset inverse (output of F2, input of B1)
  const void *Sb; const double *Sbd;  // sensitivity of S (or the band S of the loss)
  void *Lb;       double *Lbd;        // sensitivity of L
  void *Qb;       double *Qbd;        // sensitivity of Q
  const void *yb; const void *zf;     // ybar window and z for the solve term of B2
  double xscale;                      // x <- xscale * L^{-T} b
  double gl;                          // log-determinant sensitivity
  double gl1;                         // B1: gl1 / L_jj added to each Lbar_jj it writes
  int32_t sb_is_S;                    // B1: Sb holds S of tr(Q^{-1} S)
  int32_t accumulate;                 // B1: add into Lb
  // ---- workspace
  double *f1map, *f1st, *f1gmap, *f1gst;  // F1 chunk maps / states, group maps / states
  double *Pc, *Pg;                        // chunk / group products
  double *Pex;                            // exclusive prefix products within a group
  double *lmap, *lst, *lgmap, *lgst;      // linear pass maps / states
  double *lmap2;                          // second map buffer (fused summaries alternate)
  double *lmap_out;                       // replays: where the next pass's chunk maps go (or null)
  double *part;                           // 4 words per chunk: logsum, quad, trace, fail row
  // ---- per-problem outputs
  double *logdet;   // per problem
  double *parts;    // 3 per problem: logdet, y^T Q^{-1} y, tr(Q^{-1} S)
  int32_t *info;    // per problem
  double *loss;     // per problem: logdet - y^T Q^{-1} y + tr(Q^{-1} S) (or null)
  // ---- interleaved intermediates (FP64 tiled kernels only): L, S and Lb
  // point at workspace arrays in which row r of the chunk of lane l of
  // wavefront w of a launch is the record at element
  // il_off + ((w * il_rows + r) * 64 + l) * (K + 1); il_rows is the range's
  // longest chunk + K + 1, the extra rows a halo that holds the next chunk's
  // first K + 1 records of S.
  // With il the vectors z (so also bx and zf) are interleaved the same way
  // (one element per record), and the kernels read ybar from xil, an
  // interleaved copy of x (= ybar) with the same halo, instead of yb.
  int32_t il;
  int32_t il_rows;
  void *sbar_out;   // F2 replay with il: also writes (Sigma_jj, 2 Sigma_ij) here (or null)
  void *xil;        // F2 replay with il: the interleaved copy of x
  void *zcopy;      // F1 replay with il: also writes z here (a caller's vector, or null)
  int64_t il_off;   // element offset of the launch's bandwidth range (bands)
  int64_t il_voff;  // element offset of the launch's bandwidth range (vectors)
};

BO_HD const ProbDesc &prob_at(const Args &a, int32_t p) { return a.probs ? a.probs[p] : a.one; }
BO_HD int32_t prob_of_chunk(const Args &a, int32_t c) { return a.probs ? a.chunk_prob[c] : 0; }
BO_HD int32_t prob_of_group(const Args &a, int32_t g) { return a.probs ? a.group_prob[g] : 0; }

BO_HD void chunk_rows(const ProbDesc &pd, int32_t c, int64_t &a, int64_t &b) {
  a = (int64_t)(c - pd.chunk0) * pd.clen;
  b = a + pd.clen < pd.n ? a + pd.clen : pd.n;
}
BO_HD void group_chunks(const ProbDesc &pd, int32_t g, int32_t &c0, int32_t &c1) {
  const int32_t G = pd.gsize;
  c0 = pd.chunk0 + (g - pd.group0) * G;
  int32_t e = pd.chunk0 + pd.nchunk;
  c1 = c0 + G < e ? c0 + G : e;
}

template <typename T> BO_HD BandP<const T> cband(const void *p, const double *d, const ProbDesc &pd) {
  return BandP<const T>{p ? (const T *)p + pd.boff : nullptr,
                        d ? const_cast<double *>(d) + pd.voff : nullptr, pd.ld};
}
template <typename T> BO_HD BandP<T> band(void *p, double *d, const ProbDesc &pd) {
  return BandP<T>{p ? (T *)p + pd.boff : nullptr, d ? d + pd.voff : nullptr, pd.ld};
}
template <typename T> BO_HD const T *cvec(const void *p, const ProbDesc &pd) {
  return p ? (const T *)p + pd.voff : nullptr;
}
template <typename T> BO_HD T *vec(void *p, const ProbDesc &pd) { return p ? (T *)p + pd.voff : nullptr; }
// Scale of F1's diagonal addend for a problem: 1 / qdd[problem] (0 without one).
BO_HD double qdiag_scale(const Args &A, const ProbDesc &pd) {
  return (A.qdn && A.qdd) ? 1.0 / A.qdd[pd.orig] : 0.0;
}

// ============================================================== F1 items
template <int K, typename T> struct F1Summary {
  static BO_HD void run(const Args &A, int64_t i) {
    int32_t c = A.c_beg + (int32_t)i;
    const ProbDesc &pd = prob_at(A, prob_of_chunk(A, c));
    if (c == pd.chunk0 + pd.nchunk - 1) return;   // the last chunk has no successor
    int64_t a, b;
    chunk_rows(pd, c, a, b);
    F1Map<K> m;
    f1_summary_chunk<K, T>(a, b, pd.n, cband<T>(A.Q, A.Qd, pd), cvec<T>(A.y, pd), m, cvec<T>(A.qdn, pd),
                           qdiag_scale(A, pd));
    f1_store_map<K>(A.f1map + (int64_t)c * A.sw_f1map, m);
  }
};

template <int K> struct F1GroupCompose {
  static BO_HD void run(const Args &A, int64_t i) {
    int32_t g = A.g_beg + (int32_t)i;
    const ProbDesc &pd = prob_at(A, prob_of_group(A, g));
    if (g == pd.group0 + pd.ngroup - 1) return;   // the last group's map is never applied
    int32_t c0, c1;
    group_chunks(pd, g, c0, c1);
    F1Map<K> acc, m, t;
    f1_load_map<K>(A.f1map + (int64_t)c0 * A.sw_f1map, acc);
    for (int32_t c = c0 + 1; c < c1; ++c) {
      f1_load_map<K>(A.f1map + (int64_t)c * A.sw_f1map, m);
      f1_compose<K>(acc, m, t);
      acc = t;
    }
    f1_store_map<K>(A.f1gmap + (int64_t)g * A.sw_f1map, acc);
  }
};

template <int K> struct F1GroupSweep {
  static BO_HD void run(const Args &A, int64_t i) {
    int32_t p = A.p_beg + (int32_t)i;
    const ProbDesc &pd = prob_at(A, p);
    F1State<K> s, t;
    f1_zero_state<K>(s);
    for (int32_t g = pd.group0; g < pd.group0 + pd.ngroup; ++g) {
      f1_store_state<K>(A.f1gst + (int64_t)g * A.sw_f1st, s);
      if (g + 1 < pd.group0 + pd.ngroup) {
        F1Map<K> m;
        f1_load_map<K>(A.f1gmap + (int64_t)g * A.sw_f1map, m);
        f1_apply<K>(m, s, t);
        s = t;
      }
    }
  }
};

template <int K> struct F1ChunkSweep {
  static BO_HD void run(const Args &A, int64_t i) {
    int32_t g = A.g_beg + (int32_t)i;
    const ProbDesc &pd = prob_at(A, prob_of_group(A, g));
    int32_t c0, c1;
    group_chunks(pd, g, c0, c1);
    F1State<K> s, t;
    f1_load_state<K>(A.f1gst + (int64_t)g * A.sw_f1st, s);
    for (int32_t c = c0; c < c1; ++c) {
      f1_store_state<K>(A.f1st + (int64_t)c * A.sw_f1st, s);
      if (c + 1 < pd.chunk0 + pd.nchunk) {
        F1Map<K> m;
        f1_load_map<K>(A.f1map + (int64_t)c * A.sw_f1map, m);
        f1_apply<K>(m, s, t);
        s = t;
      }
    }
  }
};

template <int K, typename T> struct F1Replay {
  static BO_HD void run(const Args &A, int64_t i) {
    int32_t c = A.c_beg + (int32_t)i;
    const ProbDesc &pd = prob_at(A, prob_of_chunk(A, c));
    int64_t a, b;
    chunk_rows(pd, c, a, b);
    F1State<K> s;
    if (pd.nchunk > 1)
      f1_load_state<K>(A.f1st + (int64_t)c * A.sw_f1st, s);
    else
      f1_zero_state<K>(s);
    double ls = 0.0, qs = 0.0;
    LinMap<K> f2m;
    const bool fuse = K <= KMAX_FUSED && A.lmap_out && A.Pc;
    int64_t fail = f1_replay_chunk<K, T>(a, b, pd.n, cband<T>(A.Q, A.Qd, pd), band<T>(A.L, A.Ld, pd),
                                         cvec<T>(A.y, pd), vec<T>(A.z, pd), s,
                                         A.Pc ? A.Pc + (int64_t)c * A.sw_mat : nullptr, ls, qs,
                                         fuse ? &f2m : nullptr, cvec<T>(A.qdn, pd), qdiag_scale(A, pd));
    if (fuse) lin_store<K>(A.lmap_out + (int64_t)c * A.sw_lin, f2m);
    double *pt = A.part + 4 * (int64_t)c;
    pt[0] = ls;
    pt[1] = qs;
    pt[3] = (double)fail;
  }
};

// Chunk product P from a given factor (when F1 did not run in the same call).
template <int K, typename T> struct PcItem {
  static BO_HD void run(const Args &A, int64_t i) {
    int32_t c = A.c_beg + (int32_t)i;
    const ProbDesc &pd = prob_at(A, prob_of_chunk(A, c));
    int64_t a, b;
    chunk_rows(pd, c, a, b);
    pc_chunk<K, T>(a, b, pd.n, cband<T>(A.L, A.Ld, pd), A.Pc + (int64_t)c * A.sw_mat);
  }
};

// ======================================================= linear pass items
enum PassKind { PASS_FS = 0, PASS_F2 = 1, PASS_B1 = 2, PASS_B2 = 3 };

template <int K, typename T, int PASS, bool REPLAY>
BO_HD void run_pass(const Args &A, const ProbDesc &pd, int64_t a, int64_t b, LinMap<K> &st, double &aux,
                    LinMap<K> *next = nullptr) {
  aux = 0.0;
  if (PASS == PASS_FS) {
    fs_chunk<K, T, REPLAY>(a, b, pd.n, cband<T>(A.L, A.Ld, pd), cvec<T>(A.bx, pd), vec<T>(A.x, pd),
                           A.xscale, st, cvec<T>(A.yb, pd), A.gl, next);
  } else if (PASS == PASS_F2) {
    f2_chunk<K, T, REPLAY>(a, b, pd.n, cband<T>(A.L, A.Ld, pd), band<T>(A.S, A.Sd, pd),
                           cvec<T>(A.bx, pd), vec<T>(A.x, pd), A.xscale, st,
                           cband<T>(A.Sb, A.Sbd, pd), A.sb_is_S != 0, next);
  } else if (PASS == PASS_B1) {
    b1_chunk<K, T, REPLAY>(a, b, pd.n, cband<T>(A.L, A.Ld, pd), cband<T>(A.S, A.Sd, pd),
                           cband<T>(A.Sb, A.Sbd, pd), A.sb_is_S != 0, band<T>(A.Lb, A.Lbd, pd),
                           A.accumulate != 0, aux, st, cvec<T>(A.yb, pd), cvec<T>(A.zf, pd), A.gl,
                           next, A.gl1);
  } else {
    b2_chunk<K, T, REPLAY>(a, b, pd.n, cband<T>(A.L, A.Ld, pd), cband<T>(A.Lb, A.Lbd, pd), A.gl,
                           cvec<T>(A.yb, pd), cvec<T>(A.zf, pd), band<T>(A.Qb, A.Qbd, pd), st);
  }
}

template <int K, typename T, int PASS> struct LinSummary {
  static BO_HD void run(const Args &A, int64_t i) {
    int32_t c = A.c_beg + (int32_t)i;
    const ProbDesc &pd = prob_at(A, prob_of_chunk(A, c));
    if (pd.nchunk <= 1) return;
    int64_t a, b;
    chunk_rows(pd, c, a, b);
    LinMap<K> st;
    double aux;
    run_pass<K, T, PASS, false>(A, pd, a, b, st, aux);
    lin_store<K>(A.lmap + (int64_t)c * A.sw_lin, st);
  }
};

template <int K, typename T, int PASS> struct LinReplay {
  static BO_HD void run(const Args &A, int64_t i) {
    int32_t c = A.c_beg + (int32_t)i;
    const ProbDesc &pd = prob_at(A, prob_of_chunk(A, c));
    int64_t a, b;
    chunk_rows(pd, c, a, b);
    LinMap<K> st;
    if (pd.nchunk > 1)
      lin_load<K>(A.lst + (int64_t)c * A.sw_lin, st);
    else
      lin_zero<K>(st);
    double aux;
    LinMap<K> nm;
    const bool fuse = K <= KMAX_FUSED && A.lmap_out && (PASS == PASS_FS || PASS == PASS_F2 || PASS == PASS_B1);
    run_pass<K, T, PASS, true>(A, pd, a, b, st, aux, fuse ? &nm : nullptr);
    if (fuse) lin_store<K>(A.lmap_out + (int64_t)c * A.sw_lin, nm);
    if (PASS == PASS_B1) A.part[4 * (int64_t)c + 2] = aux;
  }
};

// Group map of a linear pass: product and composed (M, v).
template <int K, bool DESC> struct LinGroupCompose {
  static BO_HD void run(const Args &A, int64_t i) {
    constexpr int K1 = Dim<K>::K1;
    int32_t g = A.g_beg + (int32_t)i;
    const ProbDesc &pd = prob_at(A, prob_of_group(A, g));
    int32_t c0, c1;
    group_chunks(pd, g, c0, c1);
    double Gp[K1][K1], P[K1][K1];
    LinMap<K> acc, m;
    lin_zero<K>(acc);
#pragma unroll
    for (int p = 0; p < K1; ++p)
#pragma unroll
      for (int q = 0; q < K1; ++q) Gp[p][q] = (p == q) ? 1.0 : 0.0;
    for (int32_t t = 0; t < c1 - c0; ++t) {
      int32_t c = DESC ? c1 - 1 - t : c0 + t;
      mat_load<K>(A.Pc + (int64_t)c * A.sw_mat, P);
      lin_load<K>(A.lmap + (int64_t)c * A.sw_lin, m);
      lin_apply<K, DESC>(P, m, acc);
      mat_mul_acc<K, DESC>(Gp, P);
    }
    mat_store<K>(A.Pg + (int64_t)g * A.sw_mat, Gp);
    lin_store<K>(A.lgmap + (int64_t)g * A.sw_lin, acc);
  }
};

template <int K, bool DESC> struct LinGroupSweep {
  static BO_HD void run(const Args &A, int64_t i) {
    constexpr int K1 = Dim<K>::K1;
    int32_t p = A.p_beg + (int32_t)i;
    const ProbDesc &pd = prob_at(A, p);
    LinMap<K> s, m;
    double P[K1][K1];
    lin_zero<K>(s);
    for (int32_t t = 0; t < pd.ngroup; ++t) {
      int32_t g = DESC ? pd.group0 + pd.ngroup - 1 - t : pd.group0 + t;
      lin_store<K>(A.lgst + (int64_t)g * A.sw_lin, s);
      if (t + 1 < pd.ngroup) {
        mat_load<K>(A.Pg + (int64_t)g * A.sw_mat, P);
        lin_load<K>(A.lgmap + (int64_t)g * A.sw_lin, m);
        lin_apply<K, DESC>(P, m, s);
      }
    }
  }
};

template <int K, bool DESC> struct LinChunkSweep {
  static BO_HD void run(const Args &A, int64_t i) {
    constexpr int K1 = Dim<K>::K1;
    int32_t g = A.g_beg + (int32_t)i;
    const ProbDesc &pd = prob_at(A, prob_of_group(A, g));
    int32_t c0, c1;
    group_chunks(pd, g, c0, c1);
    LinMap<K> s, m;
    double P[K1][K1];
    lin_load<K>(A.lgst + (int64_t)g * A.sw_lin, s);
    for (int32_t t = 0; t < c1 - c0; ++t) {
      int32_t c = DESC ? c1 - 1 - t : c0 + t;
      lin_store<K>(A.lst + (int64_t)c * A.sw_lin, s);
      mat_load<K>(A.Pc + (int64_t)c * A.sw_mat, P);
      lin_load<K>(A.lmap + (int64_t)c * A.sw_lin, m);
      lin_apply<K, DESC>(P, m, s);
    }
  }
};

// ============================================================ finalize
// Per problem: log det = 2 sum log L_jj (compensated over chunk partials),
// y^T Q^{-1} y, the trace term and info (first failing row + 1, or 0).
struct Finalize {
  static BO_HD void run(const Args &A, int64_t i) {
    int32_t p = A.p_beg + (int32_t)i;
    const ProbDesc &pd = prob_at(A, p);
    double s = 0.0, comp = 0.0, q = 0.0, tr = 0.0;
    int64_t fail = -1;
    for (int32_t c = pd.chunk0; c < pd.chunk0 + pd.nchunk; ++c) {
      const double *pt = A.part + 4 * (int64_t)c;
      double t = pt[0], u = s + t;
      comp += (fabs(s) >= fabs(t)) ? (s - u) + t : (t - u) + s;
      s = u;
      q += pt[1];
      tr += pt[2];
      if (pt[3] >= 0.0 && fail < 0) fail = (int64_t)pt[3];
    }
    double ld = 2.0 * (s + comp);
    int32_t o = pd.orig;
    if (A.logdet) A.logdet[o] = fail >= 0 ? NAN : ld;
    if (A.parts) {
      A.parts[3 * (int64_t)o + 0] = fail >= 0 ? NAN : ld;
      A.parts[3 * (int64_t)o + 1] = q;
      A.parts[3 * (int64_t)o + 2] = tr;
    }
    if (A.info) A.info[o] = fail >= 0 ? (int32_t)(fail + 1) : 0;
  }
};

// Clear the per-chunk partials of a launch range.
struct ClearPart {
  static BO_HD void run(const Args &A, int64_t i) {
    double *pt = A.part + 4 * (A.c_beg + i);
    pt[0] = pt[1] = pt[2] = 0.0;
    pt[3] = -1.0;
  }
};

}  // namespace bo
