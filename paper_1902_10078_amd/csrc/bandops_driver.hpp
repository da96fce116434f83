// bandops_driver.hpp -- schedules and launch sequences of the banded passes.
//
// A schedule cuts every problem of a call into chunks of `clen` rows and the
// chunks into groups of G; problems are ordered by bandwidth so that the
// problems, chunks and groups sharing one bandwidth form contiguous ranges (one
// launch per bandwidth and step).  The launch sequences below are written
// against an abstract backend, `be.step(step, K, prec, args, count)`, which
// runs `count` work items of one kind; the library's backend launches one GPU
// lane per item.
#pragma once
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <vector>

#include "bandops_items.hpp"

namespace bo {

enum Step : int {
  ST_F1_SUM = 0, ST_F1_GCOMP, ST_F1_GSWEEP, ST_F1_CSWEEP, ST_F1_REP, ST_PC,
  ST_FS_SUM, ST_FS_REP, ST_F2_SUM, ST_F2_REP, ST_B1_SUM, ST_B1_REP, ST_B2_SUM, ST_B2_REP,
  ST_ASC_GCOMP, ST_ASC_GSWEEP, ST_ASC_CSWEEP, ST_DESC_GCOMP, ST_DESC_GSWEEP, ST_DESC_CSWEEP,
  ST_COUNT
};

// Bandwidths with compiled kernels.
constexpr int KMAX_SUPPORTED = 12;

struct KRange {
  int K;
  int32_t c_beg, c_cnt, g_beg, g_cnt, p_beg, p_cnt;
  int32_t max_nchunk;   // largest chunk count of a problem in the range
  int32_t il_rows;      // interleaved slot rows per lane: longest chunk + K + 1
  int64_t il_off;       // element offset of the range in each interleaved band
  int64_t il_voff;      // element offset of the range in each interleaved vector
};

struct Sched {
  std::vector<ProbDesc> probs;      // ordered by bandwidth
  std::vector<int32_t> order;       // probs[i] is the caller's problem order[i]
  std::vector<int32_t> chunk_prob, group_prob;
  std::vector<KRange> ranges;
  int32_t nchunk = 0, ngroup = 0, nprob = 0, G = 64, Kmax = 0;
  // From this bandwidth up, the chunk products of L are a pass of their own
  // after the F1 replay instead of accumulated in it (the replay's state then
  // fits in registers); above the compiled bandwidths: never.
  int32_t kpc_sep = KMAX_SUPPORTED + 1;
  int64_t rows = 0;
  // interleaved intermediates (FP64 elements per array; the arrays follow
  // the workspace proper when a call keeps L, Sigma and Lbar there)
  int64_t il_elems = 0, il_velems = 0;
  // workspace layout (bytes offsets from the workspace base)
  size_t off_tables = 0, off_f1map = 0, off_f1st = 0, off_f1gmap = 0, off_f1gst = 0, off_Pc = 0,
         off_Pg = 0, off_Pex = 0, off_lmap = 0, off_lmap2 = 0, off_lst = 0, off_lgmap = 0, off_lgst = 0, off_part = 0,
         off_out = 0, bytes = 0, off_il = 0, bytes_il = 0;
  int32_t sw_f1map = 1, sw_f1st = 1, sw_mat = 1, sw_lin = 1;
  std::vector<unsigned char> table_blob;   // probs | chunk_prob | group_prob (device image)
};

struct ProbIn {
  int64_t n;
  int32_t k, ld;
  int64_t boff, voff;
};

// Chunk length policy: spread the call's rows over about `target_chunks`
// lanes, keep every non-final chunk at least 2K+2 rows (the F1 summary needs
// K interior rows between its two boundary windows) and `min_len`, and keep
// at most G*G chunks per problem (two-level scan).
inline int64_t chunk_len_for(int64_t n, int k, int64_t rows, int64_t target_chunks, int64_t min_len,
                             int32_t G) {
  int64_t base = (rows + target_chunks - 1) / std::max<int64_t>(target_chunks, 1);
  int64_t c = std::max<int64_t>({base, min_len, 2 * (int64_t)k + 2});
  int64_t cap = (int64_t)G * G;
  if ((n + c - 1) / c > cap) c = (n + cap - 1) / cap;
  return std::max<int64_t>(c, 1);
}

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// kscale (optional, KMAX_SUPPORTED + 1 entries >= 1): the chunks of the
// problems of bandwidth k are kscale[k] times as long, so that bandwidths
// whose chunk maps are expensive to combine (the scans compose K x K maps
// serially above K = 9) get fewer of them.
inline bool build_sched(const ProbIn *in, int nprob, int64_t target_chunks, int64_t min_len, int32_t G,
                        Sched &s, const int32_t *kscale = nullptr) {
  s = Sched();
  s.G = G;
  s.nprob = nprob;
  std::vector<int32_t> ord(nprob);
  for (int i = 0; i < nprob; ++i) ord[i] = i;
  std::stable_sort(ord.begin(), ord.end(), [&](int a, int b) { return in[a].k < in[b].k; });
  for (int i = 0; i < nprob; ++i) s.rows += in[i].n;
  s.order = ord;
  int32_t c = 0, g = 0;
  for (int ii = 0; ii < nprob; ++ii) {
    const ProbIn &p = in[ord[ii]];
    if (p.k < 0 || p.k > KMAX_SUPPORTED || p.n < 0) return false;
    ProbDesc d{};
    d.n = p.n;
    d.k = p.k;
    d.ld = p.ld;
    d.boff = p.boff;
    d.voff = p.voff;
    d.orig = ord[ii];
    d.clen = p.n > 0 ? chunk_len_for(p.n, p.k, s.rows, target_chunks, min_len, G) : 1;
    if (p.n > 0 && kscale && kscale[p.k] > 1) {
      d.clen *= kscale[p.k];
      const int64_t cap = (int64_t)G * G;   // keep the two-level scan's bound
      if ((p.n + d.clen - 1) / d.clen > cap) d.clen = (p.n + cap - 1) / cap;
    }
    d.nchunk = p.n > 0 ? (int32_t)((p.n + d.clen - 1) / d.clen) : 0;
    d.chunk0 = c;
    // Two-level scan: a group's composition takes gsize serial steps and the
    // problem's group sweep ngroup, so the group size is the power of two
    // (up to the first one >= G, with at most G groups) that minimises
    // gsize + ngroup.
    d.gsize = 1;
    {
      int32_t gmax = 1;   // the smallest power of two >= G
      while (gmax < G) gmax *= 2;
      int64_t best = -1;
      for (int32_t gs = 1; gs <= gmax; gs *= 2) {
        const int64_t ng = (d.nchunk + gs - 1) / gs;
        if (ng > G && gs < gmax) continue;
        if (best < 0 || gs + ng < best) {
          best = gs + ng;
          d.gsize = gs;
        }
      }
    }
    d.ngroup = (d.nchunk + d.gsize - 1) / d.gsize;
    d.group0 = g;
    for (int32_t t = 0; t < d.nchunk; ++t) s.chunk_prob.push_back(ii);
    for (int32_t t = 0; t < d.ngroup; ++t) s.group_prob.push_back(ii);
    c += d.nchunk;
    g += d.ngroup;
    s.Kmax = std::max(s.Kmax, p.k);
    s.probs.push_back(d);
  }
  s.nchunk = c;
  s.ngroup = g;
  // bandwidth ranges
  for (int ii = 0; ii < nprob;) {
    int K = s.probs[ii].k;
    int jj = ii;
    KRange r{};
    r.K = K;
    r.p_beg = ii;
    r.c_beg = s.probs[ii].chunk0;
    r.g_beg = s.probs[ii].group0;
    r.max_nchunk = 0;
    int64_t maxclen = 0;
    while (jj < nprob && s.probs[jj].k == K) {
      r.max_nchunk = std::max(r.max_nchunk, s.probs[jj].nchunk);
      if (s.probs[jj].n > 0) maxclen = std::max<int64_t>(maxclen, std::min<int64_t>(s.probs[jj].clen, s.probs[jj].n));
      ++jj;
    }
    r.p_cnt = jj - ii;
    const ProbDesc &last = s.probs[jj - 1];
    r.c_cnt = last.chunk0 + last.nchunk - r.c_beg;
    r.g_cnt = last.group0 + last.ngroup - r.g_beg;
    r.il_rows = (int32_t)(maxclen + K + 1);
    r.il_off = s.il_elems;
    r.il_voff = s.il_velems;
    s.il_elems += (int64_t)((r.c_cnt + 63) / 64) * r.il_rows * 64 * (K + 1);
    s.il_velems += (int64_t)((r.c_cnt + 63) / 64) * r.il_rows * 64;
    s.ranges.push_back(r);
    ii = jj;
  }
  // workspace layout
  int K1 = std::max(s.Kmax, 1);
  s.sw_f1map = 3 * K1 * K1 + 2 * K1;
  s.sw_f1st = K1 * K1 + K1;
  s.sw_mat = K1 * K1;
  s.sw_lin = K1 * K1 + K1;
  size_t tb = sizeof(ProbDesc) * (size_t)nprob;
  size_t tc = sizeof(int32_t) * (size_t)s.nchunk;
  size_t tg = sizeof(int32_t) * (size_t)s.ngroup;
  s.table_blob.assign(align_up(tb) + align_up(tc) + align_up(tg), 0);
  if (nprob) std::memcpy(s.table_blob.data(), s.probs.data(), tb);
  if (s.nchunk) std::memcpy(s.table_blob.data() + align_up(tb), s.chunk_prob.data(), tc);
  if (s.ngroup) std::memcpy(s.table_blob.data() + align_up(tb) + align_up(tc), s.group_prob.data(), tg);
  size_t o = 0;
  s.off_tables = o;
  o += align_up(s.table_blob.size());
  auto take = [&](size_t words) {
    size_t at = o;
    o += align_up(words * sizeof(double));
    return at;
  };
  s.off_f1map = take((size_t)s.nchunk * s.sw_f1map);
  s.off_f1st = take((size_t)s.nchunk * s.sw_f1st);
  s.off_f1gmap = take((size_t)s.ngroup * s.sw_f1map);
  s.off_f1gst = take((size_t)s.ngroup * s.sw_f1st);
  s.off_Pc = take((size_t)s.nchunk * s.sw_mat);
  s.off_Pg = take((size_t)s.ngroup * s.sw_mat);
  s.off_Pex = take((size_t)s.nchunk * s.sw_mat);
  s.off_lmap = take((size_t)s.nchunk * s.sw_lin);
  s.off_lmap2 = take((size_t)s.nchunk * s.sw_lin);
  s.off_lst = take((size_t)s.nchunk * s.sw_lin);
  s.off_lgmap = take((size_t)s.ngroup * s.sw_lin);
  s.off_lgst = take((size_t)s.ngroup * s.sw_lin);
  s.off_part = take((size_t)s.nchunk * 4);
  // scratch per-problem results of a composite call (8 words per problem)
  s.off_out = take((size_t)nprob * 8);
  s.bytes = o;
  s.off_il = o;
  s.bytes_il = o + 3 * align_up((size_t)s.il_elems * sizeof(double)) +
               2 * align_up((size_t)s.il_velems * sizeof(double));
  return true;
}

// Fill the schedule and workspace pointers of the kernel arguments.  `single`
// passes the one problem by value (no device tables needed).
inline void bind_sched(const Sched &s, void *ws, bool single, Args &A) {
  unsigned char *w = (unsigned char *)ws;
  size_t tb = sizeof(ProbDesc) * (size_t)s.nprob, tc = sizeof(int32_t) * (size_t)s.nchunk;
  if (single) {
    A.probs = nullptr;
    A.chunk_prob = nullptr;
    A.group_prob = nullptr;
    A.one = s.probs[0];
  } else {
    A.probs = (const ProbDesc *)(w + s.off_tables);
    A.chunk_prob = (const int32_t *)(w + s.off_tables + align_up(tb));
    A.group_prob = (const int32_t *)(w + s.off_tables + align_up(tb) + align_up(tc));
  }
  A.G = s.G;
  A.sw_f1map = s.sw_f1map;
  A.sw_f1st = s.sw_f1st;
  A.sw_mat = s.sw_mat;
  A.sw_lin = s.sw_lin;
  A.f1map = (double *)(w + s.off_f1map);
  A.f1st = (double *)(w + s.off_f1st);
  A.f1gmap = (double *)(w + s.off_f1gmap);
  A.f1gst = (double *)(w + s.off_f1gst);
  A.Pc = (double *)(w + s.off_Pc);
  A.Pg = (double *)(w + s.off_Pg);
  A.Pex = (double *)(w + s.off_Pex);
  A.lmap = (double *)(w + s.off_lmap);
  A.lmap2 = (double *)(w + s.off_lmap2);
  A.lmap_out = nullptr;
  A.lst = (double *)(w + s.off_lst);
  A.lgmap = (double *)(w + s.off_lgmap);
  A.lgst = (double *)(w + s.off_lgst);
  A.part = (double *)(w + s.off_part);
}

inline void set_range(Args &A, const KRange &r) {
  A.c_beg = r.c_beg;
  A.g_beg = r.g_beg;
  A.p_beg = r.p_beg;
  A.il_rows = r.il_rows;
  A.il_off = r.il_off;
  A.il_voff = r.il_voff;
}

// Point L, S, Lb, z and the copy of x at the interleaved arrays that follow
// the workspace proper (a workspace of s.bytes_il bytes); a caller's z
// becomes the optional second copy of z.
inline void bind_il(const Sched &s, void *ws, Args &A) {
  unsigned char *w = (unsigned char *)ws + s.off_il;
  const size_t one = align_up((size_t)s.il_elems * sizeof(double));
  const size_t vone = align_up((size_t)s.il_velems * sizeof(double));
  A.il = 1;
  A.L = w;
  A.Ld = nullptr;
  A.S = w + one;
  A.Sd = nullptr;
  A.Lb = w + 2 * one;
  A.Lbd = nullptr;
  A.zcopy = A.z;
  A.z = w + 3 * one;
  A.xil = w + 3 * one + vone;
}

// ---------------------------------------------------------------- sequences
// Return codes: 0 ok, otherwise the backend's error.  A backend may restrict
// a sequence to one bandwidth range (be.range_on): the ranges touch disjoint
// problems, chunks and workspace slots, so they can run on separate streams.

template <class BE> int seq_clear(BE &be, const Sched &s, Args A) {
  for (size_t ri = 0; ri < s.ranges.size(); ++ri) {
    const KRange &r = s.ranges[ri];
    if (!be.range_on((int)ri)) continue;
    set_range(A, r);
    if (int e = be.clear(A, r.c_cnt)) return e;
  }
  return 0;
}

// F1: Cholesky + log-determinant (+ forward solve when A.y is set); with
// want_P the chunk products of L for the linear passes that follow.  rep_y,
// when given with A.y and A.z null, is read by the replay alone as the
// right-hand side of the F2 chunk maps it accumulates (A.lmap_out).
template <class BE> int seq_f1(BE &be, const Sched &s, Args A, int prec, bool want_P,
                               const void *rep_y = nullptr) {
  for (size_t ri = 0; ri < s.ranges.size(); ++ri) {
    const KRange &r = s.ranges[ri];
    if (!be.range_on((int)ri)) continue;
    set_range(A, r);
    if (r.K > 0 && r.max_nchunk > 1) {
      if (int e = be.step(ST_F1_SUM, r.K, prec, A, r.c_cnt)) return e;
      if (int e = be.step(ST_F1_GCOMP, r.K, prec, A, r.g_cnt)) return e;
      if (int e = be.step(ST_F1_GSWEEP, r.K, prec, A, r.p_cnt)) return e;
      if (int e = be.step(ST_F1_CSWEEP, r.K, prec, A, r.g_cnt)) return e;
    }
    Args B = A;
    if (!want_P || r.K == 0 || r.max_nchunk <= 1) {
      B.Pc = nullptr;
      B.lmap_out = nullptr;
    }
    if (r.K > KMAX_FUSED) B.lmap_out = nullptr;
    const bool pc_pass = B.Pc && r.K >= s.kpc_sep;
    if (pc_pass) B.Pc = nullptr;
    if (rep_y && B.lmap_out && !A.y && !A.z) B.y = rep_y;
    if (int e = be.step(ST_F1_REP, r.K, prec, B, r.c_cnt)) return e;
    if (pc_pass)
      if (int e = be.step(ST_PC, r.K, prec, A, r.c_cnt)) return e;
  }
  return 0;
}

template <class BE> int seq_pc(BE &be, const Sched &s, Args A, int prec) {
  for (size_t ri = 0; ri < s.ranges.size(); ++ri) {
    const KRange &r = s.ranges[ri];
    if (!be.range_on((int)ri)) continue;
    set_range(A, r);
    if (r.K > 0 && r.max_nchunk > 1)
      if (int e = be.step(ST_PC, r.K, prec, A, r.c_cnt)) return e;
  }
  return 0;
}

// One linear pass: zero-state summaries, the two-level scan, the replay.
template <class BE> int seq_lin(BE &be, const Sched &s, Args A, int prec, int pass,
                                 bool have_maps = false) {
  static const int sum_step[4] = {ST_FS_SUM, ST_F2_SUM, ST_B1_SUM, ST_B2_SUM};
  static const int rep_step[4] = {ST_FS_REP, ST_F2_REP, ST_B1_REP, ST_B2_REP};
  const bool desc = (pass == PASS_F2 || pass == PASS_B2);
  for (size_t ri = 0; ri < s.ranges.size(); ++ri) {
    const KRange &r = s.ranges[ri];
    if (!be.range_on((int)ri)) continue;
    set_range(A, r);
    if (r.K > 0 && r.max_nchunk > 1) {
      if (!have_maps || r.K > KMAX_FUSED)
        if (int e = be.step(sum_step[pass], r.K, prec, A, r.c_cnt)) return e;
      if (int e = be.step(desc ? ST_DESC_GCOMP : ST_ASC_GCOMP, r.K, prec, A, r.g_cnt)) return e;
      if (int e = be.step(desc ? ST_DESC_GSWEEP : ST_ASC_GSWEEP, r.K, prec, A, r.p_cnt)) return e;
      if (int e = be.step(desc ? ST_DESC_CSWEEP : ST_ASC_CSWEEP, r.K, prec, A, r.g_cnt)) return e;
    }
    Args B = A;
    if (r.K == 0 || r.max_nchunk <= 1 || r.K > KMAX_FUSED) B.lmap_out = nullptr;
    if (int e = be.step(rep_step[pass], r.K, prec, B, r.c_cnt)) return e;
  }
  return 0;
}

template <class BE> int seq_finalize(BE &be, const Sched &s, Args A) {
  A.p_beg = 0;
  return be.finalize(A, s.nprob);
}

// ---------------------------------------------------------------- pipelines
// Forward list: L = C(Q), log det, z = L^{-1} y, x = L^{-T} z, Sigma = I(L).
// Any of z (A.z), x (A.x) and Sigma (A.S) may be null; y may be null (then no
// solves).
template <class BE> int pipe_forward(BE &be, const Sched &s, Args A, int prec) {
  if (int e = seq_clear(be, s, A)) return e;
  bool lin = (A.S != nullptr) || (A.x != nullptr && A.y != nullptr);
  Args F1 = A;
  F1.lmap_out = lin ? A.lmap : nullptr;   // F1's replay also summarises F2
  if (int e = seq_f1(be, s, F1, prec, lin)) return e;
  if (lin) {
    Args F2 = A;
    F2.bx = (A.x && A.y) ? A.z : nullptr;
    F2.x = (A.x && A.y) ? A.x : nullptr;
    F2.xscale = 1.0;
    F2.Sb = nullptr;
    if (int e = seq_lin(be, s, F2, prec, PASS_F2, true)) return e;
  }
  return seq_finalize(be, s, A);
}

// loss = log det Q - y^T Q^{-1} y + tr(Q^{-1} S) with its gradients:
//   F1 (up):   L, z, log det, y^T Q^{-1} y
//   F2 (down): Sigma, ybar = -2 L^{-T} z
//   B1 (up):   Lbar from Algorithm 4 with Sigmabar = (S_jj, 2 S_ij), trace
//   B2 (down): Qbar from Algorithm 2 with the log-determinant and solve terms
// A.Sb is the band S; A.L, A.z, A.S, A.Lb, A.x (= ybar) and A.Qb are outputs.
//
// Each replay also produces the next pass's chunk maps (fused summaries), so
// after F1's own summary no pass re-reads its inputs for a summary; the maps
// alternate between the two map buffers.
template <class BE> int pipe_gauss_loss(BE &be, const Sched &s, Args A, int prec, bool fuse = true) {
  double *mapA = A.lmap, *mapB = A.lmap2;
  if (int e = seq_clear(be, s, A)) return e;
  if (!fuse) {   // separate summary kernels (reference schedule)
    if (int e = seq_f1(be, s, A, prec, true)) return e;
    Args F2 = A;
    F2.bx = A.z;
    F2.xscale = -2.0;
    F2.Sb = nullptr;
    if (int e = seq_lin(be, s, F2, prec, PASS_F2)) return e;
    Args B1 = A;
    B1.sb_is_S = 1;
    B1.accumulate = 0;
    if (int e = seq_lin(be, s, B1, prec, PASS_B1)) return e;
    Args B2 = A;
    B2.gl = 1.0;
    B2.yb = A.x;
    B2.zf = A.z;
    if (int e = seq_lin(be, s, B2, prec, PASS_B2)) return e;
    return seq_finalize(be, s, A);
  }
  Args F1 = A;
  F1.lmap_out = mapA;
  if (int e = seq_f1(be, s, F1, prec, true)) return e;
  Args F2 = A;
  F2.bx = A.z;
  F2.xscale = -2.0;
  F2.sb_is_S = 1;
  F2.lmap = mapA;
  F2.lmap_out = mapB;
  if (int e = seq_lin(be, s, F2, prec, PASS_F2, true)) return e;
  Args B1 = A;
  B1.sb_is_S = 1;
  B1.accumulate = 0;
  B1.gl = 1.0;
  B1.yb = A.x;
  B1.zf = A.z;
  B1.lmap = mapB;
  B1.lmap_out = mapA;
  if (int e = seq_lin(be, s, B1, prec, PASS_B1, true)) return e;
  Args B2 = A;
  B2.gl = 1.0;
  B2.yb = A.x;
  B2.zf = A.z;
  B2.lmap = mapA;
  B2.lmap_out = nullptr;
  if (int e = seq_lin(be, s, B2, prec, PASS_B2, true)) return e;
  return seq_finalize(be, s, A);
}

// Linear passes on a given factor L (A.L): the chunk products first.
template <class BE> int pipe_linear(BE &be, const Sched &s, Args A, int prec, int pass) {
  if (int e = seq_clear(be, s, A)) return e;
  if (int e = seq_pc(be, s, A, prec)) return e;
  return seq_lin(be, s, A, prec, pass);
}

}  // namespace bo
