// bandops_wh.hpp -- the whitened GMRF sample of gradient-based MCMC
// (Section 3.2, Algorithm 6) over a batch: L = C(Q), F = S(L^T, v) = L^{-T} v,
// and its reverse mode from a given Fbar (the likelihood's gradient in F,
// which is model-specific and the caller's):
//   vbar = L^{-1} Fbar                       (Table 1, solve row),
//   Lbar = -band(F vbar^T)                  (the same row, for L^T),
//   Qbar = Algorithm 2 applied to Lbar.
// Both directions are sequences of the library's chunked passes:
//   forward:  F1 (Cholesky, log-determinant, chunk products), then the F2
//             pass with right-hand side v and no band output (the back solve);
//   backward: the chunk products of L, the FS pass (vbar), then the B2 pass
//             with no incoming Lbar, no log-determinant term and the solve
//             term -F[j+d] vbar[j] folded into each column of Lbar.
// Summaries are fused into the replay before them (up to the fused bandwidth
// limit): the F1 replay also reads v and accumulates the F2 chunk maps, and
// the FS replay accumulates the B2 chunk maps from each vbar[j] it produces
// and F staged k+1 rows ahead.  Included by the host library.
#pragma once
#include "bandops_driver.hpp"

namespace bo_wh {

template <class BE> int pipe_whiten(BE &be, const bo::Sched &s, bo::Args A, int prec) {
  if (int e = bo::seq_clear(be, s, A)) return e;
  bo::Args F1 = A;
  F1.y = nullptr;
  F1.z = nullptr;
  F1.lmap_out = A.lmap;
  if (int e = bo::seq_f1(be, s, F1, prec, true, A.bx)) return e;
  bo::Args F2 = A;   // A.bx = v, A.x = F
  F2.S = nullptr;
  F2.Sd = nullptr;
  F2.Sb = nullptr;
  F2.xscale = 1.0;
  F2.lmap_out = nullptr;
  if (int e = bo::seq_lin(be, s, F2, prec, bo::PASS_F2, true)) return e;
  return bo::seq_finalize(be, s, A);
}

// A.L: the factor; A.bx = Fbar, A.x = vbar; A.yb = F, A.zf = vbar; A.Qb = Qbar.
// With reuse, the chunk products of L are the ones the forward call's F1
// replay left in the workspace (the linear passes' scans only read them).
template <class BE> int pipe_whiten_bwd(BE &be, const bo::Sched &s, bo::Args A, int prec, bool reuse) {
  A.lmap_out = nullptr;
  A.Lb = nullptr;
  A.Lbd = nullptr;
  A.gl = 0.0;
  A.xscale = 1.0;
  if (int e = bo::seq_clear(be, s, A)) return e;
  if (!reuse)
    if (int e = bo::seq_pc(be, s, A, prec)) return e;
  bo::Args FS = A;   // the FS replay also accumulates the B2 chunk maps
  FS.lmap_out = A.lmap2;
  if (int e = bo::seq_lin(be, s, FS, prec, bo::PASS_FS, false)) return e;
  bo::Args B2 = A;
  B2.lmap = A.lmap2;
  return bo::seq_lin(be, s, B2, prec, bo::PASS_B2, true);
}

}  // namespace bo_wh
