// bandops_step.hpp -- the row recurrences of every pass, written as steppers.
//
// A stepper holds a pass's state (the K x K window and/or K-vector of
// bandops_algo.hpp) and advances it by one row given that row's input
// records.  Drivers decide where the inputs come from: the direct drivers at
// the end of this file read global memory row by row; the GPU kernels feed the
// same steppers from LDS tiles filled by wave-cooperative loads.  Outputs are
// written by the stepper itself.
//
// Inputs that lie past the end of the matrix read as zero records.
#pragma once
#include "bandops_algo.hpp"

namespace bo {

// ============================================================ F1 summary
// Interior elimination of a chunk [a,b): rows a..a+K-1 form the boundary F,
// rows a+K..b-1 are eliminated (Cholesky of Q_II) while the coupling of the
// window to F (X), the F-block correction Z = X_F^T X_F, the window
// correction C, and the right-hand side corrections g (window) and e (F) are
// carried along.  See F1Map for the resulting map.
template <int K, typename T> struct F1SumStep {
  static constexpr int K1 = Dim<K>::K1, NS = Dim<K>::NS;
  double C[NS], Z[NS], X[K1][K1], g[K1], e[K1];

  // Boundary rows a..a+K-1: Q_FF, the coupling of rows a+K.. to F, y_F.  With
  // dn, dn[j] * ds is added to each Q_jj.
  BO_HD void begin(int64_t a, int64_t n, BandP<const T> Q, const T *y, F1Map<K> &m,
                   const T *dn = nullptr, double ds = 0.0) {
#pragma unroll
    for (int i = 0; i < NS; ++i) C[i] = Z[i] = 0.0;
#pragma unroll
    for (int p = 0; p < K1; ++p) {
      g[p] = e[p] = 0.0;
#pragma unroll
      for (int f = 0; f < K1; ++f) X[p][f] = 0.0;
    }
#pragma unroll
    for (int f = 0; f < K; ++f) {
      double rec[K + 1];
      load_rec<K, T>(Q.p, Q.diag, Q.ld, a + f, n, rec);
      if (dn) rec[0] += (double)dn[a + f] * ds;
#pragma unroll
      for (int p = f; p < K; ++p) m.A[p][f] = m.A[f][p] = rec[p - f];
#pragma unroll
      for (int p = 0; p <= f; ++p) X[p][f] = rec[K + p - f];   // Q[a+K+p, a+f]
      m.r[f] = y ? (double)y[a + f] : 0.0;
    }
  }

  BO_HD void row(const double (&q)[K + 1], double yi) {
    double s0 = q[0] - (K > 0 ? C[0] : 0.0);
    double lii = s0 > 0.0 ? sqrt(s0) : NAN;
    double inv = 1.0 / lii;
    double l[K1], xf[K1];
#pragma unroll
    for (int p = 0; p < K; ++p) l[p] = ((p + 1 < K) ? q[p + 1] - C[six(p + 1, 0)] : q[K]) * inv;
#pragma unroll
    for (int f = 0; f < K; ++f) xf[f] = X[0][f] * inv;
    double zt = (yi - (K > 0 ? g[0] : 0.0)) * inv;
#pragma unroll
    for (int f = 0; f < K; ++f) {
      e[f] += xf[f] * zt;
#pragma unroll
      for (int h = 0; h <= f; ++h) Z[six(f, h)] += xf[f] * xf[h];
    }
#pragma unroll
    for (int p = 0; p < K; ++p) {
#pragma unroll
      for (int f = 0; f < K; ++f) X[p][f] = ((p + 1 < K) ? X[p + 1][f] : 0.0) - l[p] * xf[f];
      g[p] = ((p + 1 < K) ? g[p + 1] : 0.0) + l[p] * zt;
    }
#pragma unroll
    for (int p = 0; p < K; ++p)
#pragma unroll
      for (int h = 0; h <= p; ++h)
        C[six(p, h)] = ((p + 1 < K) ? C[six(p + 1, h + 1)] : 0.0) + l[p] * l[h];
  }

  BO_HD void end(F1Map<K> &m) const {
#pragma unroll
    for (int p = 0; p < K; ++p) {
#pragma unroll
      for (int f = 0; f < K; ++f) {
        m.A[p][f] -= Z[six(p, f)];
        m.B[p][f] = -X[p][f];
        m.D[p][f] = C[six(p, f)];
      }
      m.r[p] -= e[p];
      m.d[p] = g[p];
    }
  }

  // The same with the map in memory (the layout of f1_store_map): begin_w
  // writes A = Q_FF and r = y_F there at once, so that they are not held
  // across the rows; end_w completes the map in place.
  BO_HD void begin_w(int64_t a, int64_t n, BandP<const T> Q, const T *y, double *w, const T *dn = nullptr,
                     double ds = 0.0) {
    constexpr int KK = K1 * K1;
#pragma unroll
    for (int i = 0; i < NS; ++i) C[i] = Z[i] = 0.0;
#pragma unroll
    for (int p = 0; p < K1; ++p) {
      g[p] = e[p] = 0.0;
#pragma unroll
      for (int f = 0; f < K1; ++f) X[p][f] = 0.0;
    }
#pragma unroll
    for (int f = 0; f < K; ++f) {
      double rec[K + 1];
      load_rec<K, T>(Q.p, Q.diag, Q.ld, a + f, n, rec);
      if (dn) rec[0] += (double)dn[a + f] * ds;
#pragma unroll
      for (int p = f; p < K; ++p) w[p * K1 + f] = w[f * K1 + p] = rec[p - f];
#pragma unroll
      for (int p = 0; p <= f; ++p) X[p][f] = rec[K + p - f];   // Q[a+K+p, a+f]
      w[3 * KK + f] = y ? (double)y[a + f] : 0.0;
    }
  }

  BO_HD void end_w(double *w) const {
    constexpr int KK = K1 * K1;
#pragma unroll
    for (int p = 0; p < K1; ++p) {
#pragma unroll
      for (int f = 0; f < K1; ++f) {
        const bool in = p < K && f < K;
        w[p * K1 + f] = in ? w[p * K1 + f] - Z[six(p, f)] : 0.0;
        w[KK + p * K1 + f] = in ? -X[p][f] : 0.0;
        w[2 * KK + p * K1 + f] = in ? C[six(p, f)] : 0.0;
      }
      w[3 * KK + p] = p < K ? w[3 * KK + p] - e[p] : 0.0;
      w[3 * KK + K1 + p] = p < K ? g[p] : 0.0;
    }
  }
};

// ============================================================= F1 replay
// Rows of the chunk from the exact entering state (C, g): writes L (and z),
// sums log L_jj and z_j^2, records the first non-positive pivot, and (when
// asked) accumulates the chunk product P = Kt_{b-1} ... Kt_a.
// PC: compiled with the chunk-product accumulation (without it the replay
// keeps only C and g in registers; the product then comes from PcStep).
// ZS: the stride of z (64 when it is interleaved in a workspace; then a
// caller's copy z2 may be written too).
template <int K, typename T, bool PC = true, int ZS = 1> struct F1RepStep {
  static constexpr int K1 = Dim<K>::K1, NS = Dim<K>::NS;
  double C[NS], g[K1], Pm[PC ? K1 : 1][PC ? K1 : 1];
  double M2[NS], v2[K1];   // fused summary of the F2 pass (see row())
  double ls, qs;
  int64_t fail;
  bool want_P, want_f2;
  BandP<T> L;
  VecP<T, ZS> z;
  VecP<T> z2;   // optional second copy of z (ZS = 64 only)

  // wantF2 (needs wantP): also accumulate the chunk map of the descending F2
  // pass, M = sum_j R_j^T c_j e0 e0^T R_j and v = sum_j R_j^T e0 b_j / L_jj
  // with R_j = Kt_{j-1} ... Kt_a -- the zero-state run of F2 over the chunk,
  // summed in ascending order.  The back solve's right-hand side b is the
  // forward solve's z when the replay writes z, else the replay's y input
  // itself (a back solve L^{-T} y with no forward solve).
  BO_HD void begin(const F1State<K> &st, BandP<T> L_, VecP<T, ZS> z_, bool wantP, bool wantF2 = false) {
    L = L_;
    z = z_;
    z2 = VecP<T>();
    want_P = PC && wantP;
    want_f2 = K <= KMAX_FUSED && want_P && wantF2;
    ls = qs = 0.0;
    fail = -1;
#pragma unroll
    for (int p = 0; p < K1; ++p) {
      g[p] = st.g[p];
      v2[p] = 0.0;
#pragma unroll
      for (int q = 0; q <= p; ++q) C[six(p, q)] = st.C[p][q];
      if constexpr (PC) {
#pragma unroll
        for (int q = 0; q < K1; ++q) Pm[p][q] = (p == q) ? 1.0 : 0.0;
      }
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) M2[i] = 0.0;
  }

  BO_HD void end_f2(LinMap<K> &m) const {
#pragma unroll
    for (int p = 0; p < K1; ++p) {
      m.v[p] = v2[p];
#pragma unroll
      for (int q = 0; q < K1; ++q) m.M[p][q] = (p < K && q < K) ? M2[six(p, q)] : 0.0;
    }
  }

  BO_HD void row(int64_t j, const double (&q)[K + 1], double yj) {
    if (fail >= 0) return;
    double s0 = q[0] - (K > 0 ? C[0] : 0.0);
    if (!(s0 > 0.0)) {
      fail = j;
      return;
    }
    double Ljj = sqrt(s0), inv = 1.0 / Ljj;
    double rec[K + 1], l[K1];
    rec[0] = Ljj;
#pragma unroll
    for (int p = 0; p < K; ++p) {
      l[p] = ((p + 1 < K) ? q[p + 1] - C[six(p + 1, 0)] : q[K]) * inv;
      rec[p + 1] = l[p];
    }
    store_rec<K, T>(L.p, L.diag, L.ld, j, rec);
    ls += log(Ljj);
    double zj = 0.0;
    if (z) {
      zj = (yj - (K > 0 ? g[0] : 0.0)) * inv;
      z[j] = (T)zj;
      if constexpr (ZS != 1)
        if (z2) z2[j] = (T)zj;
      qs += zj * zj;
    }
#pragma unroll
    for (int p = 0; p < K; ++p) g[p] = ((p + 1 < K) ? g[p + 1] : 0.0) + l[p] * zj;
#pragma unroll
    for (int p = 0; p < K; ++p)
#pragma unroll
      for (int h = 0; h <= p; ++h)
        C[six(p, h)] = ((p + 1 < K) ? C[six(p + 1, h + 1)] : 0.0) + l[p] * l[h];
    if (PC && want_P) {
      if (K <= KMAX_FUSED && want_f2) {
        // row 0 of R_j = Pm before this row's update
        const double cj = inv * inv, xj = (z ? zj : yj) * inv;
#pragma unroll
        for (int p = 0; p < K; ++p) {
          v2[p] += Pm[0][p] * xj;
#pragma unroll
          for (int q = 0; q <= p; ++q) M2[six(p, q)] += cj * Pm[0][p] * Pm[0][q];
        }
      }
      // P <- Kt_j P :  row p of Kt P = -u_p P[0,:] + P[p+1,:]
#pragma unroll
      for (int c = 0; c < K; ++c) {
        double p0 = Pm[0][c];
#pragma unroll
        for (int p = 0; p < K; ++p) Pm[p][c] = ((p + 1 < K) ? Pm[p + 1][c] : 0.0) - l[p] * inv * p0;
      }
    }
  }

  BO_HD void end(double *P) const {
    if constexpr (PC) {
      if (!P) return;
#pragma unroll
      for (int p = 0; p < K1; ++p)
#pragma unroll
        for (int q = 0; q < K1; ++q) P[p * K1 + q] = Pm[p][q];
    }
  }
};

// Chunk product P = Kt_{b-1} ... Kt_a of a given factor L.
template <int K> struct PcStep {
  static constexpr int K1 = Dim<K>::K1;
  double Pm[K1][K1];
  BO_HD void begin() {
#pragma unroll
    for (int p = 0; p < K1; ++p)
#pragma unroll
      for (int q = 0; q < K1; ++q) Pm[p][q] = (p == q) ? 1.0 : 0.0;
  }
  BO_HD void row(const double (&r)[K + 1]) {
    double inv = 1.0 / r[0];
#pragma unroll
    for (int c = 0; c < K; ++c) {
      double p0 = Pm[0][c];
#pragma unroll
      for (int p = 0; p < K; ++p) Pm[p][c] = ((p + 1 < K) ? Pm[p + 1][c] : 0.0) - r[p + 1] * inv * p0;
    }
  }
  BO_HD void end(double *P) const {
#pragma unroll
    for (int p = 0; p < K1; ++p)
#pragma unroll
      for (int q = 0; q < K1; ++q) P[p * K1 + q] = Pm[p][q];
  }
};

// ================================================================== FS
// Forward solve z = L^{-1} y with a given factor (ascending).  State
// g_j[p] = sum_{m<j} L[j+p,m] z_m;  g_{j+1} = Kt_j g_j + u_j y_j.
template <int K, typename T, bool REPLAY> struct FsStep {
  static constexpr int K1 = Dim<K>::K1;
  double g[K1];
  T *x;
  double xscale;
  BO_HD void begin(const LinMap<K> &st, T *x_, double xs) {
    x = x_;
    xscale = xs;
#pragma unroll
    for (int p = 0; p < K1; ++p) g[p] = REPLAY ? st.v[p] : 0.0;
  }
  // Returns the value stored at x[j] (xscale z_j, rounded to T).
  BO_HD double row(int64_t j, const double (&r)[K + 1], double yj) {
    double inv = 1.0 / r[0];
    double zj = (yj - (K > 0 ? g[0] : 0.0)) * inv;
    const T xj = (T)(xscale * zj);
    if (REPLAY) x[j] = xj;
#pragma unroll
    for (int p = 0; p < K; ++p) g[p] = ((p + 1 < K) ? g[p + 1] : 0.0) + r[p + 1] * zj;
    return (double)xj;
  }
  BO_HD void end(LinMap<K> &st) const {
#pragma unroll
    for (int p = 0; p < K1; ++p) st.v[p] = g[p];
  }
};

// ================================================================== F2
// Descending: subset inverse (Algorithm 3) and back solve x = L^{-T} b.  The
// state entering row j is the window W = Sigma[j+1..j+K, j+1..j+K] and
// xw = x[j+1..j+K].  Row j:
//   v = -W u_j                       (Sigma[j+1+p, j], Algorithm 3's sums)
//   Sigma_jj = c_j - u_j^T v
//   W' = [[Sigma_jj, v'^T], [v', W[0:K-1,0:K-1]]]   (= Kt^T W Kt + c e0 e0^T)
//   x_j = b_j / L_jj - u_j^T xw,   xw' = (x_j, xw[0:K-1])
// IL: Sigma is kept interleaved in a workspace; the replay then also writes
// the halo of the previous chunk, optionally (Sigma_jj, 2 Sigma_ij) to a
// caller's band and an interleaved copy of x with its halo.
template <int K, typename T, bool REPLAY, bool IL = false> struct F2Step {
  static constexpr int K1 = Dim<K>::K1, NS = Dim<K>::NS;
  double W[NS], xw[K1];
  double Rb[K1][K1], Mb[NS];   // fused summary of the B1 pass (see row_b1())
  double u_[K1];               // u_j of the last row() (row_b1() reuses it)
  BandP<T> S;
  VecP<T> x;
  double xscale;
  bool want_s, want_x, want_b1, sb_is_S;
  // Replays that keep Sigma interleaved also write rows j < jh to Sh, the
  // halo of the previous chunk (the B1 replay reads K + 1 records ahead).
  BandP<T> Sh{nullptr, nullptr, 0};
  int64_t jh = 0;
  // Optional copy of each Sigma record with doubled off-diagonal entries (the
  // sensitivity of tr(Q^{-1} S) with respect to S's stored entries).
  BandP<T> So{nullptr, nullptr, 0};
  // Optional second copy of x (x2) with its own halo view (xh, rows j < jh).
  VecP<T, 64> x2, xh;

  BO_HD void set_halo(BandP<T> h, int64_t j_end) {
    Sh = h;
    jh = j_end;
  }
  BO_HD void set_sym_out(BandP<T> o) { So = o; }
  BO_HD void set_x_copy(VecP<T, 64> c, VecP<T, 64> h, int64_t j_end) {
    x2 = c;
    xh = h;
    jh = j_end;
  }

  // wantB1: also accumulate the chunk map of the ascending B1 pass,
  // M = sum_j R'_j inj_j R'_j^T with R'_j = Kt_{b-1} ... Kt_{j+1} and inj_j
  // the injection of Sigmabar record j (B1Step) -- the zero-state run of B1
  // over the chunk, summed in descending order.
  BO_HD void begin(const LinMap<K> &st, BandP<T> S_, VecP<T> x_, double xs, bool ws, bool wx,
                   bool wantB1 = false, bool sbS = false) {
    S = S_;
    x = x_;
    xscale = xs;
    want_s = ws;
    want_x = wx;
    want_b1 = wantB1;
    sb_is_S = sbS;
#pragma unroll
    for (int p = 0; p < K1; ++p) {
      xw[p] = REPLAY ? st.v[p] : 0.0;
#pragma unroll
      for (int q = 0; q <= p; ++q) W[six(p, q)] = REPLAY ? st.M[p][q] : 0.0;
#pragma unroll
      for (int q = 0; q < K1; ++q) Rb[p][q] = (p == q) ? 1.0 : 0.0;
    }
#pragma unroll
    for (int i = 0; i < NS; ++i) Mb[i] = 0.0;
  }

  BO_HD void end_b1(LinMap<K> &m) const {
#pragma unroll
    for (int p = 0; p < K1; ++p) {
      m.v[p] = 0.0;
#pragma unroll
      for (int q = 0; q < K1; ++q) m.M[p][q] = (p < K && q < K) ? Mb[six(p, q)] : 0.0;
    }
  }

  // sbin = Sigmabar record j (or the band S of the trace term when sb_is_S);
  // called after row() of the same record j, whose u_j it reuses.
  BO_HD void row_b1(const double (&)[K + 1], const double (&sbin)[K + 1]) {
    const double(&u)[K1] = u_;
    double w[K1], w2[K1];
    const double f = sb_is_S ? 2.0 : 1.0;
#pragma unroll
    for (int p = 0; p < K; ++p) {
      double a1 = 0.0, a2 = 0.0;
#pragma unroll
      for (int q = 0; q < K; ++q) {
        a1 += Rb[p][q] * u[q];
        a2 += Rb[p][q] * f * sbin[1 + q];
      }
      w[p] = a1;
      w2[p] = a2;
    }
#pragma unroll
    for (int p = 0; p < K; ++p)
#pragma unroll
      for (int q = 0; q <= p; ++q)
        Mb[six(p, q)] += sbin[0] * w[p] * w[q] - 0.5 * (w2[p] * w[q] + w[p] * w2[q]);
    // R' <- R' Kt_j: column 0 = -R' u, column q = old column q-1
#pragma unroll
    for (int p = 0; p < K; ++p) {
#pragma unroll
      for (int q = K - 1; q >= 1; --q) Rb[p][q] = Rb[p][q - 1];
      Rb[p][0] = -w[p];
    }
  }

  BO_HD void row(int64_t j, const double (&r)[K + 1], double bj) {
    double inv = 1.0 / r[0];
    double(&u)[K1] = u_;
#pragma unroll
    for (int p = 0; p < K; ++p) u[p] = r[p + 1] * inv;
    if (want_s) {
      double v[K1];
      double sjj = inv * inv;
#pragma unroll
      for (int p = 0; p < K; ++p) {
        double acc = 0.0;
#pragma unroll
        for (int q = 0; q < K; ++q) acc -= W[six(p, q)] * u[q];
        v[p] = acc;
        sjj -= u[p] * acc;
      }
      if (REPLAY) {
        double o[K + 1];
        o[0] = sjj;
#pragma unroll
        for (int p = 0; p < K; ++p) o[p + 1] = v[p];
        store_rec<K, T>(S.p, S.diag, S.ld, j, o);
        if constexpr (IL) {
          if (Sh.p && j < jh) store_rec<K, T>(Sh.p, Sh.diag, Sh.ld, j, o);
          if (So.p) {
            double o2[K + 1];
            o2[0] = o[0];
#pragma unroll
            for (int p = 1; p <= K; ++p) o2[p] = 2.0 * o[p];
            store_rec<K, T>(So.p, So.diag, So.ld, j, o2);
          }
        }
      }
#pragma unroll
      for (int p = K - 1; p >= 1; --p)
#pragma unroll
        for (int q = p; q >= 1; --q) W[six(p, q)] = W[six(p - 1, q - 1)];
#pragma unroll
      for (int p = 1; p < K; ++p) W[six(p, 0)] = v[p - 1];
      if (K > 0) W[0] = sjj;
    }
    if (want_x) {
      double xj = bj * inv;
#pragma unroll
      for (int p = 0; p < K; ++p) xj -= u[p] * xw[p];
      if (REPLAY) {
        const T xv = (T)(xscale * xj);
        x[j] = xv;
        if constexpr (IL) {
          if (x2) {
            x2[j] = xv;
            if (xh && j < jh) xh[j] = xv;
          }
        }
      }
#pragma unroll
      for (int p = K - 1; p >= 1; --p) xw[p] = xw[p - 1];
      if (K > 0) xw[0] = xj;
    }
  }

  BO_HD void end(LinMap<K> &st) const {
#pragma unroll
    for (int p = 0; p < K1; ++p) {
      st.v[p] = xw[p];
#pragma unroll
      for (int q = 0; q < K1; ++q) st.M[p][q] = (q < K && p < K) ? W[six(p, q)] : 0.0;
    }
  }
};

// ============================================ B2 chunk maps, accumulated upwards
// Ascending accumulation of the chunk map of the descending B2 pass: the
// zero-state run of B2 over a chunk is M = sum_j R_j^T inj2_j R_j with
// R_j = Kt_{j-1} ... Kt_a and inj2_j the B2 injection of the total
// sensitivity of column j (a given Lbar record, the log-determinant term
// 2 gl / L_jj and the solve term -ybar[j+d] z[j]); yw = ybar[j .. j+K].  A
// replay that visits rows upwards and produces either the Lbar record (B1) or
// z (the forward solve) feeds it one row at a time.
template <int K> struct B2MapAcc {
  static constexpr int K1 = Dim<K>::K1, NS = Dim<K>::NS;
  double Rf[K1][K1], Mf[NS], yw[K + 1], glf;

  template <typename T> BO_HD void begin(int64_t a, int64_t n, const T *ybar, double gl) {
    begin_v<T, 1>(a, n, VecP<const T>(ybar), gl);
  }
  template <typename T, int S> BO_HD void begin_v(int64_t a, int64_t n, VecP<const T, S> ybar, double gl) {
    glf = gl;
#pragma unroll
    for (int p = 0; p < K1; ++p)
#pragma unroll
      for (int q = 0; q < K1; ++q) Rf[p][q] = (p == q) ? 1.0 : 0.0;
#pragma unroll
    for (int i = 0; i < NS; ++i) Mf[i] = 0.0;
#pragma unroll
    for (int d = 0; d <= K; ++d) yw[d] = (ybar && a + d < n) ? (double)ybar[a + d] : 0.0;
  }

  BO_HD void end(LinMap<K> &m) const {
#pragma unroll
    for (int p = 0; p < K1; ++p) {
      m.v[p] = 0.0;
#pragma unroll
      for (int q = 0; q < K1; ++q) m.M[p][q] = (p < K && q < K) ? Mf[six(p, q)] : 0.0;
    }
  }

  // o = Lbar record j (zeros when there is none), r = L record j (inv =
  // 1 / L_jj), zj = z[j], yahead = ybar[j+K+1] (0 past the end).
  BO_HD void row(const double (&r)[K + 1], double inv, const double (&o)[K + 1], double zj, double yahead) {
    double Lt[K + 1];
#pragma unroll
    for (int d = 0; d <= K; ++d) Lt[d] = o[d] - yw[d] * zj;
    Lt[0] += 2.0 * glf * inv;
    double qb[K + 1];
    double dot = 0.0;
#pragma unroll
    for (int p = 0; p < K; ++p) {
      qb[1 + p] = Lt[1 + p] * inv;
      dot += Lt[1 + p] * r[1 + p];
    }
    qb[0] = 0.5 * (Lt[0] - dot * inv) * inv;
    // R^T inj2 R = -(qb0 r0 r0^T + (r0 s^T + s r0^T)/2), r0 = R[0,:],
    // s = sum_{p=1}^{K-1} qb_p R[p,:]
    double sv[K1];
#pragma unroll
    for (int c = 0; c < K; ++c) {
      double acc = 0.0;
#pragma unroll
      for (int p = 1; p < K; ++p) acc += qb[p] * Rf[p][c];
      sv[c] = acc;
    }
#pragma unroll
    for (int p = 0; p < K; ++p)
#pragma unroll
      for (int q = 0; q <= p; ++q)
        Mf[six(p, q)] -= qb[0] * Rf[0][p] * Rf[0][q] + 0.5 * (Rf[0][p] * sv[q] + sv[p] * Rf[0][q]);
    // R <- Kt_j R
#pragma unroll
    for (int c = 0; c < K; ++c) {
      double p0 = Rf[0][c];
#pragma unroll
      for (int p = 0; p < K; ++p) Rf[p][c] = ((p + 1 < K) ? Rf[p + 1][c] : 0.0) - r[p + 1] * inv * p0;
    }
#pragma unroll
    for (int d = 0; d < K; ++d) yw[d] = yw[d + 1];
    yw[K] = yahead;
  }
};

// ================================================================== B1
// Ascending: reverse mode of the subset inverse (Algorithm 4).  The state
// entering row j is Wb, the sensitivity of the window W_j (symmetric, both
// halves counted).  With sb = Sigmabar record j (stored lower entries):
//   Sbjj  = sb_0 + Wb[0][0]
//   vb_p  = sb_{1+p} + 2 Wb[0][1+p]            (vb_{K-1} = sb_K)
//   ub    = -2 Sbjj v - X vb                   (X = Sigma window below j,
//                                               v = Sigma[j+1.., j])
//   Lbar[j+1+p, j] = ub_p / L_jj
//   Lbar_jj        = -2 Sbjj c_j / L_jj - (ub . u) / L_jj
//   Wb'  = shift(Wb) + Sbjj u u^T - (vb u^T + u vb^T)/2   (= Kt Wb Kt^T + ...)
// The replay keeps the K+1 Sigma records j .. j+K in registers (Sg[i] =
// record j+i) and takes record j+K+1 with each row.  With sb_is_S the
// sensitivity is (S_jj, 2 S_{j+1,j}, ...) from the band S of tr(Q^{-1} S), and
// sum_j Sigma_jj S_jj + 2 sum Sigma_ij S_ij is accumulated.  A log-determinant
// term dgl / L_jj can be added to each Lbar_jj as it is written.
template <int K, typename T, bool REPLAY, bool B2MAP = true> struct B1Step {
  static constexpr int K1 = Dim<K>::K1, NS = Dim<K>::NS;
  double Wb[NS];
  double Sg[K + 1][K + 1];
  double tr;
  double dgl;   // log-determinant term dgl / L_jj added to each Lbar_jj
  bool sb_is_S, accumulate;
  BandP<T> Lb;
  // fused summary of the descending B2 pass (B2MapAcc), fed with this pass's
  // Lbar record of each row (compiled in with B2MAP, for K <= KMAX_FUSED).
  bool want_b2;
  B2MapAcc<K> b2;

  template <int S> BO_HD void begin_b2(int64_t a, int64_t n, VecP<const T, S> ybar, double gl) {
    want_b2 = true;
    b2.template begin_v<T, S>(a, n, ybar, gl);
  }
  BO_HD void begin_b2(int64_t a, int64_t n, const T *ybar, double gl) { begin_b2<1>(a, n, VecP<const T>(ybar), gl); }

  BO_HD void end_b2(LinMap<K> &m) const { b2.end(m); }

  // Sigma records a .. a+K are read directly (once per chunk).
  BO_HD void begin(const LinMap<K> &st, int64_t a, int64_t n, BandP<const T> Sig, bool sbS,
                   BandP<T> Lb_, bool acc, double gl1 = 0.0) {
    want_b2 = false;
    sb_is_S = sbS;
    accumulate = acc;
    dgl = gl1;
    Lb = Lb_;
    tr = 0.0;
#pragma unroll
    for (int p = 0; p < K1; ++p)
#pragma unroll
      for (int q = 0; q <= p; ++q) Wb[six(p, q)] = REPLAY ? st.M[p][q] : 0.0;
    if (REPLAY) {
#pragma unroll
      for (int i = 0; i <= K; ++i) {
        if (a + i < n) {
          load_rec<K, T>(Sig.p, Sig.diag, Sig.ld, a + i, n, Sg[i]);
        } else {
#pragma unroll
          for (int d = 0; d <= K; ++d) Sg[i][d] = 0.0;
        }
      }
    }
  }

  // r = L record j, sb = Sigmabar (or S) record j, ahead = Sigma record j+K+1;
  // with the fused B2 summary also zj = z[j] and yahead = ybar[j+K+1].
  BO_HD void row(int64_t j, int64_t n, const double (&r)[K + 1], const double (&sbin)[K + 1],
                 const double (&ahead)[K + 1], double zj = 0.0, double yahead = 0.0) {
    double inv = 1.0 / r[0];
    double u[K1], sb[K + 1];
#pragma unroll
    for (int p = 0; p < K; ++p) u[p] = r[p + 1] * inv;
#pragma unroll
    for (int d = 0; d <= K; ++d) sb[d] = sbin[d];
    if (sb_is_S) {
      if (REPLAY) {
        tr += Sg[0][0] * sb[0];
#pragma unroll
        for (int d = 1; d <= K; ++d) tr += 2.0 * Sg[0][d] * sb[d];
      }
#pragma unroll
      for (int d = 1; d <= K; ++d) sb[d] *= 2.0;
    }
    double Sbjj = sb[0] + (K > 0 ? Wb[0] : 0.0);
    double vb[K1];
#pragma unroll
    for (int p = 0; p < K; ++p) vb[p] = sb[1 + p] + ((p + 1 < K) ? 2.0 * Wb[six(0, p + 1)] : 0.0);
    if (REPLAY) {
      double dot = 0.0;
      double o[K + 1];
#pragma unroll
      for (int p = 0; p < K; ++p) {
        double acc = -2.0 * Sbjj * Sg[0][1 + p];
#pragma unroll
        for (int q = 0; q < K; ++q) {
          // X[p][q] = Sigma[j+1+p, j+1+q] = record j+1+min(p,q), slot |p-q|
          double xpq = (p >= q) ? Sg[1 + q][p - q] : Sg[1 + p][q - p];
          acc -= xpq * vb[q];
        }
        dot += acc * u[p];
        o[p + 1] = (j + 1 + p < n) ? acc * inv : 0.0;
      }
      o[0] = -2.0 * Sbjj * inv * inv * inv - dot * inv;
      o[0] += dgl * inv;
      if (accumulate) {
        double old[K + 1];
        load_rec<K, T>((const T *)Lb.p, Lb.diag, Lb.ld, j, n, old);
#pragma unroll
        for (int d = 0; d <= K; ++d) o[d] += old[d];
      }
      store_rec<K, T>(Lb.p, Lb.diag, Lb.ld, j, o);
      if (B2MAP && K <= KMAX_FUSED && want_b2) b2.row(r, inv, o, zj, yahead);
#pragma unroll
      for (int i = 0; i < K; ++i)
#pragma unroll
        for (int d = 0; d <= K; ++d) Sg[i][d] = Sg[i + 1][d];
#pragma unroll
      for (int d = 0; d <= K; ++d) Sg[K][d] = ahead[d];
    }
#pragma unroll
    for (int p = 0; p < K; ++p)
#pragma unroll
      for (int q = 0; q <= p; ++q)
        Wb[six(p, q)] = ((p + 1 < K) ? Wb[six(p + 1, q + 1)] : 0.0) + Sbjj * u[p] * u[q] -
                        0.5 * (vb[p] * u[q] + u[p] * vb[q]);
  }

  BO_HD void end(LinMap<K> &st) const {
#pragma unroll
    for (int p = 0; p < K1; ++p) {
      st.v[p] = 0.0;
#pragma unroll
      for (int q = 0; q < K1; ++q) st.M[p][q] = (p < K && q < K) ? Wb[six(p, q)] : 0.0;
    }
  }
};

// ================================================================== B2
// Descending: reverse mode of the Cholesky (Algorithm 2) in the right-looking
// coordinates of F1.  The state entering row j is Cb, the sensitivity of the
// correction window C_{j+1} (symmetric, both halves).  The sensitivity of
// column j of L is assembled from the Lbar record (when given), the
// log-determinant term 2 gl / L_jj on the diagonal and the solve term
// -ybar[j+d] z[j] of Table 1 (when ybar is given); then
//   lb_p   = Lb[1+p] + 2 (Cb l)_p
//   Qbar[j+1+p, j] = lb_p / L_jj
//   Qbar_jj = (Lb[0] - lb . l / L_jj) / (2 L_jj)
//   Cb' = [[-Qbar_jj, -Qbar_{1:}^T/2], [-Qbar_{1:}/2, Cb[0:K-1,0:K-1]]]
//       (= Kt^T Cb Kt + injection)
// ybar[j+1..j+K] is kept in registers (yw).
template <int K, typename T, bool REPLAY> struct B2Step {
  static constexpr int K1 = Dim<K>::K1, NS = Dim<K>::NS;
  double Cb[NS], yw[K1];
  double gl;
  bool with_y;
  BandP<T> Qb;

  // ybar[b .. b+K-1] is read directly (once per chunk).
  BO_HD void begin(const LinMap<K> &st, int64_t b, int64_t n, const T *ybar, double gl_, BandP<T> Qb_) {
    begin_v<1>(st, b, n, VecP<const T>(ybar), gl_, Qb_);
  }
  template <int S>
  BO_HD void begin_v(const LinMap<K> &st, int64_t b, int64_t n, VecP<const T, S> ybar, double gl_,
                     BandP<T> Qb_) {
    gl = gl_;
    with_y = ybar.p != nullptr;
    Qb = Qb_;
#pragma unroll
    for (int p = 0; p < K1; ++p) {
      yw[p] = 0.0;
#pragma unroll
      for (int q = 0; q <= p; ++q) Cb[six(p, q)] = REPLAY ? st.M[p][q] : 0.0;
    }
    if (ybar) {
#pragma unroll
      for (int d = 0; d < K; ++d) yw[d] = (b + d < n) ? (double)ybar[b + d] : 0.0;
    }
  }

  // r = L record j, lbin = Lbar record j (zeros when absent), yj = ybar[j],
  // zj = z[j].
  BO_HD void row(int64_t j, int64_t n, const double (&r)[K + 1], const double (&lbin)[K + 1],
                 double yj, double zj) {
    double Lb[K + 1];
#pragma unroll
    for (int d = 0; d <= K; ++d) Lb[d] = lbin[d];
    double inv = 1.0 / r[0];
    Lb[0] += 2.0 * gl * inv;
    if (with_y) {
      Lb[0] -= yj * zj;
#pragma unroll
      for (int d = 1; d <= K; ++d) Lb[d] -= yw[d - 1] * zj;
#pragma unroll
      for (int d = K - 1; d >= 1; --d) yw[d] = yw[d - 1];
      if (K > 0) yw[0] = yj;
    }
    double qb[K + 1];
    double dot = 0.0;
#pragma unroll
    for (int p = 0; p < K; ++p) {
      double acc = Lb[1 + p];
#pragma unroll
      for (int q = 0; q < K; ++q) acc += 2.0 * Cb[six(p, q)] * r[1 + q];
      qb[1 + p] = (j + 1 + p < n) ? acc * inv : 0.0;
      dot += acc * r[1 + p];
    }
    qb[0] = 0.5 * (Lb[0] - dot * inv) * inv;
    if (REPLAY) store_rec<K, T>(Qb.p, Qb.diag, Qb.ld, j, qb);
#pragma unroll
    for (int p = K - 1; p >= 1; --p)
#pragma unroll
      for (int q = p; q >= 1; --q) Cb[six(p, q)] = Cb[six(p - 1, q - 1)];
#pragma unroll
    for (int p = 1; p < K; ++p) Cb[six(p, 0)] = -0.5 * qb[p];
    if (K > 0) Cb[0] = -qb[0];
  }

  BO_HD void end(LinMap<K> &st) const {
#pragma unroll
    for (int p = 0; p < K1; ++p) {
      st.v[p] = 0.0;
#pragma unroll
      for (int q = 0; q < K1; ++q) st.M[p][q] = (p < K && q < K) ? Cb[six(p, q)] : 0.0;
    }
  }
};

// ====================================================== direct drivers
// Row loops reading global memory directly (used where no LDS tiling runs).
template <int K, typename T>
BO_HD void load_rec_or_zero(BandP<const T> B, int64_t j, int64_t n, double (&r)[K + 1]) {
  if (B.p && j < n) {
    load_rec<K, T>(B.p, B.diag, B.ld, j, n, r);
  } else {
#pragma unroll
    for (int d = 0; d <= K; ++d) r[d] = 0.0;
  }
}

template <int K, typename T>
BO_HD void f1_summary_chunk(int64_t a, int64_t b, int64_t n, BandP<const T> Q, const T *y,
                            F1Map<K> &m, const T *dn = nullptr, double ds = 0.0) {
  F1SumStep<K, T> s;
  s.begin(a, n, Q, y, m, dn, ds);
  for (int64_t i = a + K; i < b; ++i) {
    double q[K + 1];
    load_rec<K, T>(Q.p, Q.diag, Q.ld, i, n, q);
    if (dn) q[0] += (double)dn[i] * ds;
    s.row(q, y ? (double)y[i] : 0.0);
  }
  s.end(m);
}

template <int K, typename T>
BO_HD int64_t f1_replay_chunk(int64_t a, int64_t b, int64_t n, BandP<const T> Q, BandP<T> L,
                              const T *y, T *z, const F1State<K> &st, double *P,
                              double &logsum, double &quad, LinMap<K> *f2map = nullptr,
                              const T *dn = nullptr, double ds = 0.0) {
  F1RepStep<K, T> s;
  s.begin(st, L, y ? z : nullptr, P != nullptr, f2map != nullptr);
  for (int64_t j = a; j < b && s.fail < 0; ++j) {
    double q[K + 1];
    load_rec<K, T>(Q.p, Q.diag, Q.ld, j, n, q);
    if (dn) q[0] += (double)dn[j] * ds;
    s.row(j, q, y ? (double)y[j] : 0.0);
  }
  s.end(P);
  if (f2map) s.end_f2(*f2map);
  logsum = s.ls;
  quad = s.qs;
  return s.fail;
}

template <int K, typename T>
BO_HD void pc_chunk(int64_t a, int64_t b, int64_t n, BandP<const T> L, double *P) {
  PcStep<K> s;
  s.begin();
  for (int64_t j = a; j < b; ++j) {
    double r[K + 1];
    load_rec<K, T>(L.p, L.diag, L.ld, j, n, r);
    s.row(r);
  }
  s.end(P);
}

// With b2map (replay only): also the chunk map of a B2 pass that takes this
// solve's output as its z, no Lbar record, ybar and the log-determinant
// weight gl.
template <int K, typename T, bool REPLAY>
BO_HD void fs_chunk(int64_t a, int64_t b, int64_t n, BandP<const T> L, const T *y, T *z,
                    double xscale, LinMap<K> &st, const T *ybar = nullptr, double gl = 0.0,
                    LinMap<K> *b2map = nullptr) {
  FsStep<K, T, REPLAY> s;
  s.begin(st, z, xscale);
  B2MapAcc<K> m2;
  if (REPLAY && b2map) m2.begin(a, n, ybar, gl);
  const double zero[K + 1] = {};
  for (int64_t j = a; j < b; ++j) {
    double r[K + 1];
    load_rec<K, T>(L.p, L.diag, L.ld, j, n, r);
    const double xj = s.row(j, r, (double)y[j]);
    if (REPLAY && b2map)
      m2.row(r, 1.0 / r[0], zero, xj, (ybar && j + K + 1 < n) ? (double)ybar[j + K + 1] : 0.0);
  }
  s.end(st);
  if (REPLAY && b2map) m2.end(*b2map);
}

template <int K, typename T, bool REPLAY>
BO_HD void f2_chunk(int64_t a, int64_t b, int64_t n, BandP<const T> L, BandP<T> S,
                    const T *bvec, T *x, double xscale, LinMap<K> &st,
                    BandP<const T> Sb = BandP<const T>{nullptr, nullptr, 0}, bool sbS = false,
                    LinMap<K> *b1map = nullptr) {
  F2Step<K, T, REPLAY> s;
  s.begin(st, S, x, xscale, S.p != nullptr, bvec != nullptr, b1map != nullptr, sbS);
  for (int64_t j = b - 1; j >= a; --j) {
    double r[K + 1];
    load_rec<K, T>(L.p, L.diag, L.ld, j, n, r);
    s.row(j, r, bvec ? (double)bvec[j] : 0.0);
    if (b1map) {
      double sb[K + 1];
      load_rec<K, T>(Sb.p, Sb.diag, Sb.ld, j, n, sb);
      s.row_b1(r, sb);
    }
  }
  s.end(st);
  if (b1map) s.end_b1(*b1map);
}

template <int K, typename T, bool REPLAY>
BO_HD void b1_chunk(int64_t a, int64_t b, int64_t n, BandP<const T> L, BandP<const T> Sig,
                    BandP<const T> Sb, bool sb_is_S, BandP<T> Lb, bool accumulate,
                    double &trace, LinMap<K> &st, const T *ybar = nullptr, const T *z = nullptr,
                    double gl = 0.0, LinMap<K> *b2map = nullptr, double gl1 = 0.0) {
  B1Step<K, T, REPLAY> s;
  s.begin(st, a, n, Sig, sb_is_S, Lb, accumulate, gl1);
  if (REPLAY && b2map) s.begin_b2(a, n, ybar, gl);
  for (int64_t j = a; j < b; ++j) {
    double r[K + 1], sb[K + 1], ah[K + 1];
    load_rec<K, T>(L.p, L.diag, L.ld, j, n, r);
    load_rec<K, T>(Sb.p, Sb.diag, Sb.ld, j, n, sb);
    if (REPLAY) {
      load_rec_or_zero<K, T>(Sig, j + K + 1, n, ah);
    } else {
#pragma unroll
      for (int d = 0; d <= K; ++d) ah[d] = 0.0;
    }
    double zj = (b2map && z) ? (double)z[j] : 0.0;
    double yah = (b2map && ybar && j + K + 1 < n) ? (double)ybar[j + K + 1] : 0.0;
    s.row(j, n, r, sb, ah, zj, yah);
  }
  trace = s.tr;
  s.end(st);
  if (REPLAY && b2map) s.end_b2(*b2map);
}

template <int K, typename T, bool REPLAY>
BO_HD void b2_chunk(int64_t a, int64_t b, int64_t n, BandP<const T> L, BandP<const T> Lbar,
                    double gl, const T *ybar, const T *z, BandP<T> Qb, LinMap<K> &st) {
  B2Step<K, T, REPLAY> s;
  s.begin(st, b, n, ybar, gl, Qb);
  for (int64_t j = b - 1; j >= a; --j) {
    double r[K + 1], lb[K + 1];
    load_rec<K, T>(L.p, L.diag, L.ld, j, n, r);
    load_rec_or_zero<K, T>(Lbar, j, n, lb);
    s.row(j, n, r, lb, ybar ? (double)ybar[j] : 0.0, ybar ? (double)z[j] : 0.0);
  }
  s.end(st);
}

}  // namespace bo
