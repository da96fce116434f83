// bandops_algo.hpp -- per-chunk recurrences of the banded operators.
//
// Every pass of the library walks rows of a banded matrix in order, carrying a
// small state (a k x k window and/or a k-vector).  To spread one long matrix
// over the chip, rows are cut into chunks; a chunk is processed twice:
//   * a summary: the chunk's effect on the state, independent of what enters it;
//   * after a scan over the summaries has produced every chunk's exact incoming
//     state, a replay that rewrites the chunk's outputs in natural row order.
// Nothing is permuted, so the outputs are those of the sequential algorithms
// of the paper (Algorithms 1-4 and the Table 1 compositions) up to rounding.
//
// All state lives in registers: K (the number of sub-diagonals) is a template
// parameter, so every window index below is a compile-time constant after
// unrolling.  T is the storage type of band and vector entries (double, or
// float for the mixed format whose diagonal lives in a separate FP64 array);
// arithmetic is FP64 throughout.
//
// Notation shared by the passes (0-based, record j = column j of the band):
//   l_j[p] = L[j+1+p, j]      u_j = l_j / L_jj       c_j = 1 / L_jj^2
//   Kt_j   = [ -u_j | e_0 ... e_{K-2} ]              (K x K)
// and entries whose row index is >= n are zero everywhere (the band's padding).
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#define BO_HD __host__ __device__ __forceinline__

namespace bo {

template <int K> struct Dim {
  static constexpr int K1 = K > 0 ? K : 1;                 // array extent
  static constexpr int NS = K > 0 ? K * (K + 1) / 2 : 1;   // packed symmetric
};

// Packed lower storage of a symmetric K x K matrix.
BO_HD constexpr int six(int p, int q) { return p >= q ? p * (p + 1) / 2 + q : q * (q + 1) / 2 + p; }

// ---------------------------------------------------------------- band I/O
template <int K, typename T>
BO_HD void load_rec(const T *__restrict__ band, const double *__restrict__ diag, int64_t ld,
                    int64_t j, int64_t n, double (&r)[K + 1]) {
  const T *rp = band + j * ld;
#pragma unroll
  for (int d = 0; d <= K; ++d) r[d] = (double)rp[d];
  if (diag) r[0] = diag[j];
#pragma unroll
  for (int d = 1; d <= K; ++d)
    if (j + d >= n) r[d] = 0.0;
}

template <int K, typename T>
BO_HD void store_rec(T *__restrict__ band, double *__restrict__ diag, int64_t ld, int64_t j,
                     const double (&r)[K + 1]) {
  T *rp = band + j * ld;
#pragma unroll
  for (int d = 0; d <= K; ++d) rp[d] = (T)r[d];
  if (diag) diag[j] = r[0];
}

// A band argument as the kernels see it.
template <typename T> struct BandP {
  T *p;          // records, stride ld (elements)
  double *diag;  // FP64 diagonal (mixed format) or null
  int64_t ld;
};

// ---------------------------------------------------------------- small dense
// Cholesky of a symmetric K x K matrix held full; lower factor in place.  A
// non-positive pivot turns the result into NaN (the caller's info records the
// failing row separately).
template <int K> BO_HD void chol_small(double (&M)[Dim<K>::K1][Dim<K>::K1]) {
#pragma unroll
  for (int j = 0; j < K; ++j) {
    double s = M[j][j];
#pragma unroll
    for (int m = 0; m < j; ++m) s -= M[j][m] * M[j][m];
    double r = s > 0.0 ? sqrt(s) : NAN;
    double inv = 1.0 / r;
    M[j][j] = r;
#pragma unroll
    for (int i = j + 1; i < K; ++i) {
      double t = M[i][j];
#pragma unroll
      for (int m = 0; m < j; ++m) t -= M[i][m] * M[j][m];
      M[i][j] = t * inv;
    }
  }
}

// Solve R Y = B in place (R lower, K x K; B has K rows and NC columns).
template <int K, int NC>
BO_HD void trsm_small(const double (&R)[Dim<K>::K1][Dim<K>::K1], double (&B)[Dim<K>::K1][NC]) {
#pragma unroll
  for (int i = 0; i < K; ++i) {
    double inv = 1.0 / R[i][i];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double t = B[i][c];
#pragma unroll
      for (int m = 0; m < i; ++m) t -= R[i][m] * B[m][c];
      B[i][c] = t * inv;
    }
  }
}

// ============================================================================
// F1: Cholesky (Algorithm 1) + log-determinant + forward solve z = L^{-1} y.
//
// Right-looking form of Algorithm 1: the state entering row j is the correction
// window C_j[p][q] = sum_{m<j} L[j+p,m] L[j+q,m] (p,q < K) and the right-hand
// side correction g_j[p] = sum_{m<j} L[j+p,m] z_m.  Row j reads only record j of
// Q (column j of the lower band):
//   L_jj = sqrt(Q_jj - C[0][0]),  L[j+d,j] = (Q[j+d,j] - C[d][0]) / L_jj,
//   z_j  = (y_j - g[0]) / L_jj,
//   C' = shift(C) + l l^T,  g' = shift(g) + l z_j.
// This is the same arithmetic as Algorithm 1's dot products, summed in the
// order the columns are produced.
// ============================================================================

// Map of one chunk [a,b) of F1 on its entering state (C, g): eliminate the
// chunk's interior rows I = [a+K, b) first, leaving the Schur complement on the
// chunk's first K rows F and on the K rows O = [b, b+K) after it:
//   A = Q_FF - X_F^T X_F      B = X_O^T X_F      D = X_O^T X_O
//   r = y_F  - X_F^T zt       d = X_O^T zt
// with X_* = L_I^{-1} Q_I* and zt = L_I^{-1} y_I from the Cholesky of Q_II.
// Applying the map: M = A - C_a, C_b = D + B M^{-1} B^T,
//                   g_b = d - B M^{-1} (r - g_a).
template <int K> struct F1Map {
  double A[Dim<K>::K1][Dim<K>::K1];
  double B[Dim<K>::K1][Dim<K>::K1];
  double D[Dim<K>::K1][Dim<K>::K1];
  double r[Dim<K>::K1];
  double d[Dim<K>::K1];
};
template <int K> struct F1State {
  double C[Dim<K>::K1][Dim<K>::K1];
  double g[Dim<K>::K1];
};
template <int K> constexpr int f1map_words() { return 3 * Dim<K>::K1 * Dim<K>::K1 + 2 * Dim<K>::K1; }
template <int K> constexpr int f1state_words() { return Dim<K>::K1 * Dim<K>::K1 + Dim<K>::K1; }

template <int K> BO_HD void f1_load_map(const double *w, F1Map<K> &m) {
  constexpr int K1 = Dim<K>::K1;
#pragma unroll
  for (int p = 0; p < K1; ++p)
#pragma unroll
    for (int q = 0; q < K1; ++q) {
      m.A[p][q] = w[p * K1 + q];
      m.B[p][q] = w[K1 * K1 + p * K1 + q];
      m.D[p][q] = w[2 * K1 * K1 + p * K1 + q];
    }
#pragma unroll
  for (int p = 0; p < K1; ++p) {
    m.r[p] = w[3 * K1 * K1 + p];
    m.d[p] = w[3 * K1 * K1 + K1 + p];
  }
}
template <int K> BO_HD void f1_store_map(double *w, const F1Map<K> &m) {
  constexpr int K1 = Dim<K>::K1;
#pragma unroll
  for (int p = 0; p < K1; ++p)
#pragma unroll
    for (int q = 0; q < K1; ++q) {
      w[p * K1 + q] = m.A[p][q];
      w[K1 * K1 + p * K1 + q] = m.B[p][q];
      w[2 * K1 * K1 + p * K1 + q] = m.D[p][q];
    }
#pragma unroll
  for (int p = 0; p < K1; ++p) {
    w[3 * K1 * K1 + p] = m.r[p];
    w[3 * K1 * K1 + K1 + p] = m.d[p];
  }
}
template <int K> BO_HD void f1_load_state(const double *w, F1State<K> &s) {
  constexpr int K1 = Dim<K>::K1;
#pragma unroll
  for (int p = 0; p < K1; ++p) {
#pragma unroll
    for (int q = 0; q < K1; ++q) s.C[p][q] = w[p * K1 + q];
    s.g[p] = w[K1 * K1 + p];
  }
}
template <int K> BO_HD void f1_store_state(double *w, const F1State<K> &s) {
  constexpr int K1 = Dim<K>::K1;
#pragma unroll
  for (int p = 0; p < K1; ++p) {
#pragma unroll
    for (int q = 0; q < K1; ++q) w[p * K1 + q] = s.C[p][q];
    w[K1 * K1 + p] = s.g[p];
  }
}
template <int K> BO_HD void f1_zero_state(F1State<K> &s) {
#pragma unroll
  for (int p = 0; p < Dim<K>::K1; ++p) {
#pragma unroll
    for (int q = 0; q < Dim<K>::K1; ++q) s.C[p][q] = 0.0;
    s.g[p] = 0.0;
  }
}

// Summary of chunk [a,b) (b - a >= 2K, not the problem's last chunk).
template <int K, typename T>
BO_HD void f1_summary_chunk(int64_t a, int64_t b, int64_t n, BandP<const T> Q, const T *y,
                            F1Map<K> &m) {
  constexpr int K1 = Dim<K>::K1;
  constexpr int NS = Dim<K>::NS;
  double C[NS], Z[NS], X[K1][K1], g[K1], e[K1];
#pragma unroll
  for (int i = 0; i < NS; ++i) C[i] = Z[i] = 0.0;
#pragma unroll
  for (int p = 0; p < K1; ++p) {
    g[p] = e[p] = 0.0;
#pragma unroll
    for (int f = 0; f < K1; ++f) X[p][f] = 0.0;
  }
  // Q_FF, the coupling of the first K interior rows to F, and y_F.
#pragma unroll
  for (int f = 0; f < K; ++f) {
    double rec[K + 1];
    load_rec<K, T>(Q.p, Q.diag, Q.ld, a + f, n, rec);
#pragma unroll
    for (int p = f; p < K; ++p) m.A[p][f] = m.A[f][p] = rec[p - f];
#pragma unroll
    for (int p = 0; p <= f; ++p) X[p][f] = rec[K + p - f];   // Q[a+K+p, a+f]
    m.r[f] = y ? (double)y[a + f] : 0.0;
  }
  for (int64_t i = a + K; i < b; ++i) {
    double q[K + 1];
    load_rec<K, T>(Q.p, Q.diag, Q.ld, i, n, q);
    double s0 = q[0] - (K > 0 ? C[0] : 0.0);
    double lii = s0 > 0.0 ? sqrt(s0) : NAN;
    double inv = 1.0 / lii;
    double l[K1], xf[K1];
#pragma unroll
    for (int p = 0; p < K; ++p) l[p] = ((p + 1 < K) ? q[p + 1] - C[six(p + 1, 0)] : q[K]) * inv;
#pragma unroll
    for (int f = 0; f < K; ++f) xf[f] = X[0][f] * inv;
    double zt = 0.0;
    if (y) zt = ((double)y[i] - g[0]) * inv;
    // Z += xf xf^T, e += xf zt
#pragma unroll
    for (int f = 0; f < K; ++f) {
      e[f] += xf[f] * zt;
#pragma unroll
      for (int h = 0; h <= f; ++h) Z[six(f, h)] += xf[f] * xf[h];
    }
    // shift the windows by one row
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

// State leaving a chunk given its map and the state entering it.
template <int K> BO_HD void f1_apply(const F1Map<K> &m, const F1State<K> &in, F1State<K> &out) {
  constexpr int K1 = Dim<K>::K1;
  double R[K1][K1], Y[K1][K1], t[K1][1];
#pragma unroll
  for (int p = 0; p < K1; ++p) {
#pragma unroll
    for (int q = 0; q < K1; ++q) {
      R[p][q] = m.A[p][q] - in.C[p][q];
      Y[p][q] = m.B[q][p];   // B^T
    }
    t[p][0] = m.r[p] - in.g[p];
  }
  chol_small<K>(R);
  trsm_small<K, K1>(R, Y);
  trsm_small<K, 1>(R, t);
#pragma unroll
  for (int p = 0; p < K; ++p) {
    double acc = m.d[p];
#pragma unroll
    for (int f = 0; f < K; ++f) acc -= Y[f][p] * t[f][0];
    out.g[p] = acc;
#pragma unroll
    for (int q = 0; q < K; ++q) {
      double c = m.D[p][q];
#pragma unroll
      for (int f = 0; f < K; ++f) c += Y[f][p] * Y[f][q];
      out.C[p][q] = c;
    }
  }
}

// Map of two consecutive chunks, first m1 then m2: eliminate their shared
// boundary rows O1 (N = A2 - D1, SPD as a Schur complement of Q).
template <int K> BO_HD void f1_compose(const F1Map<K> &m1, const F1Map<K> &m2, F1Map<K> &o) {
  constexpr int K1 = Dim<K>::K1;
  double R[K1][K1], Y1[K1][K1], Y2[K1][K1], t[K1][1];
#pragma unroll
  for (int p = 0; p < K1; ++p) {
#pragma unroll
    for (int q = 0; q < K1; ++q) {
      R[p][q] = m2.A[p][q] - m1.D[p][q];
      Y1[p][q] = m1.B[p][q];
      Y2[p][q] = m2.B[q][p];
    }
    t[p][0] = m2.r[p] - m1.d[p];
  }
  chol_small<K>(R);
  trsm_small<K, K1>(R, Y1);
  trsm_small<K, K1>(R, Y2);
  trsm_small<K, 1>(R, t);
#pragma unroll
  for (int p = 0; p < K; ++p) {
    double rr = m1.r[p], dd = m2.d[p];
#pragma unroll
    for (int f = 0; f < K; ++f) {
      rr += Y1[f][p] * t[f][0];
      dd -= Y2[f][p] * t[f][0];
    }
    o.r[p] = rr;
    o.d[p] = dd;
#pragma unroll
    for (int q = 0; q < K; ++q) {
      double a = m1.A[p][q], bb = 0.0, dmat = m2.D[p][q];
#pragma unroll
      for (int f = 0; f < K; ++f) {
        a -= Y1[f][p] * Y1[f][q];
        bb += Y2[f][p] * Y1[f][q];
        dmat += Y2[f][p] * Y2[f][q];
      }
      o.A[p][q] = a;
      o.B[p][q] = bb;
      o.D[p][q] = dmat;
    }
  }
}

// Replay of rows [a,b) from the exact entering state.  Writes L (and z when y
// is given); returns the first row whose pivot is not positive (or -1).
// Accumulates sum log L_jj and sum z_j^2; when P is given, also the chunk's
// product P = Kt_{b-1} ... Kt_a used by the linear passes.
template <int K, typename T>
BO_HD int64_t f1_replay_chunk(int64_t a, int64_t b, int64_t n, BandP<const T> Q, BandP<T> L,
                              const T *y, T *z, const F1State<K> &st, double *P,
                              double &logsum, double &quad) {
  constexpr int K1 = Dim<K>::K1;
  constexpr int NS = Dim<K>::NS;
  double C[NS], g[K1], Pm[K1][K1];
#pragma unroll
  for (int p = 0; p < K1; ++p) {
    g[p] = st.g[p];
#pragma unroll
    for (int q = 0; q <= p; ++q) C[six(p, q)] = st.C[p][q];
#pragma unroll
    for (int q = 0; q < K1; ++q) Pm[p][q] = (p == q) ? 1.0 : 0.0;
  }
  double ls = 0.0, qs = 0.0;
  int64_t fail = -1;
  for (int64_t j = a; j < b; ++j) {
    double q[K + 1];
    load_rec<K, T>(Q.p, Q.diag, Q.ld, j, n, q);
    double s0 = q[0] - (K > 0 ? C[0] : 0.0);
    if (!(s0 > 0.0)) {
      fail = j;
      break;
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
    if (y) {
      zj = ((double)y[j] - (K > 0 ? g[0] : 0.0)) * inv;
      z[j] = (T)zj;
      qs += zj * zj;
    }
#pragma unroll
    for (int p = 0; p < K; ++p) g[p] = ((p + 1 < K) ? g[p + 1] : 0.0) + l[p] * zj;
#pragma unroll
    for (int p = 0; p < K; ++p)
#pragma unroll
      for (int h = 0; h <= p; ++h)
        C[six(p, h)] = ((p + 1 < K) ? C[six(p + 1, h + 1)] : 0.0) + l[p] * l[h];
    if (P) {
      // P <- Kt_j P :  row p of Kt P = -u_p P[0,:] + P[p+1,:]
#pragma unroll
      for (int c = 0; c < K; ++c) {
        double p0 = Pm[0][c];
#pragma unroll
        for (int p = 0; p < K; ++p) Pm[p][c] = ((p + 1 < K) ? Pm[p + 1][c] : 0.0) - l[p] * inv * p0;
      }
    }
  }
  if (P) {
#pragma unroll
    for (int p = 0; p < K1; ++p)
#pragma unroll
      for (int q = 0; q < K1; ++q) P[p * K1 + q] = Pm[p][q];
  }
  logsum = ls;
  quad = qs;
  return fail;
}

// Product P = Kt_{b-1} ... Kt_a of a chunk of a given factor L.
template <int K, typename T>
BO_HD void pc_chunk(int64_t a, int64_t b, int64_t n, BandP<const T> L, double *P) {
  constexpr int K1 = Dim<K>::K1;
  double Pm[K1][K1];
#pragma unroll
  for (int p = 0; p < K1; ++p)
#pragma unroll
    for (int q = 0; q < K1; ++q) Pm[p][q] = (p == q) ? 1.0 : 0.0;
  for (int64_t j = a; j < b; ++j) {
    double r[K + 1];
    load_rec<K, T>(L.p, L.diag, L.ld, j, n, r);
    double inv = 1.0 / r[0];
#pragma unroll
    for (int c = 0; c < K; ++c) {
      double p0 = Pm[0][c];
#pragma unroll
      for (int p = 0; p < K; ++p) Pm[p][c] = ((p + 1 < K) ? Pm[p + 1][c] : 0.0) - r[p + 1] * inv * p0;
    }
  }
#pragma unroll
  for (int p = 0; p < K1; ++p)
#pragma unroll
    for (int q = 0; q < K1; ++q) P[p * K1 + q] = Pm[p][q];
}

// ============================================================================
// Linear passes.  With the chunk product P = Kt_{b-1} ... Kt_a, each of them
// maps the state across a chunk affinely:
//   ascending  (rows a -> b):  S_b = P S_a P^T + M,   s_b = P s_a + v
//   descending (rows b -> a):  S_a = P^T S_b P + M,   s_a = P^T s_b + v
// where (M, v) is the chunk run from a zero entering state.
// ============================================================================
template <int K> struct LinMap {   // (M, v) of one chunk or group
  double M[Dim<K>::K1][Dim<K>::K1];
  double v[Dim<K>::K1];
};
template <int K> constexpr int lin_words() { return Dim<K>::K1 * Dim<K>::K1 + Dim<K>::K1; }

template <int K> BO_HD void lin_load(const double *w, LinMap<K> &m) {
  constexpr int K1 = Dim<K>::K1;
#pragma unroll
  for (int p = 0; p < K1; ++p) {
#pragma unroll
    for (int q = 0; q < K1; ++q) m.M[p][q] = w[p * K1 + q];
    m.v[p] = w[K1 * K1 + p];
  }
}
template <int K> BO_HD void lin_store(double *w, const LinMap<K> &m) {
  constexpr int K1 = Dim<K>::K1;
#pragma unroll
  for (int p = 0; p < K1; ++p) {
#pragma unroll
    for (int q = 0; q < K1; ++q) w[p * K1 + q] = m.M[p][q];
    w[K1 * K1 + p] = m.v[p];
  }
}
template <int K> BO_HD void lin_zero(LinMap<K> &m) {
#pragma unroll
  for (int p = 0; p < Dim<K>::K1; ++p) {
#pragma unroll
    for (int q = 0; q < Dim<K>::K1; ++q) m.M[p][q] = 0.0;
    m.v[p] = 0.0;
  }
}
template <int K> BO_HD void mat_load(const double *w, double (&P)[Dim<K>::K1][Dim<K>::K1]) {
  constexpr int K1 = Dim<K>::K1;
#pragma unroll
  for (int p = 0; p < K1; ++p)
#pragma unroll
    for (int q = 0; q < K1; ++q) P[p][q] = w[p * K1 + q];
}
template <int K> BO_HD void mat_store(double *w, const double (&P)[Dim<K>::K1][Dim<K>::K1]) {
  constexpr int K1 = Dim<K>::K1;
#pragma unroll
  for (int p = 0; p < K1; ++p)
#pragma unroll
    for (int q = 0; q < K1; ++q) w[p * K1 + q] = P[p][q];
}

// s <- map(s): ascending  S = P S P^T + M, s = P s + v
//              descending S = P^T S P + M, s = P^T s + v
template <int K, bool DESC>
BO_HD void lin_apply(const double (&P)[Dim<K>::K1][Dim<K>::K1], const LinMap<K> &m, LinMap<K> &s) {
  constexpr int K1 = Dim<K>::K1;
  double W[K1][K1], v[K1];
  // W = S P^T (asc) or S P (desc);  then S' = P W (asc) or P^T W (desc)
#pragma unroll
  for (int p = 0; p < K; ++p) {
    double acc = m.v[p];
#pragma unroll
    for (int q = 0; q < K; ++q) acc += (DESC ? P[q][p] : P[p][q]) * s.v[q];
    v[p] = acc;
#pragma unroll
    for (int q = 0; q < K; ++q) {
      double w = 0.0;
#pragma unroll
      for (int r = 0; r < K; ++r) w += s.M[p][r] * (DESC ? P[r][q] : P[q][r]);
      W[p][q] = w;
    }
  }
#pragma unroll
  for (int p = 0; p < K; ++p) {
    s.v[p] = v[p];
#pragma unroll
    for (int q = 0; q < K; ++q) {
      double acc = m.M[p][q];
#pragma unroll
      for (int r = 0; r < K; ++r) acc += (DESC ? P[r][p] : P[p][r]) * W[r][q];
      s.M[p][q] = acc;
    }
  }
}

// G <- P G  (ascending group product) or G <- G P (descending traversal).
template <int K, bool RIGHT>
BO_HD void mat_mul_acc(double (&G)[Dim<K>::K1][Dim<K>::K1], const double (&P)[Dim<K>::K1][Dim<K>::K1]) {
  constexpr int K1 = Dim<K>::K1;
  double R[K1][K1];
#pragma unroll
  for (int p = 0; p < K; ++p)
#pragma unroll
    for (int q = 0; q < K; ++q) {
      double acc = 0.0;
#pragma unroll
      for (int r = 0; r < K; ++r) acc += RIGHT ? G[p][r] * P[r][q] : P[p][r] * G[r][q];
      R[p][q] = acc;
    }
#pragma unroll
  for (int p = 0; p < K; ++p)
#pragma unroll
    for (int q = 0; q < K; ++q) G[p][q] = R[p][q];
}

// ----------------------------------------------------------------------------
// FS: forward solve z = L^{-1} y with a given factor (ascending).  State
// g_j[p] = sum_{m<j} L[j+p,m] z_m;  g_{j+1} = Kt_j g_j + u_j y_j.
// ----------------------------------------------------------------------------
template <int K, typename T, bool REPLAY>
BO_HD void fs_chunk(int64_t a, int64_t b, int64_t n, BandP<const T> L, const T *y, T *z,
                    double xscale, LinMap<K> &st) {
  constexpr int K1 = Dim<K>::K1;
  double g[K1];
#pragma unroll
  for (int p = 0; p < K1; ++p) g[p] = REPLAY ? st.v[p] : 0.0;
  for (int64_t j = a; j < b; ++j) {
    double r[K + 1];
    load_rec<K, T>(L.p, L.diag, L.ld, j, n, r);
    double inv = 1.0 / r[0];
    double zj = ((double)y[j] - (K > 0 ? g[0] : 0.0)) * inv;
    if (REPLAY) z[j] = (T)(xscale * zj);
#pragma unroll
    for (int p = 0; p < K; ++p) g[p] = ((p + 1 < K) ? g[p + 1] : 0.0) + r[p + 1] * zj;
  }
#pragma unroll
  for (int p = 0; p < K1; ++p) st.v[p] = g[p];
}

// ----------------------------------------------------------------------------
// F2 (descending): subset inverse (Algorithm 3) and back solve x = L^{-T} b.
// State entering row j: the window W = Sigma[j+1..j+K, j+1..j+K] and
// xw = x[j+1..j+K].  Row j:
//   v = -W u_j                       (Sigma[j+1+p, j], Algorithm 3's sums)
//   Sigma_jj = c_j - u_j^T v
//   W' = [[Sigma_jj, v'^T], [v', W[0:K-1,0:K-1]]]   (= Kt^T W Kt + c e0 e0^T)
//   x_j = b_j / L_jj - u_j^T xw,   xw' = (x_j, xw[0:K-1])
// ----------------------------------------------------------------------------
template <int K, typename T, bool REPLAY>
BO_HD void f2_chunk(int64_t a, int64_t b, int64_t n, BandP<const T> L, BandP<T> S,
                    const T *bvec, T *x, double xscale, LinMap<K> &st) {
  constexpr int K1 = Dim<K>::K1;
  constexpr int NS = Dim<K>::NS;
  const bool want_s = S.p != nullptr, want_x = bvec != nullptr;
  double W[NS], xw[K1];
#pragma unroll
  for (int p = 0; p < K1; ++p) {
    xw[p] = REPLAY ? st.v[p] : 0.0;
#pragma unroll
    for (int q = 0; q <= p; ++q) W[six(p, q)] = REPLAY ? st.M[p][q] : 0.0;
  }
  for (int64_t j = b - 1; j >= a; --j) {
    double r[K + 1];
    load_rec<K, T>(L.p, L.diag, L.ld, j, n, r);
    double inv = 1.0 / r[0];
    double u[K1];
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
      double xj = (double)bvec[j] * inv;
#pragma unroll
      for (int p = 0; p < K; ++p) xj -= u[p] * xw[p];
      if (REPLAY) x[j] = (T)(xscale * xj);
#pragma unroll
      for (int p = K - 1; p >= 1; --p) xw[p] = xw[p - 1];
      if (K > 0) xw[0] = xj;
    }
  }
#pragma unroll
  for (int p = 0; p < K1; ++p) {
    st.v[p] = xw[p];
#pragma unroll
    for (int q = 0; q < K1; ++q) st.M[p][q] = (q < K && p < K) ? W[six(p, q)] : 0.0;
  }
}

// ----------------------------------------------------------------------------
// B1 (ascending): reverse mode of the subset inverse (Algorithm 4).  The state
// entering row j is Wb, the sensitivity of the window W_j (symmetric, both
// halves counted).  With sb = Sigmabar record j (stored lower entries):
//   Sbjj  = sb_0 + Wb[0][0]
//   vb_p  = sb_{1+p} + 2 Wb[0][1+p]            (vb_{K-1} = sb_K)
//   ub    = -2 Sbjj v - W_{j+1} vb             (W_{j+1} = Sigma window below j)
//   Lbar[j+1+p, j] = ub_p / L_jj
//   Lbar_jj        = -2 Sbjj c_j / L_jj - (ub . u) / L_jj
//   Wb'  = shift(Wb) + Sbjj u u^T - (vb u^T + u vb^T)/2   (= Kt Wb Kt^T + ...)
// With trace_w set, Sigmabar = (S_jj, 2 S_{j+1,j}, ...) is formed from the band
// S, and sum_j Sigma_jj S_jj + 2 sum Sigma_ij S_ij is accumulated.
// ----------------------------------------------------------------------------
template <int K, typename T, bool REPLAY>
BO_HD void b1_chunk(int64_t a, int64_t b, int64_t n, BandP<const T> L, BandP<const T> Sig,
                    BandP<const T> Sb, bool sb_is_S, BandP<T> Lb, bool accumulate,
                    double &trace, LinMap<K> &st) {
  constexpr int K1 = Dim<K>::K1;
  constexpr int NS = Dim<K>::NS;
  double Wb[NS];
#pragma unroll
  for (int p = 0; p < K1; ++p)
#pragma unroll
    for (int q = 0; q <= p; ++q) Wb[six(p, q)] = REPLAY ? st.M[p][q] : 0.0;
  // X = Sigma window below row j: X[p][q] = Sigma[j+1+p, j+1+q]
  double X[NS];
  if (REPLAY) {
#pragma unroll
    for (int q = 0; q < K; ++q) {
      double rec[K + 1];
      int64_t jq = a + 1 + q;
      if (jq < n) {
        load_rec<K, T>(Sig.p, Sig.diag, Sig.ld, jq, n, rec);
      } else {
#pragma unroll
        for (int d = 0; d <= K; ++d) rec[d] = 0.0;
      }
#pragma unroll
      for (int p = q; p < K; ++p) X[six(p, q)] = rec[p - q];
    }
  }
  double tr = 0.0;
  for (int64_t j = a; j < b; ++j) {
    double r[K + 1], sb[K + 1];
    load_rec<K, T>(L.p, L.diag, L.ld, j, n, r);
    load_rec<K, T>(Sb.p, Sb.diag, Sb.ld, j, n, sb);
    double inv = 1.0 / r[0];
    double u[K1];
#pragma unroll
    for (int p = 0; p < K; ++p) u[p] = r[p + 1] * inv;
    double sig[K + 1];
    if (REPLAY) load_rec<K, T>(Sig.p, Sig.diag, Sig.ld, j, n, sig);
    if (sb_is_S) {
      if (REPLAY) {
        tr += sig[0] * sb[0];
#pragma unroll
        for (int d = 1; d <= K; ++d) tr += 2.0 * sig[d] * sb[d];
      }
#pragma unroll
      for (int d = 1; d <= K; ++d) sb[d] *= 2.0;
    }
    double Sbjj = sb[0] + (K > 0 ? Wb[0] : 0.0);
    double vb[K1];
#pragma unroll
    for (int p = 0; p < K; ++p) vb[p] = sb[1 + p] + ((p + 1 < K) ? 2.0 * Wb[six(0, p + 1)] : 0.0);
    if (REPLAY) {
      double ub[K1];
      double dot = 0.0;
#pragma unroll
      for (int p = 0; p < K; ++p) {
        double acc = -2.0 * Sbjj * sig[1 + p];
#pragma unroll
        for (int q = 0; q < K; ++q) acc -= X[six(p, q)] * vb[q];
        ub[p] = acc;
        dot += acc * u[p];
      }
      double o[K + 1];
      o[0] = -2.0 * Sbjj * inv * inv * inv - dot * inv;
#pragma unroll
      for (int p = 0; p < K; ++p) o[p + 1] = (j + 1 + p < n) ? ub[p] * inv : 0.0;
      if (accumulate) {
        double old[K + 1];
        load_rec<K, T>((const T *)Lb.p, Lb.diag, Lb.ld, j, n, old);
#pragma unroll
        for (int d = 0; d <= K; ++d) o[d] += old[d];
      }
      store_rec<K, T>(Lb.p, Lb.diag, Lb.ld, j, o);
      // slide X down one row: X'[p][q] = X[p+1][q+1]; new row K-1 is
      // Sigma[j+1+K, j+2+q] = record (j+2+q) slot (K-1-q).
#pragma unroll
      for (int p = 0; p + 1 < K; ++p)
#pragma unroll
        for (int q = 0; q <= p; ++q) X[six(p, q)] = X[six(p + 1, q + 1)];
#pragma unroll
      for (int q = 0; q < K; ++q) {
        int64_t jr = j + 2 + q;
        double val = 0.0;
        if (jr < n && jr + (K - 1 - q) < n) {
          const T *rp = Sig.p + jr * Sig.ld;
          val = (K - 1 - q == 0 && Sig.diag) ? Sig.diag[jr] : (double)rp[K - 1 - q];
        }
        if (K > 0) X[six(K - 1, q)] = val;
      }
    }
    // Wb' = shift(Wb) + Sbjj u u^T - (vb u^T + u vb^T) / 2
#pragma unroll
    for (int p = 0; p < K; ++p)
#pragma unroll
      for (int q = 0; q <= p; ++q)
        Wb[six(p, q)] = ((p + 1 < K) ? Wb[six(p + 1, q + 1)] : 0.0) + Sbjj * u[p] * u[q] -
                        0.5 * (vb[p] * u[q] + u[p] * vb[q]);
  }
  trace = tr;
#pragma unroll
  for (int p = 0; p < K1; ++p) {
    st.v[p] = 0.0;
#pragma unroll
    for (int q = 0; q < K1; ++q) st.M[p][q] = (p < K && q < K) ? Wb[six(p, q)] : 0.0;
  }
}

// ----------------------------------------------------------------------------
// B2 (descending): reverse mode of the Cholesky (Algorithm 2), in the
// right-looking coordinates of F1.  The state entering row j is Cb, the
// sensitivity of the correction window C_{j+1} (symmetric, both halves).
// The sensitivity of column j of L is assembled from
//   Lbar record j (when given), the log-determinant term 2 gl / L_jj on the
//   diagonal, and the solve term -ybar[j+d] z[j] of Table 1 (when given);
// then
//   lb_p   = Lb[1+p] + 2 (Cb l)_p
//   Qbar[j+1+p, j] = lb_p / L_jj
//   Qbar_jj = (Lb[0] - lb . l / L_jj) / (2 L_jj)
//   Cb' = [[-Qbar_jj, -Qbar_{1:}^T/2], [-Qbar_{1:}/2, Cb[0:K-1,0:K-1]]]
//       (= Kt^T Cb Kt + injection)
// ----------------------------------------------------------------------------
template <int K, typename T, bool REPLAY>
BO_HD void b2_chunk(int64_t a, int64_t b, int64_t n, BandP<const T> L, BandP<const T> Lbar,
                    double gl, const T *ybar, const T *z, BandP<T> Qb, LinMap<K> &st) {
  constexpr int K1 = Dim<K>::K1;
  constexpr int NS = Dim<K>::NS;
  double Cb[NS];
#pragma unroll
  for (int p = 0; p < K1; ++p)
#pragma unroll
    for (int q = 0; q <= p; ++q) Cb[six(p, q)] = REPLAY ? st.M[p][q] : 0.0;
  // ybar window: before row j, yw[d] = ybar[j+1+d] for d = 0..K-1
  double yw[K1];
  if (ybar) {
#pragma unroll
    for (int d = 0; d < K; ++d) yw[d] = (b + d < n) ? (double)ybar[b + d] : 0.0;
  }
  for (int64_t j = b - 1; j >= a; --j) {
    double r[K + 1], Lb[K + 1];
    load_rec<K, T>(L.p, L.diag, L.ld, j, n, r);
    if (Lbar.p) {
      load_rec<K, T>(Lbar.p, Lbar.diag, Lbar.ld, j, n, Lb);
    } else {
#pragma unroll
      for (int d = 0; d <= K; ++d) Lb[d] = 0.0;
    }
    double inv = 1.0 / r[0];
    Lb[0] += 2.0 * gl * inv;
    if (ybar) {
      double yj = (double)ybar[j], zj = (double)z[j];
      Lb[0] -= yj * zj;
#pragma unroll
      for (int d = 1; d <= K; ++d) Lb[d] -= yw[d - 1] * zj;
#pragma unroll
      for (int d = K - 1; d >= 1; --d) yw[d] = yw[d - 1];
      if (K > 0) yw[0] = yj;
    }
    double lb[K1], qb[K + 1];
    double dot = 0.0;
#pragma unroll
    for (int p = 0; p < K; ++p) {
      double acc = Lb[1 + p];
#pragma unroll
      for (int q = 0; q < K; ++q) acc += 2.0 * Cb[six(p, q)] * r[1 + q];
      lb[p] = acc;
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
    (void)lb;
  }
#pragma unroll
  for (int p = 0; p < K1; ++p) {
    st.v[p] = 0.0;
#pragma unroll
    for (int q = 0; q < K1; ++q) st.M[p][q] = (p < K && q < K) ? Cb[six(p, q)] : 0.0;
  }
}

}  // namespace bo
