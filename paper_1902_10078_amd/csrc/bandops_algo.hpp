// bandops_algo.hpp -- state algebra of the chunked banded passes.
//
// Every pass of the library walks rows of a banded matrix in order, carrying a
// small state (a k x k window and/or a k-vector); the row steppers are in
// bandops_step.hpp.  To spread one long matrix over the chip, rows are cut into
// chunks; a chunk is processed twice:
//   * a summary: the chunk's effect on the state, independent of what enters it;
//   * after a scan over the summaries has produced every chunk's exact incoming
//     state, a replay that rewrites the chunk's outputs in natural row order.
// Nothing is permuted, so the outputs are those of the sequential algorithms
// of the paper (Algorithms 1-4 and the Table 1 compositions) up to rounding.
// This file holds the summaries' types and how they compose and apply.
//
// All state lives in registers: K (the number of sub-diagonals) is a template
// parameter, so every window index is a compile-time constant after
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

// Largest bandwidth whose replays also produce the next pass's chunk maps.
// Above it the fused replay kernels no longer fit in registers (they spill)
// and gave wrong next-pass maps on gfx950 while the same code is exact on the
// host; those bandwidths run separate summary kernels instead, and their
// steppers and kernels are compiled without the fused accumulations.
#ifndef BO_KMAX_FUSED
#define BO_KMAX_FUSED 5
#endif
constexpr int KMAX_FUSED = BO_KMAX_FUSED;

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

// A vector argument: element j at p[j * S] (S = 1 for a caller's vector; a
// chunk-interleaved workspace vector has S = 64).
template <typename T, int S = 1> struct VecP {
  T *p = nullptr;
  BO_HD VecP() {}
  BO_HD VecP(T *q) : p(q) {}
  BO_HD explicit operator bool() const { return p != nullptr; }
  BO_HD T &operator[](int64_t j) const { return p[j * S]; }
};

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

// Composite of two consecutive linear maps, first (P1, m1) then (P2, m2),
// written into (P1, m1).
template <int K, bool DESC>
BO_HD void lin_compose(double (&P1)[Dim<K>::K1][Dim<K>::K1], LinMap<K> &m1,
                       const double (&P2)[Dim<K>::K1][Dim<K>::K1], const LinMap<K> &m2) {
  mat_mul_acc<K, DESC>(P1, P2);
  lin_apply<K, DESC>(P2, m2, m1);
}

}  // namespace bo
