// bandops_tile.hpp -- LDS-tiled row streaming for the chunked passes (device).
//
// Each lane of a wavefront walks its own chunk of rows.  Reading records lane
// by lane makes every load instruction touch 64 separate cache lines and stalls
// on every row.  Instead the wave streams tiles: for TR rows at a time it
// copies every lane's next TR records of each input array into LDS with
// wave-cooperative loads (consecutive lanes read consecutive elements of one
// lane's contiguous record run, written straight into LDS), waits once, and
// then each lane's stepper consumes its rows from LDS.  One workgroup is one
// wavefront.  Records must be packed (stride K+1).
#pragma once
#include "bandops_step.hpp"

namespace bo {
namespace tile {

constexpr int kWave = 64;
// LDS bytes one wavefront may use for its tiles (tiles plus tables stay under 40 KB: four wavefronts per CU).
constexpr int kTileBytes = 34816;

template <typename T> constexpr int band_row_bytes(int K) {
  return (K + 1) * (int)sizeof(T) + (sizeof(T) == 4 ? 8 : 0);   // + FP64 diagonal
}
template <int K, typename T, int NB, int NV> constexpr int tile_rows() {
  int bytes = NB * band_row_bytes<T>(K) + NV * (int)sizeof(T);
  int tr = bytes > 0 ? kTileBytes / (kWave * bytes) : 16;
  return tr < 2 ? 2 : (tr > 32 ? 32 : tr);
}

// Maximum over the wavefront (one workgroup = one wavefront).
__device__ __forceinline__ int64_t wave_max(int64_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    int64_t o = __shfl_xor(v, off, kWave);
    v = o > v ? o : v;
  }
  return v;
}

// LDS layout of one staged array: 64 segments (one per lane) of TR rows x W
// elements, copied as 4-byte pieces.  The segment pitch (in pieces) is padded
// so that lanes reading the same row offset hit different banks.
template <typename E, int W, int TR> struct Geom {
  static constexpr int PPS = TR * W * (int)sizeof(E) / 4;   // pieces per segment
  static constexpr int PITCH = sizeof(E) == 8 ? (((PPS / 2) % 2 == 0) ? PPS + 2 : PPS)
                                              : ((PPS % 2 == 0) ? PPS + 1 : PPS);
  static constexpr int WORDS = kWave * PITCH;               // 4-byte words
};

typedef __attribute__((address_space(3))) void *lds_ptr_t;

// Fill an LDS tile: for every lane s of the wave, the first cnt[s] * W
// elements at src[s] (contiguous records) land at dst + s * PITCH words.  Each
// instruction moves 64 consecutive 4-byte pieces of the flattened tile
// straight from global memory into LDS (no registers), so all loads of a tile
// are in flight together; the caller waits once.
template <typename E, int W, int TR>
__device__ __forceinline__ void lds_fill(uint32_t *dst, const E *const *src, const int *cnt, int lane) {
  using G = Geom<E, W, TR>;
#pragma unroll 8
  for (int k = 0; k < G::PITCH; ++k) {
    const int p = k * kWave + lane;
    const int s = p / G::PITCH;
    const int q = p - s * G::PITCH;
    const char *sp = (const char *)src[s];
    if (sp && q * 4 < cnt[s] * W * (int)sizeof(E))
      __builtin_amdgcn_global_load_lds((const void *)(sp + q * 4), (lds_ptr_t)(dst + k * kWave), 4, 0, 0);
  }
}

// A staged band input: records of the lane's problem (null when absent) and,
// in the mixed format, its FP64 diagonal.  `shift` offsets the staged rows
// from the processed rows (the B1 replay reads Sigma K+1 rows ahead).
template <typename T> struct BandIn {
  const T *p;
  const double *diag;
  int shift;
};
template <typename T> struct VecIn {
  const T *p;
  int shift;   // staged rows = processed rows + shift (values past n read 0)
};

// Streams rows [lo, hi) of each lane (ascending, or descending when DESC) and
// calls body(j, rec, val) per row with rec[b] = record j(+shift_b) of band b
// (slots past the matrix end zeroed) and val[v] = vector v at row j.
template <int K, typename T, int NB, int NV, bool DESC, class Body>
__device__ __forceinline__ void stream_rows(const BandIn<T> (&bands)[NB > 0 ? NB : 1],
                                            const VecIn<T> (&vecs)[NV > 0 ? NV : 1], int64_t lo,
                                            int64_t hi, int64_t n, int64_t ld, Body &&body) {
  constexpr int W = K + 1;
  constexpr int TR = tile_rows<K, T, NB, NV>();
  constexpr bool MIXED = sizeof(T) == 4;
  constexpr int NB1 = NB > 0 ? NB : 1, NV1 = NV > 0 ? NV : 1;
  using GB = Geom<T, W, TR>;
  using GD = Geom<double, 1, TR>;
  using GV = Geom<T, 1, TR>;
  __shared__ uint32_t sb[NB1][GB::WORDS];
  __shared__ uint32_t sd[MIXED ? NB1 : 1][MIXED ? GD::WORDS : 1];
  __shared__ uint32_t sv[NV1][NV > 0 ? GV::WORDS : 1];
  __shared__ const T *pb[NB1][kWave];
  __shared__ const double *pd[NB1][kWave];
  __shared__ const T *pv[NV1][kWave];
  __shared__ int cb[NB1][kWave];
  __shared__ int cv[NV1][kWave];

  const int lane = threadIdx.x;
  const int64_t len = hi > lo ? hi - lo : 0;
  const int64_t maxlen = wave_max(len);
  for (int64_t t0 = 0; t0 < maxlen; t0 += TR) {
    const int cnt = (int)(len - t0 < TR ? (len - t0 > 0 ? len - t0 : 0) : TR);
    const int64_t r0 = DESC ? hi - t0 - cnt : lo + t0;   // first row of this tile
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) {
      int64_t s0 = r0 + bands[bi].shift;
      int c = cnt;
      if (s0 + c > n) c = (int)(n - s0 > 0 ? n - s0 : 0);
      const bool on = bands[bi].p && c > 0;
      pb[bi][lane] = on ? bands[bi].p + s0 * ld : nullptr;
      pd[bi][lane] = (on && bands[bi].diag) ? bands[bi].diag + s0 : nullptr;
      cb[bi][lane] = c;
    }
#pragma unroll
    for (int vi = 0; vi < NV; ++vi) {
      int64_t s0 = r0 + vecs[vi].shift;
      int c = cnt;
      if (s0 + c > n) c = (int)(n - s0 > 0 ? n - s0 : 0);
      pv[vi][lane] = (vecs[vi].p && c > 0) ? vecs[vi].p + s0 : nullptr;
      cv[vi][lane] = c;
    }
    __syncthreads();
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) {
      lds_fill<T, W, TR>(sb[bi], pb[bi], cb[bi], lane);
      if (MIXED) lds_fill<double, 1, TR>(sd[MIXED ? bi : 0], pd[bi], cb[bi], lane);
    }
#pragma unroll
    for (int vi = 0; vi < NV; ++vi) lds_fill<T, 1, TR>(sv[vi], pv[vi], cv[vi], lane);
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
#pragma unroll 1
    for (int t = 0; t < TR; ++t) {
      if (t < cnt) {
        const int r = DESC ? cnt - 1 - t : t;
        const int64_t j = r0 + r;
        double rec[NB1][K + 1];
        double val[NV1];
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
          const int64_t js = j + bands[bi].shift;
          const T *row = (const T *)(sb[bi] + lane * GB::PITCH) + r * W;
#pragma unroll
          for (int d = 0; d <= K; ++d) {
            double x = (double)row[d];
            if (d == 0 && MIXED && bands[bi].diag)
              x = ((const double *)(sd[MIXED ? bi : 0] + lane * GD::PITCH))[r];
            rec[bi][d] = (bands[bi].p && js + d < n) ? x : 0.0;
          }
        }
#pragma unroll
        for (int vi = 0; vi < NV; ++vi)
          val[vi] = (vecs[vi].p && j + vecs[vi].shift < n)
                        ? (double)((const T *)(sv[vi] + lane * GV::PITCH))[r] : 0.0;
        body(j, rec, val);
      }
    }
    __syncthreads();
  }
}

}  // namespace tile
}  // namespace bo
