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
#include <type_traits>

#include "bandops_step.hpp"

namespace bo {
namespace tile {

constexpr int kWave = 64;
// LDS bytes one wavefront may use for its tiles: a quarter of the CU's 160 KB,
// so that four wavefronts (one per SIMD) stay resident.
#ifndef BO_TILE_BYTES
#define BO_TILE_BYTES 40960
#endif
constexpr int kTileBytes = BO_TILE_BYTES;
// Tile buffers per array.  With 2, the loads of a wave's next tile are issued
// before it steps through the current one (each buffer gets half the budget).
// The wait at the next tile then also covers the stores the row work has just
// issued (one counter tracks loads and stores), and halving the tiles doubles
// those waits: measured slower on every kernel that writes, so 1 is the
// default.
#ifndef BO_TILE_BUFS
#define BO_TILE_BUFS 1
#endif
constexpr int kTileBufs = BO_TILE_BUFS;

// Maximum over the wavefront (one workgroup = one wavefront).
__device__ __forceinline__ int64_t wave_max(int64_t v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    int64_t o = __shfl_xor(v, off, kWave);
    v = o > v ? o : v;
  }
  return v;
}

// LDS layout of one staged array: 64 segments (one per lane) of up to TR rows
// x W elements, packed back to back.  A segment occupies PPI pieces (16-byte
// pieces when every segment start of the tile is 16-byte aligned, else 4-byte
// pieces); PPI is made odd so that lanes reading the same row offset fall in
// different banks.  Geom gives both layouts and the LDS size of the larger.
template <typename E, int W, int TR> struct Geom {
  static constexpr int SEGB = TR * W * (int)sizeof(E);   // data bytes per segment
  static constexpr int odd(int x) { return x % 2 == 0 ? x + 1 : x; }
  static constexpr int PPI16 = odd((SEGB + 15) / 16);
  static constexpr int PPI4 = odd((SEGB + 3) / 4);
  static constexpr int BYTES16 = kWave * PPI16 * 16, BYTES4 = kWave * PPI4 * 4;
  static constexpr int WORDS = (BYTES16 > BYTES4 ? BYTES16 : BYTES4) / 4;
};

// LDS bytes of the tiles of NB bands and NV vectors at TR rows per tile.
template <int K, typename T, int NB, int NV, int TR> constexpr int tile_lds_bytes() {
  return NB * Geom<T, K + 1, TR>::WORDS * 4 + (sizeof(T) == 4 ? NB * Geom<double, 1, TR>::WORDS * 4 : 0) +
         NV * Geom<T, 1, TR>::WORDS * 4;
}
// Rows per tile: the most (up to 32) whose tiles (kTileBufs sets) fit the
// budget, at least 2.
template <int K, typename T, int NB, int NV, int TR = 32> constexpr int tile_rows() {
  if constexpr (TR <= 2) {
    return 2;
  } else {
    if constexpr (kTileBufs * tile_lds_bytes<K, T, NB, NV, TR>() <= kTileBytes) return TR;
    else return tile_rows<K, T, NB, NV, TR - 1>();
  }
}

// Vectors are staged VM band tiles at a time (VM * TR rows per vector tile):
// a vector segment is only 8 bytes per row, so short vector tiles waste most
// of every cache line they touch.  VM is the largest (up to 8) that keeps all
// tiles inside the budget, with 2 KB left for the compiler's own LDS.
template <int K, typename T, int NB, int NV, int TR, int VM = 8> constexpr int vec_mult() {
  if constexpr (VM <= 1 || NV == 0) {
    return 1;
  } else {
    constexpr int bands = NB * Geom<T, K + 1, TR>::WORDS * 4 + (sizeof(T) == 4 ? NB * Geom<double, 1, TR>::WORDS * 4 : 0);
    if constexpr (kTileBufs * (bands + NV * Geom<T, 1, TR * VM>::WORDS * 4) <= kTileBytes - 2048) return VM;
    else return vec_mult<K, T, NB, NV, TR, VM - 1>();
  }
}

typedef __attribute__((address_space(3))) void *lds_ptr_t;
template <typename E> using lds_cptr = const __attribute__((address_space(3))) E *;

// Load the pieces of every segment of a tile, PPI pieces of PIECE bytes per
// segment, segment s at d + s * PPI * PIECE.  When a segment fits in one
// instruction (PPI <= 64), each instruction covers 64 / PPI consecutive
// segments and a lane learns its segment's source address by a cross-lane
// shuffle; otherwise each segment takes ceil(PPI / 64) instructions and its
// address is read from its lane (uniform).
// One piece load into LDS (the size operand of the builtin must be a literal).
template <int PIECE>
__device__ __forceinline__ void load_piece(uint64_t src, __attribute__((address_space(3))) char *dst) {
  if constexpr (PIECE == 16)
    __builtin_amdgcn_global_load_lds((const void *)src, (lds_ptr_t)dst, 16, 0, 0);
  else
    __builtin_amdgcn_global_load_lds((const void *)src, (lds_ptr_t)dst, 4, 0, 0);
}

template <int PPI, int PIECE>
__device__ __forceinline__ void fill_pieces(__attribute__((address_space(3))) char *d, uint64_t my_src,
                                            int my_bytes, int lane) {
  if constexpr (PPI <= kWave) {
    constexpr int NSEG = kWave / PPI;
    constexpr int NI = (kWave + NSEG - 1) / NSEG;
    const int sl = lane / PPI, q = lane - sl * PPI;
#pragma unroll 4
    for (int i = 0; i < NI; ++i) {
      const int s = i * NSEG + sl;
      const int ss = s < kWave ? s : kWave - 1;
      const uint64_t sp = __shfl(my_src, ss, kWave);
      const int nb = __shfl(my_bytes, ss, kWave);
      if (sl < NSEG && s < kWave && q * PIECE < nb) load_piece<PIECE>(sp + q * PIECE, d + i * NSEG * PPI * PIECE);
    }
  } else {
    constexpr int IPS = (PPI + kWave - 1) / kWave;
#pragma unroll 2
    for (int s = 0; s < kWave; ++s) {
      const uint64_t sp = ((uint64_t)__builtin_amdgcn_readlane((uint32_t)(my_src >> 32), s) << 32) |
                          (uint32_t)__builtin_amdgcn_readlane((uint32_t)my_src, s);
      const int nb = __builtin_amdgcn_readlane(my_bytes, s);
      if (nb <= 0) continue;
#pragma unroll
      for (int p = 0; p < IPS; ++p) {
        const int q = p * kWave + lane;
        if (q * PIECE < nb) load_piece<PIECE>(sp + q * PIECE, d + (s * PPI + p * kWave) * PIECE);
      }
    }
  }
}

// Fill an LDS tile: lane s's cnt_s * W elements at src_s (contiguous records;
// src_s, cnt_s are lane s's my_src, my_cnt) land in segment s, straight from
// global memory into LDS so that every load of a tile is in flight at once;
// the caller waits once.  Uses 16-byte pieces when every segment start is
// 16-byte aligned, else 4-byte pieces.  Returns the segment pitch in bytes.
template <typename E, int W, int TR>
__device__ __forceinline__ int lds_fill(uint32_t *dst, const E *my_src, int my_cnt, int lane) {
  using G = Geom<E, W, TR>;
  const int my_bytes = (my_src && my_cnt > 0) ? my_cnt * W * (int)sizeof(E) : 0;
  const bool ok16 = my_bytes == 0 || (((uint64_t)my_src & 15) == 0);
  __attribute__((address_space(3))) char *d = (__attribute__((address_space(3))) char *)(lds_ptr_t)dst;
  if (__all(ok16)) {
    fill_pieces<G::PPI16, 16>(d, (uint64_t)my_src, my_bytes, lane);
    return G::PPI16 * 16;
  }
  fill_pieces<G::PPI4, 4>(d, (uint64_t)my_src, my_bytes, lane);
  return G::PPI4 * 4;
}

// Fill an LDS tile from an interleaved band: `bytes` contiguous bytes (a
// multiple of 16, 16-byte aligned source) copied in 16-byte pieces, piece q
// by lane q % 64 of instruction q / 64; LDS receives the block unchanged.
__device__ __forceinline__ void il_fill(uint32_t *dst, const void *src, int bytes, int lane) {
  __attribute__((address_space(3))) char *d = (__attribute__((address_space(3))) char *)(lds_ptr_t)dst;
  const char *sp = (const char *)src;
  const int np = bytes >> 4;
#pragma unroll 4
  for (int i = 0; i < np; i += kWave)
    if (i + lane < np) load_piece<16>((uint64_t)(sp + (int64_t)(i + lane) * 16), d + i * 16);
}

// A staged band input: records of the lane's problem (null when absent) and,
// in the mixed format, its FP64 diagonal.  `shift` offsets the staged rows
// from the processed rows (the B1 replay reads Sigma K+1 rows ahead).
//
// An interleaved band (a bit of stream_rows' ILB mask) holds the chunks of one
// wavefront row by row: row r of the chunk of lane l (global row lo_l + r) is
// record r * 64 + l of the array that p points at, so one tile of every lane
// is one contiguous block.  Interleaved bands are FP64 only (no diag).
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
//
// Tiles are laid out in chunk-relative rows r = j - lo: ascending, tile i
// covers r in [i TR, (i+1) TR); descending, tile i covers r in
// [top - (i+1) TR, top - i TR), with top the lane's own chunk length, or the
// wave's longest chunk when an interleaved array is staged (then a lane with a
// shorter chunk starts later, and the tile's rows are common to the wave).
// Each lane takes the rows of a tile that lie in [0, hi - lo).
//
// Tile i of every array goes to buffer i % kTileBufs.  With two buffers the
// order per tile is: wait for tile i's loads, barrier, issue tile i+1's loads
// into the other buffer (whose tile i-1 every lane has finished with at the
// barrier), step through tile i.  A vector tile spans VM band tiles and
// alternates between its own two buffers the same way.
//
// ILB / ILV: bit b set when band (vector) b is interleaved (FP64 only); a
// vector is then interleaved like a band of one element per record.
template <int K, typename T, int NB, int NV, bool DESC, unsigned ILB = 0u, unsigned ILV = 0u, class Body>
__device__ __forceinline__ void stream_rows(const BandIn<T> (&bands)[NB > 0 ? NB : 1],
                                            const VecIn<T> (&vecs)[NV > 0 ? NV : 1], int64_t lo,
                                            int64_t hi, int64_t n, int64_t ld, Body &&body) {
  constexpr int W = K + 1;
  constexpr int TR = tile_rows<K, T, NB, NV>();
  constexpr int VM = vec_mult<K, T, NB, NV, TR>();
  constexpr int VR = TR * VM;   // rows per vector tile
  constexpr bool MIXED = sizeof(T) == 4;
  constexpr int NB1 = NB > 0 ? NB : 1, NV1 = NV > 0 ? NV : 1;
  constexpr int NBUF = kTileBufs;
  static_assert(NBUF == 1 || NBUF == 2, "one or two tile buffers");
  static_assert((ILB == 0u && ILV == 0u) || !MIXED, "interleaved arrays are FP64");
  using GB = Geom<T, W, TR>;
  using GD = Geom<double, 1, TR>;
  using GV = Geom<T, 1, VR>;
  static_assert(kWave * TR * W * (int)sizeof(T) <= GB::WORDS * 4, "an interleaved tile fits the band buffer");
  static_assert(kWave * VR * (int)sizeof(T) <= GV::WORDS * 4, "an interleaved vector tile fits its buffer");
  __shared__ __attribute__((aligned(16))) uint32_t sb[NBUF][NB1][GB::WORDS];
  __shared__ __attribute__((aligned(16))) uint32_t sd[NBUF][MIXED ? NB1 : 1][MIXED ? GD::WORDS : 1];
  __shared__ __attribute__((aligned(16))) uint32_t sv[NBUF][NV1][NV > 0 ? GV::WORDS : 1];

  const int lane = threadIdx.x;
  const int64_t len = hi > lo ? hi - lo : 0;
  const int64_t maxlen = wave_max(len);
  // Descending tiles count down from `top`: the wave's longest chunk when an
  // interleaved array is staged (its tiles are blocks common to the wave),
  // else each lane's own chunk end.
  constexpr bool any_il = (ILB | ILV) != 0u;
  const int64_t top = any_il ? maxlen : len;
  // Per band: where the lane's rows of the current tile start in LDS (bytes)
  // and the LDS distance between consecutive rows.  A segment band keeps the
  // lane's rows together (pitch per lane); an interleaved band keeps the
  // block as loaded (64 records per row).
  int rbase[NBUF][NB1], dbase[NBUF][NB1];
  int pv0[NV1], pv1[NV1];   // vector: lane's start (bytes) per buffer
  int64_t vb0 = 0, vb1 = 0;
  auto band_il = [](int bi) constexpr { return ((ILB >> bi) & 1u) != 0u; };
  auto vec_il = [](int vi) constexpr { return ((ILV >> vi) & 1u) != 0u; };
#pragma unroll
  for (int vi = 0; vi < NV1; ++vi) pv0[vi] = pv1[vi] = 0;
#pragma unroll
  for (int bi = 0; bi < NB1; ++bi)
#pragma unroll
    for (int u = 0; u < NBUF; ++u) rbase[u][bi] = dbase[u][bi] = 0;
  // chunk-relative rows [r_lo, r_hi) of tile `it` (the wave's block) and the
  // lane's share [r_lo, min(r_hi, len)) of it
  auto tile_span = [&](int64_t it, int rows, int64_t &r_lo, int64_t &r_hi) {
    const int64_t t0 = it * TR;
    if (DESC) {
      r_hi = top - t0;
      r_lo = r_hi - rows > 0 ? r_hi - rows : 0;
    } else {
      r_lo = t0;
      r_hi = t0 + rows < maxlen ? t0 + rows : maxlen;
    }
  };
  // Issue the loads of tile `it` into band buffer U.
  auto fill = [&](int64_t it, auto Uc) {
    constexpr int U = decltype(Uc)::value;
    int64_t r_lo, r_hi;
    tile_span(it, TR, r_lo, r_hi);
    const int64_t mine = (r_hi < len ? r_hi : len) - r_lo;
    const int cnt = (int)(mine > 0 ? mine : 0);
    const int64_t r0 = lo + r_lo;
#pragma unroll
    for (int bi = 0; bi < NB; ++bi) {
      if (band_il(bi)) {
        // the wave's block of rows [r_lo, r_hi) (shifted), every lane's slot
        const int64_t b0 = r_lo + bands[bi].shift;
        const int rows = (int)(r_hi - r_lo);
        if (bands[bi].p && rows > 0)
          il_fill(sb[U][bi], bands[bi].p + b0 * kWave * W, rows * kWave * W * (int)sizeof(T), lane);
        rbase[U][bi] = lane * W * (int)sizeof(T);
      } else {
        int64_t s0 = r0 + bands[bi].shift;
        int c = cnt;
        if (s0 + c > n) c = (int)(n - s0 > 0 ? n - s0 : 0);
        const bool on = bands[bi].p && c > 0;
        rbase[U][bi] = lane * lds_fill<T, W, TR>(sb[U][bi], on ? bands[bi].p + s0 * ld : nullptr, c, lane);
        if (MIXED)
          dbase[U][bi] = lane * lds_fill<double, 1, TR>(sd[U][MIXED ? bi : 0],
                                                        (on && bands[bi].diag) ? bands[bi].diag + s0 : nullptr, c,
                                                        lane);
      }
    }
    if (NV > 0 && it % VM == 0) {   // next vector tile: rows of the following VM band tiles
      const bool v1 = NBUF > 1 && ((it / VM) & 1);
      int64_t v_lo, v_hi;
      tile_span(it, VR, v_lo, v_hi);
      const int64_t vmine = (v_hi < len ? v_hi : len) - v_lo;
      const int vcnt = (int)(vmine > 0 ? vmine : 0);
      const int64_t vb = lo + v_lo;
      if (v1) vb1 = vb;
      else vb0 = vb;
#pragma unroll
      for (int vi = 0; vi < NV; ++vi) {
        // buffer 1 of vector vi lies NV1 * GV::WORDS words past buffer 0
        uint32_t *vdst = &sv[0][vi][0] + (v1 ? (NBUF - 1) * NV1 * GV::WORDS : 0);
        int pv;
        if (vec_il(vi)) {
          const int rows = (int)(v_hi - v_lo);
          if (vecs[vi].p && rows > 0)
            il_fill(vdst, vecs[vi].p + (v_lo + vecs[vi].shift) * kWave, rows * kWave * (int)sizeof(T), lane);
          pv = lane * (int)sizeof(T);
        } else {
          int64_t s0 = vb + vecs[vi].shift;
          int c = vcnt;
          if (s0 + c > n) c = (int)(n - s0 > 0 ? n - s0 : 0);
          const T *src = (vecs[vi].p && c > 0) ? vecs[vi].p + s0 : nullptr;
          pv = lane * lds_fill<T, 1, VR>(vdst, src, c, lane);
        }
        if (v1) pv1[vi] = pv;
        else pv0[vi] = pv;
      }
    }
  };
  // Step through the rows of tile `it`, staged in band buffer U.
  auto consume = [&](int64_t it, auto Uc) {
    constexpr int U = decltype(Uc)::value;
    const bool v1 = NBUF > 1 && ((it / VM) & 1);
    const int64_t vbase = v1 ? vb1 : vb0;
    int64_t r_lo, r_hi;
    tile_span(it, TR, r_lo, r_hi);
    // the lane's rows of the tile: [r_lo, r_lo + cnt), visited downwards when
    // descending (the per-row work below is 32-bit)
    const int64_t mine = (r_hi < len ? r_hi : len) - r_lo;
    const int cnt = (int)(mine > 0 ? mine : 0);
    const int64_t row0 = lo + r_lo;
#pragma unroll 1
    for (int t = 0; t < TR; ++t) {
      if (t < cnt) {
        const int lr = DESC ? cnt - 1 - t : t;   // row within the tile
        const int64_t j = row0 + lr;
        double rec[NB1][K + 1];
        double val[NV1];
#pragma unroll
        for (int bi = 0; bi < NB; ++bi) {
          const int64_t js = j + bands[bi].shift;
          constexpr int rs0 = W * (int)sizeof(T);
          const int rstride = band_il(bi) ? kWave * rs0 : rs0;
          lds_cptr<T> row = (lds_cptr<T>)((lds_cptr<char>)(lds_ptr_t)sb[U][bi] + rbase[U][bi] + lr * rstride);
#pragma unroll
          for (int d = 0; d <= K; ++d) {
            double x = (double)row[d];
            if (d == 0 && MIXED && bands[bi].diag)
              x = ((lds_cptr<double>)((lds_cptr<char>)(lds_ptr_t)sd[U][MIXED ? bi : 0] + dbase[U][bi]))[lr];
            rec[bi][d] = (bands[bi].p && js + d < n) ? x : 0.0;
          }
        }
        const int rv = (int)(j - vbase);
#pragma unroll
        for (int vi = 0; vi < NV; ++vi) {
          // buffer 1 of vector vi lies NV1 * GV::WORDS words past buffer 0
          const int voff = v1 ? (NBUF - 1) * NV1 * GV::WORDS * 4 + pv1[vi] : pv0[vi];
          const int vstride = (vec_il(vi) ? kWave : 1) * (int)sizeof(T);
          lds_cptr<char> vrow = (lds_cptr<char>)(lds_ptr_t)sv[0][vi] + voff + rv * vstride;
          val[vi] = (vecs[vi].p && j + vecs[vi].shift < n) ? (double)*(lds_cptr<T>)vrow : 0.0;
        }
        body(j, rec, val);
      }
    }
  };
  using C0 = std::integral_constant<int, 0>;
  using CL = std::integral_constant<int, NBUF - 1>;
  const int64_t ntile = (maxlen + TR - 1) / TR;
  if constexpr (NBUF == 1) {
#pragma unroll 1
    for (int64_t it = 0; it < ntile; ++it) {
      fill(it, C0{});
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      consume(it, C0{});
      __syncthreads();
    }
  } else {
    // wait for tile it, barrier (every lane is done with the other buffer),
    // issue tile it+1 into the other buffer, step through tile it
    if (ntile > 0) fill(0, C0{});
#pragma unroll 1
    for (int64_t it = 0; it < ntile; it += 2) {
      __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      if (it + 1 < ntile) fill(it + 1, CL{});
      consume(it, C0{});
      if (it + 1 < ntile) {
        __builtin_amdgcn_s_waitcnt(0);
        __syncthreads();
        if (it + 2 < ntile) fill(it + 2, C0{});
        consume(it + 1, CL{});
      }
    }
  }
}

}  // namespace tile
}  // namespace bo
