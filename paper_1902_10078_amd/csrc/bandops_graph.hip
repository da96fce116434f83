// bandops_graph.hip -- GMRF precisions on graphs (Section 2: a precision with
// Q_ij = 0 off the graph's edges is sparse, and its bandwidth depends on the
// node ordering; Section 5 orders a road network with reverse Cuthill-McKee
// before using the banded operators).
//   bo_rcm               host: the reverse Cuthill-McKee ordering of a CSR
//                        pattern;
//   bo_csr_permute       host: the pattern of P Q P^T (rows in the new order,
//                        columns sorted) and where each of its entries was;
//   bo_csr_to_band       GPU: the lower band of a symmetric CSR matrix whose
//                        rows are in band order, for several value sets;
//   bo_band_to_csr_grad  GPU: the gradient with respect to Q's CSR entries
//                        from the gradient with respect to the band.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstdint>
#include <functional>
#include <string>
#include <utility>
#include <vector>

#include "bandops.h"

bo_status bo_set_error(bo_status st, const std::string &msg);
int bo_profile_graph(int which, hipStream_t s, const std::function<int()> &launch);

namespace {

bo_status gfail(bo_status s, const std::string &m) { return bo_set_error(s, m); }

// Validates a CSR pattern on the host: indptr[0] = 0, non-decreasing, column
// indices in [0, n).
bool csr_ok(int64_t n, const int64_t *indptr, const int64_t *indices) {
  if (indptr[0] != 0) return false;
  for (int64_t i = 0; i < n; ++i)
    if (indptr[i + 1] < indptr[i]) return false;
  for (int64_t e = 0; e < indptr[n]; ++e)
    if (indices[e] < 0 || indices[e] >= n) return false;
  return true;
}

constexpr int kRows = 256;
constexpr int kStageLd = 16;   // records of at most 16 elements are staged in LDS (32 KB in FP64)

__global__ void __launch_bounds__(kRows) k_zero_counter(int64_t *c) {
  if (threadIdx.x == 0) c[0] = 0;
}

// One thread per (value set, band record) of a CSR matrix whose rows are
// already in band order: record j is row j from the diagonal rightwards,
// the entries (j, c), c >= j, at slot c - j (the matrix is symmetric).  The
// record is built in registers and written whole (pads 0); entries past the
// band are counted.
template <typename T, int W>
__global__ void __launch_bounds__(kRows)
    k_csr_to_band(int64_t n, int32_t nsets, const int64_t *indptr, const int64_t *indices, const double *vals,
                  int64_t nnz, int32_t k, int64_t ld, T *band, double *diag, int64_t *dropped) {
  const int64_t total = n * nsets;
  const int64_t t0 = (int64_t)blockIdx.x * kRows, t = t0 + threadIdx.x;
  const bool valid = t < total;
  double rec[W];
#pragma unroll
  for (int s = 0; s < W; ++s) rec[s] = 0.0;
  if (valid) {
    const int64_t set = t / n, j = t - set * n;
    const double *v = vals + set * nnz;
    int64_t lost = 0;
    for (int64_t e = indptr[j]; e < indptr[j + 1]; ++e) {
      const int64_t d = indices[e] - j;
      if (d < 0) continue;
      if (d > k) {
        ++lost;
        continue;
      }
#pragma unroll
      for (int s = 0; s < W; ++s)
        if (s == d) rec[s] = v[e];
    }
    if (diag) diag[t] = rec[0];
    if (lost) atomicAdd((unsigned long long *)dropped, (unsigned long long)lost);
  }
  // Record t of the launch lives at band + t ld (t = set n + j), so a
  // block's records form one contiguous range.  Narrow records go through LDS
  // and out with consecutive threads on consecutive elements (every thread of
  // the block reaches the barrier); wide ones are stored directly.
  if (ld <= kStageLd) {
    __shared__ T stage[kRows * kStageLd];
    const int64_t cnt = total - t0 < kRows ? total - t0 : kRows;
    if (valid) {
#pragma unroll
      for (int s = 0; s < W; ++s)
        if (s < ld) stage[threadIdx.x * ld + s] = (T)rec[s];
      for (int64_t s = W; s < ld; ++s) stage[threadIdx.x * ld + s] = (T)0;
    }
    __syncthreads();
    T *dst = band + t0 * ld;
    for (int64_t e = threadIdx.x; e < cnt * ld; e += kRows) dst[e] = stage[e];
    return;
  }
  if (!valid) return;
  T *out = band + t * ld;
#pragma unroll
  for (int s = 0; s < W; ++s)
    if (s < ld) out[s] = (T)rec[s];
  for (int64_t s = W; s < ld; ++s) out[s] = (T)0;
}

// The reverse: the entries of row j that record j read get the band's
// gradient there, the row's other entries 0.  Narrow records come in through
// LDS like the assembly's go out (every thread of the block reaches the
// barrier).
template <typename T>
__global__ void __launch_bounds__(kRows)
    k_band_to_csr(int64_t n, int32_t nsets, const int64_t *indptr, const int64_t *indices, int64_t nnz, int32_t k,
                  int64_t ld, const T *gband, const double *gdiag, double *gvals) {
  const int64_t total = n * nsets;
  const int64_t t0 = (int64_t)blockIdx.x * kRows, t = t0 + threadIdx.x;
  const T *g = gband + t * ld;
  if (ld <= kStageLd) {
    __shared__ T stage[kRows * kStageLd];
    const int64_t cnt = total - t0 < kRows ? total - t0 : kRows;
    const T *src = gband + t0 * ld;
    for (int64_t e = threadIdx.x; e < cnt * ld; e += kRows) stage[e] = src[e];
    __syncthreads();
    g = stage + threadIdx.x * ld;
  }
  if (t >= total) return;
  const int64_t set = t / n, j = t - set * n;
  double *gv = gvals + set * nnz;
  for (int64_t e = indptr[j]; e < indptr[j + 1]; ++e) {
    const int64_t d = indices[e] - j;
    double x = 0.0;
    if (d >= 0 && d <= k) x = (d == 0 && gdiag) ? gdiag[t] : (double)g[d];
    gv[e] = x;
  }
}

unsigned grid_for(int64_t count) { return (unsigned)((count + kRows - 1) / kRows); }

}  // namespace

extern "C" bo_status bo_rcm(int64_t n, const int64_t *indptr, const int64_t *indices, int64_t *perm, int64_t *iperm,
                            int64_t *bandwidth) {
  if (n < 0 || !indptr || (n > 0 && (!indices || !perm))) return gfail(BO_EINVAL, "bo_rcm: bad argument");
  if (!csr_ok(n, indptr, indices)) return gfail(BO_EINVAL, "bo_rcm: malformed CSR pattern");
  // adjacency without self-loops or repeats
  std::vector<int64_t> adj_ptr(n + 1, 0), adj;
  adj.reserve(indptr[n]);
  for (int64_t i = 0; i < n; ++i) {
    const size_t s = adj.size();
    for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e)
      if (indices[e] != i) adj.push_back(indices[e]);
    std::sort(adj.begin() + s, adj.end());
    adj.erase(std::unique(adj.begin() + s, adj.end()), adj.end());
    adj_ptr[i + 1] = (int64_t)adj.size();
  }
  std::vector<int64_t> deg(n);
  for (int64_t i = 0; i < n; ++i) deg[i] = adj_ptr[i + 1] - adj_ptr[i];
  auto before = [&](int64_t x, int64_t y) { return deg[x] != deg[y] ? deg[x] < deg[y] : x < y; };
  std::vector<int64_t> starts(n);
  for (int64_t i = 0; i < n; ++i) starts[i] = i;
  std::sort(starts.begin(), starts.end(), before);
  // Cuthill-McKee: breadth-first from each component's lowest (degree, index)
  // node; a visited node's unvisited neighbours join by (degree, index)
  std::vector<char> seen(n, 0);
  std::vector<int64_t> order;
  order.reserve(n);
  std::vector<int64_t> fresh;
  for (int64_t s : starts) {
    if (seen[s]) continue;
    seen[s] = 1;
    order.push_back(s);
    for (size_t head = order.size() - 1; head < order.size(); ++head) {
      const int64_t i = order[head];
      fresh.clear();
      for (int64_t e = adj_ptr[i]; e < adj_ptr[i + 1]; ++e)
        if (!seen[adj[e]]) fresh.push_back(adj[e]);
      std::sort(fresh.begin(), fresh.end(), before);
      for (int64_t j : fresh) {
        seen[j] = 1;
        order.push_back(j);
      }
    }
  }
  int64_t bw = 0;
  for (int64_t t = 0; t < n; ++t) perm[t] = order[n - 1 - t];
  std::vector<int64_t> inv(n);
  for (int64_t t = 0; t < n; ++t) inv[perm[t]] = t;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e) bw = std::max<int64_t>(bw, std::llabs(inv[i] - inv[indices[e]]));
  if (iperm)
    for (int64_t i = 0; i < n; ++i) iperm[i] = inv[i];
  if (bandwidth) *bandwidth = bw;
  return BO_OK;
}

extern "C" bo_status bo_csr_permute(int64_t n, const int64_t *indptr, const int64_t *indices, const int64_t *perm,
                                    const int64_t *iperm, int64_t *out_indptr, int64_t *out_indices, int64_t *map) {
  if (n < 0 || !indptr || !out_indptr || (n > 0 && (!indices || !perm || !iperm || !out_indices || !map)))
    return gfail(BO_EINVAL, "bo_csr_permute: bad argument");
  if (!csr_ok(n, indptr, indices)) return gfail(BO_EINVAL, "bo_csr_permute: malformed CSR pattern");
  for (int64_t t = 0; t < n; ++t)
    if (perm[t] < 0 || perm[t] >= n || iperm[perm[t]] != t)
      return gfail(BO_EINVAL, "bo_csr_permute: perm and iperm are not inverse permutations");
  std::vector<std::pair<int64_t, int64_t>> row;
  out_indptr[0] = 0;
  int64_t o = 0;
  for (int64_t j = 0; j < n; ++j) {
    const int64_t i = perm[j];
    row.clear();
    for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e) row.emplace_back(iperm[indices[e]], e);
    std::sort(row.begin(), row.end());
    for (const auto &ce : row) {
      out_indices[o] = ce.first;
      map[o] = ce.second;
      ++o;
    }
    out_indptr[j + 1] = o;
  }
  return BO_OK;
}

template <typename T>
int launch_csr_to_band(int64_t n, int32_t nsets, const int64_t *indptr, const int64_t *indices, const double *vals,
                       int64_t nnz, int32_t k, int64_t ld, T *band, double *diag, int64_t *dropped,
                       hipStream_t stream) {
  const dim3 grid(grid_for(n * nsets)), blk(kRows);
#define BO_CSR_W(WW)                                                                                          \
  hipLaunchKernelGGL((k_csr_to_band<T, WW>), grid, blk, 0, stream, n, nsets, indptr, indices, vals, nnz, k, ld, \
                     band, diag, dropped)
  if (k < 4) BO_CSR_W(4);
  else if (k < 8) BO_CSR_W(8);
  else if (k < 13) BO_CSR_W(13);
  else if (k < 32) BO_CSR_W(32);
  else BO_CSR_W(65);
#undef BO_CSR_W
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

extern "C" bo_status bo_csr_to_band(bo_prec prec, int64_t n, int32_t nsets, const int64_t *indptr,
                                    const int64_t *indices, int64_t nnz, const double *vals, int32_t k, int64_t ld,
                                    void *band, double *diag, int64_t *dropped, hipStream_t stream) {
  if (prec != BO_F64 && prec != BO_MIXED) return gfail(BO_EINVAL, "unknown precision");
  if (n < 0 || nsets < 0 || nnz < 0 || k < 0 || k > 64 || ld < k + 1)
    return gfail(BO_EINVAL, "bo_csr_to_band: bad sizes");
  if (n > 0 && nsets > 0 && (!indptr || !indices || !vals || !band || !dropped))
    return gfail(BO_EINVAL, "bo_csr_to_band: null array");
  if ((prec == BO_MIXED) != (diag != nullptr))
    return gfail(BO_EINVAL, "bo_csr_to_band: the FP64 diagonal is for BO_MIXED only, and required there");
  if (n == 0 || nsets == 0) return BO_OK;
  int e = bo_profile_graph(0, stream, [&] {
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(kRows), 0, stream, dropped);
    return prec == BO_F64 ? launch_csr_to_band<double>(n, nsets, indptr, indices, vals, nnz, k, ld, (double *)band,
                                                      diag, dropped, stream)
                          : launch_csr_to_band<float>(n, nsets, indptr, indices, vals, nnz, k, ld, (float *)band, diag,
                                                     dropped, stream);
  });
  return e ? gfail(BO_EDEVICE, "bo_csr_to_band: kernel launch failed") : BO_OK;
}

extern "C" bo_status bo_band_to_csr_grad(bo_prec prec, int64_t n, int32_t nsets, const int64_t *indptr,
                                         const int64_t *indices, int64_t nnz, int32_t k, int64_t ld,
                                         const void *gband, const double *gdiag, double *gvals, hipStream_t stream) {
  if (prec != BO_F64 && prec != BO_MIXED) return gfail(BO_EINVAL, "unknown precision");
  if (n < 0 || nsets < 0 || nnz < 0 || k < 0 || ld < k + 1) return gfail(BO_EINVAL, "bo_band_to_csr_grad: bad sizes");
  if (n > 0 && nsets > 0 && (!indptr || !indices || !gband || !gvals))
    return gfail(BO_EINVAL, "bo_band_to_csr_grad: null array");
  if ((prec == BO_MIXED) != (gdiag != nullptr))
    return gfail(BO_EINVAL, "bo_band_to_csr_grad: the FP64 diagonal is for BO_MIXED only, and required there");
  if (n == 0 || nsets == 0) return BO_OK;
  int e = bo_profile_graph(1, stream, [&] {
    const dim3 grid(grid_for(n * nsets)), blk(kRows);
    if (prec == BO_F64)
      hipLaunchKernelGGL(k_band_to_csr<double>, grid, blk, 0, stream, n, nsets, indptr, indices, nnz, k, ld,
                         (const double *)gband, gdiag, gvals);
    else
      hipLaunchKernelGGL(k_band_to_csr<float>, grid, blk, 0, stream, n, nsets, indptr, indices, nnz, k, ld,
                         (const float *)gband, gdiag, gvals);
    return hipGetLastError() == hipSuccess ? 0 : -2;
  });
  return e ? gfail(BO_EDEVICE, "bo_band_to_csr_grad: kernel launch failed") : BO_OK;
}
