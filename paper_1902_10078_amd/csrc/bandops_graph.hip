// bandops_graph.hip -- GMRF precisions on graphs (Section 2: a precision with
// Q_ij = 0 off the graph's edges is sparse, and its bandwidth depends on the
// node ordering; Section 5 orders a road network with reverse Cuthill-McKee
// before using the banded operators).
//   bo_rcm               host: the reverse Cuthill-McKee ordering of a CSR
//                        pattern;
//   bo_csr_to_band       GPU: the lower band of P Q P^T from Q's CSR entries;
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

template <typename T> __global__ void __launch_bounds__(kRows) k_fill_band(int64_t count, T *p, double *d, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * kRows + threadIdx.x;
  if (t < count) p[t] = (T)0;
  if (d && t < n) d[t] = 0.0;
}

__global__ void __launch_bounds__(kRows) k_zero_counter(int64_t *c) {
  if (threadIdx.x == 0) c[0] = 0;
}

// One thread per row of Q: its entries (i, j) with inv[i] >= inv[j] land at
// record inv[j], slot inv[i] - inv[j] of the band; entries below the band are
// counted.
template <typename T>
__global__ void __launch_bounds__(kRows)
    k_csr_to_band(int64_t n, const int64_t *indptr, const int64_t *indices, const double *vals, const int64_t *iperm,
                  int32_t k, int64_t ld, T *band, double *diag, int64_t *dropped) {
  const int64_t i = (int64_t)blockIdx.x * kRows + threadIdx.x;
  if (i >= n) return;
  const int64_t a = iperm[i];
  int64_t lost = 0;
  for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e) {
    const int64_t b = iperm[indices[e]];
    if (a < b) continue;
    if (a - b > k) {
      ++lost;
      continue;
    }
    band[b * ld + (a - b)] = (T)vals[e];
    if (a == b && diag) diag[b] = vals[e];
  }
  if (lost) atomicAdd((unsigned long long *)dropped, (unsigned long long)lost);
}

// One thread per row of Q: the entry (i, j) that the band assembly placed
// gets the band's gradient there; the entries it did not read get 0.
template <typename T>
__global__ void __launch_bounds__(kRows)
    k_band_to_csr(int64_t n, const int64_t *indptr, const int64_t *indices, const int64_t *iperm, int32_t k,
                  int64_t ld, const T *gband, const double *gdiag, double *gvals) {
  const int64_t i = (int64_t)blockIdx.x * kRows + threadIdx.x;
  if (i >= n) return;
  const int64_t a = iperm[i];
  for (int64_t e = indptr[i]; e < indptr[i + 1]; ++e) {
    const int64_t b = iperm[indices[e]];
    double g = 0.0;
    if (a >= b && a - b <= k) g = (a == b && gdiag) ? gdiag[b] : (double)gband[b * ld + (a - b)];
    gvals[e] = g;
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

extern "C" bo_status bo_csr_to_band(bo_prec prec, int64_t n, const int64_t *indptr, const int64_t *indices,
                                    const double *vals, const int64_t *iperm, int32_t k, int64_t ld, void *band,
                                    double *diag, int64_t *dropped, hipStream_t stream) {
  if (prec != BO_F64 && prec != BO_MIXED) return gfail(BO_EINVAL, "unknown precision");
  if (n < 0 || k < 0 || ld < k + 1) return gfail(BO_EINVAL, "bo_csr_to_band: bad sizes");
  if (n > 0 && (!indptr || !indices || !vals || !iperm || !band || !dropped))
    return gfail(BO_EINVAL, "bo_csr_to_band: null array");
  if ((prec == BO_MIXED) != (diag != nullptr))
    return gfail(BO_EINVAL, "bo_csr_to_band: the FP64 diagonal is for BO_MIXED only, and required there");
  if (n == 0) return BO_OK;
  const bool f64 = prec == BO_F64;
  const int64_t cnt = n * ld;
  int e = bo_profile_graph(0, stream, [&] {
    hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(kRows), 0, stream, dropped);
    if (f64) {
      hipLaunchKernelGGL(k_fill_band<double>, dim3(grid_for(cnt)), dim3(kRows), 0, stream, cnt, (double *)band, diag, n);
      hipLaunchKernelGGL(k_csr_to_band<double>, dim3(grid_for(n)), dim3(kRows), 0, stream, n, indptr, indices, vals,
                         iperm, k, ld, (double *)band, diag, dropped);
    } else {
      hipLaunchKernelGGL(k_fill_band<float>, dim3(grid_for(cnt)), dim3(kRows), 0, stream, cnt, (float *)band, diag, n);
      hipLaunchKernelGGL(k_csr_to_band<float>, dim3(grid_for(n)), dim3(kRows), 0, stream, n, indptr, indices, vals,
                         iperm, k, ld, (float *)band, diag, dropped);
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
  });
  return e ? gfail(BO_EDEVICE, "bo_csr_to_band: kernel launch failed") : BO_OK;
}

extern "C" bo_status bo_band_to_csr_grad(bo_prec prec, int64_t n, const int64_t *indptr, const int64_t *indices,
                                         const int64_t *iperm, int32_t k, int64_t ld, const void *gband,
                                         const double *gdiag, double *gvals, hipStream_t stream) {
  if (prec != BO_F64 && prec != BO_MIXED) return gfail(BO_EINVAL, "unknown precision");
  if (n < 0 || k < 0 || ld < k + 1) return gfail(BO_EINVAL, "bo_band_to_csr_grad: bad sizes");
  if (n > 0 && (!indptr || !indices || !iperm || !gband || !gvals))
    return gfail(BO_EINVAL, "bo_band_to_csr_grad: null array");
  if ((prec == BO_MIXED) != (gdiag != nullptr))
    return gfail(BO_EINVAL, "bo_band_to_csr_grad: the FP64 diagonal is for BO_MIXED only, and required there");
  if (n == 0) return BO_OK;
  int e = bo_profile_graph(1, stream, [&] {
    if (prec == BO_F64)
      hipLaunchKernelGGL(k_band_to_csr<double>, dim3(grid_for(n)), dim3(kRows), 0, stream, n, indptr, indices, iperm,
                         k, ld, (const double *)gband, gdiag, gvals);
    else
      hipLaunchKernelGGL(k_band_to_csr<float>, dim3(grid_for(n)), dim3(kRows), 0, stream, n, indptr, indices, iperm,
                         k, ld, (const float *)gband, gdiag, gvals);
    return hipGetLastError() == hipSuccess ? 0 : -2;
  });
  return e ? gfail(BO_EDEVICE, "bo_band_to_csr_grad: kernel launch failed") : BO_OK;
}
