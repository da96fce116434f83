// bandops_kern.hip -- kernels of one bandwidth K (compiled once per K with
// -DBO_K=<k>).  Every kernel runs one work item per lane; the item types are
// the per-chunk / per-group / per-problem steps of bandops_items.hpp.
#include "bandops_steps.hpp"

#ifndef BO_K
#error "compile with -DBO_K=<bandwidth>"
#endif

#define BO_CAT2(a, b) a##b
#define BO_CAT(a, b) BO_CAT2(a, b)

namespace {

constexpr int kBlock = 64;   // one wavefront per workgroup

template <class Item>
__global__ void __launch_bounds__(kBlock) k_item(const bo::Args a, int64_t count) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) Item::run(a, i);
}

struct Launch {
  const bo::Args &a;
  int64_t count;
  hipStream_t s;
  template <class Item> int go() {
    if (count <= 0) return 0;
    int64_t grid = (count + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_item<Item>, dim3((unsigned)grid), dim3(kBlock), 0, s, a, count);
    return hipGetLastError() == hipSuccess ? 0 : -2;
  }
};

}  // namespace

// Runs `count` items of `step` for bandwidth BO_K; prec 0 = FP64 storage,
// 1 = FP32 storage with FP64 diagonals.
extern "C" int BO_CAT(bo_step_k, BO_K)(int step, int prec, const bo::Args *a, int64_t count,
                                        hipStream_t s) {
  Launch l{*a, count, s};
  if (prec == 0) return bo::with_item<BO_K, double>(step, l);
  return bo::with_item<BO_K, float>(step, l);
}
