// bandops_lib.hip -- host side of the C ABI (include/bandops.h): argument
// checks, schedules, launch sequences; plus the bandwidth-independent kernels
// (per-problem finalisation, band products, band-restricted outer products,
// log-determinant sensitivity).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/bandops.h"
#include "bandops_driver.hpp"
#include "bandops_ml.hpp"
#include "bandops_ng.hpp"
#include "bandops_wh.hpp"

using bo::Args;
using bo::Sched;

// ------------------------------------------------------------------ errors
static thread_local std::string g_err;

static bo_status fail(bo_status st, const std::string &msg) {
  g_err = msg;
  return st;
}

// Shared with the other translation units of the library (C++ linkage).
bo_status bo_set_error(bo_status st, const std::string &msg) { return fail(st, msg); }

extern "C" const char *bo_last_error(void) { return g_err.c_str(); }

extern "C" const char *bo_status_string(int s) {
  switch (s) {
    case BO_OK: return "ok";
    case BO_EINVAL: return "invalid argument";
    case BO_EDEVICE: return "device error";
    case BO_EWORKSPACE: return "workspace too small";
    case BO_EUNSUPPORTED: return "unsupported";
    default: return "unknown status";
  }
}

// ----------------------------------------------------- per-bandwidth steps
typedef int (*StepFn)(int, int, const Args *, int64_t, hipStream_t);
extern "C" {
int bo_step_k0(int, int, const Args *, int64_t, hipStream_t);
int bo_step_k1(int, int, const Args *, int64_t, hipStream_t);
int bo_step_k2(int, int, const Args *, int64_t, hipStream_t);
int bo_step_k3(int, int, const Args *, int64_t, hipStream_t);
int bo_step_k4(int, int, const Args *, int64_t, hipStream_t);
int bo_step_k5(int, int, const Args *, int64_t, hipStream_t);
int bo_step_k6(int, int, const Args *, int64_t, hipStream_t);
int bo_step_k7(int, int, const Args *, int64_t, hipStream_t);
int bo_step_k8(int, int, const Args *, int64_t, hipStream_t);
int bo_step_k9(int, int, const Args *, int64_t, hipStream_t);
int bo_step_k10(int, int, const Args *, int64_t, hipStream_t);
int bo_step_k11(int, int, const Args *, int64_t, hipStream_t);
int bo_step_k12(int, int, const Args *, int64_t, hipStream_t);
}
static const StepFn g_steps[bo::KMAX_SUPPORTED + 1] = {
    bo_step_k0, bo_step_k1, bo_step_k2, bo_step_k3, bo_step_k4,  bo_step_k5, bo_step_k6,
    bo_step_k7, bo_step_k8, bo_step_k9, bo_step_k10, bo_step_k11, bo_step_k12};

namespace {

constexpr int kBlock = 64;

template <class Item>
__global__ void __launch_bounds__(kBlock) k_item(const Args a, int64_t count) {
  int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
  if (i < count) Item::run(a, i);
}

template <class Item> int launch_items(const Args &a, int64_t count, hipStream_t s) {
  if (count <= 0) return 0;
  int64_t grid = (count + kBlock - 1) / kBlock;
  hipLaunchKernelGGL(k_item<Item>, dim3((unsigned)grid), dim3(kBlock), 0, s, a, count);
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// Per-problem results from the per-chunk partials: one workgroup per problem;
// lane t takes chunks t, t+64, ... (Neumaier-compensated sums), the partial
// sums are combined in LDS.  Same quantities as bo::Finalize.
__global__ void __launch_bounds__(kBlock) k_finalize(const Args A) {
  __shared__ double sh_s[kBlock], sh_c[kBlock], sh_q[kBlock], sh_t[kBlock];
  __shared__ long long sh_f[kBlock];
  const int32_t p = A.p_beg + (int32_t)blockIdx.x;
  const bo::ProbDesc &pd = bo::prob_at(A, p);
  double s = 0.0, comp = 0.0, q = 0.0, tr = 0.0;
  long long fail = -1;
  for (int32_t c = pd.chunk0 + (int32_t)threadIdx.x; c < pd.chunk0 + pd.nchunk; c += kBlock) {
    const double *pt = A.part + 4 * (int64_t)c;
    double t = pt[0], u = s + t;
    comp += (fabs(s) >= fabs(t)) ? (s - u) + t : (t - u) + s;
    s = u;
    q += pt[1];
    tr += pt[2];
    if (pt[3] >= 0.0 && fail < 0) fail = (long long)pt[3];   // chunks ascend in rows
  }
  sh_s[threadIdx.x] = s;
  sh_c[threadIdx.x] = comp;
  sh_q[threadIdx.x] = q;
  sh_t[threadIdx.x] = tr;
  sh_f[threadIdx.x] = fail;
  __syncthreads();
  if (threadIdx.x != 0) return;
  s = 0.0;
  comp = 0.0;
  q = 0.0;
  tr = 0.0;
  fail = -1;
  for (int i = 0; i < kBlock; ++i) {
    double t = sh_s[i], u = s + t;
    comp += (fabs(s) >= fabs(t)) ? (s - u) + t : (t - u) + s;
    s = u;
    comp += sh_c[i];
    q += sh_q[i];
    tr += sh_t[i];
    if (sh_f[i] >= 0 && (fail < 0 || sh_f[i] < fail)) fail = sh_f[i];
  }
  double ld = 2.0 * (s + comp);
  int32_t o = pd.orig;
  if (A.logdet) A.logdet[o] = fail >= 0 ? NAN : ld;
  if (A.parts) {
    A.parts[3 * (int64_t)o + 0] = fail >= 0 ? NAN : ld;
    A.parts[3 * (int64_t)o + 1] = q;
    A.parts[3 * (int64_t)o + 2] = tr;
  }
  if (A.info) A.info[o] = fail >= 0 ? (int32_t)(fail + 1) : 0;
  if (A.loss) A.loss[o] = fail >= 0 ? NAN : ld - q + tr;
}

// ------------------------------------------------------------ profiling
// When enabled, every launch is bracketed by a pair of events on its stream;
// bo_profile_read() waits for them and sums the durations per step kind.
// + clear, finalize, the four wide passes, the KL term's row kernels, the
// three launches of Algorithm 5 and its reverse mode
constexpr int kProfSlots = bo::ST_COUNT + 27;
constexpr int kSlotViPre = bo::ST_COUNT + 6, kSlotViPost = bo::ST_COUNT + 7, kSlotViNeg = bo::ST_COUNT + 8;
constexpr int kSlotSolveMat = bo::ST_COUNT + 9, kSlotSolveMatG = bo::ST_COUNT + 10, kSlotSolveMatOut = bo::ST_COUNT + 11;
constexpr int kSlotMlPost = bo::ST_COUNT + 13, kSlotMlFinal = bo::ST_COUNT + 14;   // + 12: unused
constexpr int kSlotNgPre = bo::ST_COUNT + 15, kSlotNgPost = bo::ST_COUNT + 16, kSlotNgNeg = bo::ST_COUNT + 17,
              kSlotNgFinal = bo::ST_COUNT + 18;
struct ProfRec {
  int slot;
  hipEvent_t a, b;
};
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
std::vector<hipEvent_t> g_prof_pool;
double g_prof_ms[kProfSlots];
int64_t g_prof_n[kProfSlots];

hipEvent_t prof_event() {
  if (!g_prof_pool.empty()) {
    hipEvent_t e = g_prof_pool.back();
    g_prof_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

template <class F> int profiled(int slot, hipStream_t s, F &&launch) {
  if (!g_prof_on) return launch();
  ProfRec r{slot, prof_event(), prof_event()};
  (void)hipEventRecord(r.a, s);
  int e = launch();
  (void)hipEventRecord(r.b, s);
  g_prof_pending.push_back(r);
  return e;
}

}  // namespace

// Launch timing of the graph kernels (the band assembly and its gradient's
// gather): slots ST_COUNT + 19 + which, which = 0..1.
int bo_profile_graph(int which, hipStream_t s, const std::function<int()> &launch) {
  return profiled(bo::ST_COUNT + 19 + which, s, launch);
}

// Launch timing for the other translation units of the library (C++ linkage):
// the wide passes' replays use slots ST_COUNT + 2 + which, which = 0..3, their
// summaries, scans and finalisation ST_COUNT + 21 + (which - 4), which = 4..9.
int bo_profile_wide(int which, hipStream_t s, const std::function<int()> &launch) {
  return profiled(which < 4 ? bo::ST_COUNT + 2 + which : bo::ST_COUNT + 21 + (which - 4), s, launch);
}

namespace {

struct GpuBE {
  hipStream_t s;
  int only = -1;   // >= 0: run the sequences of this bandwidth range alone, no finalisation
  bool range_on(int r) const { return only < 0 || only == r; }
  int step(int st, int K, int prec, const Args &a, int64_t count) {
    if (K < 0 || K > bo::KMAX_SUPPORTED) return -4;
    if (count <= 0) return 0;
    return profiled(st, s, [&] { return g_steps[K](st, prec, &a, count, s); });
  }
  int clear(const Args &a, int64_t count) {
    if (count <= 0) return 0;
    return profiled(bo::ST_COUNT, s, [&] { return launch_items<bo::ClearPart>(a, count, s); });
  }
  int finalize(const Args &a, int64_t count) {
    if (count <= 0 || only >= 0) return 0;
    return profiled(bo::ST_COUNT + 1, s, [&] {
      hipLaunchKernelGGL(k_finalize, dim3((unsigned)count), dim3(kBlock), 0, s, a);
      return hipGetLastError() == hipSuccess ? 0 : -2;
    });
  }
};

int64_t default_target_chunks() {
  static int64_t v = [] {
    const char *e = std::getenv("BANDOPS_TARGET_CHUNKS");
    long long t = e ? std::atoll(e) : 0;
    return (int64_t)(t > 0 ? t : 196608);
  }();
  return v;
}
int64_t default_min_len() {
  static int64_t v = [] {
    const char *e = std::getenv("BANDOPS_MIN_CHUNK");
    long long t = e ? std::atoll(e) : 0;
    return (int64_t)(t > 0 ? t : 32);
  }();
  return v;
}
// Per-bandwidth chunk-length factors "k:f,k:f" from BANDOPS_KSCALE, a switch
// for schedule experiments (unset: every factor 1, the measured best).
const int32_t *env_kscale() {
  static int32_t v[bo::KMAX_SUPPORTED + 1];
  static bool any = [] {
    for (int k = 0; k <= bo::KMAX_SUPPORTED; ++k) v[k] = 1;
    const char *e = std::getenv("BANDOPS_KSCALE");
    bool set = false;
    while (e && *e) {
      int k = 0, f = 0;
      if (std::sscanf(e, "%d:%d", &k, &f) == 2 && k >= 0 && k <= bo::KMAX_SUPPORTED && f >= 1) {
        v[k] = f;
        set = true;
      }
      const char *c = std::strchr(e, ',');
      e = c ? c + 1 : nullptr;
    }
    return set;
  }();
  return any ? v : nullptr;
}
// Launch order of the bandwidth ranges (BANDOPS_RANGE_ORDER=desc: widest
// first, a switch for schedule experiments; default narrowest first).
bool ranges_widest_first() {
  static bool v = [] {
    const char *e = std::getenv("BANDOPS_RANGE_ORDER");
    return e && std::strcmp(e, "desc") == 0;
  }();
  return v;
}
// First bandwidth whose chunk products get a pass of their own after the F1
// replay (BANDOPS_PC_SEPARATE, a switch for schedule experiments; 13: never).
int32_t pc_separate_from() {
  static int32_t v = [] {
    const char *e = std::getenv("BANDOPS_PC_SEPARATE");
    int t = e ? std::atoi(e) : 11;
    return (int32_t)(t >= 1 ? t : 11);
  }();
  return v;
}
bool fuse_summaries() {
  static bool v = [] {
    const char *e = std::getenv("BANDOPS_FUSE");
    return !(e && e[0] == '0');
  }();
  return v;
}

int32_t group_size() {
  static int32_t v = [] {
    const char *e = std::getenv("BANDOPS_GROUP");
    int t = e ? std::atoi(e) : 0;
    return (int32_t)(t >= 2 && t <= 1024 ? t : 64);
  }();
  return v;
}

bo_status dev_status(int e, const char *what) {
  if (e == 0) return BO_OK;
  if (e == -4) return fail(BO_EUNSUPPORTED, std::string(what) + ": bandwidth without compiled kernels");
  return fail(BO_EDEVICE, std::string(what) + ": kernel launch failed: " +
                              hipGetErrorString(hipGetLastError()));
}

// ---------------------------------------------------------- argument checks
bo_status check_band(const bo_band *b, bo_prec prec, const char *name, bool need_lower) {
  if (!b) return fail(BO_EINVAL, std::string(name) + ": null descriptor");
  if (b->n < 0 || b->l < 0 || b->u < 0) return fail(BO_EINVAL, std::string(name) + ": negative size");
  if (b->ld < b->l + b->u + 1) return fail(BO_EINVAL, std::string(name) + ": ld < l+u+1");
  if (need_lower && b->u != 0) return fail(BO_EINVAL, std::string(name) + ": must be a lower band (u = 0)");
  if (b->n > 0 && !b->band) return fail(BO_EINVAL, std::string(name) + ": null band pointer");
  if (prec == BO_MIXED && b->n > 0 && !b->diag64)
    return fail(BO_EINVAL, std::string(name) + ": BO_MIXED needs the FP64 diagonal array");
  if (prec == BO_F64 && b->diag64) return fail(BO_EINVAL, std::string(name) + ": diag64 must be NULL for BO_F64");
  if (prec != BO_F64 && prec != BO_MIXED) return fail(BO_EINVAL, "unknown precision");
  return BO_OK;
}

bo_status check_same(const bo_band *a, const bo_band *b, const char *what) {
  if (a->n != b->n) return fail(BO_EINVAL, std::string(what) + ": matrix orders differ");
  if (a->l != b->l) return fail(BO_EINVAL, std::string(what) + ": bandwidths differ");
  if (a->ld != b->ld) return fail(BO_EINVAL, std::string(what) + ": record strides differ");
  return BO_OK;
}

// Schedule of one problem (n, k, ld) and the kernel arguments bound to ws.
bo_status single_sched(int64_t n, int32_t k, int32_t ld, void *ws, size_t ws_bytes, Sched &s,
                       Args &A) {
  if (k > bo::KMAX_SUPPORTED)
    return fail(BO_EUNSUPPORTED, "bandwidth k = " + std::to_string(k) + " exceeds BO_KMAX");
  bo::ProbIn pi{n, k, ld, 0, 0};
  if (!bo::build_sched(&pi, 1, default_target_chunks(), default_min_len(), group_size(), s))
    return fail(BO_EINVAL, "bad problem shape");
  if (!ws || ws_bytes < s.bytes)
    return fail(BO_EWORKSPACE, "workspace needs " + std::to_string(s.bytes) + " bytes");
  A = Args{};
  bo::bind_sched(s, ws, true, A);
  return BO_OK;
}

#include "bandops_gbk.hpp"

}  // namespace

// ======================================================== C ABI: profiling
static const char *const kStepNames[kProfSlots] = {
    "f1_summary", "f1_group_compose", "f1_group_sweep", "f1_chunk_sweep", "f1_replay",
    "chunk_product", "fs_summary", "fs_replay", "f2_summary", "f2_replay", "b1_summary",
    "b1_replay", "b2_summary", "b2_replay", "asc_group_compose", "asc_group_sweep",
    "asc_chunk_sweep", "desc_group_compose", "desc_group_sweep", "desc_chunk_sweep",
    "clear_partials", "finalize", "wide_f1", "wide_f2", "wide_b1", "wide_b2", "vi_pre", "vi_post", "vi_neg", "solve_mat", "solve_mat_g", "solve_mat_out",
    "reserved", "ml_post", "ml_finalize", "ng_pre", "ng_post", "ng_neg", "ng_finalize", "csr_to_band",
    "band_to_csr", "wide_f1_sum", "wide_f1_scan", "wide_lin_sum", "wide_lin_scan", "wide_b2_sum", "wide_finalize"};

extern "C" int bo_profile_slots(void) { return kProfSlots; }

extern "C" const char *bo_profile_slot_name(int slot) {
  return (slot >= 0 && slot < kProfSlots) ? kStepNames[slot] : "";
}

extern "C" bo_status bo_profile_enable(int on) {
  g_prof_on = on != 0;
  return BO_OK;
}

extern "C" bo_status bo_profile_read(double *ms, int64_t *launches, int nslots) {
  for (const ProfRec &r : g_prof_pending) {
    if (hipEventSynchronize(r.b) != hipSuccess) return fail(BO_EDEVICE, "bo_profile_read: event wait failed");
    float t = 0.f;
    (void)hipEventElapsedTime(&t, r.a, r.b);
    g_prof_ms[r.slot] += t;
    g_prof_n[r.slot] += 1;
    g_prof_pool.push_back(r.a);
    g_prof_pool.push_back(r.b);
  }
  g_prof_pending.clear();
  for (int i = 0; i < nslots && i < kProfSlots; ++i) {
    if (ms) ms[i] = g_prof_ms[i];
    if (launches) launches[i] = g_prof_n[i];
    g_prof_ms[i] = 0.0;
    g_prof_n[i] = 0;
  }
  return BO_OK;
}

// ========================================================== C ABI: queries
extern "C" size_t bo_workspace_size(int64_t n, int32_t k) {
  if (n < 0 || k < 0 || k > bo::KMAX_SUPPORTED) return 0;
  bo::ProbIn pi{n, k, k + 1, 0, 0};
  Sched s;
  if (!bo::build_sched(&pi, 1, default_target_chunks(), default_min_len(), group_size(), s)) return 0;
  return s.bytes;
}

// ====================================================== C ABI: forward ops
extern "C" bo_status bo_chol(bo_prec prec, const bo_band *Q, bo_band *L, const void *y, void *z,
                             double *logdet, int32_t *info, void *ws, size_t ws_bytes,
                             hipStream_t stream) {
  if (bo_status e = check_band(Q, prec, "Q", true)) return e;
  if (bo_status e = check_band(L, prec, "L", true)) return e;
  if (bo_status e = check_same(Q, L, "bo_chol")) return e;
  if ((y == nullptr) != (z == nullptr)) return fail(BO_EINVAL, "bo_chol: y and z go together");
  if (!info) return fail(BO_EINVAL, "bo_chol: info is required");
  Sched s;
  Args A;
  if (bo_status e = single_sched(Q->n, Q->l, Q->ld, ws, ws_bytes, s, A)) return e;
  A.Q = Q->band;
  A.Qd = Q->diag64;
  A.L = L->band;
  A.Ld = L->diag64;
  A.y = y;
  A.z = z;
  A.logdet = logdet;
  A.info = info;
  GpuBE be{stream};
  return dev_status(bo::pipe_forward(be, s, A, (int)prec), "bo_chol");
}

// ------------------------------------------ Cholesky without allocation
// The workspace of bo_chol_noalloc lives in this file-scope device array; each
// GPU the library runs on holds its own copy until the process ends.  Host
// code never passes the array's name to a kernel (on the host it is only a
// stand-in): the entry point looks up the array's device address once per
// device with hipGetSymbolAddress and uses that pointer.
constexpr size_t kScratchBytes = (size_t)BO_NOALLOC_SCRATCH_MB << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void *g_scratch_ptr[kMaxDevices];

// Device address of the scratch array on the current device (looked up on the
// first call there).
static bo_status scratch_on_current_device(void **out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(BO_EDEVICE, "bo_chol_noalloc: no current HIP device");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void *ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(BO_EDEVICE, std::string("bo_chol_noalloc: scratch address lookup failed: ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return BO_OK;
}

extern "C" size_t bo_chol_noalloc_scratch_bytes(void) { return kScratchBytes; }

extern "C" bo_status bo_chol_noalloc(bo_prec prec, const bo_band *Q, bo_band *L, const void *y, void *z,
                                     double *logdet, int32_t *info, hipStream_t stream) {
  if (bo_status e = check_band(Q, prec, "Q", true)) return e;
  if (bo_status e = check_band(L, prec, "L", true)) return e;
  if (bo_status e = check_same(Q, L, "bo_chol_noalloc")) return e;
  if ((y == nullptr) != (z == nullptr)) return fail(BO_EINVAL, "bo_chol_noalloc: y and z go together");
  if (!info) return fail(BO_EINVAL, "bo_chol_noalloc: info is required");
  if (Q->l > bo::KMAX_SUPPORTED)
    return fail(BO_EUNSUPPORTED, "bo_chol_noalloc: bandwidth k = " + std::to_string(Q->l) + " exceeds BO_KMAX");
  // The schedule of bo_chol, with fewer chunks when its workspace would not fit.
  bo::ProbIn pi{Q->n, Q->l, Q->ld, 0, 0};
  Sched s;
  int64_t target = default_target_chunks();
  for (;;) {
    if (!bo::build_sched(&pi, 1, target, default_min_len(), group_size(), s))
      return fail(BO_EINVAL, "bo_chol_noalloc: bad problem shape");
    if (s.bytes <= kScratchBytes) break;
    if (target <= 1)
      return fail(BO_EWORKSPACE, "bo_chol_noalloc: the workspace (" + std::to_string(s.bytes) +
                                     " bytes) exceeds the scratch array (" + std::to_string(kScratchBytes) + " bytes)");
    target /= 2;
  }
  void *ws = nullptr;
  if (bo_status e = scratch_on_current_device(&ws)) return e;
  Args A{};
  bo::bind_sched(s, ws, true, A);
  A.Q = Q->band;
  A.Qd = Q->diag64;
  A.L = L->band;
  A.Ld = L->diag64;
  A.y = y;
  A.z = z;
  A.logdet = logdet;
  A.info = info;
  GpuBE be{stream};
  return dev_status(bo::pipe_forward(be, s, A, (int)prec), "bo_chol_noalloc");
}

extern "C" bo_status bo_trsv(bo_prec prec, const bo_band *L, int trans, const void *b, void *x,
                             int64_t nrhs, int64_t ldx, void *ws, size_t ws_bytes, hipStream_t stream) {
  if (bo_status e = check_band(L, prec, "L", true)) return e;
  if (nrhs < 0) return fail(BO_EINVAL, "bo_trsv: negative nrhs");
  if (nrhs > 1 && ldx < L->n) return fail(BO_EINVAL, "bo_trsv: ldx < n");
  if (L->n > 0 && nrhs > 0 && (!b || !x)) return fail(BO_EINVAL, "bo_trsv: null vector");
  Sched s;
  Args A;
  if (bo_status e = single_sched(L->n, L->l, L->ld, ws, ws_bytes, s, A)) return e;
  if (nrhs == 0 || L->n == 0) return BO_OK;
  A.L = L->band;
  A.Ld = L->diag64;
  A.xscale = 1.0;
  const size_t esz = prec == BO_F64 ? sizeof(double) : sizeof(float);
  GpuBE be{stream};
  const int pass = trans ? bo::PASS_F2 : bo::PASS_FS;
  for (int64_t c = 0; c < nrhs; ++c) {
    A.bx = (const char *)b + (size_t)(c * ldx) * esz;
    A.x = (char *)x + (size_t)(c * ldx) * esz;
    // the chunk products of L stay in ws from the first column's pipeline
    const int e = c == 0 ? bo::pipe_linear(be, s, A, (int)prec, pass) : bo::seq_lin(be, s, A, (int)prec, pass);
    if (e) return dev_status(e, "bo_trsv");
  }
  return BO_OK;
}

extern "C" size_t bo_subset_inv_workspace_size(int64_t n, int32_t k, int32_t kout) {
  if (n < 0 || k < 0 || kout < k || kout > bo::KMAX_SUPPORTED) return 0;
  if (kout == k) return bo_workspace_size(n, k);
  const size_t base = bo_workspace_size(n, kout);
  return base ? bo::align_up((size_t)n * (size_t)(kout + 1) * sizeof(double)) + base : 0;
}

extern "C" bo_status bo_subset_inv(bo_prec prec, const bo_band *L, bo_band *Sig, void *ws,
                                   size_t ws_bytes, hipStream_t stream) {
  if (bo_status e = check_band(L, prec, "L", true)) return e;
  if (bo_status e = check_band(Sig, prec, "Sigma", true)) return e;
  if (Sig->l < L->l) return fail(BO_EINVAL, "bo_subset_inv: Sigma narrower than L");
  if (Sig->l == L->l) {
    if (bo_status e = check_same(L, Sig, "bo_subset_inv")) return e;
    Sched s;
    Args A;
    if (bo_status e = single_sched(L->n, L->l, L->ld, ws, ws_bytes, s, A)) return e;
    A.L = L->band;
    A.Ld = L->diag64;
    A.S = Sig->band;
    A.Sd = Sig->diag64;
    GpuBE be{stream};
    return dev_status(bo::pipe_linear(be, s, A, (int)prec, bo::PASS_F2), "bo_subset_inv");
  }
  // a wider output: Algorithm 3 on L widened to kout sub-diagonals with zeros
  const int32_t kout = Sig->l;
  const int64_t n = L->n;
  if (Sig->n != n) return fail(BO_EINVAL, "bo_subset_inv: matrix orders differ");
  if (kout > bo::KMAX_SUPPORTED)
    return fail(BO_EUNSUPPORTED, "bo_subset_inv: output width k_out = " + std::to_string(kout) + " exceeds BO_KMAX");
  if (Sig->ld != kout + 1) return fail(BO_EINVAL, "bo_subset_inv: a wider Sigma must be packed (ld = k_out + 1)");
  const size_t need = bo_subset_inv_workspace_size(n, L->l, kout);
  if (!ws || ws_bytes < need)
    return fail(BO_EWORKSPACE, "bo_subset_inv: workspace needs " + std::to_string(need) + " bytes");
  const size_t pad = bo::align_up((size_t)n * (size_t)(kout + 1) * sizeof(double));
  Sched s;
  Args A;
  if (bo_status e = single_sched(n, kout, kout + 1, (char *)ws + pad, ws_bytes - pad, s, A)) return e;
  if (n == 0) return BO_OK;
  const int64_t el = n * (int64_t)(kout + 1);
  if (prec == BO_F64)
    hipLaunchKernelGGL(k_widen_lower<double>, dim3(blocks_for(el, 256)), dim3(256), 0, stream, n,
                       (const double *)L->band, (int64_t)L->ld, L->l, (double *)ws, kout);
  else
    hipLaunchKernelGGL(k_widen_lower<float>, dim3(blocks_for(el, 256)), dim3(256), 0, stream, n,
                       (const float *)L->band, (int64_t)L->ld, L->l, (float *)ws, kout);
  if (hipGetLastError() != hipSuccess) return dev_status(-2, "bo_subset_inv");
  A.L = ws;
  A.Ld = L->diag64;
  A.S = Sig->band;
  A.Sd = Sig->diag64;
  GpuBE be{stream};
  return dev_status(bo::pipe_linear(be, s, A, (int)prec, bo::PASS_F2), "bo_subset_inv");
}

extern "C" bo_status bo_gbmm(bo_prec prec, const bo_band *A, int tA, const bo_band *B, int tB,
                             bo_band *C, hipStream_t stream) {
  if (bo_status e = check_band(A, prec, "A", false)) return e;
  if (bo_status e = check_band(B, prec, "B", false)) return e;
  if (bo_status e = check_band(C, prec, "C", false)) return e;
  if (A->n != B->n || A->n != C->n) return fail(BO_EINVAL, "bo_gbmm: matrix orders differ");
  int64_t n = C->n, w = (int64_t)C->l + C->u + 1;
  if (n == 0) return BO_OK;
  if (prec == BO_F64)
    hipLaunchKernelGGL(k_gbmm<double>, dim3(blocks_for(n * w, 256)), dim3(256), 0, stream, n,
                       gb<double>(A), tA, gb<double>(B), tB, gb<double>(C));
  else
    hipLaunchKernelGGL(k_gbmm<float>, dim3(blocks_for(n * w, 256)), dim3(256), 0, stream, n,
                       gb<float>(A), tA, gb<float>(B), tB, gb<float>(C));
  return dev_status(hipGetLastError() == hipSuccess ? 0 : -2, "bo_gbmm");
}

extern "C" bo_status bo_solve_band_mat(bo_prec prec, const bo_band *L, const bo_band *R, bo_band *O,
                                       hipStream_t stream) {
  if (bo_status e = check_band(L, prec, "L", true)) return e;
  if (bo_status e = check_band(R, prec, "R", false)) return e;
  if (bo_status e = check_band(O, prec, "O", false)) return e;
  if (L->n != R->n || L->n != O->n) return fail(BO_EINVAL, "bo_solve_band_mat: matrix orders differ");
  if (O->l != L->l || O->u != R->u)
    return fail(BO_EINVAL, "bo_solve_band_mat: O must have L's lower and R's upper width");
  if (L->l > 12 || R->u > 12) return fail(BO_EUNSUPPORTED, "bo_solve_band_mat: widths above 12");
  const int64_t n = O->n;
  if (n == 0) return BO_OK;
  const int e = profiled(kSlotSolveMat, stream, [&] {
    int TC = 256;
    while (TC > 64 && solve_mat_lds(TC, L->l, R->l, R->u) > 48 * 1024) TC /= 2;
    const size_t lds = solve_mat_lds(TC, L->l, R->l, R->u);
    if (prec == BO_F64)
      hipLaunchKernelGGL(k_solve_mat<double>, dim3(blocks_for(n, TC)), dim3(TC), lds, stream, n, gb<double>(L),
                         gb<double>(R), gb<double>(O));
    else
      hipLaunchKernelGGL(k_solve_mat<float>, dim3(blocks_for(n, TC)), dim3(TC), lds, stream, n, gb<float>(L),
                         gb<float>(R), gb<float>(O));
    return hipGetLastError() == hipSuccess ? 0 : -2;
  });
  return dev_status(e, "bo_solve_band_mat");
}

extern "C" size_t bo_solve_band_mat_workspace(int64_t n, int32_t k, int32_t u) {
  return n > 0 ? (size_t)n * (size_t)(k + u + 1) * sizeof(double) : 0;
}

extern "C" bo_status bo_solve_band_mat_bwd(bo_prec prec, const bo_band *L, const bo_band *O,
                                           const bo_band *Obar, bo_band *Rbar, bo_band *Lbar, void *ws,
                                           size_t ws_bytes, hipStream_t stream) {
  if (bo_status e = check_band(L, prec, "L", true)) return e;
  if (bo_status e = check_band(O, prec, "O", false)) return e;
  if (bo_status e = check_band(Obar, prec, "Obar", false)) return e;
  if (bo_status e = check_band(Rbar, prec, "Rbar", false)) return e;
  if (bo_status e = check_band(Lbar, prec, "Lbar", true)) return e;
  const int64_t n = O->n;
  if (L->n != n || Obar->n != n || Rbar->n != n || Lbar->n != n)
    return fail(BO_EINVAL, "bo_solve_band_mat_bwd: matrix orders differ");
  if (O->l != L->l || Obar->l != O->l || Obar->u != O->u || Rbar->u != O->u || Lbar->l != L->l)
    return fail(BO_EINVAL, "bo_solve_band_mat_bwd: band widths do not match the forward call");
  if (L->l > 12 || O->u > 12) return fail(BO_EUNSUPPORTED, "bo_solve_band_mat_bwd: widths above 12");
  if (n == 0) return BO_OK;
  if (!ws || ws_bytes < bo_solve_band_mat_workspace(n, L->l, O->u))
    return fail(BO_EWORKSPACE, "bo_solve_band_mat_bwd: workspace smaller than bo_solve_band_mat_workspace()");
  double *G = (double *)ws;
  const int k = L->l, u = O->u;
  const bool f64 = prec == BO_F64;
  int e = profiled(kSlotSolveMatG, stream, [&] {
    int TC = 256;
    while (TC > 64 && solve_mat_g_lds(TC, k, u) > 48 * 1024) TC /= 2;
    const size_t lds = solve_mat_g_lds(TC, k, u);
    if (f64)
      hipLaunchKernelGGL(k_solve_mat_g<double>, dim3(blocks_for(n, TC)), dim3(TC), lds, stream, n, gb<double>(L),
                         gb<double>(Obar), G, gb<double>(Rbar));
    else
      hipLaunchKernelGGL(k_solve_mat_g<float>, dim3(blocks_for(n, TC)), dim3(TC), lds, stream, n, gb<float>(L),
                         gb<float>(Obar), G, gb<float>(Rbar));
    return hipGetLastError() == hipSuccess ? 0 : -2;
  });
  if (e == 0)
    e = profiled(kSlotSolveMatOut, stream, [&] {
      int TC = 256;
      while (TC > 64 && solve_mat_lbar_lds(TC, k, u) > 48 * 1024) TC /= 2;
      const size_t lds = solve_mat_lbar_lds(TC, k, u);
      if (f64)
        hipLaunchKernelGGL(k_solve_mat_lbar<double>, dim3(blocks_for(n, TC)), dim3(TC), lds, stream, n, k, u,
                           (const double *)G, gb<double>(O), gb<double>(Lbar));
      else
        hipLaunchKernelGGL(k_solve_mat_lbar<float>, dim3(blocks_for(n, TC)), dim3(TC), lds, stream, n, k, u,
                           (const double *)G, gb<float>(O), gb<float>(Lbar));
      return hipGetLastError() == hipSuccess ? 0 : -2;
    });
  return dev_status(e, "bo_solve_band_mat_bwd");
}

extern "C" bo_status bo_gbmv(bo_prec prec, const bo_band *A, int tA, const void *x, void *y,
                             hipStream_t stream) {
  if (bo_status e = check_band(A, prec, "A", false)) return e;
  int64_t n = A->n;
  if (n == 0) return BO_OK;
  if (!x || !y) return fail(BO_EINVAL, "bo_gbmv: null vector");
  if (prec == BO_F64)
    hipLaunchKernelGGL(k_gbmv<double>, dim3(blocks_for(n, 256)), dim3(256), 0, stream, n,
                       gb<double>(A), tA, (const double *)x, (double *)y);
  else
    hipLaunchKernelGGL(k_gbmv<float>, dim3(blocks_for(n, 256)), dim3(256), 0, stream, n,
                       gb<float>(A), tA, (const float *)x, (float *)y);
  return dev_status(hipGetLastError() == hipSuccess ? 0 : -2, "bo_gbmv");
}

extern "C" bo_status bo_outer_band(bo_prec prec, const void *m, const void *v, double alpha,
                                   int accumulate, bo_band *O, hipStream_t stream) {
  if (bo_status e = check_band(O, prec, "O", false)) return e;
  int64_t n = O->n, w = (int64_t)O->l + O->u + 1;
  if (n == 0) return BO_OK;
  if (!m || !v) return fail(BO_EINVAL, "bo_outer_band: null vector");
  if (prec == BO_F64)
    hipLaunchKernelGGL(k_outer<double>, dim3(blocks_for(n * w, 256)), dim3(256), 0, stream, n,
                       (const double *)m, (const double *)v, alpha, accumulate, gb<double>(O));
  else
    hipLaunchKernelGGL(k_outer<float>, dim3(blocks_for(n * w, 256)), dim3(256), 0, stream, n,
                       (const float *)m, (const float *)v, alpha, accumulate, gb<float>(O));
  return dev_status(hipGetLastError() == hipSuccess ? 0 : -2, "bo_outer_band");
}

// ===================================================== C ABI: reverse mode
extern "C" bo_status bo_chol_bwd(bo_prec prec, const bo_band *L, const bo_band *Lbar,
                                 bo_band *Qbar, void *ws, size_t ws_bytes, hipStream_t stream) {
  if (bo_status e = check_band(L, prec, "L", true)) return e;
  if (bo_status e = check_band(Lbar, prec, "Lbar", true)) return e;
  if (bo_status e = check_band(Qbar, prec, "Qbar", true)) return e;
  if (bo_status e = check_same(L, Lbar, "bo_chol_bwd")) return e;
  if (bo_status e = check_same(L, Qbar, "bo_chol_bwd")) return e;
  Sched s;
  Args A;
  if (bo_status e = single_sched(L->n, L->l, L->ld, ws, ws_bytes, s, A)) return e;
  A.L = L->band;
  A.Ld = L->diag64;
  A.Lb = Lbar->band;
  A.Lbd = Lbar->diag64;
  A.Qb = Qbar->band;
  A.Qbd = Qbar->diag64;
  A.gl = 0.0;
  GpuBE be{stream};
  return dev_status(bo::pipe_linear(be, s, A, (int)prec, bo::PASS_B2), "bo_chol_bwd");
}

extern "C" bo_status bo_subset_inv_bwd(bo_prec prec, const bo_band *L, const bo_band *Sig,
                                       const bo_band *Sigbar, bo_band *Lbar, int accumulate,
                                       void *ws, size_t ws_bytes, hipStream_t stream) {
  if (bo_status e = check_band(L, prec, "L", true)) return e;
  if (bo_status e = check_band(Sig, prec, "Sigma", true)) return e;
  if (bo_status e = check_band(Sigbar, prec, "Sigmabar", true)) return e;
  if (bo_status e = check_band(Lbar, prec, "Lbar", true)) return e;
  if (bo_status e = check_same(L, Sig, "bo_subset_inv_bwd")) return e;
  if (bo_status e = check_same(L, Sigbar, "bo_subset_inv_bwd")) return e;
  if (bo_status e = check_same(L, Lbar, "bo_subset_inv_bwd")) return e;
  Sched s;
  Args A;
  if (bo_status e = single_sched(L->n, L->l, L->ld, ws, ws_bytes, s, A)) return e;
  A.L = L->band;
  A.Ld = L->diag64;
  A.S = Sig->band;
  A.Sd = Sig->diag64;
  A.Sb = Sigbar->band;
  A.Sbd = Sigbar->diag64;
  A.Lb = Lbar->band;
  A.Lbd = Lbar->diag64;
  A.sb_is_S = 0;
  A.accumulate = accumulate ? 1 : 0;
  GpuBE be{stream};
  return dev_status(bo::pipe_linear(be, s, A, (int)prec, bo::PASS_B1), "bo_subset_inv_bwd");
}

extern "C" bo_status bo_trsv_bwd(bo_prec prec, const bo_band *L, int trans, const void *x,
                                 const void *xbar, void *bbar, bo_band *Lbar, int accumulate,
                                 void *ws, size_t ws_bytes, hipStream_t stream) {
  if (bo_status e = check_band(L, prec, "L", true)) return e;
  if (Lbar) {
    if (bo_status e = check_band(Lbar, prec, "Lbar", true)) return e;
    if (bo_status e = check_same(L, Lbar, "bo_trsv_bwd")) return e;
  }
  if (L->n > 0 && (!x || !xbar || !bbar)) return fail(BO_EINVAL, "bo_trsv_bwd: null vector");
  Sched s;
  Args A;
  if (bo_status e = single_sched(L->n, L->l, L->ld, ws, ws_bytes, s, A)) return e;
  A.L = L->band;
  A.Ld = L->diag64;
  A.bx = xbar;
  A.x = bbar;
  A.xscale = 1.0;
  GpuBE be{stream};
  // bbar = L^{-T} xbar (trans = 0) or L^{-1} xbar (trans = 1)
  if (bo_status e = dev_status(bo::pipe_linear(be, s, A, (int)prec, trans ? bo::PASS_FS : bo::PASS_F2),
                               "bo_trsv_bwd"))
    return e;
  if (!Lbar) return BO_OK;
  // Lbar = -bbar x^T (trans = 0) or -x bbar^T (trans = 1) on the lower band
  return bo_outer_band(prec, trans ? x : bbar, trans ? bbar : x, -1.0, accumulate, Lbar, stream);
}

extern "C" bo_status bo_logdet_bwd(bo_prec prec, const bo_band *L, const double *gbar,
                                   bo_band *Lbar, int accumulate, hipStream_t stream) {
  if (bo_status e = check_band(L, prec, "L", true)) return e;
  if (bo_status e = check_band(Lbar, prec, "Lbar", true)) return e;
  if (bo_status e = check_same(L, Lbar, "bo_logdet_bwd")) return e;
  if (!gbar) return fail(BO_EINVAL, "bo_logdet_bwd: null gbar");
  int64_t n = L->n, w = (int64_t)L->l + 1;
  if (n == 0) return BO_OK;
  if (prec == BO_F64)
    hipLaunchKernelGGL(k_logdet_bwd<double>, dim3(blocks_for(n * w, 256)), dim3(256), 0, stream, n,
                       gb<double>(L), gbar, accumulate, gb<double>(Lbar));
  else
    hipLaunchKernelGGL(k_logdet_bwd<float>, dim3(blocks_for(n * w, 256)), dim3(256), 0, stream, n,
                       gb<float>(L), gbar, accumulate, gb<float>(Lbar));
  return dev_status(hipGetLastError() == hipSuccess ? 0 : -2, "bo_logdet_bwd");
}

// ============================================================ C ABI: plans
struct bo_plan {
  Sched s;
  void *pinned = nullptr;   // host copy of the device tables (pinned)
  // One stream per bandwidth range after the first (default priority) and the
  // events that fork them from the caller's stream and join them back.
  std::vector<hipStream_t> aux;
  hipEvent_t fork = nullptr;
  std::vector<hipEvent_t> join;
};

// Run `pipe` (a pass sequence that takes a GpuBE) once per bandwidth range,
// each range on its own stream forked from `stream` and joined back to it
// before the per-problem finalisation: the ranges share no problem, chunk or
// workspace slot, so their scans (serial, narrow launches at the wide
// bandwidths) overlap the other ranges' streaming passes.  Event records and
// waits are stream-ordered and graph-capturable (the captured graph holds the
// ranges as parallel branches).  Plans with one range, or without streams,
// run on `stream` alone.
template <class F>
static int run_ranges(const bo_plan *plan, hipStream_t stream, const Args &A, F &&pipe) {
  const int nr = (int)plan->s.ranges.size();
  if (nr <= 1 || (int)plan->aux.size() + 1 < nr || !plan->fork) {
    GpuBE be{stream};
    return pipe(be);
  }
  if (hipEventRecord(plan->fork, stream) != hipSuccess) return -2;
  const bool desc = ranges_widest_first();
  for (int i = 0; i < nr; ++i) {
    const int r = desc ? nr - 1 - i : i;
    hipStream_t st = r == 0 ? stream : plan->aux[r - 1];
    if (r > 0 && hipStreamWaitEvent(st, plan->fork, 0) != hipSuccess) return -2;
    GpuBE be{st};
    be.only = r;
    if (int e = pipe(be)) return e;
    if (r > 0 && (hipEventRecord(plan->join[r - 1], st) != hipSuccess ||
                  hipStreamWaitEvent(stream, plan->join[r - 1], 0) != hipSuccess))
      return -2;
  }
  GpuBE be{stream};
  return bo::seq_finalize(be, plan->s, A);
}

extern "C" bo_status bo_plan_create(const bo_problem *probs, int32_t nprob, int64_t target_chunks,
                                    bo_plan **out) {
  if (!out) return fail(BO_EINVAL, "bo_plan_create: null output");
  *out = nullptr;
  if (nprob <= 0 || !probs) return fail(BO_EINVAL, "bo_plan_create: no problems");
  std::vector<bo::ProbIn> in(nprob);
  for (int i = 0; i < nprob; ++i) {
    const bo_problem &p = probs[i];
    if (p.n < 0 || p.k < 0 || p.boff < 0 || p.voff < 0)
      return fail(BO_EINVAL, "bo_plan_create: problem " + std::to_string(i) + " has a negative field");
    if (p.k > bo::KMAX_SUPPORTED)
      return fail(BO_EUNSUPPORTED, "bo_plan_create: problem " + std::to_string(i) + " has k > BO_KMAX");
    in[i] = bo::ProbIn{p.n, p.k, p.k + 1, p.boff, p.voff};
  }
  bo_plan *pl = new bo_plan();
  if (!bo::build_sched(in.data(), nprob, target_chunks > 0 ? target_chunks : default_target_chunks(),
                       default_min_len(), group_size(), pl->s, env_kscale())) {
    delete pl;
    return fail(BO_EINVAL, "bo_plan_create: bad problem table");
  }
  pl->s.kpc_sep = pc_separate_from();
  size_t tb = pl->s.table_blob.size();
  if (hipHostMalloc(&pl->pinned, tb ? tb : 1, hipHostMallocDefault) != hipSuccess) {
    delete pl;
    return fail(BO_EDEVICE, "bo_plan_create: pinned host allocation failed");
  }
  if (tb) std::memcpy(pl->pinned, pl->s.table_blob.data(), tb);
  const int nr = (int)pl->s.ranges.size();
  if (nr > 1) {
    bool ok = hipEventCreateWithFlags(&pl->fork, hipEventDisableTiming) == hipSuccess;
    for (int r = 1; r < nr && ok; ++r) {
      hipStream_t st = nullptr;
      hipEvent_t ev = nullptr;
      ok = hipStreamCreateWithFlags(&st, hipStreamNonBlocking) == hipSuccess;
      if (ok) pl->aux.push_back(st);
      ok = ok && hipEventCreateWithFlags(&ev, hipEventDisableTiming) == hipSuccess;
      if (ok) pl->join.push_back(ev);
    }
    if (!ok) {
      bo_plan_destroy(pl);
      return fail(BO_EDEVICE, "bo_plan_create: stream or event creation failed");
    }
  }
  *out = pl;
  return BO_OK;
}

extern "C" bo_status bo_plan_workspace_size(const bo_plan *plan, size_t *bytes) {
  if (!plan || !bytes) return fail(BO_EINVAL, "bo_plan_workspace_size: null argument");
  *bytes = plan->s.bytes;
  return BO_OK;
}

extern "C" bo_status bo_plan_loss_workspace_size(const bo_plan *plan, size_t *bytes) {
  if (!plan || !bytes) return fail(BO_EINVAL, "bo_plan_loss_workspace_size: null argument");
  *bytes = plan->s.bytes_il;
  return BO_OK;
}

extern "C" bo_status bo_plan_upload(const bo_plan *plan, void *ws, hipStream_t stream) {
  if (!plan || !ws) return fail(BO_EINVAL, "bo_plan_upload: null argument");
  size_t tb = plan->s.table_blob.size();
  if (!tb) return BO_OK;
  if (hipMemcpyAsync((char *)ws + plan->s.off_tables, plan->pinned, tb, hipMemcpyHostToDevice,
                     stream) != hipSuccess)
    return fail(BO_EDEVICE, "bo_plan_upload: copy failed");
  return BO_OK;
}

static bo_status plan_args(const bo_plan *plan, bo_prec prec, const bo_batch_io *io, void *ws,
                           Args &A, bool need_L = true) {
  if (!plan || !io || !ws) return fail(BO_EINVAL, "plan call: null argument");
  if (prec != BO_F64 && prec != BO_MIXED) return fail(BO_EINVAL, "unknown precision");
  if (!io->Q || (need_L && !io->L)) return fail(BO_EINVAL, "plan call: Q and L are required");
  if (prec == BO_MIXED && (!io->Qd || !io->Ld))
    return fail(BO_EINVAL, "plan call: BO_MIXED needs FP64 diagonals of Q and L");
  A = Args{};
  bo::bind_sched(plan->s, ws, false, A);
  A.Q = io->Q;
  A.Qd = io->Qd;
  A.L = io->L;
  A.Ld = io->Ld;
  A.y = io->y;
  A.z = io->z;
  A.x = io->x;
  A.S = io->Sig;
  A.Sd = io->Sigd;
  A.Sb = io->S;
  A.Sbd = io->Sd;
  A.Lb = io->Lbar;
  A.Lbd = io->Lbard;
  A.Qb = io->Qbar;
  A.Qbd = io->Qbard;
  A.logdet = io->logdet;
  A.parts = io->parts;
  A.info = io->info;
  A.loss = io->loss;
  return BO_OK;
}

// out = s_p * in over every problem of a plan (bo_plan_scale's kinds).
static bo_status plan_scale_launch(const bo_plan *plan, bo_prec prec, int32_t kind, const double *g,
                                   const void *in, const double *ind, void *out, double *outd, void *ws,
                                   hipStream_t stream) {
  const Sched &s = plan->s;
  if (kind == BO_SCALE_PROBLEM) {
    hipLaunchKernelGGL(k_problem_scale, dim3(blocks_for(s.nprob, 256)), dim3(256), 0, stream, (int64_t)s.nprob, g,
                       (const double *)in, (double *)out);
    return hipGetLastError() == hipSuccess ? BO_OK : dev_status(-2, "bo_plan_scale");
  }
  if (s.nchunk == 0) return BO_OK;
  Args A{};
  bo::bind_sched(s, ws, false, A);
  if (prec == BO_F64)
    hipLaunchKernelGGL(k_plan_scale<double>, dim3((unsigned)s.nchunk), dim3(256), 0, stream, A.probs, A.chunk_prob,
                       (int)kind, g, (const double *)in, (const double *)nullptr, (double *)out, (double *)nullptr);
  else
    hipLaunchKernelGGL(k_plan_scale<float>, dim3((unsigned)s.nchunk), dim3(256), 0, stream, A.probs, A.chunk_prob,
                       (int)kind, g, (const float *)in, kind == BO_SCALE_VEC ? nullptr : ind, (float *)out,
                       kind == BO_SCALE_VEC ? nullptr : outd);
  return hipGetLastError() == hipSuccess ? BO_OK : dev_status(-2, "bo_plan_scale");
}

extern "C" bo_status bo_plan_forward(const bo_plan *plan, bo_prec prec, const bo_batch_io *io,
                                     void *ws, hipStream_t stream) {
  Args A;
  if (bo_status e = plan_args(plan, prec, io, ws, A)) return e;
  if ((io->z || io->x) && !io->y) return fail(BO_EINVAL, "bo_plan_forward: solves need y");
  if (io->x && !io->z) return fail(BO_EINVAL, "bo_plan_forward: x needs z");
  if (io->Sig && prec == BO_MIXED && !io->Sigd) return fail(BO_EINVAL, "bo_plan_forward: Sigd needed");
  A.Sb = nullptr;
  return dev_status(run_ranges(plan, stream, A, [&](GpuBE &be) { return bo::pipe_forward(be, plan->s, A, (int)prec); }),
                    "bo_plan_forward");
}

extern "C" bo_status bo_plan_gauss_loss(const bo_plan *plan, bo_prec prec, const bo_batch_io *io,
                                        void *ws, hipStream_t stream) {
  Args A;
  // L, Sig and Lbar all NULL: the intermediates stay in the workspace,
  // interleaved by chunk (FP64; ws of bo_plan_loss_workspace_size bytes)
  const bool keep = io && !io->L && !io->Sig && !io->Lbar;
  if (bo_status e = plan_args(plan, prec, io, ws, A, !keep)) return e;
  if (keep && prec != BO_F64)
    return fail(BO_EINVAL, "bo_plan_gauss_loss: intermediates in the workspace need BO_F64");
  if (!io->y || !io->S || (!keep && (!io->z || !io->Sig || !io->Lbar)) || !io->x || !io->Qbar || !io->parts ||
      !io->info)
    return fail(BO_EINVAL, "bo_plan_gauss_loss: y, S, z, x, Sig, Lbar, Qbar, parts, info required");
  if (keep) {
    bo::bind_il(plan->s, ws, A);
    A.sbar_out = io->Sbar;
  }
  if (prec == BO_MIXED && (!io->Sd || !io->Sigd || !io->Lbard || !io->Qbard))
    return fail(BO_EINVAL, "bo_plan_gauss_loss: BO_MIXED needs every FP64 diagonal");
  if (io->Sbar && prec == BO_MIXED && !io->Sbard)
    return fail(BO_EINVAL, "bo_plan_gauss_loss: BO_MIXED needs Sbard with Sbar");
  if (bo_status e = dev_status(run_ranges(plan, stream, A,
                                          [&](GpuBE &be) {
                                            return bo::pipe_gauss_loss(be, plan->s, A, (int)prec, fuse_summaries());
                                          }),
                               "bo_plan_gauss_loss"))
    return e;
  if (!io->Sbar || keep) return BO_OK;
  // d tr(Q^{-1} S) / dS on S's stored entries: Sigma_ii, 2 Sigma_ij
  return plan_scale_launch(plan, prec, BO_SCALE_BAND_SYM, nullptr, io->Sig, io->Sigd, io->Sbar, io->Sbard, ws,
                           stream);
}

extern "C" bo_status bo_plan_scale(const bo_plan *plan, bo_prec prec, int32_t kind, const double *g, const void *in,
                                   const double *ind, void *out, double *outd, void *ws, hipStream_t stream) {
  if (!plan || !ws) return fail(BO_EINVAL, "bo_plan_scale: null plan or workspace");
  if (prec != BO_F64 && prec != BO_MIXED) return fail(BO_EINVAL, "unknown precision");
  if (kind != BO_SCALE_BAND && kind != BO_SCALE_BAND_SYM && kind != BO_SCALE_VEC && kind != BO_SCALE_PROBLEM)
    return fail(BO_EINVAL, "bo_plan_scale: unknown kind");
  if ((plan->s.rows > 0 || kind == BO_SCALE_PROBLEM) && (!in || !out))
    return fail(BO_EINVAL, "bo_plan_scale: null array");
  if ((kind == BO_SCALE_BAND || kind == BO_SCALE_BAND_SYM) && prec == BO_MIXED && plan->s.rows > 0 && (!ind || !outd))
    return fail(BO_EINVAL, "bo_plan_scale: BO_MIXED bands need their FP64 diagonals");
  if (prec == BO_F64 && (ind || outd)) return fail(BO_EINVAL, "bo_plan_scale: diagonals must be NULL for BO_F64");
  return plan_scale_launch(plan, prec, kind, g, in, ind, out, outd, ws, stream);
}

extern "C" bo_status bo_plan_vi_kl(const bo_plan *plan, bo_prec prec, const bo_kl_io *io, void *ws,
                                   hipStream_t stream) {
  if (!plan || !io || !ws) return fail(BO_EINVAL, "bo_plan_vi_kl: null argument");
  if (prec != BO_F64 && prec != BO_MIXED) return fail(BO_EINVAL, "unknown precision");
  if (!io->Lq || !io->Lp || !io->mq || !io->mp || !io->Sig || !io->Lqbar || !io->Lpbar || !io->mqbar ||
      !io->mpbar || !io->parts)
    return fail(BO_EINVAL, "bo_plan_vi_kl: every array is required");
  if (prec == BO_MIXED && (!io->Lqd || !io->Lpd || !io->Sigd || !io->Lqbard || !io->Lpbard))
    return fail(BO_EINVAL, "bo_plan_vi_kl: BO_MIXED needs every FP64 diagonal");
  if (prec == BO_F64 && (io->Lqd || io->Lpd || io->Sigd || io->Lqbard || io->Lpbard))
    return fail(BO_EINVAL, "bo_plan_vi_kl: FP64 diagonals are for BO_MIXED only");
  Args A = Args{};
  bo::bind_sched(plan->s, ws, false, A);
  A.L = const_cast<void *>(io->Lq);   // read only: the passes below never write L
  A.Ld = const_cast<double *>(io->Lqd);
  A.S = io->Sig;
  A.Sd = io->Sigd;
  A.Sb = io->Lpbar;
  A.Sbd = io->Lpbard;
  A.Lb = io->Lqbar;
  A.Lbd = io->Lqbard;
  const bo_vi::KLP P{io->Lp, io->Lpd, io->mq, io->mp, io->Lpbar, io->Lpbard, io->mqbar, io->mpbar, io->parts};
  GpuBE be{stream};
  auto launch = [&](int which, int64_t count, const Args &a, int k) -> int {
    if (count <= 0) return 0;
    const dim3 grid((unsigned)count);
    const size_t pre_lds = bo_vi::pre_lds_bytes(k + 1), post_lds = bo_vi::post_lds_bytes(k + 1);
    const int slot = which == 0 ? kSlotViPre : which == 1 ? kSlotViPost : which == 2 ? kSlotViNeg : bo::ST_COUNT + 1;
    return profiled(slot, stream, [&] {
      const bool f64 = prec == BO_F64;
      const dim3 rows(bo_vi::kRowBlock);
      switch (which) {
        case 0:
          if (f64) hipLaunchKernelGGL(bo_vi::k_kl_pre<double>, grid, rows, pre_lds, stream, a, P);
          else hipLaunchKernelGGL(bo_vi::k_kl_pre<float>, grid, rows, pre_lds, stream, a, P);
          break;
        case 1:
          if (f64) hipLaunchKernelGGL(bo_vi::k_kl_post<double>, grid, rows, post_lds, stream, a, P);
          else hipLaunchKernelGGL(bo_vi::k_kl_post<float>, grid, rows, post_lds, stream, a, P);
          break;
        case 2:
          if (f64) hipLaunchKernelGGL(bo_vi::k_kl_neg<double>, grid, rows, 0, stream, a, P);
          else hipLaunchKernelGGL(bo_vi::k_kl_neg<float>, grid, rows, 0, stream, a, P);
          break;
        default:
          hipLaunchKernelGGL(bo_vi::k_kl_finalize, grid, dim3(64), 0, stream, a, P.parts);
      }
      return hipGetLastError() == hipSuccess ? 0 : -2;
    });
  };
  return dev_status(bo_vi::pipe_vi_kl(be, plan->s, A, (int)prec, launch), "bo_plan_vi_kl");
}

extern "C" bo_status bo_plan_marglik(const bo_plan *plan, bo_prec prec, const bo_ml_io *io, void *ws,
                                     hipStream_t stream) {
  if (!plan || !io || !ws) return fail(BO_EINVAL, "bo_plan_marglik: null argument");
  if (prec != BO_F64 && prec != BO_MIXED) return fail(BO_EINVAL, "unknown precision");
  if (!io->Q || !io->mask || !io->b || !io->tau2 || !io->L || !io->Sig || !io->x || !io->Qbar || !io->bbar ||
      !io->tau2bar || !io->parts || !io->info)
    return fail(BO_EINVAL, "bo_plan_marglik: every array is required");
  if (prec == BO_MIXED && (!io->Qd || !io->Ld || !io->Sigd || !io->Qbard))
    return fail(BO_EINVAL, "bo_plan_marglik: BO_MIXED needs every FP64 diagonal");
  if (prec == BO_F64 && (io->Qd || io->Ld || io->Sigd || io->Qbard))
    return fail(BO_EINVAL, "bo_plan_marglik: FP64 diagonals are for BO_MIXED only");
  const Sched &s = plan->s;
  double *sc = (double *)((unsigned char *)ws + s.off_out);   // 8 words per problem
  // first forward list: C(Q) into L, I(L_Q) into Qbar
  Args prior = Args{};
  bo::bind_sched(s, ws, false, prior);
  prior.Q = io->Q;
  prior.Qd = io->Qd;
  prior.L = io->L;
  prior.Ld = io->Ld;
  prior.S = io->Qbar;
  prior.Sd = io->Qbard;
  prior.parts = sc;
  prior.info = (int32_t *)(sc + 6 * (size_t)s.nprob);
  // second forward list: Q1 = Q + mask / tau2 (added to the diagonal as F1
  // reads Q) with the right-hand side b
  Args post = Args{};
  bo::bind_sched(s, ws, false, post);
  post.Q = io->Q;
  post.Qd = io->Qd;
  post.qdn = io->mask;
  post.qdd = io->tau2;
  post.L = io->L;
  post.Ld = io->Ld;
  post.y = io->b;
  post.z = io->bbar;
  post.x = io->x;
  post.S = io->Sig;
  post.Sd = io->Sigd;
  post.parts = sc + 3 * (size_t)s.nprob;
  post.info = io->info;
  const bo_ml::MLP P{io->Q,     io->Qd,   io->mask,    io->b,      io->tau2,   io->Sig,  io->Sigd,
                     io->x,     io->Qbar, io->Qbard,   io->bbar,   io->tau2bar, io->parts, io->info,
                     prior.parts, post.parts, prior.info};
  GpuBE be{stream};
  auto launch = [&](int which, int64_t count, const Args &a, int) -> int {
    if (count <= 0) return 0;
    const dim3 grid((unsigned)count);
    const int slot = which == 1 ? kSlotMlPost : kSlotMlFinal;
    return profiled(slot, stream, [&] {
      const bool f64 = prec == BO_F64;
      const dim3 rows(bo_ml::kRowBlock);
      switch (which) {
        case 1:
          if (f64) hipLaunchKernelGGL(bo_ml::k_ml_post<double>, grid, rows, 0, stream, a, P);
          else hipLaunchKernelGGL(bo_ml::k_ml_post<float>, grid, rows, 0, stream, a, P);
          break;
        default:
          hipLaunchKernelGGL(bo_ml::k_ml_finalize, grid, dim3(64), 0, stream, a, P);
      }
      return hipGetLastError() == hipSuccess ? 0 : -2;
    });
  };
  return dev_status(bo_ml::pipe_marglik(be, s, prior, post, (int)prec, launch), "bo_plan_marglik");
}

extern "C" bo_status bo_plan_natgp(const bo_plan *plan, bo_prec prec, const bo_natgp_io *io, void *ws,
                                   hipStream_t stream) {
  if (!plan || !io || !ws) return fail(BO_EINVAL, "bo_plan_natgp: null argument");
  if (prec != BO_F64 && prec != BO_MIXED) return fail(BO_EINVAL, "unknown precision");
  if (!io->Lpr || !io->etapr || !io->Llik || !io->etalik || !io->L || !io->Sig || !io->x || !io->Lprbar ||
      !io->Llikbar || !io->etaprbar || !io->parts || !io->info)
    return fail(BO_EINVAL, "bo_plan_natgp: every array is required");
  const bool mixed = prec == BO_MIXED;
  const bool any_d = io->Lprd || io->Llikd || io->Ld || io->Sigd || io->Lprbard || io->Llikbard;
  const bool all_d = io->Lprd && io->Llikd && io->Ld && io->Sigd && io->Lprbard && io->Llikbard;
  if (mixed && !all_d) return fail(BO_EINVAL, "bo_plan_natgp: BO_MIXED needs every FP64 diagonal");
  if (!mixed && any_d) return fail(BO_EINVAL, "bo_plan_natgp: FP64 diagonals are for BO_MIXED only");
  const Sched &s = plan->s;
  double *sc = (double *)((unsigned char *)ws + s.off_out);   // 8 words per problem
  // first forward list: Lam_pr with eta_pr
  Args prior = Args{};
  bo::bind_sched(s, ws, false, prior);
  prior.Q = io->Lpr;
  prior.Qd = io->Lprd;
  prior.L = io->L;
  prior.Ld = io->Ld;
  prior.y = io->etapr;
  prior.z = io->x;
  prior.x = io->etaprbar;
  prior.S = io->Lprbar;
  prior.Sd = io->Lprbard;
  prior.parts = sc;
  prior.info = io->info;
  // second forward list: Lam_po (written into Sig by pre) with eta_po (in x)
  Args post = Args{};
  bo::bind_sched(s, ws, false, post);
  post.Q = io->Sig;
  post.Qd = io->Sigd;
  post.L = io->L;
  post.Ld = io->Ld;
  post.y = io->x;
  post.z = io->Llikbar;
  post.x = io->x;
  post.S = io->Sig;
  post.Sd = io->Sigd;
  post.parts = sc + 3 * (size_t)s.nprob;
  post.info = (int32_t *)(sc + 6 * (size_t)s.nprob);
  const bo_ng::NGP P{io->Lpr,     io->Lprd,     io->etapr,    io->Llik,    io->Llikd,  io->etalik, io->Sig,
                     io->Sigd,    io->x,        io->Sig,      io->Sigd,    io->Lprbar, io->Lprbard, io->Llikbar,
                     io->Llikbard, io->etaprbar, io->parts,   io->info,    prior.parts, post.parts, post.info};
  GpuBE be{stream};
  auto launch = [&](int which, int64_t count, const Args &a) -> int {
    if (count <= 0) return 0;
    static const int slots[4] = {kSlotNgPre, kSlotNgPost, kSlotNgNeg, kSlotNgFinal};
    return profiled(slots[which], stream, [&] {
      const bool f64 = prec == BO_F64;
      const dim3 grid((unsigned)count), rows(bo_ng::kRowBlock);
      switch (which) {
        case 0:
          if (f64) hipLaunchKernelGGL(bo_ng::k_ng_pre<double>, grid, rows, 0, stream, a, P);
          else hipLaunchKernelGGL(bo_ng::k_ng_pre<float>, grid, rows, 0, stream, a, P);
          break;
        case 1:
          if (f64) hipLaunchKernelGGL(bo_ng::k_ng_post<double>, grid, rows, 0, stream, a, P);
          else hipLaunchKernelGGL(bo_ng::k_ng_post<float>, grid, rows, 0, stream, a, P);
          break;
        case 2:
          if (f64) hipLaunchKernelGGL(bo_ng::k_ng_neg<double>, grid, rows, 0, stream, a, P);
          else hipLaunchKernelGGL(bo_ng::k_ng_neg<float>, grid, rows, 0, stream, a, P);
          break;
        default:
          hipLaunchKernelGGL(bo_ng::k_ng_finalize, dim3((unsigned)((count + 63) / 64)), dim3(64), 0, stream, a, P,
                             (int32_t)count);
      }
      return hipGetLastError() == hipSuccess ? 0 : -2;
    });
  };
  return dev_status(bo_ng::pipe_natgp(be, s, prior, post, (int)prec, launch), "bo_plan_natgp");
}

extern "C" bo_status bo_plan_whiten(const bo_plan *plan, bo_prec prec, const bo_whiten_io *io, void *ws,
                                    hipStream_t stream) {
  if (!plan || !io || !ws) return fail(BO_EINVAL, "bo_plan_whiten: null argument");
  if (prec != BO_F64 && prec != BO_MIXED) return fail(BO_EINVAL, "unknown precision");
  if (!io->Q || !io->v || !io->L || !io->F) return fail(BO_EINVAL, "bo_plan_whiten: Q, v, L and F are required");
  if (prec == BO_MIXED && (!io->Qd || !io->Ld))
    return fail(BO_EINVAL, "bo_plan_whiten: BO_MIXED needs FP64 diagonals of Q and L");
  if (prec == BO_F64 && (io->Qd || io->Ld)) return fail(BO_EINVAL, "bo_plan_whiten: FP64 diagonals are for BO_MIXED only");
  Args A = Args{};
  bo::bind_sched(plan->s, ws, false, A);
  A.Q = io->Q;
  A.Qd = io->Qd;
  A.L = io->L;
  A.Ld = io->Ld;
  A.bx = io->v;
  A.x = io->F;
  A.logdet = io->logdet;
  A.info = io->info;
  GpuBE be{stream};
  return dev_status(bo_wh::pipe_whiten(be, plan->s, A, (int)prec), "bo_plan_whiten");
}

extern "C" bo_status bo_plan_whiten_bwd(const bo_plan *plan, bo_prec prec, const bo_whiten_io *io, void *ws,
                                        hipStream_t stream) {
  if (!plan || !io || !ws) return fail(BO_EINVAL, "bo_plan_whiten_bwd: null argument");
  if (prec != BO_F64 && prec != BO_MIXED) return fail(BO_EINVAL, "unknown precision");
  if (!io->L || !io->F || !io->Fbar || !io->vbar || !io->Qbar)
    return fail(BO_EINVAL, "bo_plan_whiten_bwd: L, F, Fbar, vbar and Qbar are required");
  if (prec == BO_MIXED && (!io->Ld || !io->Qbard))
    return fail(BO_EINVAL, "bo_plan_whiten_bwd: BO_MIXED needs FP64 diagonals of L and Qbar");
  if (prec == BO_F64 && (io->Ld || io->Qbard))
    return fail(BO_EINVAL, "bo_plan_whiten_bwd: FP64 diagonals are for BO_MIXED only");
  Args A = Args{};
  bo::bind_sched(plan->s, ws, false, A);
  A.L = io->L;
  A.Ld = io->Ld;
  A.bx = io->Fbar;
  A.x = io->vbar;
  A.yb = io->F;
  A.zf = io->vbar;
  A.Qb = io->Qbar;
  A.Qbd = io->Qbard;
  GpuBE be{stream};
  return dev_status(bo_wh::pipe_whiten_bwd(be, plan->s, A, (int)prec, io->reuse != 0), "bo_plan_whiten_bwd");
}

extern "C" bo_status bo_plan_stats(const bo_plan *plan, int64_t out[5]) {
  if (!plan || !out) return fail(BO_EINVAL, "bo_plan_stats: null argument");
  out[0] = plan->s.nprob;
  out[1] = plan->s.nchunk;
  out[2] = plan->s.ngroup;
  out[3] = plan->s.rows;
  out[4] = plan->s.Kmax;
  return BO_OK;
}

extern "C" bo_status bo_plan_destroy(bo_plan *plan) {
  if (!plan) return BO_OK;
  if (plan->pinned) (void)hipHostFree(plan->pinned);
  for (hipStream_t st : plan->aux) (void)hipStreamDestroy(st);
  for (hipEvent_t ev : plan->join) (void)hipEventDestroy(ev);
  if (plan->fork) (void)hipEventDestroy(plan->fork);
  delete plan;
  return BO_OK;
}
