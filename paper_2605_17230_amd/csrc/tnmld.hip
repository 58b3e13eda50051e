// Boundary-MPS coset contraction for the rotated surface code on gfx950, and
// the C ABI declared in include/tnmld.h.
//
// Forward contraction of one (syndrome, coset) pair (paper Sec. 3.2.1):
//   1. reference error: the coset's base error f = R(s) * L_m, with R(s) a
//      product of check-flipping strings and L_m a logical representative;
//      the result is filed under its class lambda(R) xor lambda(L_m);
//   2. for each anti-diagonal row u of the 45-degree lattice: apply the row's
//      MPO (bond 2, entries p_q(f_q xor P) resolved from codes) to the MPS,
//      bring the product to right-canonical form by a right-to-left sweep of
//      Householder LQ factorisations, then sweep left-to-right with a QR of
//      every site matrix, and on each bond that exceeds chi a one-sided Jacobi
//      SVD of the triangular factor keeping the chi largest singular values
//      (the paper's successive SVD truncations); the removed log-norms go to
//      an FP64 accumulator;
//   3. the last row leaves a product over columns that is summed out.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/tnmld.h"
#include "adjoint.hpp"
#include "contract.hpp"
#include "plan.hpp"
#include "sweep.hpp"

// GEMM mode of the bf16 precision form (split bf16x3 keeps ~16 mantissa bits)
#ifndef BF16_GEMM_MODE
#define BF16_GEMM_MODE GEMM_BF16X3
#endif

// The forward kernel built for 256-thread work-groups (tnmld_small.hip).
namespace tnmld_small {
int small_wgs_per_cu(int precision, int lds_bytes, bool xg);
int launch_fwd_small(int precision, const void* jt, unsigned long long* counter, char* scratch, int64_t stride,
                     int64_t snap_ofs, const void* lay, int lds_bytes, int nwg, hipStream_t st);
int small_bwd_wgs_per_cu(int precision, int lds_bytes);
int launch_bwd_small(int precision, const void* jt, char* scratch, int64_t stride, const void* lay, int lds_bytes,
                     int flags, double* partials, int64_t pstride, int nwg, hipStream_t st);
}  // namespace tnmld_small

// The same kernel built for three 256-thread work-groups per CU (tnmld_small3.hip).
namespace tnmld_small3 {
int wgs_per_cu(int precision, int lds_bytes);
int launch_fwd(int precision, const void* jt, unsigned long long* counter, char* scratch, int64_t stride,
               int64_t snap_ofs, const void* lay, int lds_bytes, int nwg, hipStream_t st);
}  // namespace tnmld_small3

namespace tnmld {

// Forward: persistent work-groups take syndromes (all four cosets each) from
// an atomic counter.  Per-group scratch: the MPS site regions, then (at
// snap_ofs elements) the saved MPS after the rows common to the cosets.
template <typename Real, typename Fac, int GM>
__global__ __launch_bounds__(NT) void fwd_kernel(JobTable jt, unsigned long long* counter, char* scratch,
                                                  int64_t scratch_stride, int64_t snap_ofs, LdsLayout lay) {
  extern __shared__ __align__(16) uint8_t smem[];
  Real* scr = reinterpret_cast<Real*>(scratch + (int64_t)blockIdx.x * scratch_stride);
  Real* snap = scr + snap_ofs;
  __shared__ long long s_item;
  for (;;) {
    if (threadIdx.x == 0) s_item = (long long)atomicAdd(counter, 1ull);
    __syncthreads();
    const int64_t item = s_item;
    __syncthreads();
    if (item >= jt.nitems) break;
    int jb = 0;
    while (jb + 1 < jt.n && jt.j[jb + 1].item_begin <= item) ++jb;
    const JobDev& job = jt.j[jb];
    contract_syndrome<Real, Fac, GM>(job, item - job.item_begin, smem, lay, scr, snap);
    __syncthreads();
  }
}

// Backward: each work-group walks a fixed stride of items (deterministic order)
// and accumulates into its own FP64 partial gradient.
template <typename Real, typename Fac, int GM>
// flags: bit 0 writes log Z and log P(s); bits 1-2 the ADJ_* mode.
__global__ __launch_bounds__(NT) void bwd_kernel(JobTable jt, char* scratch, int64_t scratch_stride, LdsLayout lay,
                                                  int flags, double* partials, int64_t part_stride) {
  extern __shared__ __align__(16) uint8_t smem[];
  Real* scr = reinterpret_cast<Real*>(scratch + (int64_t)blockIdx.x * scratch_stride);
  double* mypart = partials + (int64_t)blockIdx.x * part_stride;
  for (int64_t item = blockIdx.x; item < jt.nitems; item += gridDim.x) {
    int jb = 0;
    while (jb + 1 < jt.n && jt.j[jb + 1].item_begin <= item) ++jb;
    const JobDev& job = jt.j[jb];
    adjoint_syndrome<Real, Fac, GM>(job, item - job.item_begin, smem, lay, scr, flags & 1, mypart + job.part_ofs,
                                    flags >> 1);
    __syncthreads();
  }
}

__global__ void fill_zero_f64(double* p, int64_t n) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0.0;
}

// out[i] += sum over work-groups w (in order) of partials[w * stride + ofs + i]
__global__ void reduce_partials(const double* partials, int64_t stride, int nwg, int64_t ofs, int64_t len,
                                double* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= len) return;
  double acc = 0.0;
  for (int w = 0; w < nwg; ++w) acc += partials[(int64_t)w * stride + ofs + i];
  out[i] += acc;
}

__global__ void zero_counter(unsigned long long* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0ull;
}

__global__ void zero_status(unsigned* st) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    st[0] = 0u;
    *reinterpret_cast<unsigned long long*>(st + 2) = 0ull;
  }
}

// log P(s) = logsumexp over the four cosets and the tie-tolerant argmax
__global__ void decide_kernel(const double* logz, int64_t count, double tie_tol, double* logp, uint8_t* cls) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= count) return;
  double z[4];
  double mx = -INFINITY;
  for (int k = 0; k < 4; ++k) {
    z[k] = logz[4 * b + k];
    mx = z[k] > mx ? z[k] : mx;
  }
  double lp = -INFINITY;
  int c = 0;
  if (mx > -INFINITY) {
    double s = 0.0;
    for (int k = 0; k < 4; ++k) s += exp(z[k] - mx);
    lp = mx + log(s);
    const double tau = tie_tol * (fabs(mx) > 1.0 ? fabs(mx) : 1.0);
    for (int k = 3; k >= 0; --k)
      if (z[k] >= mx - tau) c = k;
  }
  if (logp) logp[b] = lp;
  if (cls) cls[b] = (uint8_t)c;
}

// Host helpers shared with the planar exact solver (kacward.hip).
int report_error(int code, const std::string& msg);
void launch_zero_status(unsigned* st, hipStream_t stream) { zero_status<<<1, 64, 0, stream>>>(st); }
void launch_decide(const double* logz, int64_t count, double tie_tol, double* logp, uint8_t* cls,
                   hipStream_t stream) {
  if (count > 0 && (logp || cls))
    decide_kernel<<<(unsigned)((count + 255) / 256), 256, 0, stream>>>(logz, count, tie_tol, logp, cls);
}

// Fixed device array of the allocation-free entry point (tn_decode_batch_noalloc),
// 128 MiB on every device the library runs on, for the life of the process.
constexpr size_t kNoAllocBytes = 128ull << 20;
__device__ __align__(256) char scratch[kNoAllocBytes];

// ------------------------------------------------------------------ host side
namespace {

thread_local std::string g_err;
int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

struct DevPlan {
  Plan plan;
  uint8_t* dev = nullptr;
};

std::mutex g_mu;
std::map<std::tuple<int, int, int, int, int>, DevPlan*> g_plans;  // (device, d, chi, group, rounds)

struct DevInfo {
  int cus = 0;
  int lds_max = 0;
};
std::map<int, DevInfo> g_dev;

int device_info(DevInfo* out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(TN_EDEVICE, "no HIP device");
  std::lock_guard<std::mutex> lk(g_mu);
  auto it = g_dev.find(dev);
  if (it == g_dev.end()) {
    DevInfo di;
    if (hipDeviceGetAttribute(&di.cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
      return fail(TN_EDEVICE, "hipDeviceGetAttribute failed");
    if (hipDeviceGetAttribute(&di.lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      return fail(TN_EDEVICE, "hipDeviceGetAttribute failed");
    it = g_dev.emplace(dev, di).first;
  }
  *out = it->second;
  return TN_OK;
}

// element sizes of the MPS storage / GEMM type and of the factorisation type
int real_bytes(int precision) { return precision == TN_FP64 ? 8 : 4; }
int fac_bytes(int precision) { return (precision == TN_FP32_PLAIN || precision == TN_BF16) ? 4 : 8; }
bool precision_built(int precision) {
  return precision >= TN_FP64 && precision <= TN_BF16_F64;
}

// largest usable LDS per block on gfx950 when no device is queried
constexpr int kLdsLimit = 160 * 1024;

constexpr int kLdsPerCU = 160 * 1024;
constexpr int kMaxWgPerCU = 1024 / NT > 1 ? 1024 / NT : 1;  // 4 waves per SIMD at most for 512-thread groups

// Tuned launch shapes, set by tn_set_tuning (the autotuner's cache).
struct Tune {
  int group, wgs, threads;  // threads: 0 = either build, 512 or 256 = that build
};
std::map<std::tuple<int, int, int>, Tune> g_tune;

// Raise a kernel's dynamic-LDS limit once per (kernel, size) and remember it,
// so that warm calls enqueue kernels only (a stream being captured into a
// graph sees no attribute calls).
int ensure_lds_attr(const void* kern, int bytes) {
  static std::map<const void*, int> done;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  int& cur = done[kern];
  if (cur >= bytes) return TN_OK;
  if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess)
    return fail(TN_EDEVICE, "hipFuncSetAttribute failed");
  cur = bytes;
  return TN_OK;
}

const void* fwd_kernel_of(int precision) {
  if (precision == TN_FP64) return reinterpret_cast<const void*>(fwd_kernel<double, double, GEMM_F64>);
  if (precision == TN_FP32) return reinterpret_cast<const void*>(fwd_kernel<float, double, GEMM_F32>);
  if (precision == TN_BF16) return reinterpret_cast<const void*>(fwd_kernel<float, float, BF16_GEMM_MODE>);
  if (precision == TN_BF16_F64) return reinterpret_cast<const void*>(fwd_kernel<float, double, GEMM_BF16>);
  return reinterpret_cast<const void*>(fwd_kernel<float, float, GEMM_F32>);
}
// (no adjoint for TN_BF16_F64: the backward planner rejects it before asking)
const void* bwd_kernel_of(int precision) {
  if (precision == TN_FP64) return reinterpret_cast<const void*>(bwd_kernel<double, double, GEMM_VALU>);
  if (precision == TN_FP32) return reinterpret_cast<const void*>(bwd_kernel<float, double, GEMM_F32>);
  if (precision == TN_BF16) return reinterpret_cast<const void*>(bwd_kernel<float, float, BF16_GEMM_MODE>);
  return reinterpret_cast<const void*>(bwd_kernel<float, float, GEMM_F32>);
}

// Work-groups of `kern` that one CU holds at once with lds_bytes of dynamic
// LDS: the smaller of the LDS fit and the register-file fit reported by the
// runtime (the sweep kernels use up to 256 VGPRs, i.e. one 512-thread group
// per CU).  Without a device only the LDS fit is known.
int wgs_for(int lds_bytes, const void* kern = nullptr) {
  int w = kLdsPerCU / (lds_bytes + 256);
  w = w < 1 ? 0 : (w > kMaxWgPerCU ? kMaxWgPerCU : w);
  if (!kern || w == 0) return w;
  static std::map<std::pair<const void*, int>, int> cache;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  auto key = std::make_pair(kern, lds_bytes);
  auto it = cache.find(key);
  if (it == cache.end()) {
    int nb = 0;
    if (ensure_lds_attr(kern, lds_bytes) != TN_OK ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, NT, (size_t)lds_bytes) != hipSuccess || nb < 1)
      nb = w;
    it = cache.emplace(key, nb).first;
  }
  return std::min(w, it->second);
}

// Choose the column grouping (1 or 2 columns per site): a tuned entry if one
// exists, else the grouping that fits the most work-groups per CU (ties: 2).
int choose_group(int d, int chi, int precision, int lds_limit, Plan* out, std::string* why, int rounds = 1) {
  int forced = rounds > 1 ? 1 : 0;  // repeated rounds: one column (2^T values) per site
  if (rounds <= 1) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tune.find(std::make_tuple(d, chi, precision));
    if (it != g_tune.end()) forced = it->second.group;
  }
  int best_g = -1, best_w = 0;
  Plan best;
  for (int g = 2; g >= 1; --g) {
    if (forced && g != forced) continue;
    Plan p;
    std::string e = build_plan(d, chi, g, &p, rounds);
    if (!e.empty()) {
      *why = e;
      return -1;
    }
    LdsLayout lay = lds_layout(p.h, real_bytes(precision), fac_bytes(precision));
    if (lay.bytes > lds_limit) {
      *why = "chi=" + std::to_string(chi) + " needs " + std::to_string(lay.bytes) + " B of LDS";
      continue;
    }
    const int w = wgs_for(lay.bytes, fwd_kernel_of(precision));
    if (w > best_w) {
      best_w = w;
      best_g = g;
      best = std::move(p);
    }
  }
  if (best_g > 0) *out = std::move(best);
  return best_g;
}

// Plans are kept per (device, d, chi, group).  upload = false: the plan is
// built and kept on the host only (dev stays null), for the allocation-free
// entry point, which copies the blob into its own fixed device array.
int get_plan(int d, int chi, int precision, int lds_limit, DevPlan** out, bool upload = true, int rounds = 1) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(TN_EDEVICE, "no HIP device");
  Plan p;
  std::string why;
  int g = choose_group(d, chi, precision, lds_limit, &p, &why, rounds);
  if (g < 0) return fail(TN_EUNSUPPORTED, why);
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_tuple(dev, d, chi, g, rounds);
  auto it = g_plans.find(key);
  if (it != g_plans.end() && (it->second->dev || !upload)) {
    *out = it->second;
    return TN_OK;
  }
  DevPlan* dp = it != g_plans.end() ? it->second : new DevPlan;
  if (it == g_plans.end()) {
    dp->plan = std::move(p);
    g_plans[key] = dp;
  }
  if (!upload) {
    *out = dp;
    return TN_OK;
  }
  uint8_t* devp = nullptr;
  if (hipMalloc(&devp, dp->plan.blob.size()) != hipSuccess) return fail(TN_ENOMEM, "hipMalloc of plan failed");
  if (hipMemcpy(devp, dp->plan.blob.data(), dp->plan.blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(devp);
    return fail(TN_EDEVICE, "plan upload failed");
  }
  dp->dev = devp;
  *out = dp;
  return TN_OK;
}

int validate(const tn_segment* segs, int32_t nseg) {
  if (!segs || nseg < 1 || nseg > TN_MAX_SEGMENTS) return fail(TN_EINVAL, "nseg must be in [1, 16]");
  for (int i = 0; i < nseg; ++i) {
    const tn_segment& s = segs[i];
    if (s.d < 3 || s.d > TN_MAX_D || s.d % 2 == 0) return fail(TN_EINVAL, "d must be odd in [3, 31]");
    if (s.chi < 0) return fail(TN_EINVAL, "chi must be >= 0");
    if (s.precision < TN_FP64 || s.precision > TN_BF16_F64) return fail(TN_EINVAL, "bad precision");
    if (s.n_models < 1) return fail(TN_EINVAL, "n_models must be >= 1");
    if (s.count < 0) return fail(TN_EINVAL, "count must be >= 0");
    if (s.count > 0 && (!s.rates || !s.syndromes || !s.out_logz)) return fail(TN_EINVAL, "null pointer");
    if (s.rounds < 0 || s.rounds > TN_MAX_ROUNDS) return fail(TN_EINVAL, "rounds must be in [0, TN_MAX_ROUNDS]");
    if (s.rounds > 1 && s.count > 0 && !s.meas_rates) return fail(TN_EINVAL, "repeated rounds need meas_rates");
  }
  return TN_OK;
}

// Plans whose site matrices have at most 64 rows (chi <= 32 with a bond-2
// MPO) and at most 256 columns run on the 256-thread build of the forward
// kernel when at least two of its work-groups fit a CU (LDS and registers):
// in practice chi <= 24, the larger plans need more than half the LDS.
constexpr int kSmallNT = 256;

// LDS of the 256-thread build within half a CU: the plain layout, else without
// the MPO step's LDS copy of the input site (read from its site region), else
// (FP32 factorisations) with the LQ matrix of the right-to-left sweep in the
// work-group's scratch, which frees enough of that phase for the input site's
// copy to return, else with both in scratch.  Returns the bytes, or -1.
int small_layout(const PlanHeader& h, int precision, bool* aj_global, bool* x_global) {
  const int limit = kLdsPerCU / 2 - 256;
  const int rb = real_bytes(precision), fb = fac_bytes(precision);
  for (int v = 0; v < 4; ++v) {
    const bool aj = v == 1 || v == 3, xg = v >= 2;
    if (xg && fb != 4) break;
    const int lb = lds_layout(h, rb, fb, aj, xg).bytes;
    if (lb <= limit) {
      *aj_global = aj;
      *x_global = xg;
      return lb;
    }
  }
  return -1;
}

bool small_plan(const PlanHeader& h, int precision) {
  // rows the 256-thread build keeps in registers: 4 per 16-lane group with
  // FP32 factorisations, 2 with FP64 ones
  const int rpg = fac_bytes(precision) == 4 ? 4 : 2;
  if (h.max_m > rpg * (kSmallNT / 16) || h.max_n > 256 || h.max_bond > kSmallNT) return false;
  bool aj = false, xg = false;
  const int lb = small_layout(h, precision, &aj, &xg);
  if (lb < 0) return false;
  return tnmld_small::small_wgs_per_cu(precision, lb, xg) >= 2;
}

// LDS of the three-groups-per-CU build within a third of a CU (plain layout,
// else without the input site's LDS copy); -1 if neither fits.
int small3_layout(const PlanHeader& h, int precision, bool* aj_global) {
  const int limit = kLdsPerCU / 3 - 256;
  for (int v = 0; v < 2; ++v) {
    const int lb = lds_layout(h, real_bytes(precision), fac_bytes(precision), v == 1).bytes;
    if (lb <= limit) {
      *aj_global = v == 1;
      return lb;
    }
  }
  return -1;
}

// Plans whose factorisations all run in registers with at most 8 columns per
// lane (site matrices of at most 128 columns in both sweeps) and whose LDS fits
// a third of a CU run on the three-groups-per-CU build.
bool small3_plan(const PlanHeader& h, int precision) {
  const int rpg = fac_bytes(precision) == 4 ? 4 : 2;
  if (h.max_m > rpg * (kSmallNT / 16) || h.max_kr > rpg * (kSmallNT / 16) || h.max_n > 128 ||
      h.max_rows > 128 || h.max_bond > kSmallNT)
    return false;
  bool aj = false;
  const int lb = small3_layout(h, precision, &aj);
  if (lb < 0) return false;
  return tnmld_small3::wgs_per_cu(precision, lb) >= 3;
}

// launch classes: the 512-thread build, the 256-thread build at two
// work-groups per CU, and at three
enum { BUILD_512 = 0, BUILD_256 = 1, BUILD_256X3 = 2, kNumBuilds = 3 };
constexpr int kMaxLaunches = kNumBuilds * (TN_BF16_F64 + 1);  // one per precision and size class

struct Launch {
  const Plan* host_plan[TN_MAX_SEGMENTS];  // plan of each job (host copy)
  int build;       // BUILD_*
  bool small;      // a 256-thread build
  bool aj_global;  // small launch whose MPO step reads the input site from its region (LDS)
  bool x_global;   // small launch whose LQ matrix lives in the work-group's scratch (LDS)
  int precision;
  JobTable jt;  // forward items are syndromes
  PlanHeader merged;
  int64_t scratch_elems;  // site regions (max over the merged plans)
  int64_t mps_elems;      // one compact MPS (max over the merged plans)
  int nwg;  // persistent work-groups of this launch
};

constexpr size_t kAlign = kWorkspaceAlign;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Bytes of one work-group's scratch: the site regions and the saved MPS of the
// rows common to the cosets, then (x_global) the LQ matrix.
size_t group_bytes(const Launch& L) {
  size_t b = align_up((size_t)(L.scratch_elems + L.mps_elems) * real_bytes(L.precision));
  if (L.x_global) b += align_up((size_t)L.merged.max_X * fac_bytes(L.precision));
  return b;
}

LdsLayout launch_layout(const Launch& L) {
  LdsLayout lay = lds_layout(L.merged, real_bytes(L.precision), fac_bytes(L.precision), L.aj_global, L.x_global);
  if (L.x_global) lay.xg = (int32_t)align_up((size_t)(L.scratch_elems + L.mps_elems) * real_bytes(L.precision));
  return lay;
}

// Workspace header (the first kAlign bytes): one work counter per launch, then
// the status word of the last call (ST_* bits, read by tn_workspace_status)
// and, 8 bytes on, its 64-bit count of unresolved cosets.
constexpr size_t kStatusOfs = kStatusOffset;
static_assert(sizeof(unsigned long long) * kMaxLaunches <= kStatusOfs, "header layout");
unsigned* status_word(void* workspace) {
  return reinterpret_cast<unsigned*>(reinterpret_cast<char*>(workspace) + kStatusOfs);
}

// Build the launch groups (one per precision) and the workspace layout.
int plan_launches(const tn_segment* segs, int32_t nseg, int lds_limit, std::vector<Launch>* out, size_t* ws_bytes,
                  int* nwg, bool allow_small = true, bool upload = true) {
  int rc = validate(segs, nseg);
  if (rc) return rc;
  DevInfo di;
  if ((rc = device_info(&di))) return rc;
  *nwg = 0;
  // order segments: larger d first so the heaviest items start first
  std::vector<int> order(nseg);
  for (int i = 0; i < nseg; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return segs[a].d > segs[b].d; });
  out->clear();
  // the build each segment runs on: the 512-thread one when tuned so or when
  // its plan needs it, else three 256-thread groups per CU where the plan
  // fits (and no tuning says two), else two
  std::vector<int> cls(nseg, BUILD_512);
  std::vector<DevPlan*> plans(nseg, nullptr);
  std::vector<Tune> tunes(nseg, Tune{0, 0, 0});
  bool needs2[TN_BF16_F64 + 1] = {};
  for (int i = 0; i < nseg; ++i) {
    const tn_segment& s = segs[i];
    if (s.count == 0) continue;
    if (!precision_built(s.precision)) return fail(TN_EUNSUPPORTED, "precision not built");
    const int rounds = s.rounds > 1 ? s.rounds : 1;
    if ((rc = get_plan(s.d, s.chi, s.precision, lds_limit, &plans[i], upload, rounds))) return rc;
    if (rounds == 1) {  // the tuned shapes are for one-round plans
      std::lock_guard<std::mutex> lk(g_mu);
      auto it = g_tune.find(std::make_tuple(s.d, s.chi, s.precision));
      if (it != g_tune.end()) tunes[i] = it->second;
    }
    const Tune& tu = tunes[i];
    const PlanHeader& h = plans[i]->plan.h;
    if (!allow_small || tu.threads == NT) continue;
    const bool two = tu.threads == kSmallNT && tu.wgs > 0 && tu.wgs < 3;
    if (!two && small3_plan(h, s.precision)) cls[i] = BUILD_256X3;
    else if (small_plan(h, s.precision)) cls[i] = BUILD_256;
    if (cls[i] == BUILD_256) needs2[s.precision] = true;
  }
  // one persistent launch per precision and build: a precision whose call has
  // plans on the two-group build runs its three-group plans there too
  for (int i = 0; i < nseg; ++i)
    if (cls[i] == BUILD_256X3 && needs2[segs[i].precision]) cls[i] = BUILD_256;
  for (int launch = 0; launch < kMaxLaunches; ++launch) {
    const int prec = launch / kNumBuilds;
    const int build = launch % kNumBuilds;
    Launch L{};
    L.build = build;
    L.small = build != BUILD_512;
    L.precision = prec;
    int64_t items = 0;
    for (int oi : order) {
      const tn_segment& s = segs[oi];
      if (s.precision != prec || s.count == 0 || cls[oi] != build) continue;
      DevPlan* dp = plans[oi];
      const Tune& tu = tunes[oi];
      const int rounds = s.rounds > 1 ? s.rounds : 1;
      L.host_plan[L.jt.n] = &dp->plan;
      JobDev& j = L.jt.j[L.jt.n++];
      j.plan = dp->dev;
      j.rates = s.rates;
      j.model_index = s.model_index;
      j.syn = s.syndromes;
      j.logz = s.out_logz;
      j.count = s.count;
      j.item_begin = items;
      j.n_models = s.n_models;
      j.rounds = rounds;
      j.meas = rounds > 1 ? s.meas_rates : nullptr;
      items += s.count;
      merge_maxima(&L.merged, dp->plan.h);
      L.scratch_elems = std::max<int64_t>(L.scratch_elems, dp->plan.h.scratch_elems);
      L.mps_elems = std::max<int64_t>(L.mps_elems, dp->plan.h.mps_elems);
      // a tuned work-groups-per-CU count applies to the build it was tuned on
      const bool small = L.small;
      const int tw = (tu.threads == (small ? kSmallNT : NT) || (tu.threads == 0 && !small)) ? tu.wgs : 0;
      if (tw > 0) L.nwg = L.nwg ? std::min(L.nwg, tw) : tw;  // per-CU count for now
    }
    L.jt.nitems = items;
    L.aj_global = L.x_global = false;
    if (build == BUILD_256X3) {
      if (small3_layout(L.merged, prec, &L.aj_global) < 0) L.aj_global = true;  // merged: the compact layout
    } else if (build == BUILD_256 && small_layout(L.merged, prec, &L.aj_global, &L.x_global) < 0) {
      // plans that fit one by one, merged: the most compact layout (the
      // work-groups per CU below follow from its LDS)
      L.aj_global = true;
      L.x_global = fac_bytes(prec) == 4;
    }
    if (L.jt.n > 0) out->push_back(L);
  }
  size_t bytes = align_up(sizeof(unsigned long long) * kMaxLaunches);
  for (auto& L : *out) {
    if (L.merged.max_bond > NT) return fail(TN_EUNSUPPORTED, "bond dimension above the work-group size");
    const int lb = launch_layout(L).bytes;
    int w = wgs_for(lb, fwd_kernel_of(L.precision));
    if (L.small) {
      const int ws = L.build == BUILD_256X3 ? tnmld_small3::wgs_per_cu(L.precision, lb)
                                            : tnmld_small::small_wgs_per_cu(L.precision, lb, L.x_global);
      w = std::min(kLdsPerCU / (lb + 256), ws > 0 ? ws : 1);
      if (L.nwg > 0) w = std::min(w, L.nwg);  // tuned for the 256-thread build
    } else if (L.nwg > 0) {
      w = std::min(w, L.nwg);  // tuned work-groups per CU (tuned for the 512-thread build)
    }
    if (w < 1) return fail(TN_EUNSUPPORTED, "LDS of the merged plans exceeds one CU");
    L.nwg = w * di.cus;
    *nwg = std::max(*nwg, L.nwg);
    bytes += (size_t)L.nwg * group_bytes(L);
  }
  *ws_bytes = bytes;
  return TN_OK;
}

template <typename Real, typename Fac, int GM>
int launch_fwd(const Launch& L, int nwg, char* ws_scratch, unsigned long long* counter, hipStream_t st) {
  LdsLayout lay = launch_layout(L);
  auto kern = fwd_kernel<Real, Fac, GM>;
  if (int rc = ensure_lds_attr(reinterpret_cast<const void*>(kern), lay.bytes)) return rc;
  zero_counter<<<1, 64, 0, st>>>(counter);
  const int64_t stride = (int64_t)group_bytes(L);
  const int64_t snap_ofs = L.scratch_elems;
  hipLaunchKernelGGL(kern, dim3(nwg), dim3(NT), lay.bytes, st, L.jt, counter, ws_scratch, stride, snap_ofs, lay);
  if (hipGetLastError() != hipSuccess) return fail(TN_EDEVICE, "kernel launch failed");
  return TN_OK;
}

// Enqueue the planned launches.  header: workspace header (counters and
// status word); regions: start of the per-work-group regions, launch after
// launch (nwg of each x its aligned per-group bytes).
int enqueue_forward(std::vector<Launch>& launches, char* header, char* regions, hipStream_t st) {
  unsigned* status = status_word(header);
  zero_status<<<1, 64, 0, st>>>(status);
  size_t off = 0;
  int li = 0, rc = TN_OK;
  for (auto& L : launches) {
    for (int i = 0; i < L.jt.n; ++i) L.jt.j[i].status = status;
    unsigned long long* counter = reinterpret_cast<unsigned long long*>(header) + li;
    char* scr = regions + off;
    off += (size_t)L.nwg * group_bytes(L);
    if (L.small) {
      const LdsLayout lay = launch_layout(L);
      const int64_t stride = (int64_t)group_bytes(L);
      const int r = L.build == BUILD_256X3
                        ? tnmld_small3::launch_fwd(L.precision, &L.jt, counter, scr, stride, L.scratch_elems, &lay,
                                                   lay.bytes, L.nwg, st)
                        : tnmld_small::launch_fwd_small(L.precision, &L.jt, counter, scr, stride, L.scratch_elems,
                                                        &lay, lay.bytes, L.nwg, st);
      if (r != 0) return fail(TN_EDEVICE, "kernel launch failed");
      ++li;
      continue;
    }
    if (L.precision == TN_FP64) rc = launch_fwd<double, double, GEMM_F64>(L, L.nwg, scr, counter, st);
    else if (L.precision == TN_FP32) rc = launch_fwd<float, double, GEMM_F32>(L, L.nwg, scr, counter, st);
    else if (L.precision == TN_BF16) rc = launch_fwd<float, float, BF16_GEMM_MODE>(L, L.nwg, scr, counter, st);
    else if (L.precision == TN_BF16_F64) rc = launch_fwd<float, double, GEMM_BF16>(L, L.nwg, scr, counter, st);
    else rc = launch_fwd<float, float, GEMM_F32>(L, L.nwg, scr, counter, st);
    if (rc) return rc;
    ++li;
  }
  return TN_OK;
}

int run_forward(const tn_segment* segs, int32_t nseg, void* workspace, size_t ws_bytes, void* stream) {
  std::vector<Launch> launches;
  size_t need = 0;
  int nwg = 0;
  DevInfo di;
  int rc = validate(segs, nseg);
  if (rc) return rc;
  if ((rc = device_info(&di))) return rc;
  if ((rc = plan_launches(segs, nseg, std::min(di.lds_max, kLdsLimit), &launches, &need, &nwg))) return rc;
  if (launches.empty()) return TN_OK;
  if (!workspace || ws_bytes < need) return fail(TN_EINVAL, "workspace too small: need " + std::to_string(need));
  char* base = reinterpret_cast<char*>(workspace);
  return enqueue_forward(launches, base, base + align_up(sizeof(unsigned long long) * kMaxLaunches),
                         reinterpret_cast<hipStream_t>(stream));
}

// ---- allocation-free entry point ---------------------------------------------
// Device memory of tn_decode_batch_noalloc: a fixed array that every device the
// library runs on holds for the life of the process.  Layout: workspace header
// (kAlign bytes), the plan blobs of the call (kNoAllocPlanBytes), then the
// per-work-group regions.  Host code never passes `scratch` itself to a kernel
// or a copy: it uses the device address that hipGetSymbolAddress returned for
// the current device (noalloc_base).
constexpr size_t kNoAllocPlanBytes = 4ull << 20;

std::mutex g_noalloc_mu;
std::map<int, char*> g_noalloc_base;  // device -> address of `scratch` on that device

int noalloc_base(char** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(TN_EDEVICE, "no HIP device");
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  auto it = g_noalloc_base.find(dev);
  if (it == g_noalloc_base.end()) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p)
      return fail(TN_EDEVICE, "hipGetSymbolAddress of the fixed scratch array failed");
    it = g_noalloc_base.emplace(dev, reinterpret_cast<char*>(p)).first;
  }
  *out = it->second;
  return TN_OK;
}

int run_forward_noalloc(const tn_segment* segs, int32_t nseg, void* stream) {
  std::vector<Launch> launches;
  size_t need = 0;
  int nwg = 0;
  DevInfo di;
  int rc = validate(segs, nseg);
  if (rc) return rc;
  if ((rc = device_info(&di))) return rc;
  char* base = nullptr;
  if ((rc = noalloc_base(&base))) return rc;
  if ((rc = plan_launches(segs, nseg, std::min(di.lds_max, kLdsLimit), &launches, &need, &nwg, true, false)))
    return rc;
  if (launches.empty()) return TN_OK;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  // plan blobs (one copy per distinct plan) after the header
  std::map<const Plan*, size_t> placed;
  size_t pofs = 0;
  for (auto& L : launches)
    for (int i = 0; i < L.jt.n; ++i) {
      const Plan* p = L.host_plan[i];
      auto it = placed.find(p);
      if (it == placed.end()) {
        if (pofs + align_up(p->blob.size()) > kNoAllocPlanBytes)
          return fail(TN_EINVAL, "plans of this call exceed the allocation-free entry point's plan area");
        it = placed.emplace(p, pofs).first;
        pofs += align_up(p->blob.size());
      }
      L.jt.j[i].plan = reinterpret_cast<const uint8_t*>(base + kAlign + it->second);
    }
  // persistent work-groups: as many as the fixed regions hold, up to the usual count
  const size_t avail = kNoAllocBytes - kAlign - kNoAllocPlanBytes;
  size_t per_round = 0, full = 0;
  for (auto& L : launches) {
    const size_t pw = group_bytes(L);
    per_round += pw;
    full += (size_t)L.nwg * pw;
  }
  if (per_round > avail)
    return fail(TN_EINVAL, "one work-group of each launch needs " + std::to_string(per_round) +
                               " bytes; the allocation-free entry point holds " + std::to_string(avail));
  if (full > avail) {
    const double f = (double)avail / (double)full;
    for (auto& L : launches) {
      int w = (int)((double)L.nwg * f);
      L.nwg = std::max(1, std::min(L.nwg, w));
    }
  }
  for (const auto& kv : placed)
    if (hipMemcpyAsync(base + kAlign + kv.second, kv.first->blob.data(), kv.first->blob.size(),
                       hipMemcpyHostToDevice, st) != hipSuccess)
      return fail(TN_EDEVICE, "plan copy failed");
  return enqueue_forward(launches, base, base + kAlign + kNoAllocPlanBytes, st);
}

// Layout of the backward call: one launch (all segments share a precision).
struct BwdLayout {
  int precision = 0;
  JobTable jt{};
  int seg_of_job[TN_MAX_SEGMENTS] = {};
  PlanHeader merged{};
  int nwg = 0;
  bool small = false;      // 256-thread build (two or more work-groups per CU)
  bool aj_global = false;  // small build without the LDS copy of the input site
  int64_t scratch_stride = 0, part_stride = 0;
  size_t hdr_bytes = 0, total = 0;
  // caller memory of the two-call backward: each job's top-sweep states
  int64_t states_elems[TN_MAX_SEGMENTS] = {};  // per syndrome
  size_t states_ofs[TN_MAX_SEGMENTS] = {};     // bytes from the start of the buffer
  size_t states_total = 0;
};

int plan_backward(const tn_segment* segs, int32_t nseg, BwdLayout* bl) {
  std::vector<Launch> launches;
  size_t fwd = 0;
  int nwgf = 0;
  DevInfo di;
  int rc = validate(segs, nseg);
  if (rc) return rc;
  for (int i = 0; i < nseg; ++i) {
    if (segs[i].rounds > 1) return fail(TN_EUNSUPPORTED, "the gradient takes segments of one syndrome round");
    if (segs[i].precision == TN_BF16_F64 && segs[i].count > 0)
      return fail(TN_EUNSUPPORTED, "the gradient is not built for TN_BF16_F64");
  }
  if ((rc = device_info(&di))) return rc;
  bl->hdr_bytes = kAlign;  // counters and the status word
  if ((rc = plan_launches(segs, nseg, std::min(di.lds_max, kLdsLimit), &launches, &fwd, &nwgf, false))) return rc;
  if (launches.size() > 1) return fail(TN_EUNSUPPORTED, "backward segments must share one precision");
  if (launches.empty()) {
    bl->total = bl->hdr_bytes;
    return TN_OK;
  }
  const Launch& L = launches[0];
  bl->precision = L.precision;
  bl->jt = L.jt;
  bl->merged = L.merged;
  {
    // backward items are syndromes (the four cosets of one in a work-group)
    int64_t items = 0;
    for (int i = 0; i < bl->jt.n; ++i) {
      bl->jt.j[i].item_begin = items;
      items += bl->jt.j[i].count;
    }
    bl->jt.nitems = items;
  }
  // map jobs back to segments (same order as plan_launches: by decreasing d, stable)
  std::vector<int> order(nseg);
  for (int i = 0; i < nseg; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return segs[a].d > segs[b].d; });
  int ji = 0;
  int64_t part = 0, per_item = 0;
  for (int oi : order) {
    if (segs[oi].count == 0) continue;
    bl->seg_of_job[ji] = oi;
    JobDev& j = bl->jt.j[ji];
    j.logp = segs[oi].out_logp;
    j.part_ofs = part;
    part += (int64_t)segs[oi].n_models * segs[oi].d * segs[oi].d * 3;
    const PlanHeader* H = nullptr;
    {
      std::lock_guard<std::mutex> lk(g_mu);
      for (auto& kv : g_plans)
        if (kv.second->dev == j.plan) H = &kv.second->plan.h;
    }
    if (!H) return fail(TN_EDEVICE, "internal: plan not cached");
    // work and bottom regions, the stored top states (the shared rows once,
    // the rest per coset), environments and three temporaries
    const int S = std::min(H->shared_rows, H->nstep);
    const int64_t st_elems = (int64_t)(S + 4 * (H->nstep - S)) * H->mps_elems;
    per_item = std::max<int64_t>(per_item, 2 * H->scratch_elems + st_elems + H->env_elems + 3 * H->tmp_elems);
    bl->states_elems[ji] = st_elems;
    bl->states_ofs[ji] = bl->states_total;
    bl->states_total += align_up((size_t)segs[oi].count * (size_t)st_elems * real_bytes(L.precision));
    ++ji;
  }
  const int lb = lds_layout(L.merged, real_bytes(L.precision), fac_bytes(L.precision)).bytes;
  bl->nwg = std::max(1, wgs_for(lb, bwd_kernel_of(L.precision))) * di.cus;
  {
    // the 256-thread build when its plan fits (as for the forward pass) and
    // at least two of its work-groups share a CU
    const int rpg = fac_bytes(L.precision) == 4 ? 4 : 2;
    const PlanHeader& h = L.merged;
    if (h.max_m <= rpg * (kSmallNT / 16) && h.max_n <= 256 && h.max_bond <= kSmallNT) {
      const int limit = kLdsPerCU / 2 - 256;
      bool ajg = false;
      int sb = lb;
      if (sb > limit) {
        sb = lds_layout(h, real_bytes(L.precision), fac_bytes(L.precision), true).bytes;
        ajg = true;
      }
      const int ws = sb <= limit ? tnmld_small::small_bwd_wgs_per_cu(L.precision, sb) : 0;
      if (ws >= 2) {
        bl->small = true;
        bl->aj_global = ajg;
        bl->nwg = std::min(ws, kLdsPerCU / (sb + 256)) * di.cus;
      }
    }
  }
  bl->scratch_stride = (int64_t)align_up((size_t)per_item * real_bytes(L.precision));
  bl->part_stride = (part + 31) / 32 * 32;
  bl->total = bl->hdr_bytes + align_up((size_t)bl->nwg * bl->part_stride * sizeof(double)) +
              (size_t)bl->nwg * bl->scratch_stride;
  return TN_OK;
}

}  // namespace

int report_error(int code, const std::string& msg) { return fail(code, msg); }

}  // namespace tnmld

using namespace tnmld;

extern "C" {

size_t tn_workspace_size(const tn_segment* segs, int32_t nseg, int32_t with_backward) {
  if (with_backward) {
    BwdLayout bl;
    if (plan_backward(segs, nseg, &bl)) return 0;
    return bl.total;
  }
  std::vector<Launch> launches;
  size_t need = 0;
  int nwg = 0;
  DevInfo di;
  if (validate(segs, nseg)) return 0;
  if (device_info(&di)) return 0;
  if (plan_launches(segs, nseg, std::min(di.lds_max, kLdsLimit), &launches, &need, &nwg)) return 0;
  return need;
}

int tn_coset_loglik(const tn_segment* segs, int32_t nseg, void* workspace, size_t ws_bytes, void* stream) {
  int rc = run_forward(segs, nseg, workspace, ws_bytes, stream);
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  for (int i = 0; i < nseg; ++i)
    if (segs[i].out_logp && segs[i].count > 0)
      decide_kernel<<<(unsigned)((segs[i].count + 255) / 256), 256, 0, st>>>(segs[i].out_logz, segs[i].count, 1e-9,
                                                                           segs[i].out_logp, nullptr);
  if (hipGetLastError() != hipSuccess) return fail(TN_EDEVICE, "decide launch failed");
  return TN_OK;
}

int tn_decode_batch(const tn_segment* segs, int32_t nseg, double tie_tol, void* workspace, size_t ws_bytes,
                    void* stream) {
  if (!(tie_tol > 0.0)) tie_tol = 1e-9;
  int rc = run_forward(segs, nseg, workspace, ws_bytes, stream);
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  for (int i = 0; i < nseg; ++i)
    if (segs[i].count > 0 && (segs[i].out_logp || segs[i].out_class))
      decide_kernel<<<(unsigned)((segs[i].count + 255) / 256), 256, 0, st>>>(segs[i].out_logz, segs[i].count, tie_tol,
                                                                           segs[i].out_logp, segs[i].out_class);
  if (hipGetLastError() != hipSuccess) return fail(TN_EDEVICE, "decide launch failed");
  return TN_OK;
}

int tn_decode_batch_noalloc(const tn_segment* segs, int32_t nseg, double tie_tol, void* stream) {
  if (!(tie_tol > 0.0)) tie_tol = 1e-9;
  int rc = run_forward_noalloc(segs, nseg, stream);
  if (rc) return rc;
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  for (int i = 0; i < nseg; ++i)
    if (segs[i].count > 0 && (segs[i].out_logp || segs[i].out_class))
      decide_kernel<<<(unsigned)((segs[i].count + 255) / 256), 256, 0, st>>>(segs[i].out_logz, segs[i].count, tie_tol,
                                                                           segs[i].out_logp, segs[i].out_class);
  if (hipGetLastError() != hipSuccess) return fail(TN_EDEVICE, "decide launch failed");
  return TN_OK;
}

}  // extern "C"

namespace tnmld {
namespace {

// The backward launch in one of three modes (ADJ_FUSED, ADJ_TOP, ADJ_BOTTOM;
// adjoint.hpp).  ADJ_TOP takes no gradient arrays and writes log Z / log P(s);
// the other two accumulate into grad_log_rates.
int run_backward(const tn_segment* segs, int32_t nseg, const double* const* grad_logp, double* const* grad_log_rates,
                 int write_fwd, int mode, void* states, size_t states_bytes, void* workspace, size_t ws_bytes,
                 void* stream) {
  BwdLayout bl;
  int rc = plan_backward(segs, nseg, &bl);
  if (rc) return rc;
  const bool grads = mode != ADJ_TOP;
  if (grads && (!grad_logp || !grad_log_rates)) return fail(TN_EINVAL, "null gradient arrays");
  for (int i = 0; i < nseg; ++i) {
    if (segs[i].count > 0 && (!segs[i].out_logp || (grads && (!grad_logp[i] || !grad_log_rates[i]))))
      return fail(TN_EINVAL, "backward needs grad_logp, grad_log_rates and out_logp for every segment");
  }
  if (mode != ADJ_FUSED && (!states || states_bytes < bl.states_total))
    return fail(TN_EINVAL, "states buffer too small: need " + std::to_string(bl.states_total));
  if (!workspace || ws_bytes < bl.total) return fail(TN_EINVAL, "workspace too small: need " + std::to_string(bl.total));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  unsigned* status = status_word(workspace);
  zero_status<<<1, 64, 0, st>>>(status);
  if (bl.jt.n == 0) return TN_OK;
  char* base = reinterpret_cast<char*>(workspace) + bl.hdr_bytes;
  double* partials = reinterpret_cast<double*>(base);
  char* scratch_base = base + align_up((size_t)bl.nwg * bl.part_stride * sizeof(double));
  if (grads) fill_zero_f64<<<256, 256, 0, st>>>(partials, (int64_t)bl.nwg * bl.part_stride);
  JobTable jt = bl.jt;
  for (int i = 0; i < jt.n; ++i) {
    jt.j[i].gradp = grads ? grad_logp[bl.seg_of_job[i]] : nullptr;
    jt.j[i].status = status;
    jt.j[i].states = mode == ADJ_FUSED ? nullptr : static_cast<char*>(states) + bl.states_ofs[i];
    jt.j[i].states_stride = bl.states_elems[i];
  }
  LdsLayout lay = lds_layout(bl.merged, real_bytes(bl.precision), fac_bytes(bl.precision), bl.aj_global);
  int flags = (write_fwd ? 1 : 0) | (mode << 1);
  int64_t sstride = bl.scratch_stride, pstride = bl.part_stride;
  if (bl.small) {
    if (tnmld_small::launch_bwd_small(bl.precision, &jt, scratch_base, sstride, &lay, lay.bytes, flags, partials,
                                      pstride, bl.nwg, st) != 0)
      return fail(TN_EDEVICE, "backward launch failed");
  } else {
    const void* kern = bwd_kernel_of(bl.precision);
    if ((rc = ensure_lds_attr(kern, lay.bytes))) return rc;
    void* args[] = {&jt, &scratch_base, &sstride, &lay, &flags, &partials, &pstride};
    if (hipLaunchKernel(kern, dim3(bl.nwg), dim3(NT), args, lay.bytes, st) != hipSuccess)
      return fail(TN_EDEVICE, "backward launch failed");
  }
  if (grads)
    for (int i = 0; i < jt.n; ++i) {
      const tn_segment& sg = segs[bl.seg_of_job[i]];
      const int64_t len = (int64_t)sg.n_models * sg.d * sg.d * 3;
      reduce_partials<<<(unsigned)((len + 255) / 256), 256, 0, st>>>(partials, pstride, bl.nwg, jt.j[i].part_ofs,
                                                                     len, grad_log_rates[bl.seg_of_job[i]]);
    }
  if (hipGetLastError() != hipSuccess) return fail(TN_EDEVICE, "reduction launch failed");
  return TN_OK;
}

}  // namespace
}  // namespace tnmld

extern "C" {

int tn_coset_loglik_backward(const tn_segment* segs, int32_t nseg, const double* const* grad_logp,
                             double* const* grad_log_rates, int32_t forward_done, void* workspace, size_t ws_bytes,
                             void* stream) {
  return run_backward(segs, nseg, grad_logp, grad_log_rates, forward_done ? 0 : 1, ADJ_FUSED, nullptr, 0, workspace,
                      ws_bytes, stream);
}

size_t tn_states_size(const tn_segment* segs, int32_t nseg) {
  BwdLayout bl;
  if (plan_backward(segs, nseg, &bl)) return 0;
  return bl.states_total > 0 ? bl.states_total : 256;
}

int tn_coset_loglik_save(const tn_segment* segs, int32_t nseg, void* states, size_t states_bytes, void* workspace,
                         size_t ws_bytes, void* stream) {
  return run_backward(segs, nseg, nullptr, nullptr, 1, ADJ_TOP, states, states_bytes, workspace, ws_bytes, stream);
}

int tn_coset_loglik_backward_saved(const tn_segment* segs, int32_t nseg, const double* const* grad_logp,
                                   double* const* grad_log_rates, const void* states, size_t states_bytes,
                                   void* workspace, size_t ws_bytes, void* stream) {
  return run_backward(segs, nseg, grad_logp, grad_log_rates, 0, ADJ_BOTTOM, const_cast<void*>(states), states_bytes,
                      workspace, ws_bytes, stream);
}

int tn_code_stabilizers(int32_t d, int32_t* type_out, int32_t* support_out) {
  if (d < 3 || d > TN_MAX_D || d % 2 == 0 || !type_out || !support_out) return fail(TN_EINVAL, "bad arguments");
  int j = 0;
  for (int pass = 0; pass < 2; ++pass)
    for (int r = -1; r <= d - 1; ++r)
      for (int c = -1; c <= d - 1; ++c) {
        bool is_x = ((r + c) & 1) == 0;
        bool bulk = r >= 0 && c >= 0 && r <= d - 2 && c <= d - 2;
        bool tb = (r == -1 || r == d - 1) && is_x && c >= 0 && c <= d - 2;
        bool lr = (c == -1 || c == d - 1) && !is_x && r >= 0 && r <= d - 2;
        if (!(bulk || tb || lr) || ((pass == 0) == is_x)) continue;
        type_out[j] = is_x ? 0 : 1;
        int k = 0;
        for (int dr = 0; dr < 2; ++dr)
          for (int dc = 0; dc < 2; ++dc) {
            int rr = r + dr, cc = c + dc;
            if (rr >= 0 && rr < d && cc >= 0 && cc < d) support_out[4 * j + k++] = rr * d + cc;
          }
        for (; k < 4; ++k) support_out[4 * j + k] = -1;
        ++j;
      }
  return j;
}

int tn_plan_adjoint_flops(int32_t d, int32_t chi, int32_t precision, double* out) {
  if (!out || precision < TN_FP64 || precision > TN_BF16_F64) return fail(TN_EINVAL, "bad arguments");
  Plan p;
  std::string why;
  if (choose_group(d, chi, precision, kLdsLimit, &p, &why) < 0) return fail(TN_EUNSUPPORTED, why);
  out[0] = p.h.flops_bu;
  out[1] = p.h.flops_env;
  out[2] = p.h.flops_shared + 4.0 * (p.h.flops_fwd - p.h.flops_shared) + 4.0 * (p.h.flops_bu + p.h.flops_env);
  return TN_OK;
}

int tn_plan_gemm_flops(int32_t d, int32_t chi, int32_t precision, double* out) {
  if (!out || precision < TN_FP64 || precision > TN_BF16_F64) return fail(TN_EINVAL, "bad arguments");
  Plan p;
  std::string why;
  if (choose_group(d, chi, precision, kLdsLimit, &p, &why) < 0) return fail(TN_EUNSUPPORTED, why);
  out[0] = p.h.flops_gemm;
  out[1] = p.h.flops_gemm_shared + 4.0 * (p.h.flops_gemm - p.h.flops_gemm_shared);
  return TN_OK;
}

int tn_plan_info(int32_t d, int32_t chi, int32_t precision, double* info) {
  return tn_plan_info_rounds(d, chi, precision, 1, info);
}

int tn_plan_info_rounds(int32_t d, int32_t chi, int32_t precision, int32_t rounds, double* info) {
  if (!info || precision < TN_FP64 || precision > TN_BF16_F64 || rounds < 0 || rounds > TN_MAX_ROUNDS)
    return fail(TN_EINVAL, "bad arguments");
  if (rounds < 1) rounds = 1;
  Plan p;
  std::string why;
  int g = choose_group(d, chi, precision, kLdsLimit, &p, &why, rounds);
  if (g < 0) return fail(TN_EUNSUPPORTED, why);
  info[0] = p.h.flops_fwd;
  info[1] = (double)p.h.scratch_elems * real_bytes(precision);
  info[2] = lds_layout(p.h, real_bytes(precision), fac_bytes(precision)).bytes;
  info[3] = p.h.nsite;
  info[4] = p.h.nstep;
  info[5] = g;
  info[6] = wgs_for((int)info[2], fwd_kernel_of(precision));
  info[7] = p.h.flops_shared + 4.0 * (p.h.flops_fwd - p.h.flops_shared);
  if (rounds == 1) {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tune.find(std::make_tuple(d, chi, precision));
    if (it != g_tune.end() && it->second.wgs > 0) info[6] = std::min<double>(info[6], it->second.wgs);
  }
  return TN_OK;
}

int tn_set_tuning_ex(int32_t d, int32_t chi, int32_t precision, int32_t group, int32_t wg_per_cu,
                     int32_t threads) {
  if (d < 3 || d > TN_MAX_D || d % 2 == 0 || chi < 0 || precision < TN_FP64 || precision > TN_BF16_F64 ||
      group < 0 || group > 2 || wg_per_cu < 0 || wg_per_cu > 4 || (threads != 0 && threads != NT && threads != kSmallNT))
    return fail(TN_EINVAL, "bad tuning arguments");
  std::lock_guard<std::mutex> lk(g_mu);
  if (group == 0 && wg_per_cu == 0 && threads == 0) g_tune.erase(std::make_tuple(d, chi, precision));
  else g_tune[std::make_tuple(d, chi, precision)] = Tune{group, wg_per_cu, threads};
  return TN_OK;
}

int tn_set_tuning(int32_t d, int32_t chi, int32_t precision, int32_t group, int32_t wg_per_cu) {
  if (wg_per_cu > kMaxWgPerCU) return fail(TN_EINVAL, "bad tuning arguments");
  return tn_set_tuning_ex(d, chi, precision, group, wg_per_cu, 0);
}

int tn_get_launch(int32_t d, int32_t chi, int32_t precision, int32_t* shape) {
  if (!shape || precision < TN_FP64 || precision > TN_BF16_F64) return fail(TN_EINVAL, "bad arguments");
  // a one-segment call of this bucket: which build and how many groups per CU
  tn_segment sg{};
  sg.d = d;
  sg.chi = chi;
  sg.precision = precision;
  sg.n_models = 1;
  sg.count = 1;
  sg.rates = reinterpret_cast<const double*>(1);  // never dereferenced: only the plan is built
  sg.syndromes = reinterpret_cast<const uint8_t*>(1);
  sg.out_logz = reinterpret_cast<double*>(1);
  std::vector<Launch> launches;
  size_t need = 0;
  int nwg = 0;
  DevInfo di;
  int rc = device_info(&di);
  if (rc) return rc;
  if ((rc = plan_launches(&sg, 1, std::min(di.lds_max, kLdsLimit), &launches, &need, &nwg))) return rc;
  if (launches.size() != 1) return fail(TN_EUNSUPPORTED, "no launch");
  shape[0] = launches[0].host_plan[0]->h.group;
  shape[1] = launches[0].nwg / std::max(1, di.cus);
  shape[2] = launches[0].small ? kSmallNT : NT;
  return TN_OK;
}

int tn_get_launches(const tn_segment* segs, int32_t nseg, int32_t* out, int32_t max_launches, int32_t* count) {
  if (!out || !count || max_launches < 0) return fail(TN_EINVAL, "bad arguments");
  std::vector<Launch> launches;
  size_t need = 0;
  int nwg = 0;
  DevInfo di;
  int rc = device_info(&di);
  if (rc) return rc;
  if ((rc = plan_launches(segs, nseg, std::min(di.lds_max, kLdsLimit), &launches, &need, &nwg))) return rc;
  *count = (int32_t)launches.size();
  for (size_t i = 0; i < launches.size() && i < (size_t)max_launches; ++i) {
    const Launch& L = launches[i];
    out[4 * i] = L.precision;
    out[4 * i + 1] = L.small ? kSmallNT : NT;
    out[4 * i + 2] = L.nwg / std::max(1, di.cus);
    out[4 * i + 3] = L.jt.n;
  }
  return TN_OK;
}

int tn_workspace_status(const void* workspace, size_t ws_bytes, void* stream, int64_t* unresolved_cosets) {
  if (!workspace) {  // the allocation-free entry point's fixed array on the current device
    char* base = nullptr;
    if (int rc = noalloc_base(&base)) return rc;
    workspace = base;
    ws_bytes = kAlign;
  }
  if (ws_bytes < kAlign) return fail(TN_EINVAL, "workspace too small for a status word");
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  if (hipStreamSynchronize(st) != hipSuccess) return fail(TN_EDEVICE, "stream synchronisation failed");
  unsigned v[4] = {0u, 0u, 0u, 0u};
  if (hipMemcpy(v, status_word(const_cast<void*>(workspace)), sizeof(v), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(TN_EDEVICE, "status read failed");
  unsigned long long cnt = 0;
  std::memcpy(&cnt, v + 2, sizeof(cnt));
  if (unresolved_cosets) *unresolved_cosets = (v[0] & ST_UNRESOLVED) ? (int64_t)cnt : 0;
  if (v[0] & ST_BAD_INPUT)
    return fail(TN_EINVAL, "invalid input values: a syndrome byte above 1, a model index out of range, or rates "
                           "outside [0, 1] / NaN / p_X + p_Y + p_Z > 1 (those syndromes were given log Z = -inf)");
  if (v[0] & ST_NUMERIC)
    return fail(TN_ENUMERIC, "precision breakdown: all four cosets of a syndrome of a strictly positive noise "
                             "model contracted to Z <= 0 (reported as log Z = -inf)");
  return TN_OK;
}

const char* tn_last_error(void) { return g_err.c_str(); }

}  // extern "C"
