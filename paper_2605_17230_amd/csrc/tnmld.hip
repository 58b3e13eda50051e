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
//      Householder LQ factorisations, then sweep left-to-right truncating every
//      bond to chi by a one-sided Jacobi SVD (the paper's "successive SVD
//      truncations"), and add the removed log-norm to an FP64 accumulator;
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
#include "contract.hpp"
#include "plan.hpp"
#include "sweep.hpp"

namespace tnmld {

template <typename Real, typename Fac>
__global__ __launch_bounds__(NT) void fwd_kernel(JobTable jt, unsigned long long* counter, char* scratch,
                                                  int64_t scratch_stride, LdsLayout lay) {
  extern __shared__ __align__(16) uint8_t smem[];
  Real* scr = reinterpret_cast<Real*>(scratch + (int64_t)blockIdx.x * scratch_stride);
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
    const int64_t local = item - job.item_begin;
    const int64_t b = local >> 2;
    const int mlog = (int)(local & 3);
    int label = 0;
    const double lz = contract_one<Real, Fac>(job, b, mlog, smem, lay, scr, &label);
    if (threadIdx.x == 0) job.logz[b * 4 + label] = lz;
    __syncthreads();
  }
}

__global__ void zero_counter(unsigned long long* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0ull;
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
std::map<std::tuple<int, int, int, int>, DevPlan*> g_plans;  // (device, d, chi, group)

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
int fac_bytes(int precision) { return precision == TN_FP32_PLAIN ? 4 : 8; }
bool precision_built(int precision) {
  return precision == TN_FP64 || precision == TN_FP32 || precision == TN_FP32_PLAIN;
}

// largest usable LDS per block on gfx950 when no device is queried
constexpr int kLdsLimit = 160 * 1024;

constexpr int kLdsPerCU = 160 * 1024;
constexpr int kMaxWgPerCU = 1024 / NT > 1 ? 1024 / NT : 1;  // <= 128 VGPRs: 4 waves per SIMD, 1024 threads per CU

// Tuned launch shapes, set by tn_set_tuning (the autotuner's cache).
struct Tune {
  int group, wgs;
};
std::map<std::tuple<int, int, int>, Tune> g_tune;

int wgs_for(int lds_bytes) {
  const int w = kLdsPerCU / (lds_bytes + 256);
  return w < 1 ? 0 : (w > kMaxWgPerCU ? kMaxWgPerCU : w);
}

// Choose the column grouping (1 or 2 columns per site): a tuned entry if one
// exists, else the grouping that fits the most work-groups per CU (ties: 2).
int choose_group(int d, int chi, int precision, int lds_limit, Plan* out, std::string* why) {
  int forced = 0;
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tune.find(std::make_tuple(d, chi, precision));
    if (it != g_tune.end()) forced = it->second.group;
  }
  int best_g = -1, best_w = 0;
  Plan best;
  for (int g = 2; g >= 1; --g) {
    if (forced && g != forced) continue;
    Plan p;
    std::string e = build_plan(d, chi, g, &p);
    if (!e.empty()) {
      *why = e;
      return -1;
    }
    LdsLayout lay = lds_layout(p.h, real_bytes(precision), fac_bytes(precision));
    if (lay.bytes > lds_limit) {
      *why = "chi=" + std::to_string(chi) + " needs " + std::to_string(lay.bytes) + " B of LDS";
      continue;
    }
    const int w = wgs_for(lay.bytes);
    if (w > best_w) {
      best_w = w;
      best_g = g;
      best = std::move(p);
    }
  }
  if (best_g > 0) *out = std::move(best);
  return best_g;
}

int get_plan(int d, int chi, int precision, int lds_limit, DevPlan** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return fail(TN_EDEVICE, "no HIP device");
  Plan p;
  std::string why;
  int g = choose_group(d, chi, precision, lds_limit, &p, &why);
  if (g < 0) return fail(TN_EUNSUPPORTED, why);
  std::lock_guard<std::mutex> lk(g_mu);
  auto key = std::make_tuple(dev, d, chi, g);
  auto it = g_plans.find(key);
  if (it != g_plans.end()) {
    *out = it->second;
    return TN_OK;
  }
  DevPlan* dp = new DevPlan;
  dp->plan = std::move(p);
  if (hipMalloc(&dp->dev, dp->plan.blob.size()) != hipSuccess) {
    delete dp;
    return fail(TN_ENOMEM, "hipMalloc of plan failed");
  }
  if (hipMemcpy(dp->dev, dp->plan.blob.data(), dp->plan.blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
    (void)hipFree(dp->dev);
    delete dp;
    return fail(TN_EDEVICE, "plan upload failed");
  }
  g_plans[key] = dp;
  *out = dp;
  return TN_OK;
}

int validate(const tn_segment* segs, int32_t nseg) {
  if (!segs || nseg < 1 || nseg > TN_MAX_SEGMENTS) return fail(TN_EINVAL, "nseg must be in [1, 16]");
  for (int i = 0; i < nseg; ++i) {
    const tn_segment& s = segs[i];
    if (s.d < 3 || s.d > TN_MAX_D || s.d % 2 == 0) return fail(TN_EINVAL, "d must be odd in [3, 31]");
    if (s.chi < 0) return fail(TN_EINVAL, "chi must be >= 0");
    if (s.precision < TN_FP64 || s.precision > TN_FP32_PLAIN) return fail(TN_EINVAL, "bad precision");
    if (s.n_models < 1) return fail(TN_EINVAL, "n_models must be >= 1");
    if (s.count < 0) return fail(TN_EINVAL, "count must be >= 0");
    if (s.count > 0 && (!s.rates || !s.syndromes || !s.out_logz)) return fail(TN_EINVAL, "null pointer");
  }
  return TN_OK;
}

struct Launch {
  int precision;
  JobTable jt;
  PlanHeader merged;
  int64_t scratch_elems;
  int nwg;  // persistent work-groups of this launch
};

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Build the launch groups (one per precision) and the workspace layout.
int plan_launches(const tn_segment* segs, int32_t nseg, int lds_limit, std::vector<Launch>* out, size_t* ws_bytes,
                  int* nwg) {
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
  for (int prec = TN_FP64; prec <= TN_FP32_PLAIN; ++prec) {
    Launch L{};
    L.precision = prec;
    int64_t items = 0;
    for (int oi : order) {
      const tn_segment& s = segs[oi];
      if (s.precision != prec || s.count == 0) continue;
      if (!precision_built(prec)) return fail(TN_EUNSUPPORTED, "precision not built");
      DevPlan* dp = nullptr;
      if ((rc = get_plan(s.d, s.chi, prec, lds_limit, &dp))) return rc;
      JobDev& j = L.jt.j[L.jt.n++];
      j.plan = dp->dev;
      j.rates = s.rates;
      j.model_index = s.model_index;
      j.syn = s.syndromes;
      j.logz = s.out_logz;
      j.count = s.count;
      j.item_begin = items;
      j.n_models = s.n_models;
      items += 4 * s.count;
      merge_maxima(&L.merged, dp->plan.h);
      L.scratch_elems = std::max<int64_t>(L.scratch_elems, dp->plan.h.scratch_elems);
      int tw = 0;
      {
        std::lock_guard<std::mutex> lk(g_mu);
        auto it = g_tune.find(std::make_tuple(s.d, s.chi, prec));
        if (it != g_tune.end()) tw = it->second.wgs;
      }
      if (tw > 0) L.nwg = L.nwg ? std::min(L.nwg, tw) : tw;  // per-CU count for now
    }
    L.jt.nitems = items;
    if (L.jt.n > 0) out->push_back(L);
  }
  size_t bytes = align_up(sizeof(unsigned long long) * 4);
  for (auto& L : *out) {
    if (L.merged.max_bond > NT) return fail(TN_EUNSUPPORTED, "bond dimension above the work-group size");
    const int lb = lds_layout(L.merged, real_bytes(L.precision), fac_bytes(L.precision)).bytes;
    int w = wgs_for(lb);
    if (L.nwg > 0) w = std::min(w, L.nwg);
    if (w < 1) return fail(TN_EUNSUPPORTED, "LDS of the merged plans exceeds one CU");
    L.nwg = w * di.cus;
    *nwg = std::max(*nwg, L.nwg);
    bytes += (size_t)L.nwg * align_up((size_t)L.scratch_elems * real_bytes(L.precision));
  }
  *ws_bytes = bytes;
  return TN_OK;
}

template <typename Real, typename Fac>
int launch_fwd(const Launch& L, int nwg, char* ws_scratch, unsigned long long* counter, hipStream_t st) {
  LdsLayout lay = lds_layout(L.merged, sizeof(Real), sizeof(Fac));
  auto kern = fwd_kernel<Real, Fac>;
  if (hipFuncSetAttribute(reinterpret_cast<const void*>(kern), hipFuncAttributeMaxDynamicSharedMemorySize,
                          lay.bytes) != hipSuccess)
    return fail(TN_EDEVICE, "hipFuncSetAttribute failed");
  zero_counter<<<1, 64, 0, st>>>(counter);
  const int64_t stride = (int64_t)align_up((size_t)L.scratch_elems * sizeof(Real));
  hipLaunchKernelGGL(kern, dim3(nwg), dim3(NT), lay.bytes, st, L.jt, counter, ws_scratch, stride, lay);
  if (hipGetLastError() != hipSuccess) return fail(TN_EDEVICE, "kernel launch failed");
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
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* base = reinterpret_cast<char*>(workspace);
  size_t off = align_up(sizeof(unsigned long long) * 4);
  int li = 0;
  for (auto& L : launches) {
    unsigned long long* counter = reinterpret_cast<unsigned long long*>(base) + li;
    char* scr = base + off;
    off += (size_t)L.nwg * align_up((size_t)L.scratch_elems * real_bytes(L.precision));
    if (L.precision == TN_FP64) rc = launch_fwd<double, double>(L, L.nwg, scr, counter, st);
    else if (L.precision == TN_FP32) rc = launch_fwd<float, double>(L, L.nwg, scr, counter, st);
    else rc = launch_fwd<float, float>(L, L.nwg, scr, counter, st);
    if (rc) return rc;
    ++li;
  }
  return TN_OK;
}

}  // namespace
}  // namespace tnmld

using namespace tnmld;

extern "C" {

size_t tn_workspace_size(const tn_segment* segs, int32_t nseg, int32_t with_backward) {
  (void)with_backward;
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

int tn_coset_loglik_backward(const tn_segment* segs, int32_t nseg, const double* const* grad_logp,
                             double* const* grad_log_rates, void* workspace, size_t ws_bytes, void* stream) {
  (void)segs;
  (void)nseg;
  (void)grad_logp;
  (void)grad_log_rates;
  (void)workspace;
  (void)ws_bytes;
  (void)stream;
  return fail(TN_EUNSUPPORTED, "backward not built yet");
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

int tn_plan_info(int32_t d, int32_t chi, int32_t precision, double* info) {
  if (!info || precision < TN_FP64 || precision > TN_FP32_PLAIN) return fail(TN_EINVAL, "bad arguments");
  Plan p;
  std::string why;
  int g = choose_group(d, chi, precision, kLdsLimit, &p, &why);
  if (g < 0) return fail(TN_EUNSUPPORTED, why);
  info[0] = p.h.flops_fwd;
  info[1] = (double)p.h.scratch_elems * real_bytes(precision);
  info[2] = lds_layout(p.h, real_bytes(precision), fac_bytes(precision)).bytes;
  info[3] = p.h.nsite;
  info[4] = p.h.nstep;
  info[5] = g;
  info[6] = wgs_for((int)info[2]);
  {
    std::lock_guard<std::mutex> lk(g_mu);
    auto it = g_tune.find(std::make_tuple(d, chi, precision));
    if (it != g_tune.end() && it->second.wgs > 0) info[6] = std::min<double>(info[6], it->second.wgs);
  }
  return TN_OK;
}

int tn_set_tuning(int32_t d, int32_t chi, int32_t precision, int32_t group, int32_t wg_per_cu) {
  if (d < 3 || d > TN_MAX_D || d % 2 == 0 || chi < 0 || precision < TN_FP64 || precision > TN_FP32_PLAIN ||
      group < 0 || group > 2 || wg_per_cu < 0 || wg_per_cu > kMaxWgPerCU)
    return fail(TN_EINVAL, "bad tuning arguments");
  std::lock_guard<std::mutex> lk(g_mu);
  if (group == 0 && wg_per_cu == 0) g_tune.erase(std::make_tuple(d, chi, precision));
  else g_tune[std::make_tuple(d, chi, precision)] = Tune{group, wg_per_cu};
  return TN_OK;
}

const char* tn_last_error(void) { return g_err.c_str(); }

}  // extern "C"
