// The forward and backward kernels built for 256-thread work-groups, for plans
// whose LQ rows fit this size's register rows (at most 64 rows with FP32
// factorisations, 32 with FP64 ones; at most 256 columns): such items leave
// much of a 512-thread group idle, and with 256 threads two work-groups share
// a CU and hide each other's barrier and reduction latency.  Plans of at most
// 128 columns run three groups per CU instead (tnmld_small3.hip).  Same device
// code as the 512-thread build, compiled here in its own namespace; the host
// side of tnmld.hip launches it through the functions at the end.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <tuple>

#define TNMLD_NT 256
#define tnmld tnmld_small
#include "adjoint.hpp"

#ifndef BF16_GEMM_MODE
#define BF16_GEMM_MODE GEMM_BF16X3
#endif

namespace tnmld_small {

// Two waves per SIMD (two groups per CU) is what this build is for; the
// 16-column register code sits at the edge of that budget, so it is stated.
template <typename Real, typename Fac, int GM, bool XG = false>
__global__ __launch_bounds__(NT, 2) void fwd_kernel_small(JobTable jt, unsigned long long* counter, char* scratch,
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
    contract_syndrome<Real, Fac, GM, XG>(job, item - job.item_begin, smem, lay, scr, snap);
    __syncthreads();
  }
}

// Backward on 256-thread work-groups (see bwd_kernel in tnmld.hip).
template <typename Real, typename Fac, int GM>
__global__ __launch_bounds__(NT) void bwd_kernel_small(JobTable jt, char* scratch, int64_t scratch_stride,
                                                        LdsLayout lay, int flags, double* partials,
                                                        int64_t part_stride) {
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

__global__ void zero_one(unsigned long long* c) {
  if (threadIdx.x == 0) *c = 0ull;
}

namespace {
// xg: the variant whose LQ matrix lives in global scratch (built for the forms
// with FP32 factorisations, the only ones whose plans need it)
const void* kernel_of(int precision, bool xg = false) {
  if (xg) {
    if (precision == TN_BF16)
      return reinterpret_cast<const void*>(fwd_kernel_small<float, float, BF16_GEMM_MODE, true>);
    if (precision == TN_FP32_PLAIN) return reinterpret_cast<const void*>(fwd_kernel_small<float, float, GEMM_F32, true>);
    return nullptr;
  }
  if (precision == TN_FP64) return reinterpret_cast<const void*>(fwd_kernel_small<double, double, GEMM_F64>);
  if (precision == TN_FP32) return reinterpret_cast<const void*>(fwd_kernel_small<float, double, GEMM_F32>);
  if (precision == TN_BF16) return reinterpret_cast<const void*>(fwd_kernel_small<float, float, BF16_GEMM_MODE>);
  if (precision == TN_BF16_F64) return reinterpret_cast<const void*>(fwd_kernel_small<float, double, GEMM_BF16>);
  return reinterpret_cast<const void*>(fwd_kernel_small<float, float, GEMM_F32>);
}

const void* bwd_kernel_of(int precision) {
  if (precision == TN_BF16_F64) return nullptr;  // forward only
  if (precision == TN_FP64) return reinterpret_cast<const void*>(bwd_kernel_small<double, double, GEMM_VALU>);
  if (precision == TN_FP32) return reinterpret_cast<const void*>(bwd_kernel_small<float, double, GEMM_F32>);
  if (precision == TN_BF16) return reinterpret_cast<const void*>(bwd_kernel_small<float, float, BF16_GEMM_MODE>);
  return reinterpret_cast<const void*>(bwd_kernel_small<float, float, GEMM_F32>);
}

int raise_lds(const void* kern, int bytes) {
  static std::map<const void*, int> done;
  static std::mutex mu;
  std::lock_guard<std::mutex> lk(mu);
  int& cur = done[kern];
  if (cur >= bytes) return 0;
  if (hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize, bytes) != hipSuccess) return -1;
  cur = bytes;
  return 0;
}
}  // namespace

// Work-groups of the small kernel that one CU holds with lds_bytes of LDS
// (0 if the runtime cannot say).
int small_wgs_per_cu(int precision, int lds_bytes, bool xg) {
  static std::map<std::tuple<int, int, bool>, int> cache;
  static std::mutex mu;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(std::make_tuple(precision, lds_bytes, xg));
    if (it != cache.end()) return it->second;
  }
  const void* kern = kernel_of(precision, xg);
  int nb = 0;
  if (!kern || raise_lds(kern, lds_bytes) != 0 ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, NT, (size_t)lds_bytes) != hipSuccess)
    nb = 0;
  std::lock_guard<std::mutex> lk(mu);
  cache[std::make_tuple(precision, lds_bytes, xg)] = nb;
  return nb;
}

// Enqueue the counter reset and the persistent small kernel.  jt and lay are
// the caller's JobTable and LdsLayout (same definitions, other namespace).
int launch_fwd_small(int precision, const void* jt, unsigned long long* counter, char* scratch, int64_t stride,
                     int64_t snap_ofs, const void* lay, int lds_bytes, int nwg, hipStream_t st) {
  LdsLayout l = *reinterpret_cast<const LdsLayout*>(lay);
  const void* kern = kernel_of(precision, l.X < 0);
  if (!kern || raise_lds(kern, lds_bytes) != 0) return -1;
  zero_one<<<1, 64, 0, st>>>(counter);
  JobTable t = *reinterpret_cast<const JobTable*>(jt);
  void* args[] = {&t, &counter, &scratch, &stride, &snap_ofs, &l};
  if (hipLaunchKernel(kern, dim3(nwg), dim3(NT), args, (size_t)lds_bytes, st) != hipSuccess) return -1;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

// Work-groups of the small backward kernel that one CU holds (0 if unknown).
int small_bwd_wgs_per_cu(int precision, int lds_bytes) {
  const void* kern = bwd_kernel_of(precision);
  int nb = 0;
  if (!kern || raise_lds(kern, lds_bytes) != 0 ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, NT, (size_t)lds_bytes) != hipSuccess)
    nb = 0;
  return nb;
}

// Enqueue the small backward kernel (jt, lay: the caller's JobTable / LdsLayout).
int launch_bwd_small(int precision, const void* jt, char* scratch, int64_t stride, const void* lay, int lds_bytes,
                     int flags, double* partials, int64_t pstride, int nwg, hipStream_t st) {
  const void* kern = bwd_kernel_of(precision);
  if (!kern || raise_lds(kern, lds_bytes) != 0) return -1;
  JobTable t = *reinterpret_cast<const JobTable*>(jt);
  LdsLayout l = *reinterpret_cast<const LdsLayout*>(lay);
  void* args[] = {&t, &scratch, &stride, &l, &flags, &partials, &pstride};
  if (hipLaunchKernel(kern, dim3(nwg), dim3(NT), args, (size_t)lds_bytes, st) != hipSuccess) return -1;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace tnmld_small
