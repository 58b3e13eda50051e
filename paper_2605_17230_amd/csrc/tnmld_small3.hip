// The forward kernel built for three 256-thread work-groups per CU, for plans
// whose site matrices have at most 128 columns (d <= 9 at chi = 16, and the
// like).  Two groups per CU leave the factorisations' barrier and reduction
// latency partly exposed; a third one needs the registers of three waves per
// SIMD (168 per lane), which this build gets by leaving out the 16-column
// register code (the plans it takes never run it).  Same device code as the
// other builds, compiled here in its own namespace; the host side of
// tnmld.hip launches it through the two functions at the end.
#include <hip/hip_runtime.h>

#include <map>
#include <mutex>

#define TNMLD_NT 256
#define TNMLD_MAX_NPL 8
#define tnmld tnmld_small3
#include "contract.hpp"

#ifndef BF16_GEMM_MODE
#define BF16_GEMM_MODE GEMM_BF16X3
#endif

namespace tnmld_small3 {

template <typename Real, typename Fac, int GM>
__global__ __launch_bounds__(NT, 3) void fwd_kernel_small3(JobTable jt, unsigned long long* counter, char* scratch,
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

__global__ void zero_one3(unsigned long long* c) {
  if (threadIdx.x == 0) *c = 0ull;
}

namespace {
const void* kernel_of(int precision) {
  if (precision == TN_FP64) return reinterpret_cast<const void*>(fwd_kernel_small3<double, double, GEMM_F64>);
  if (precision == TN_FP32) return reinterpret_cast<const void*>(fwd_kernel_small3<float, double, GEMM_F32>);
  if (precision == TN_BF16) return reinterpret_cast<const void*>(fwd_kernel_small3<float, float, BF16_GEMM_MODE>);
  if (precision == TN_BF16_F64) return reinterpret_cast<const void*>(fwd_kernel_small3<float, double, GEMM_BF16>);
  return reinterpret_cast<const void*>(fwd_kernel_small3<float, float, GEMM_F32>);
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

// Work-groups of this build that one CU holds with lds_bytes of LDS (0 if the
// runtime cannot say).
int wgs_per_cu(int precision, int lds_bytes) {
  static std::map<std::pair<int, int>, int> cache;
  static std::mutex mu;
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = cache.find(std::make_pair(precision, lds_bytes));
    if (it != cache.end()) return it->second;
  }
  const void* kern = kernel_of(precision);
  int nb = 0;
  if (raise_lds(kern, lds_bytes) != 0 ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, NT, (size_t)lds_bytes) != hipSuccess)
    nb = 0;
  std::lock_guard<std::mutex> lk(mu);
  cache[std::make_pair(precision, lds_bytes)] = nb;
  return nb;
}

// Enqueue the counter reset and the persistent kernel.  jt and lay are the
// caller's JobTable and LdsLayout (same definitions, other namespace).
int launch_fwd(int precision, const void* jt, unsigned long long* counter, char* scratch, int64_t stride,
               int64_t snap_ofs, const void* lay, int lds_bytes, int nwg, hipStream_t st) {
  const void* kern = kernel_of(precision);
  if (raise_lds(kern, lds_bytes) != 0) return -1;
  zero_one3<<<1, 64, 0, st>>>(counter);
  JobTable t = *reinterpret_cast<const JobTable*>(jt);
  LdsLayout l = *reinterpret_cast<const LdsLayout*>(lay);
  void* args[] = {&t, &counter, &scratch, &stride, &snap_ofs, &l};
  if (hipLaunchKernel(kern, dim3(nwg), dim3(NT), args, (size_t)lds_bytes, st) != hipSuccess) return -1;
  return hipGetLastError() == hipSuccess ? 0 : -1;
}

}  // namespace tnmld_small3
