// Planar exact coset partition functions under bit-flip noise (paper Sec.
// 3.1.3, exact solutions on planar graphs: the Kac-Ward determinant), and the
// C ABI entry points tn_bitflip_workspace_size / tn_bitflip_decode.
//
// Per (syndrome, coset I or X) a persistent work-group of 256 threads
//   1. checks the inputs and forms the coset's reference error (X strings of
//      the fired Z-type checks, plus the X representative on the last column
//      for coset X), hence the bond weights t_q = eta_q (1 - 2 p_q);
//   2. assembles the dense complex FP64 matrix I - Lambda of the plan
//      (kw_plan.hpp) in its scratch region (row-major, rows padded to 16);
//   3. factorises it by right-looking blocked LU with partial pivoting: panels
//      of 32 columns on the vector units (one thread per row), the row swaps
//      and the unit-lower solve of the panel's rows one thread per column, and
//      the trailing update as a complex GEMM on the FP64 matrix cores
//      (v_mfma_f64_16x16x4_f64, four real products per complex product);
//   4. log Z = (m_X - n) ln 2 + log|det| / 2 (the determinant is the square
//      of a positive sum: its phase must come out zero).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/tnmld.h"
#include "kw_plan.hpp"
#include "plan.hpp"

namespace tnmld {

int report_error(int code, const std::string& msg);
void launch_zero_status(unsigned* st, hipStream_t stream);
void launch_decide(const double* logz, int64_t count, double tie_tol, double* logp, uint8_t* cls,
                   hipStream_t stream);

namespace kw {

constexpr int NT = 256;
constexpr int WAVE = 64;
constexpr int NB = 32;  // panel width (a multiple of 4: the matrix-core k-step)
constexpr unsigned ST_BAD_INPUT = 1u, ST_NUMERIC = 2u, ST_UNRESOLVED = 4u;  // same bits as the boundary-MPS path

typedef double f64x4 __attribute__((ext_vector_type(4)));

struct Job {
  const uint8_t* plan;
  const double* rates;
  const int32_t* model_index;
  const uint8_t* syn;
  double* logz;
  int64_t count;
  int64_t item_begin;  // first item (two per syndrome) of this job
  int32_t n_models;
  int32_t pad;
};

struct Jobs {
  Job j[TN_MAX_SEGMENTS];
  int32_t n;
  int32_t pad;
  int64_t nitems;
  unsigned* status;
};

__device__ inline double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ inline double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

// (value, index) maximum with ties to the lower index, over the work-group;
// every thread gets the result (index -1 when no thread had a candidate).
__device__ inline int block_argmax(double v, int i, double* rv, int* ri, double* best) {
  const int tid = threadIdx.x, lane = tid % WAVE, w = tid / WAVE;
  for (int off = WAVE / 2; off > 0; off >>= 1) {
    const double v2 = __shfl_xor(v, off, WAVE);
    const int i2 = __shfl_xor(i, off, WAVE);
    if (i2 >= 0 && (i < 0 || v2 > v || (v2 == v && i2 < i))) {
      v = v2;
      i = i2;
    }
  }
  if (lane == 0) {
    rv[w] = v;
    ri[w] = i;
  }
  __syncthreads();
  double bv = rv[0];
  int bi = ri[0];
  for (int k = 1; k < NT / WAVE; ++k)
    if (ri[k] >= 0 && (bi < 0 || rv[k] > bv || (rv[k] == bv && ri[k] < bi))) {
      bv = rv[k];
      bi = ri[k];
    }
  *best = bv;
  return bi;
}

// One (syndrome, coset) item.  A: this work-group's scratch, ld x ld complex.
__device__ void kw_item(const Job& job, int64_t b, int coset, double2* A, unsigned* status) {
  const KwHeader* H = reinterpret_cast<const KwHeader*>(job.plan);
  const int d = H->d, n = H->n, m = H->m, N = H->N, ld = H->ld, tid = threadIdx.x;
  const KwEntry* ent = reinterpret_cast<const KwEntry*>(job.plan + H->nz_ofs);
  const int8_t* zc = reinterpret_cast<const int8_t*>(job.plan + H->zcheck_ofs);
  __shared__ double s_t[TN_MAX_D * TN_MAX_D + 1];
  __shared__ uint8_t s_syn[TN_MAX_D * TN_MAX_D];
  __shared__ uint8_t s_f[TN_MAX_D * TN_MAX_D];
  __shared__ double2 s_prow[NB];
  __shared__ double2 s_L[NB][NB];
  __shared__ double2 s_Li[NB][NB];
  __shared__ int s_ipiv[NB];
  __shared__ double s_rv[NT / WAVE];
  __shared__ int s_ri[NT / WAVE];
  __shared__ int s_label;

  // --- 1. input checks, reference error, bond weights ----------------------
  const int raw = job.model_index ? job.model_index[b] : 0;
  const bool mok = raw >= 0 && raw < job.n_models;
  const double* rates = job.rates + (int64_t)(mok ? raw : 0) * n * 3;
  int bad = mok ? 0 : 1, pos = 1, imp = 0;
  for (int j = tid; j < m; j += NT) {
    const uint8_t s = job.syn[b * m + j];
    s_syn[j] = s;
    if (s > 1) bad = 1;
    if (j >= m / 2 && s) imp = 1;  // an X-type check fired: needs a Z error
  }
  for (int q = tid; q < n; q += NT) {
    const double px = rates[3 * q], py = rates[3 * q + 1], pz = rates[3 * q + 2];
    if (!(px >= 0.0 && px <= 1.0) || py != 0.0 || pz != 0.0) bad = 1;
    if (!(px > 0.0 && px < 1.0)) pos = 0;
  }
  bad = __syncthreads_or(bad);
  pos = __syncthreads_and(pos);
  imp = __syncthreads_or(imp);
  if (bad) {
    if (tid < 4) job.logz[b * 4 + tid] = -INFINITY;
    if (tid == 0) atomicOr(status, ST_BAD_INPUT);
    __syncthreads();
    return;
  }
  for (int q = tid; q < n; q += NT) {
    const int r = q / d, c = q % d;
    int x = 0;
    for (int j = 0; j < m / 2; ++j)
      if (s_syn[j] && zc[2 * j] == c && r <= zc[2 * j + 1]) x ^= 1;
    if (coset == 1 && c == d - 1) x ^= 1;
    s_f[q] = (uint8_t)x;
    s_t[q] = (x ? -1.0 : 1.0) * (1.0 - 2.0 * rates[3 * q]);
  }
  if (tid == 0) s_t[n] = 1.0;
  __syncthreads();
  if (tid == 0) {
    int a = 0;  // class of the reference: x-parity on row 0 (I = 0, X = 1)
    for (int c = 0; c < d; ++c) a ^= s_f[c];
    s_label = a;
    if (coset == 0) job.logz[b * 4 + 2] = job.logz[b * 4 + 3] = -INFINITY;  // Y, Z: impossible under bit flips
    if (imp) job.logz[b * 4 + a] = -INFINITY;
  }
  __syncthreads();
  if (imp) return;

  // --- 2. I - Lambda ---------------------------------------------------------
  const int64_t tot = (int64_t)ld * ld;
  for (int64_t e = tid; e < tot; e += NT) A[e] = make_double2(0.0, 0.0);
  __syncthreads();
  for (int i = tid; i < N; i += NT) A[(int64_t)i * ld + i] = make_double2(1.0, 0.0);
  for (int z = tid; z < H->nnz; z += NT) {
    const KwEntry en = ent[z];
    const double t = s_t[en.edge];
    A[(int64_t)en.row * ld + en.col] = make_double2(-t * en.re, -t * en.im);
  }
  __syncthreads();

  // --- 3. blocked LU with partial pivoting -----------------------------------
  double logdet = 0.0, arg = 0.0;  // thread 0
  int swaps = 0, singular = 0;
  double bv = -1.0;
  int bi = -1;
  for (int i = tid; i < N; i += NT) {
    const double v = cabs2(A[(int64_t)i * ld]);
    if (v > bv) {
      bv = v;
      bi = i;
    }
  }
  for (int k0 = 0; k0 < N && !singular; k0 += NB) {
    const int k1 = min(k0 + NB, N), kb = k1 - k0;
    for (int j = k0; j < k1; ++j) {
      double pbest = 0.0;
      const int piv = block_argmax(bv, bi, s_rv, s_ri, &pbest);
      if (piv < 0 || !(pbest > 0.0)) {  // a zero or NaN column: the same decision in every thread
        singular = 1;
        break;
      }
      if (tid < kb) {
        const int c = k0 + tid;
        const double2 x = A[(int64_t)j * ld + c], y = A[(int64_t)piv * ld + c];
        if (piv != j) {
          A[(int64_t)j * ld + c] = y;
          A[(int64_t)piv * ld + c] = x;
        }
        s_prow[tid] = piv != j ? y : x;
      }
      if (tid == 0) s_ipiv[j - k0] = piv;
      __syncthreads();
      const double2 p = s_prow[j - k0];
      const double p2 = cabs2(p);
      if (!(p2 > 0.0)) {
        singular = 1;
        break;
      }
      if (tid == 0) {
        logdet += 0.5 * log(p2);
        arg += atan2(p.y, p.x);
        swaps += piv != j;
      }
      const double2 inv = make_double2(p.x / p2, -p.y / p2);
      bv = -1.0;
      bi = -1;
      for (int i = j + 1 + tid; i < N; i += NT) {
        double2* row = A + (int64_t)i * ld;
        const double2 l = cmul(row[j], inv);
        row[j] = l;
        for (int c = j + 1; c < k1; ++c) {
          const double2 u = s_prow[c - k0];
          const double2 a = row[c];
          row[c] = make_double2(a.x - (l.x * u.x - l.y * u.y), a.y - (l.x * u.y + l.y * u.x));
        }
        if (j + 1 < k1) {
          const double v = cabs2(row[j + 1]);
          if (v > bv) {
            bv = v;
            bi = i;
          }
        }
      }
      __syncthreads();
    }
    if (singular || k1 >= N) break;
    // rows k0..k1-1 of the trailing columns: the panel's row swaps (thread per
    // column, in pivot order), then U12 = L11^-1 A12 with the inverse of the
    // unit-lower L11 formed in LDS and applied on the matrix cores
    for (int c = k1 + tid; c < N; c += NT)
      for (int jj = 0; jj < kb; ++jj) {
        const int r = k0 + jj, pr = s_ipiv[jj];
        if (pr != r) {
          const double2 x = A[(int64_t)r * ld + c];
          A[(int64_t)r * ld + c] = A[(int64_t)pr * ld + c];
          A[(int64_t)pr * ld + c] = x;
        }
      }
    for (int e = tid; e < NB * NB; e += NT) {
      const int r = e / NB, c = e % NB;
      s_L[r][c] = (r < kb && c < kb) ? A[(int64_t)(k0 + r) * ld + k0 + c] : make_double2(0.0, 0.0);
      s_Li[r][c] = make_double2(r == c && r < kb ? 1.0 : 0.0, 0.0);
    }
    __syncthreads();
    if (tid < kb) {  // column j of L11^-1 by forward substitution, in LDS
      const int j = tid;
      for (int i = j + 1; i < kb; ++i) {
        double2 acc = s_L[i][j];
        for (int mm = j + 1; mm < i; ++mm) {
          const double2 l = s_L[i][mm], x = s_Li[mm][j];
          acc = make_double2(acc.x + (l.x * x.x - l.y * x.y), acc.y + (l.x * x.y + l.y * x.x));
        }
        s_Li[i][j] = make_double2(-acc.x, -acc.y);
      }
    }
    __syncthreads();
    const int lane = tid % WAVE, wv = tid / WAVE;
    const int nks = kb >> 2;  // k-steps of 4 (kb is a multiple of 4: N = 2(d^2 + 1) and NB are)
    {
      // one wave per block of 16 columns: its kb rows are read into registers
      // before either 16-row half of the product is written back in place
      const int nct = (ld - k1) / 16;
      for (int cb = wv; cb < nct; cb += NT / WAVE) {
        const int c0 = k1 + 16 * cb;
        double2 bq[NB / 4];
#pragma unroll
        for (int s2 = 0; s2 < NB / 4; ++s2)
          if (s2 < nks) bq[s2] = A[(int64_t)(k0 + 4 * s2 + lane / 16) * ld + c0 + lane % 16];
#pragma unroll
        for (int h = 0; h < NB / 16; ++h) {
          if (16 * h >= kb) break;
          f64x4 cr = {0.0, 0.0, 0.0, 0.0}, ci = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
          for (int s2 = 0; s2 < NB / 4; ++s2)
            if (s2 < nks) {
              const double2 a = s_Li[16 * h + lane % 16][4 * s2 + lane / 16], bb = bq[s2];
              cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, bb.x, cr, 0, 0, 0);
              cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, bb.y, cr, 0, 0, 0);
              ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, bb.y, ci, 0, 0, 0);
              ci = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, bb.x, ci, 0, 0, 0);
            }
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const int r = 16 * h + lane / 16 + 4 * v;
            if (r < kb) A[(int64_t)(k0 + r) * ld + c0 + lane % 16] = make_double2(cr[v], ci[v]);
          }
        }
      }
    }
    __syncthreads();
    // trailing update A[k1:, k1:] -= A[k1:, k0:k1] A[k0:k1, k1:] on the matrix cores:
    // 16 x 16 complex tiles; v_mfma_f64_16x16x4_f64 takes A[l % 16][l / 16] and
    // B[l / 16][l % 16] from lane l and leaves D[l / 16 + 4 v][l % 16] in its v-th value
    const int nt = (ld - k1) / 16;
    bv = -1.0;
    bi = -1;
    for (int t = wv; t < nt * nt; t += NT / WAVE) {
      const int i0 = k1 + 16 * (t / nt), c0 = k1 + 16 * (t % nt);
      // every operand of the tile is loaded before the matrix-core chain, so
      // the loads overlap instead of waiting one k-step at a time
      double2 av[NB / 4], bv2[NB / 4];
#pragma unroll
      for (int s = 0; s < NB / 4; ++s)
        if (s < nks) {
          const int ks = k0 + 4 * s;
          av[s] = A[(int64_t)(i0 + lane % 16) * ld + ks + lane / 16];
          bv2[s] = A[(int64_t)(ks + lane / 16) * ld + c0 + lane % 16];
        }
      f64x4 cr, ci;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double2 x = A[(int64_t)(i0 + lane / 16 + 4 * v) * ld + c0 + lane % 16];
        cr[v] = x.x;
        ci[v] = x.y;
      }
#pragma unroll
      for (int s = 0; s < NB / 4; ++s)
        if (s < nks) {
          const double2 a = av[s], bb = bv2[s];
          cr = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.x, bb.x, cr, 0, 0, 0);
          cr = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, bb.y, cr, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.x, bb.y, ci, 0, 0, 0);
          ci = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, bb.x, ci, 0, 0, 0);
        }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = i0 + lane / 16 + 4 * v;
        A[(int64_t)r * ld + c0 + lane % 16] = make_double2(cr[v], ci[v]);
        if (c0 == k1 && lane % 16 == 0 && r < N) {  // pivot candidates of the next panel's first column
          const double vv = cr[v] * cr[v] + ci[v] * ci[v];
          if (vv > bv) {
            bv = vv;
            bi = r;
          }
        }
      }
    }
    __syncthreads();
  }

  // --- 4. log Z ----------------------------------------------------------------
  if (tid == 0) {
    double lz = -INFINITY;
    if (!singular) {
      // det = |det| e^{i (arg + pi swaps)} must be real and positive
      const double ph = arg + M_PI * (double)(swaps & 1);
      if (cos(ph) > 0.5) lz = H->log_pref + 0.5 * logdet;
    }
    if (!(lz > -INFINITY && lz < INFINITY)) {
      // under a strictly positive model Z > 0: a precision loss (kw_finish
      // tells one lost coset from a lost syndrome)
      lz = -INFINITY;
      if (pos) {
        atomicOr(status, ST_UNRESOLVED);
        atomicAdd(reinterpret_cast<unsigned long long*>(status + 2), 1ull);
      }
    }
    job.logz[b * 4 + s_label] = lz;
  }
  __syncthreads();
}

__global__ __launch_bounds__(NT) void kw_kernel(Jobs jb, unsigned long long* counter, char* scratch, int64_t stride) {
  __shared__ long long s_item;
  double2* A = reinterpret_cast<double2*>(scratch + (int64_t)blockIdx.x * stride);
  for (;;) {
    if (threadIdx.x == 0) s_item = (long long)atomicAdd(counter, 1ull);
    __syncthreads();
    const int64_t item = s_item;
    __syncthreads();
    if (item >= jb.nitems) break;
    int k = 0;
    while (k + 1 < jb.n && jb.j[k + 1].item_begin <= item) ++k;
    const int64_t local = item - jb.j[k].item_begin;
    kw_item(jb.j[k], local >> 1, (int)(local & 1), A, jb.status);
  }
}

// After the items: a syndrome that needs no Z error, under a strictly
// positive model, whose cosets I and X both came out -inf lost log P(s):
// ST_NUMERIC.  One thread per syndrome.
__global__ void kw_finish(Job job, unsigned* status) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= job.count) return;
  if (job.logz[b * 4] > -INFINITY || job.logz[b * 4 + 1] > -INFINITY) return;
  const KwHeader* H = reinterpret_cast<const KwHeader*>(job.plan);
  const int n = H->n, m = H->m;
  for (int j = m / 2; j < m; ++j)
    if (job.syn[b * m + j]) return;  // impossible syndrome: -inf is exact
  const int raw = job.model_index ? job.model_index[b] : 0;
  if (raw < 0 || raw >= job.n_models) return;  // reported as bad input
  const double* r = job.rates + (int64_t)raw * n * 3;
  for (int q = 0; q < n; ++q)
    if (!(r[3 * q] > 0.0 && r[3 * q] < 1.0) || r[3 * q + 1] != 0.0 || r[3 * q + 2] != 0.0) return;
  atomicOr(status, ST_NUMERIC);
}

__global__ void kw_zero_counter(unsigned long long* c) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *c = 0ull;
}

// ------------------------------------------------------------------ host side
namespace {

int kfail(int code, const std::string& msg) { return report_error(code, msg); }

struct KwDev {
  KwPlan plan;
  uint8_t* dev = nullptr;
};
std::mutex g_kw_mu;
std::map<std::pair<int, int>, KwDev*> g_kw_plans;  // (device, d)

int kw_plan_for(int d, bool upload, KwDev** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return kfail(TN_EDEVICE, "no HIP device");
  std::lock_guard<std::mutex> lk(g_kw_mu);
  auto key = std::make_pair(dev, d);
  auto it = g_kw_plans.find(key);
  KwDev* kd = nullptr;
  if (it == g_kw_plans.end()) {
    kd = new KwDev;
    std::string e = build_kw_plan(d, &kd->plan);
    if (!e.empty()) {
      delete kd;
      return kfail(TN_EINVAL, e);
    }
    g_kw_plans[key] = kd;
  } else {
    kd = it->second;
  }
  if (upload && !kd->dev) {
    uint8_t* p = nullptr;
    if (hipMalloc(&p, kd->plan.blob.size()) != hipSuccess) return kfail(TN_ENOMEM, "hipMalloc of plan failed");
    if (hipMemcpy(p, kd->plan.blob.data(), kd->plan.blob.size(), hipMemcpyHostToDevice) != hipSuccess) {
      (void)hipFree(p);
      return kfail(TN_EDEVICE, "plan upload failed");
    }
    kd->dev = p;
  }
  *out = kd;
  return TN_OK;
}

int kw_validate(const tn_segment* segs, int32_t nseg) {
  if (!segs || nseg < 1 || nseg > TN_MAX_SEGMENTS) return kfail(TN_EINVAL, "nseg must be in [1, 16]");
  for (int i = 0; i < nseg; ++i) {
    const tn_segment& s = segs[i];
    if (s.d < 3 || s.d > TN_MAX_D || s.d % 2 == 0) return kfail(TN_EINVAL, "d must be odd in [3, 31]");
    if (s.precision != TN_FP64) return kfail(TN_EINVAL, "the planar exact solver computes in FP64 (precision = TN_FP64)");
    if (s.n_models < 1) return kfail(TN_EINVAL, "n_models must be >= 1");
    if (s.count < 0) return kfail(TN_EINVAL, "count must be >= 0");
    if (s.count > 0 && (!s.rates || !s.syndromes || !s.out_logz)) return kfail(TN_EINVAL, "null pointer");
    if (s.rounds > 1) return kfail(TN_EINVAL, "the planar exact solver takes one syndrome round");
  }
  return TN_OK;
}

// persistent work-groups: as many as fit a CU (at most 4), on every CU
int kw_workgroups(int* cus_out) {
  static int cached = 0, cached_cus = 0;
  if (!cached) {
    int dev = 0, cus = 0, nb = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, reinterpret_cast<const void*>(kw_kernel), NT, 0) !=
            hipSuccess ||
        nb < 1)
      nb = 1;
    cached = std::min(nb, 4) * cus;
    cached_cus = cus;
  }
  *cus_out = cached_cus;
  return cached;
}

// Launch layout: items (two per syndrome) of every segment, the largest d first.
int kw_plan_call(const tn_segment* segs, int32_t nseg, Jobs* jb, int64_t* stride, int* nwg, size_t* bytes) {
  int rc = kw_validate(segs, nseg);
  if (rc) return rc;
  std::vector<int> order(nseg);
  for (int i = 0; i < nseg; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return segs[a].d > segs[b].d; });
  *jb = Jobs{};
  int64_t items = 0, ldmax = 16;
  for (int oi : order) {
    const tn_segment& s = segs[oi];
    if (s.count == 0) continue;
    KwDev* kd = nullptr;
    if ((rc = kw_plan_for(s.d, true, &kd))) return rc;
    Job& j = jb->j[jb->n++];
    j.plan = kd->dev;
    j.rates = s.rates;
    j.model_index = s.model_index;
    j.syn = s.syndromes;
    j.logz = s.out_logz;
    j.count = s.count;
    j.item_begin = items;
    j.n_models = s.n_models;
    items += 2 * s.count;
    ldmax = std::max<int64_t>(ldmax, kd->plan.h.ld);
  }
  jb->nitems = items;
  *stride = (ldmax * ldmax * (int64_t)sizeof(double2) + 255) / 256 * 256;
  int cus = 0;
  *nwg = kw_workgroups(&cus);
  if (*nwg < 1) return kfail(TN_EDEVICE, "device query failed");
  if (*stride > (int64_t)(16 << 20)) *nwg = std::min(*nwg, cus);  // large d: one matrix per CU
  *bytes = kWorkspaceAlign + (size_t)(*nwg) * (size_t)(*stride);
  return TN_OK;
}

}  // namespace
}  // namespace kw
}  // namespace tnmld

using namespace tnmld;
using namespace tnmld::kw;

extern "C" {

size_t tn_bitflip_workspace_size(const tn_segment* segs, int32_t nseg) {
  Jobs jb;
  int64_t stride = 0;
  int nwg = 0;
  size_t bytes = 0;
  if (kw_plan_call(segs, nseg, &jb, &stride, &nwg, &bytes)) return 0;
  return bytes;
}

int tn_bitflip_decode(const tn_segment* segs, int32_t nseg, double tie_tol, void* workspace, size_t ws_bytes,
                      void* stream) {
  if (!(tie_tol > 0.0)) tie_tol = 1e-9;
  Jobs jb;
  int64_t stride = 0;
  int nwg = 0;
  size_t bytes = 0;
  int rc = kw_plan_call(segs, nseg, &jb, &stride, &nwg, &bytes);
  if (rc) return rc;
  if (jb.nitems == 0) return TN_OK;
  if (!workspace || ws_bytes < bytes) return kfail(TN_EINVAL, "workspace too small: need " + std::to_string(bytes));
  hipStream_t st = reinterpret_cast<hipStream_t>(stream);
  char* base = reinterpret_cast<char*>(workspace);
  unsigned long long* counter = reinterpret_cast<unsigned long long*>(base);
  jb.status = reinterpret_cast<unsigned*>(base + kStatusOffset);
  launch_zero_status(jb.status, st);
  kw_zero_counter<<<1, 64, 0, st>>>(counter);
  hipLaunchKernelGGL(kw_kernel, dim3(nwg), dim3(NT), 0, st, jb, counter, base + kWorkspaceAlign, stride);
  for (int i = 0; i < jb.n; ++i)
    kw_finish<<<(unsigned)((jb.j[i].count + 255) / 256), 256, 0, st>>>(jb.j[i], jb.status);
  if (hipGetLastError() != hipSuccess) return kfail(TN_EDEVICE, "kernel launch failed");
  for (int i = 0; i < nseg; ++i)
    launch_decide(segs[i].out_logz, segs[i].count, tie_tol, segs[i].out_logp, segs[i].out_class, st);
  if (hipGetLastError() != hipSuccess) return kfail(TN_EDEVICE, "decide launch failed");
  return TN_OK;
}

int tn_bitflip_plan_info(int32_t d, double* info) {
  if (!info) return kfail(TN_EINVAL, "null info");
  KwPlan p;
  std::string e = build_kw_plan(d, &p);
  if (!e.empty()) return kfail(TN_EINVAL, e);
  const double N = p.h.N;
  info[0] = N;                                   // directed edges: the matrix order
  info[1] = p.h.nnz;                             // entries of Lambda
  info[2] = 8.0 / 3.0 * N * N * N;               // real flops of one complex LU (leading term)
  info[3] = (double)p.h.ld * p.h.ld * 16.0;      // scratch bytes per work-group
  info[4] = p.h.log_pref;                        // (m_X - n) ln 2
  return TN_OK;
}

}  // extern "C"
