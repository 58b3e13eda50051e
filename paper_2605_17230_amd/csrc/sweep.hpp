// Device building blocks of the boundary-MPS sweep (gfx950, wave64).
//
// One work-group of NT = 512 threads contracts one (syndrome, coset) pair at a
// time.  Every dense matrix of a site step lives in LDS; the MPS itself lives
// in a per-work-group scratch region of HBM (it does not fit in LDS at
// chi = 32: 33 sites x 8-64 KB).  Routines here are work-group collective:
// every thread of the block must call them with identical arguments.
#pragma once
#ifndef TNMLD_EMU
#include <hip/hip_runtime.h>
#endif
#include <stdint.h>

#include <type_traits>

#include "plan.hpp"

namespace tnmld {

// Threads per work-group (512; a second build of the forward kernel uses 256).
#ifndef TNMLD_NT
#define TNMLD_NT 512
#endif
constexpr int NT = TNMLD_NT;
constexpr int WAVE = 64;

// Element types in a named address space, for the arguments of out-of-line
// device functions (a generic pointer would turn every LDS access into a flat
// one): LDS and global memory.
#ifndef TNMLD_EMU
template <typename T>
using lds_t = __attribute__((address_space(3))) T;
template <typename T>
using glb_t = __attribute__((address_space(1))) T;
#else
template <typename T>
using lds_t = T;
template <typename T>
using glb_t = T;
#endif

// A generic pointer known to address LDS: the assumption lets the compiler use
// DS instructions for it where it cannot trace the pointer back to LDS itself
// (in out-of-line functions).  in_global: the same statement for global
// memory, for the reader (no assumption is available).
template <typename T>
__device__ inline T* in_lds(T* p) {
#if defined(__HIP_DEVICE_COMPILE__)
  __builtin_assume(__builtin_amdgcn_is_shared((const void*)p));
#endif
  return p;
}
template <typename T>
__device__ inline T* in_global(T* p) {
  return p;
}

template <typename Real>
struct Eps;
template <>
struct Eps<double> {
  static constexpr double v = 2.220446049250313e-16;
};
template <>
struct Eps<float> {
  static constexpr float v = 1.1920929e-07f;
};
// relative cosine between columns below which the SVD of a bond that is
// being truncated is converged: the kept subspace is then exact to that
// angle and the kept weight to its square
template <typename Fac>
struct SplitTol;
template <>
struct SplitTol<double> {
  static constexpr double v = 1e-10;
};
template <>
struct SplitTol<float> {
  static constexpr double v = 1e-5;
};
// norms below this are treated as exact zeros (1/norm must stay finite in Real)
template <typename Real>
struct TinyNorm;
template <>
struct TinyNorm<double> {
  static constexpr double v = 1e-290;
};
template <>
struct TinyNorm<float> {
  static constexpr double v = 1e-30;
};

#ifndef TNMLD_EMU
// Lane moves inside a row of 16 lanes by DPP (a VALU operand modifier: no LDS
// traffic).  Controls: 0xB1 quad_perm [1,0,3,2], 0x4E quad_perm [2,3,0,1],
// 0x141 row_half_mirror (lane i <- 7-i in each half-row), 0x140 row_mirror
// (lane i <- 15-i).  Every lane of the row must be active.
// The FP32 move names 0 (the sum's identity) as the value of a lane with no
// source, so that the compiler folds it into the add that consumes it
// (v_add_f32_dpp): one instruction per reduction step instead of two.
template <int CTRL>
__device__ inline float dpp_move(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
template <int CTRL>
__device__ inline double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffLL), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
// Value of v on lane src of the wave (src uniform), to every lane.
__device__ inline float lane_read(float v, int src) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ inline double lane_read(double v, int src) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffLL), src);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), src);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}
#endif

// Square root and reciprocal of a normal, finite FP64 value, for the
// reflector scalars of FP32 rows (rounded to FP32 afterwards): the hardware
// estimates refined by Newton steps (two for the reciprocal; for the root a
// coupled root/half-inverse-root step and two residual corrections), about
// an ulp of FP64, without the range scaling and special-value handling of
// the IEEE forms.  The argument of sqrt_normal may be 0: the result is then
// NaN, which the caller's tests treat as no reflection.
__device__ inline double sqrt_normal(double s) {
#ifdef TNMLD_EMU
  return sqrt(s);
#else
  const double y = __builtin_amdgcn_rsq(s);
  double g = s * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  g = fma(fma(-g, g, s), h, g);
  return fma(fma(-g, g, s), h, g);
#endif
}
__device__ inline double recip_normal(double p) {
#ifdef TNMLD_EMU
  return 1.0 / p;
#else
  double r = __builtin_amdgcn_rcp(p);
  r = fma(r, fma(-p, r, 1.0), r);
  return fma(r, fma(-p, r, 1.0), r);
#endif
}

// Sum over aligned groups of G consecutive lanes (G a power of two <= 64),
// returned to every lane of the group.  Partners add in commutative pairs, so
// every lane of a group holds the bitwise-identical sum.  G <= 16 stays inside
// a DPP row: groups may then diverge from each other; G >= 32 needs the whole
// wave active.
template <typename Real>
__device__ inline Real group_sum(Real v, int G) {
#ifdef TNMLD_EMU
  for (int off = G >> 1; off > 0; off >>= 1) v += emu_shfl_xor(v, off, G);
#else
  if (G >= 2) v += dpp_move<0xB1>(v);
  if (G >= 4) v += dpp_move<0x4E>(v);
  if (G >= 8) v += dpp_move<0x141>(v);
  if (G >= 16) v += dpp_move<0x140>(v);
  if (G >= 32) v += __shfl_xor(v, 16, WAVE);
  if (G >= 64) v += __shfl_xor(v, 32, WAVE);
#endif
  return v;
}

// block-wide sum, result returned to every thread; red holds >= NT/WAVE reals
template <typename Real>
__device__ inline Real block_sum(Real v, Real* red) {
  v = group_sum(v, WAVE);
  const int w = threadIdx.x / WAVE;
  __syncthreads();
  if ((threadIdx.x & (WAVE - 1)) == 0) red[w] = v;
  __syncthreads();
  Real s = 0;
  for (int i = 0; i < NT / WAVE; ++i) s += red[i];
  return s;
}

// Visit every (i, j) of an R x C index space; element i*C + j goes to thread
// (i*C + j) mod NT, as in a flat loop, but without a division per element.
template <typename F>
__device__ inline void for_2d(int R, int C, F f) {
  if (R <= 0 || C <= 0) return;
  const int di = NT / C, dj = NT - di * C;
  int i = (int)threadIdx.x / C, j = (int)threadIdx.x - i * C;
  while (i < R) {
    f(i, j);
    i += di;
    j += dj;
    if (j >= C) {
      j -= C;
      ++i;
    }
  }
}

// C = A (MxK, row-major lda) * B (KxN, row-major ldb); store(i, j, value).
// 4x4 register tiles; threads sweep tiles row-major.
template <typename Real, typename Store>
__device__ inline void gemm_lds(int M, int N, int K, const Real* A, int lda, const Real* B, int ldb, Store store) {
  const int tm = (M + 3) >> 2, tn = (N + 3) >> 2;
  for (int t = threadIdx.x; t < tm * tn; t += NT) {
    const int i0 = (t / tn) << 2, j0 = (t % tn) << 2;
    Real acc[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b) acc[a][b] = 0;
    const bool fullm = i0 + 4 <= M, fulln = j0 + 4 <= N;
    for (int k = 0; k < K; ++k) {
      Real av[4], bv[4];
#pragma unroll
      for (int a = 0; a < 4; ++a) av[a] = (fullm || i0 + a < M) ? A[(i0 + a) * lda + k] : Real(0);
#pragma unroll
      for (int b = 0; b < 4; ++b) bv[b] = (fulln || j0 + b < N) ? B[k * ldb + j0 + b] : Real(0);
#pragma unroll
      for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) acc[a][b] += av[a] * bv[b];
    }
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
      for (int b = 0; b < 4; ++b)
        if (i0 + a < M && j0 + b < N) store(i0 + a, j0 + b, acc[a][b]);
  }
}

// GEMM on the matrix cores: C (MxN) = A (MxK) B (KxN) with A, B read through
// aload(i, k) / bload(k, j) as floats, rounded to bf16, accumulated in FP32 by
// v_mfma_f32_16x16x32_bf16 (one 16x16 output tile per wave at a time).  With
// SPLIT each operand is split into bf16 hi + lo parts and the three leading
// products hi*hi + hi*lo + lo*hi are accumulated (about 16 mantissa bits).
// Lane layout of the instruction: A lane l holds row l%16, k = 8(l/16)+i;
// B lane l holds column l%16, k = 8(l/16)+i; D lane l value i is row
// 4(l/16)+i, column l%16.
#ifndef TNMLD_EMU
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));

template <bool SPLIT, typename ALoad, typename BLoad, typename Store>
__device__ inline void gemm_mfma_bf16(int M, int N, int K, ALoad aload, BLoad bload, Store store) {
  const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int tm = (M + 15) >> 4, tn = (N + 15) >> 4;
  const int lr = lane & 15, lk = (lane >> 4) * 8;
  for (int t = wave; t < tm * tn; t += NT / WAVE) {
    const int i0 = (t / tn) << 4, j0 = (t % tn) << 4;
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    const int r = i0 + lr, c = j0 + lr;
    for (int k0 = 0; k0 < K; k0 += 32) {
      bf16x8_t ah, bh, al, bl;
#pragma unroll
      for (int i = 0; i < 8; ++i) {
        const int kk = k0 + lk + i;
        const float a = (r < M && kk < K) ? aload(r, kk) : 0.f;
        const float b = (kk < K && c < N) ? bload(kk, c) : 0.f;
        ah[i] = (__bf16)a;
        bh[i] = (__bf16)b;
        if (SPLIT) {
          al[i] = (__bf16)(a - (float)ah[i]);
          bl[i] = (__bf16)(b - (float)bh[i]);
        }
      }
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
      if (SPLIT) {
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rr = i0 + (lane >> 4) * 4 + i;
      if (rr < M && c < N) store(rr, c, acc[i]);
    }
  }
}

// Batched FP32 GEMM on the matrix cores: for bt < nb, C_bt (M x N) = A_bt
// (M x K) B_bt (K x N) with operands read through aload(bt, i, k) and
// bload(bt, k, j), FP32 products accumulated in FP32 by v_mfma_f32_16x16x4_f32
// (one 16x16 output tile per wave at a time, the tiles of every batch spread
// over the waves).  Lane layout: A lane l holds row l%16, k = l/16; B lane l
// holds column l%16, k = l/16; D lane l value i is row 4(l/16)+i, column l%16.
template <typename ALoad, typename BLoad, typename Store>
__device__ inline void gemm_mfma_f32(int nb, int M, int N, int K, ALoad aload, BLoad bload, Store store) {
  const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int tm = (M + 15) >> 4, tn = (N + 15) >> 4, per = tm * tn;
  const int lr = lane & 15, lk = lane >> 4;
  for (int t = wave; t < nb * per; t += NT / WAVE) {
    const int bt = t / per, tt = t - bt * per;
    const int i0 = (tt / tn) << 4, j0 = (tt % tn) << 4;
    const int r = i0 + lr, c = j0 + lr;
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int kk = k0 + lk;
      const float a = (r < M && kk < K) ? aload(bt, r, kk) : 0.f;
      const float b = (kk < K && c < N) ? bload(bt, kk, c) : 0.f;
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rr = i0 + lk * 4 + i;
      if (rr < M && c < N) store(bt, rr, c, acc[i]);
    }
  }
}

// The same on the FP64 matrix cores (v_mfma_f64_16x16x4_f64: FP64 products
// accumulated in FP64).  Operand lanes as above; output lane l value i is
// row l/16 + 4i, column l%16 (the rows interleave, unlike the FP32 form).
typedef double f64x4_t __attribute__((ext_vector_type(4)));
template <typename ALoad, typename BLoad, typename Store>
__device__ inline void gemm_mfma_f64(int nb, int M, int N, int K, ALoad aload, BLoad bload, Store store) {
  const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int tm = (M + 15) >> 4, tn = (N + 15) >> 4, per = tm * tn;
  const int lr = lane & 15, lk = lane >> 4;
  for (int t = wave; t < nb * per; t += NT / WAVE) {
    const int bt = t / per, tt = t - bt * per;
    const int i0 = (tt / tn) << 4, j0 = (tt % tn) << 4;
    const int r = i0 + lr, c = j0 + lr;
    f64x4_t acc = {0.0, 0.0, 0.0, 0.0};
    for (int k0 = 0; k0 < K; k0 += 4) {
      const int kk = k0 + lk;
      const double a = (r < M && kk < K) ? aload(bt, r, kk) : 0.0;
      const double b = (kk < K && c < N) ? bload(bt, kk, c) : 0.0;
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rr = i0 + lk + 4 * i;
      if (rr < M && c < N) store(bt, rr, c, acc[i]);
    }
  }
}

// FP32 -> bf16 hi + lo (bits), the split of the three-product GEMMs.
__device__ inline void split_bf16(float x, uint16_t& hi, uint16_t& lo) {
  const __bf16 h = (__bf16)x;
  hi = __builtin_bit_cast(uint16_t, h);
  lo = __builtin_bit_cast(uint16_t, (__bf16)(x - (float)h));
}

typedef unsigned int u32x4_t __attribute__((ext_vector_type(4)));
__device__ inline bf16x8_t load_bf16x8(const uint16_t* p, bool ok) {
  u32x4_t v = {0u, 0u, 0u, 0u};
  if (ok) v = *reinterpret_cast<const u32x4_t*>(p);
  return __builtin_bit_cast(bf16x8_t, v);
}

// C (M x N) = A (M x K) B (K x N) on the matrix cores, from operands already
// split into bf16 planes: A row-major (Ah, Al, leading dimension lda), B
// stored transposed (row c of Bh, Bl holds column c of B, leading dimension
// ldb).  lda and ldb are multiples of 8, the planes 16-byte aligned, and
// columns K..pad8(K)-1 of both hold zeros.  Same three products and lane
// layout as gemm_mfma_bf16, with one 16-byte load per operand and k-step;
// without SPLIT only the high planes are read (one product: operands rounded
// once to bf16).
template <bool SPLIT = true, typename Store>
__device__ inline void gemm_mfma_planes(int M, int N, int K, const uint16_t* Ah, const uint16_t* Al, int lda,
                                        const uint16_t* Bh, const uint16_t* Bl, int ldb, Store store) {
  const int wave = threadIdx.x / WAVE, lane = threadIdx.x % WAVE;
  const int tm = (M + 15) >> 4, tn = (N + 15) >> 4;
  const int lr = lane & 15, lk = (lane >> 4) * 8, K8 = (K + 7) & ~7;
  for (int t = wave; t < tm * tn; t += NT / WAVE) {
    const int i0 = (t / tn) << 4, j0 = (t % tn) << 4;
    const int r = i0 + lr, c = j0 + lr;
    f32x4_t acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 32) {
      const int kk = k0 + lk;
      const bool oka = r < M && kk < K8, okb = c < N && kk < K8;
      const bf16x8_t ah = load_bf16x8(Ah + r * lda + kk, oka);
      const bf16x8_t bh = load_bf16x8(Bh + c * ldb + kk, okb);
      acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc, 0, 0, 0);
      if constexpr (SPLIT) {
        const bf16x8_t al = load_bf16x8(Al + r * lda + kk, oka);
        const bf16x8_t bl = load_bf16x8(Bl + c * ldb + kk, okb);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc, 0, 0, 0);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int rr = i0 + (lane >> 4) * 4 + i;
      if (rr < M && c < N) store(rr, c, acc[i]);
    }
  }
}

#endif  // TNMLD_EMU

// Householder LQ of X (m x n, row-major, leading dimension ld), in place:
// X = L Q with L lower-trapezoidal (m x k) and Q (k x n) with orthonormal rows,
// k = min(m, n).  Reflectors follow the LAPACK convention H = I - tau v v^T
// with v_0 = 1 (implicit), so tau is in [1, 2] and v = O(1) whatever the
// scale of the row: tiny rows (graded matrices) keep their relative accuracy.
// Norms and dot products accumulate in FP64 so that FP32 squares of small
// entries cannot underflow.  On return row i holds v_i in columns i+1..n-1,
// the strictly lower part holds L, diag[i] = L[i][i], tau[i] = tau_i.
//
// One barrier per reflector: lane group 0 (16 lanes) owns the next row.  It
// updates that row, takes its tail norm and builds the next reflector while
// the other groups are still applying the current one to the rows below; the
// FP64 tau of step i is handed over in red[i & 1].
template <typename Real>
__device__ __attribute__((noinline)) void lq_factor(Real* X, int m, int n, int ld, Real* tau, Real* diag,
                                                   double* red) {
  const int k = m < n ? m : n;
  const int tid = threadIdx.x, lane = tid & 15, grp = tid >> 4;
  constexpr int NG = NT / 16;
  double tail2 = 0.0;  // group 0: squared norm of row i beyond column i
  if (grp == 0 && k > 0) {
    for (int c = 1 + lane; c < n; c += 16) tail2 += (double)X[c] * (double)X[c];
    tail2 = group_sum(tail2, 16);
  }
  for (int i = 0; i < k; ++i) {
    Real* xi = X + i * ld;
    if (grp == 0) {
      const double x0 = (double)xi[i];
      const double nrm = sqrt(tail2 + x0 * x0);
      // reflector; rows at the bottom of the real range are treated as exact zeros
      const bool live = tail2 > 0.0 && nrm > TinyNorm<Real>::v;
      double beta = x0, t = 0.0;
      if (live) {
        beta = x0 >= 0.0 ? -nrm : nrm;
        t = (beta - x0) / beta;
        const double scale = 1.0 / (x0 - beta);
        for (int c = i + 1 + lane; c < n; c += 16) xi[c] = Real((double)xi[c] * scale);
      }
      if (lane == 0) {
        tau[i] = Real(t);
        diag[i] = Real(beta);
        red[i & 1] = t;
      }
    }
    __syncthreads();
    const double t = red[i & 1];
    if (grp == 0) {
      const int r = i + 1;
      if (r < m) {
        Real* xr = X + r * ld;
        double nt2 = 0.0;
        if (t != 0.0) {
          const double xri = (double)xr[i];  // read before lane 0 rewrites it
          double dot = 0.0;
          for (int c = i + 1 + lane; c < n; c += 16) dot += (double)xr[c] * (double)xi[c];
          dot = group_sum(dot, 16);
          const Real w = Real((dot + xri) * t);
          if (lane == 0) xr[i] -= w;
          for (int c = i + 1 + lane; c < n; c += 16) {
            const Real y = xr[c] - w * xi[c];
            xr[c] = y;
            if (c > r) nt2 += (double)y * (double)y;
          }
        } else {
          for (int c = r + 1 + lane; c < n; c += 16) nt2 += (double)xr[c] * (double)xr[c];
        }
        tail2 = group_sum(nt2, 16);
      }
    } else if (t != 0.0) {
      for (int r = i + 1 + grp; r < m; r += NG - 1) {
        Real* xr = X + r * ld;
        const double xri = (double)xr[i];
        double dot = 0.0;
        for (int c = i + 1 + lane; c < n; c += 16) dot += (double)xr[c] * (double)xi[c];
        dot = group_sum(dot, 16);
        const Real w = Real((dot + xri) * t);
        if (lane == 0) xr[i] -= w;
        for (int c = i + 1 + lane; c < n; c += 16) xr[c] -= w * xi[c];
      }
    }
    // no barrier: the next reflector touches only row i + 1, which group 0 owns
  }
  __syncthreads();
}

// After lq_factor and after L has been copied out: overwrite rows 0..k-1 of X
// with the explicit Q = [I_k 0] H_{k-1} ... H_0.  v is scratch of length 2n
// (the reflector of step i is staged in v + (i & 1) * n one step ahead, so a
// step needs a single barrier).
template <typename Real>
__device__ __attribute__((noinline)) void lq_form_q(Real* X, int m, int n, int ld, const Real* tau, Real* v) {
  const int k = m < n ? m : n;
  const int tid = threadIdx.x, lane = tid & 15, grp = tid >> 4;
  if (k == 0) return;
  {
    Real* vb = v + ((k - 1) & 1) * n;
    const Real* xi = X + (k - 1) * ld;
    for (int c = tid; c < n; c += NT) vb[c] = c < k - 1 ? Real(0) : (c == k - 1 ? Real(1) : xi[c]);
  }
  __syncthreads();
  for (int i = k - 1; i >= 0; --i) {
    const Real* vb = v + (i & 1) * n;
    const Real t = tau[i];
    if (t != Real(0)) {
      for (int r = i + 1 + grp; r < k; r += NT / 16) {
        Real* xr = X + r * ld;
        double dot = 0;
        for (int c = i + lane; c < n; c += 16) dot += (double)xr[c] * (double)vb[c];
        dot = group_sum(dot, 16);
        const Real w = Real(dot) * t;
        for (int c = i + lane; c < n; c += 16) xr[c] -= w * vb[c];
      }
    }
    Real* xi = X + i * ld;
    for (int c = tid; c < n; c += NT) xi[c] = c < i ? Real(0) : ((c == i ? Real(1) : Real(0)) - t * vb[c]);
    if (i > 0) {
      Real* vn = v + ((i - 1) & 1) * n;
      const Real* xp = X + (i - 1) * ld;
      for (int c = tid; c < n; c += NT) vn[c] = c < i - 1 ? Real(0) : (c == i - 1 ? Real(1) : xp[c]);
    }
    __syncthreads();
  }
}

// Register-resident Householder LQ for m <= 64 rows and n <= 256 columns:
// lane group g (16 lanes) keeps rows g and g + 32 in registers, lane l holds
// columns l + 16 c.  Same reflectors and output layout as lq_factor, except
// that the dot products of the row updates accumulate in the factorisation
// type (FP32 in the FP32 forms: the reflector's leading entry is 1, so the
// dot keeps the scale of the row's own entry and only terms far below it can
// underflow); row norms stay FP64.  Only the
// reflector of each step goes through LDS, staged over all 16 NPL columns with
// explicit zeros (left of i and past n) and the implicit one, in
// vb + (i & 1) * 16 NPL, so the row update loads it with no bounds test.  The
// owner of row i + 1 builds the next reflector as soon as it has updated that
// row: one barrier per step.  vb: LDS scratch of 32 NPL.
// lq_rpg: rows per lane group: 2 with 512 threads; with 256 threads 4 for FP32
// factorisations (64-row matrices in registers, as in the 512-thread build)
// and 2 for FP64 ones (four rows of doubles would halve the waves per SIMD).
// Widest register row a build compiles (columns per lane; 8 or 16): a build for
// small plans leaves out the 16-column code, whose register use would cap its
// occupancy.  Wider matrices take the LDS-resident factorisation there.
#ifndef TNMLD_MAX_NPL
#define TNMLD_MAX_NPL 16
#endif
constexpr int kMaxNpl = TNMLD_MAX_NPL;
template <typename Real>
constexpr int lq_rpg() {
  return NT >= 512 ? 2 : (sizeof(Real) == 4 ? 4 : 2);
}
template <typename Real>
__device__ inline bool lq_regs_fit(int m, int n) {
  return m <= lq_rpg<Real>() * (NT / 16) && n <= kMaxNpl * 16;
}
// Row held in slot j by lane group g in the explicit-Q builder: slots pair a
// row with its mirror (g and 2 NG - 1 - g, then 2 NG + g and 4 NG - 1 - g), so
// every group's rows need the same number of reflector steps in total.
__device__ inline int lq_q_row(int j, int g, int ng) {
  const int base = 2 * ng * (j >> 1);
  return (j & 1) ? base + 2 * ng - 1 - g : base + g;
}

// NPL: columns per lane held in registers (n <= 16 NPL); instantiated for 8
// and 16 so that 128-column matrices do not run 256-column loops.  XT: the
// element type of X with its address space (LDS, or global scratch); the other
// buffers are LDS.  Out of line, with typed pointers so that LDS accesses stay
// DS instructions.
template <typename Real, int NPL, typename XT>
__device__ __attribute__((noinline)) void lq_factor_regs(XT* X, int m, int n, int ld, lds_t<Real>* tau,
                                                        lds_t<Real>* diag, lds_t<double>* red, lds_t<Real>* vb) {
  constexpr int LQR_RPG = lq_rpg<Real>();
  const int k = m < n ? m : n;
  const int tid = threadIdx.x, lane = tid & 15, grp = tid >> 4;
  constexpr int NG = NT / 16;
  Real x[LQR_RPG][NPL];
#pragma unroll
  for (int j = 0; j < LQR_RPG; ++j) {
    const int r = grp + NG * j;
#pragma unroll
    for (int c = 0; c < NPL; ++c) {
      const int col = lane + 16 * c;
      x[j][c] = (r < m && col < n) ? X[r * ld + col] : Real(0);
    }
  }
  // reflector of row i held in slot j of this group (all 16 lanes call it).
  // Norm and reflector scalars in FP64; the tail is scaled in the storage type.
  auto reflector = [&](int i, Real* xr) {
    double tp[4] = {0.0, 0.0, 0.0, 0.0};  // four partial sums: short FMA chains
    Real x0r = Real(0);
#pragma unroll
    for (int c = 0; c < NPL; ++c) {
      const int col = lane + 16 * c;
      const Real xt = col > i ? xr[c] : Real(0);
      tp[c & 3] += (double)xt * (double)xt;
      if (col == i) x0r = xr[c];
    }
    const double t2 = group_sum((tp[0] + tp[1]) + (tp[2] + tp[3]), 16);
#ifdef TNMLD_EMU
    const double x0 = (double)group_sum(x0r, 16);  // one lane holds it: the sum is exact
#else
    // one lane holds it: read it there.  Only this group's lanes are active
    // here (the caller's branch on the row it owns), so the first active
    // lane gives the group's base lane in the wave.
    const int src = __builtin_amdgcn_readfirstlane((int)threadIdx.x & (WAVE - 16)) + (i & 15);
    const double x0 = (double)lane_read(x0r, src);
#endif
    const double nrm = sizeof(Real) == 4 ? sqrt_normal(t2 + x0 * x0) : sqrt(t2 + x0 * x0);
    const bool live = t2 > 0.0 && nrm > TinyNorm<Real>::v;
    double beta = x0, td = 0.0, sd = 0.0;
    if (live) {
      beta = x0 >= 0.0 ? -nrm : nrm;
      if constexpr (sizeof(Real) == 4) {
        // one division: a = x0 - beta has |a| >= nrm, and beta a stays far
        // inside the FP64 range for FP32 rows
        const double a = x0 - beta;
        const double rp = recip_normal(beta * a);
        td = -(a * a) * rp;  // (beta - x0) / beta
        sd = beta * rp;      // 1 / (x0 - beta)
      } else {
        td = (beta - x0) / beta;
        sd = 1.0 / (x0 - beta);
      }
    }
    // with no reflection the tail is scaled by 1: exact, and no select per column
    const Real t = Real(td), scale = live ? Real(sd) : Real(1);
    lds_t<Real>* v = vb + (i & 1) * (16 * NPL);
#pragma unroll
    for (int c = 0; c < NPL; ++c) {
      const int col = lane + 16 * c;
      if (col > i) xr[c] *= scale;
      v[col] = col < i ? Real(0) : (col == i ? Real(1) : xr[c]);  // past column n, xr stays 0
    }
    if (lane == 0) {
      tau[i] = t;
      diag[i] = Real(beta);
      red[i & 1] = (double)t;
    }
  };
  if (k > 0 && grp == 0) reflector(0, x[0]);
  __syncthreads();
  for (int i = 0; i < k; ++i) {
    const Real t = Real(red[i & 1]);
    const lds_t<Real>* v = vb + (i & 1) * (16 * NPL);
    Real vv[NPL];
#pragma unroll
    for (int c = 0; c < NPL; ++c) vv[c] = v[lane + 16 * c];  // staged with its zeros: no bounds test
#pragma unroll
    for (int j = 0; j < LQR_RPG; ++j) {
      const int r = grp + NG * j;
      if (r > i && r < m) {
        if (t != Real(0)) {
          Real dp[4] = {Real(0), Real(0), Real(0), Real(0)};
#pragma unroll
          for (int c = 0; c < NPL; ++c) dp[c & 3] += x[j][c] * vv[c];
          const Real w = group_sum((dp[0] + dp[1]) + (dp[2] + dp[3]), 16) * t;
#pragma unroll
          for (int c = 0; c < NPL; ++c) x[j][c] -= w * vv[c];
        }
        if (r == i + 1 && r < k) reflector(r, x[j]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < LQR_RPG; ++j) {
    const int r = grp + NG * j;
#pragma unroll
    for (int c = 0; c < NPL; ++c) {
      const int col = lane + 16 * c;
      if (r < m && col < n) X[r * ld + col] = x[j][c];
    }
  }
  __syncthreads();
}

// Register-resident explicit Q after lq_factor (k = min(m, n) <= 64): row r
// of Q = [I_k 0] H_{k-1} ... H_0 is e_r - tau_r v_r pushed through
// H_{r-1}, ..., H_0, which involves no other row of Q, so each lane group
// builds its rows (lq_q_row: mirrored pairs, balancing the step counts) with no barrier,
// reading the reflectors from X.  The strictly lower part of X (L, already
// copied out by the caller) is first overwritten with the zeros and the
// diagonal with the ones of the reflectors, so the loop reads rows with no
// index tests; FULL (n == 16 NPL) drops the bounds test on the columns too.
// One barrier before the rows are stored.
template <typename Real, int NPL, bool FULL>
__device__ __attribute__((noinline)) void lq_form_q_regs(lds_t<Real>* X, int m, int n, int ld,
                                                        const lds_t<Real>* tau) {
  constexpr int LQR_RPG = lq_rpg<Real>();
  const int k = m < n ? m : n;
  const int tid = threadIdx.x, lane = tid & 15, grp = tid >> 4;
  constexpr int NG = NT / 16;
  for_2d(k, k, [&](int r, int c) {
    if (c <= r) X[r * ld + c] = c == r ? Real(1) : Real(0);
  });
  __syncthreads();
  Real q[LQR_RPG][NPL];
#pragma unroll
  for (int j = 0; j < LQR_RPG; ++j) {
    const int r = lq_q_row(j, grp, NG);
    if (r >= k) continue;
    {
      const Real t = tau[r];
      const lds_t<Real>* xr = X + r * ld;
#pragma unroll
      for (int c = 0; c < NPL; ++c) {
        const int col = lane + 16 * c;
        const Real vc = (FULL || col < n) ? xr[col] : Real(0);
        q[j][c] = (col == r ? Real(1) : Real(0)) - t * vc;
      }
    }
    for (int i = r - 1; i >= 0; --i) {
      const Real t = tau[i];  // tau = 0 (no reflection) leaves q as it is
      const lds_t<Real>* xi = X + i * ld;
      Real vv[NPL];
      Real dp[4] = {Real(0), Real(0), Real(0), Real(0)};
#pragma unroll
      for (int c = 0; c < NPL; ++c) {
        const int col = lane + 16 * c;
        vv[c] = (FULL || col < n) ? xi[col] : Real(0);
        dp[c & 3] += q[j][c] * vv[c];
      }
      const Real dot = group_sum((dp[0] + dp[1]) + (dp[2] + dp[3]), 16);
      const Real w = Real(dot) * t;
#pragma unroll
      for (int c = 0; c < NPL; ++c) q[j][c] -= w * vv[c];
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < LQR_RPG; ++j) {
    const int r = lq_q_row(j, grp, NG);
    if (r >= k) continue;
#pragma unroll
    for (int c = 0; c < NPL; ++c) {
      const int col = lane + 16 * c;
      if (FULL || col < n) X[r * ld + col] = q[j][c];
    }
  }
  __syncthreads();
}

// Explicit Q as lq_form_q_regs, for reflectors kept outside LDS (the LQ
// matrix in the work-group's global scratch, lq_factor output as is: L below
// the diagonal).  The reflectors go through LDS in chunks of up to cap (buf:
// cap x 16 NPL elements of LDS), from k-1 down; within a chunk each lane group
// takes its rows through the chunk's reflectors with no barrier, as
// lq_form_q_regs does with all of them.  Row r starts as e_r - tau_r v_r in the
// chunk that holds reflector r and takes reflectors r-1..0 after it: per row,
// the operations and their order are those of lq_form_q_regs.  Two barriers
// per chunk.  Rows 0..k-1 of Q go to out (leading dimension ldo).  Out of
// line: inlined into the sweep, its four live row slots push the 256-thread
// build past the registers of two waves per SIMD.
template <typename Fac, typename Out, int NPL>
__device__ __attribute__((noinline)) void lq_form_q_staged(const glb_t<Fac>* X, int m, int n, int ld,
                                                           const lds_t<Fac>* tau, lds_t<Fac>* buf, int cap,
                                                           glb_t<Out>* out, int ldo) {
  constexpr int RPG = lq_rpg<Fac>();
  constexpr int NG = NT / 16;
  constexpr int W = 16 * NPL;  // staged row: columns 0..W-1, zeros past n
  const int k = m < n ? m : n;
  const int tid = threadIdx.x, lane = tid & 15, grp = tid >> 4;
  Fac q[RPG][NPL];
#pragma unroll
  for (int j = 0; j < RPG; ++j)
#pragma unroll
    for (int c = 0; c < NPL; ++c) q[j][c] = Fac(0);
  for (int hi = k - 1; hi >= 0; hi -= cap) {
    const int lo = hi - cap + 1 > 0 ? hi - cap + 1 : 0;
    // reflectors lo..hi as full rows: zeros left of i, the implicit one, the tail
    for (int e = tid; e < (hi - lo + 1) * W; e += NT) {
      const int i = lo + e / W, c = e % W;
      buf[e] = c < i ? Fac(0) : (c == i ? Fac(1) : (c < n ? X[i * ld + c] : Fac(0)));
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < RPG; ++j) {
      const int r = lq_q_row(j, grp, NG);
      if (r >= k || r < lo) continue;  // a row below the chunk starts in a later one
      int i = hi;
      if (r <= hi) {
        const Fac t = tau[r];
        const lds_t<Fac>* v = buf + (r - lo) * W + lane;
#pragma unroll
        for (int c = 0; c < NPL; ++c) q[j][c] = (lane + 16 * c == r ? Fac(1) : Fac(0)) - t * v[16 * c];
        i = r - 1;
      }
      for (; i >= lo; --i) {
        const Fac t = tau[i];  // tau = 0 (no reflection) leaves q as it is
        const lds_t<Fac>* v = buf + (i - lo) * W + lane;
        Fac vv[NPL];
        Fac dp[4] = {Fac(0), Fac(0), Fac(0), Fac(0)};
#pragma unroll
        for (int c = 0; c < NPL; ++c) {
          vv[c] = v[16 * c];
          dp[c & 3] += q[j][c] * vv[c];
        }
        const Fac dot = group_sum((dp[0] + dp[1]) + (dp[2] + dp[3]), 16);
        const Fac w = Fac(dot) * t;
#pragma unroll
        for (int c = 0; c < NPL; ++c) q[j][c] -= w * vv[c];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int j = 0; j < RPG; ++j) {
    const int r = lq_q_row(j, grp, NG);
    if (r >= k) continue;
    glb_t<Out>* o = out + (int64_t)r * ldo + lane;  // one address per row, immediate offsets per column
#pragma unroll
    for (int c = 0; c < NPL; ++c)
      if (lane + 16 * c < n) o[16 * c] = Out(q[j][c]);
  }
}

// Dispatch: registers when the matrix fits, else the LDS-resident version.
// tau, diag, red and vb are LDS; X is LDS, or global scratch when XGL.
template <typename Real, bool XGL = false>
__device__ inline __attribute__((always_inline)) void lq_factor_any(Real* X, int m, int n, int ld, Real* tau,
                                                                    Real* diag, double* red, Real* vb) {
  using XT = typename std::conditional<XGL, glb_t<Real>, lds_t<Real>>::type;
  if (lq_regs_fit<Real>(m, n)) {
    auto tl = (lds_t<Real>*)tau;
    auto dl = (lds_t<Real>*)diag;
    auto rl = (lds_t<double>*)red;
    auto vl = (lds_t<Real>*)vb;
    if (n <= 128) lq_factor_regs<Real, 8, XT>((XT*)X, m, n, ld, tl, dl, rl, vl);
    else if constexpr (kMaxNpl >= 16) lq_factor_regs<Real, 16, XT>((XT*)X, m, n, ld, tl, dl, rl, vl);
  } else {
    lq_factor<Real>(X, m, n, ld, tau, diag, red);
  }
}
// X and tau are LDS.
template <typename Real>
__device__ inline __attribute__((always_inline)) void lq_form_q_any(Real* X, int m, int n, int ld, const Real* tau,
                                                                    Real* v) {
  if (lq_regs_fit<Real>(m, n)) {
    auto xl = (lds_t<Real>*)X;
    auto tl = (const lds_t<Real>*)tau;
    if (n == 128) lq_form_q_regs<Real, 8, true>(xl, m, n, ld, tl);
    else if (n < 128) lq_form_q_regs<Real, 8, false>(xl, m, n, ld, tl);
    else if constexpr (kMaxNpl >= 16) {
      if (n == 256) lq_form_q_regs<Real, 16, true>(xl, m, n, ld, tl);
      else lq_form_q_regs<Real, 16, false>(xl, m, n, ld, tl);
    }
  } else {
    lq_form_q<Real>(X, m, n, ld, tau, v);
  }
}

// One-sided (Hestenes) Jacobi on the columns of M (rows x cols, column-major,
// leading dimension ldm), accumulating the rotations in V (cols x cols,
// column-major, ldv), which must hold the identity on entry.  Afterwards the
// columns of M are mutually orthogonal: M_in V = M_out, and the column norms
// are the singular values.  Parallel cyclic ordering (circle method): each
// round rotates n'/2 disjoint pairs, one pair per group of G lanes, with the
// pair's columns held in registers.
//
// Columns whose norm is below k eps |M|_F (k = sqrt(rows)) are rounding noise
// of the matrix: they are left out of the rotations altogether (they keep
// their place and an identity column of V), so a graded matrix with n live
// columns costs n - 1 rounds per sweep instead of cols - 1.  Among the live
// columns a pair is left alone once its cosine is below tol, or once what a
// rotation would remove is below the rounding level of the storage type:
// |a.b| <= k eps max(|a|^2, |b|^2), or |a.b| <= (k eps |M|_F)^2.  Without
// these tests, columns at the rounding floor keep rotating forever.  The
// iteration stops after a sweep in which no rotated pair had a cosine above
// sqrt(tol / cols): with quadratic convergence the pairs are then below tol.
// eps: rounding unit of the data (of the storage type, which may be coarser
// than Real).  lst: int scratch of cols entries.  Returns the number of sweeps.
template <typename Real>
__device__ __attribute__((noinline)) int jacobi_svd_lds(lds_t<Real>* M, int rows, int cols, int ldm, lds_t<Real>* V,
                                                        int ldv, double tol, double eps, lds_t<int>* flag,
                                                        lds_t<double>* red, lds_t<double>* nrm, lds_t<int>* lst) {
  constexpr int MAXR = 4;  // rows (and V rows) lane + j G, j < MAXR, live in registers; the rest stream from LDS
  if (cols < 2) return 0;
  const int tid = threadIdx.x;
  (void)red;
  // squared column norms, the Frobenius norm as their sum, and the live columns
  for (int c = tid >> 4; c < cols; c += NT / 16) {
    double sq = 0;
    for (int r = tid & 15; r < rows; r += 16) sq += (double)M[c * ldm + r] * (double)M[c * ldm + r];
    sq = group_sum(sq, 16);
    if ((tid & 15) == 0) nrm[c] = sq;
  }
  __syncthreads();
  double nf2 = 0;
  for (int c = 0; c < cols; ++c) nf2 += nrm[c];  // same order in every thread
  const double keps = sqrt((double)rows) * eps;
  const double floor2 = keps * keps * nf2;
  int nlive = 0;
  for (int c = 0; c < cols; ++c) nlive += nrm[c] > floor2;
  for (int c = tid; c < cols; c += NT) {
    if (nrm[c] > floor2) {
      int rank = 0;
      for (int c2 = 0; c2 < c; ++c2) rank += nrm[c2] > floor2;
      lst[rank] = c;
    }
  }
  __syncthreads();
  if (nlive < 2) return 1;
  const int N = nlive + (nlive & 1);
  const int P = N >> 1;
  int G = WAVE;
  while (G > 1 && G * P > NT) G >>= 1;
  const int g = tid / G, lane = tid % G;
  const int nr = (rows + G - 1) / G, nc = (cols + G - 1) / G;
  // a sweep whose largest rotated cosine is below sqrt(tol / cols) leaves every
  // pair below tol (convergence is quadratic), so no confirming sweep follows
  const double big2 = tol / (double)cols;
  int sweep = 0;
  for (; sweep < 40; ++sweep) {
    if (tid == 0) *flag = 0;
    if (sweep > 0) {
      // exact squared norms of the live columns at the start of every sweep;
      // rotations update them in closed form (|a'|^2 = |a|^2 - t a.b, |b'|^2 = |b|^2 + t a.b)
      for (int i0 = 0; i0 < nlive; i0 += NT / G) {
        const int i = i0 + g;
        const int c = i < nlive ? lst[i] : 0;
        double sq = 0;
        if (i < nlive)
          for (int r = lane; r < rows; r += G) sq += (double)M[c * ldm + r] * (double)M[c * ldm + r];
        sq = group_sum(sq, G);
        if (i < nlive && lane == 0) nrm[c] = sq;
      }
    }
    __syncthreads();
    // circle method: group g pairs (rd + g, rd - g) mod (N - 1), group 0 pairs
    // (rd, N - 1); the two indices advance by one per round (no divisions)
    int pp = g == 0 ? 0 : (g < N - 1 ? g : g % (N - 1));
    int qq = g == 0 ? N - 1 : (N - 1 - pp == N - 1 ? 0 : N - 1 - pp);
    for (int rd = 0; rd < N - 1; ++rd) {
      int p = pp, q = qq;
      if (p > q) {
        const int t = p;
        p = q;
        q = t;
      }
      if (g != 0) {
        pp = pp + 1 == N - 1 ? 0 : pp + 1;
        qq = qq + 1 == N - 1 ? 0 : qq + 1;
      } else {
        pp = pp + 1;
      }
      const bool act = g < P && q < nlive;
      const int cp = act ? lst[p] : 0, cq = act ? lst[q] : 0;
      lds_t<Real>* a = M + cp * ldm;
      lds_t<Real>* b = M + cq * ldm;
      Real xa[MAXR], xb[MAXR];
      double gp[2] = {0.0, 0.0};  // FP64 sums: no underflow of small columns
#pragma unroll
      for (int j = 0; j < MAXR; ++j) {
        const int r = lane + j * G;
        xa[j] = xb[j] = Real(0);
        if (act && j < nr && r < rows) {
          xa[j] = a[r];
          xb[j] = b[r];
        }
        gp[j & 1] += (double)xa[j] * (double)xb[j];
      }
      if (act)
        for (int r = lane + MAXR * G; r < rows; r += G) gp[0] += (double)a[r] * (double)b[r];
      // the rotation's V columns are loaded now so that their latency overlaps the reduction
      lds_t<Real>* va = V + cp * ldv;
      lds_t<Real>* vb = V + cq * ldv;
      Real ya[MAXR], yb[MAXR];
#pragma unroll
      for (int j = 0; j < MAXR; ++j) {
        const int r = lane + j * G;
        ya[j] = yb[j] = Real(0);
        if (act && j < nc && r < cols) {
          ya[j] = va[r];
          yb[j] = vb[r];
        }
      }
      const double al = act ? nrm[cp] : 0.0, be = act ? nrm[cq] : 0.0;
      const double ga = group_sum(gp[0] + gp[1], G);
      const double aga = fabs(ga);
      // squared form of |ga| > tol |a| |b| (the pair is far above the noise floor here)
      const bool rot = act && aga > keps * (al > be ? al : be) && aga > floor2 && ga * ga > tol * tol * al * be &&
                       (sizeof(Real) == 8 || (float)ga != 0.0f);
      if (rot) {
        Real c, s;
        double tn;
        if constexpr (sizeof(Real) == 4) {
          // the rotation of FP32 columns only needs an FP32 angle
          const float z = (float)(be - al) / (2.0f * (float)ga);
          const float az = fabsf(z);
          const float tt = az > 1e15f ? 0.5f / z : (z >= 0.0f ? 1.0f : -1.0f) / (az + sqrtf(1.0f + z * z));
          c = 1.0f / sqrtf(1.0f + tt * tt);
          s = c * tt;
          tn = (double)tt;
        } else {
          const double zeta = (be - al) / (2.0 * ga);
          double tt;
          if (fabs(zeta) > 1e16) tt = 0.5 / zeta;
          else tt = (zeta >= 0.0 ? 1.0 : -1.0) / (fabs(zeta) + sqrt(1.0 + zeta * zeta));
          const double cd = 1.0 / sqrt(1.0 + tt * tt);
          c = Real(cd);
          s = Real(cd * tt);
          tn = tt;
        }
#pragma unroll
        for (int j = 0; j < MAXR; ++j) {
          const int r = lane + j * G;
          if (j < nr && r < rows) {
            a[r] = c * xa[j] - s * xb[j];
            b[r] = s * xa[j] + c * xb[j];
          }
        }
        for (int r = lane + MAXR * G; r < rows; r += G) {
          const Real x = a[r], y = b[r];
          a[r] = c * x - s * y;
          b[r] = s * x + c * y;
        }
#pragma unroll
        for (int j = 0; j < MAXR; ++j) {
          const int r = lane + j * G;
          if (j < nc && r < cols) {
            va[r] = c * ya[j] - s * yb[j];
            vb[r] = s * ya[j] + c * yb[j];
          }
        }
        for (int r = lane + MAXR * G; r < cols; r += G) {
          const Real x = va[r], y = vb[r];
          va[r] = c * x - s * y;
          vb[r] = s * x + c * y;
        }
        if (lane == 0) {
          if (ga * ga > big2 * al * be) *flag = 1;
          nrm[cp] = fmax(al - tn * ga, 0.0);
          nrm[cq] = fmax(be + tn * ga, 0.0);
        }
      }
      __syncthreads();
    }
    const int f = *flag;
    __syncthreads();
    if (!f) return sweep + 1;
  }
  return sweep;
}

// jacobi_svd_lds on buffers that are all in LDS (the caller's pointers).
template <typename Real>
__device__ inline __attribute__((always_inline)) int jacobi_svd(Real* M, int rows, int cols, int ldm, Real* V,
                                                                int ldv, double tol, double eps, int* flag,
                                                                double* red, double* nrm, int* lst) {
  return jacobi_svd_lds<Real>((lds_t<Real>*)M, rows, cols, ldm, (lds_t<Real>*)V, ldv, tol, eps, (lds_t<int>*)flag,
                              (lds_t<double>*)red, (lds_t<double>*)nrm, (lds_t<int>*)lst);
}


}  // namespace tnmld
