// Device-side forward contraction of one (syndrome, coset) pair (paper
// Sec. 3.2.1): reference error, row MPO application, right-to-left LQ sweep,
// left-to-right SVD truncation, FP64 log-norm accumulation.  Included by the
// HIP translation unit; collective over one work-group of NT threads.
#pragma once
#ifndef TNMLD_EMU
#include <hip/hip_runtime.h>
#endif
#include <stdint.h>

#include "../../include/tnmld.h"
#include "plan.hpp"
#include "sweep.hpp"

namespace tnmld {

struct JobDev {
  const uint8_t* plan;
  const double* rates;
  const int32_t* model_index;
  const uint8_t* syn;
  double* logz;
  const double* logp;   // backward: log P(s) of the forward pass
  const double* gradp;  // backward: d loss / d log P(s)
  int64_t count;
  int64_t item_begin;
  int64_t part_ofs;     // backward: offset of this segment in a work-group's partial gradient
  int32_t n_models;
  int32_t rounds;       // syndrome rounds per item (0 or 1: one perfect round)
  unsigned* status;     // status word of the call (ST_* bits), in the workspace header
  const double* meas;   // repeated rounds: [n_models][m] measurement flip probabilities
  void* states;         // backward in two calls: this job's top-sweep states (caller memory), or null
  int64_t states_stride;  // elements of one syndrome's states
};

struct JobTable {
  JobDev j[TN_MAX_SEGMENTS];
  int32_t n;
  int32_t pad;
  int64_t nitems;
};

__device__ inline int pauli_code(int x, int z) { return x ? (z ? 2 : 1) : (z ? 3 : 0); }
__device__ inline int pauli_x(int p) { return p == 1 || p == 2; }
__device__ inline int pauli_z(int p) { return p == 2 || p == 3; }

// p_q(f_q xor P) for the four P, from FP64 rates; p_I = 1 - p_X - p_Y - p_Z,
// never below zero (sums a rounding step above one are accepted as inputs)
template <typename Real>
__device__ inline Real pauli_weight(const double* rq, int fb, int P) {
  const int x = pauli_x(P) ^ (fb & 1), z = pauli_z(P) ^ (fb >> 1);
  const int e = pauli_code(x, z);
  if (e == 0) return Real(fmax(1.0 - rq[0] - rq[1] - rq[2], 0.0));
  return Real(rq[e - 1]);
}

// Repeated rounds: the qubit tensor of code 2 + k (see the MPO code comment
// in plan.hpp), in FP64.  rq: the qubit's rates; fb: bits of f_q.
__device__ inline double pauli_prob2(const double* rq, int c) {  // c = x | z << 1
  if (c == 0) return fmax(1.0 - rq[0] - rq[1] - rq[2], 0.0);
  return rq[c == 1 ? 0 : (c == 3 ? 1 : 2)];
}
__device__ inline double rounds_tensor(const double* rq, int fb, int k, int T) {
  const int dT = (k >> (2 * (T - 1))) & 3;
  const int cT = dT ^ fb;  // C_T = f_q P_T as (x | z << 1)
  double acc = 0.0;
  const int nh = 1 << (2 * (T - 1));
  for (int h = 0; h < nh; ++h) {  // intermediate accumulated Paulis C_1..C_{T-1}
    double prod = 1.0;
    int prev = 0, sgn = 0;
    for (int t = 0; t < T - 1; ++t) {
      const int c = (h >> (2 * t)) & 3;
      const int dg = (k >> (2 * t)) & 3;  // (bX, bZ) of round t+1
      prod *= pauli_prob2(rq, prev ^ c);
      sgn ^= ((dg & 1) & (c >> 1)) ^ ((dg >> 1) & (c & 1));
      prev = c;
    }
    prod *= pauli_prob2(rq, prev ^ cT);
    acc += sgn ? -prod : prod;
  }
  return acc;
}
// Measurement weights of check j carried by the T-bit variable value `idx`:
// prod over rounds t < T-1 of g(bit t), g(0) = 1/2, g(1) = (1 - 2 q_j)/2 (-1)^{s_tj}.
__device__ inline double rounds_check_weight(const double* meas, const uint8_t* syn, int m, int j, int idx, int T) {
  double v = 1.0;
  const double h1 = 0.5 * (1.0 - 2.0 * meas[j]);
  for (int t = 0; t < T - 1; ++t) v *= ((idx >> t) & 1) ? (syn[t * m + j] ? -h1 : h1) : 0.5;
  return v;
}

// Bits a call ORs into the status word of its workspace.  The status word is
// followed (8 bytes on) by a 64-bit count of unresolved cosets.
enum : unsigned {
  ST_BAD_INPUT = 1u,   // an item had a syndrome byte above 1, a model index out of range, or invalid rates
  ST_NUMERIC = 2u,     // all four cosets of a strictly positive model came out with Z <= 0: log P(s) was lost
  ST_UNRESOLVED = 4u   // some (not all) cosets of a strictly positive model came out with Z <= 0: they lie
                       // below the resolution of the form at that syndrome and are reported as -inf
};
// Slack on p_X + p_Y + p_Z <= 1 for rates that were rounded from a sum of one
constexpr double kRateSlack = 1e-12;

struct ItemCheck {
  int model;      // model index to read (0 when the item is invalid)
  bool valid;     // the item may be contracted
  bool positive;  // every Pauli of every qubit has probability > 0: every coset then has Z > 0
};

// Syndrome rounds of a job's items (at least 1) and the bytes of one item.
__device__ inline int job_rounds(const JobDev& job) { return job.rounds > 1 ? job.rounds : 1; }

// Input check of syndrome b (collective): syndrome bytes in {0, 1}, model
// index in [0, n_models), and the model's rates in [0, 1] (NaN fails) with
// p_X + p_Y + p_Z <= 1.  An invalid item raises ST_BAD_INPUT.
__device__ inline ItemCheck check_item(const JobDev& job, int64_t b, int n, int m) {
  const int tid = threadIdx.x;
  const int raw = job.model_index ? job.model_index[b] : 0;
  const bool mok = raw >= 0 && raw < job.n_models;
  const int model = mok ? raw : 0;
  const int R = job_rounds(job);
  const uint8_t* sy = job.syn + b * (int64_t)m * R;
  int bad = mok ? 0 : 1;
  for (int j = tid; j < m * R; j += NT) bad |= sy[j] > 1 ? 1 : 0;
  if (R > 1) {  // measurement flip probabilities in [0, 1] (NaN fails)
    const double* mq = job.meas + (int64_t)model * m;
    for (int j = tid; j < m; j += NT) bad |= (mq[j] >= 0.0 && mq[j] <= 1.0) ? 0 : 1;
  }
  const double* r = job.rates + (int64_t)model * n * 3;
  int pos = 1;
  for (int q = tid; q < n; q += NT) {
    const double a = r[3 * q], bb = r[3 * q + 1], c = r[3 * q + 2];
    const bool in01 = a >= 0.0 && a <= 1.0 && bb >= 0.0 && bb <= 1.0 && c >= 0.0 && c <= 1.0;
    const double s = a + bb + c;
    if (!in01 || !(s <= 1.0 + kRateSlack)) bad = 1;
    if (!(a > 0.0 && bb > 0.0 && c > 0.0 && s < 1.0)) pos = 0;
  }
  bad = __syncthreads_or(bad);
  pos = __syncthreads_and(pos);
  if (bad && tid == 0 && job.status) atomicOr(job.status, ST_BAD_INPUT);
  return ItemCheck{model, bad == 0, bad == 0 && pos != 0};
}

// log Z of a finished coset, never NaN: a result that is not finite (the
// state vanished or the closing sum was <= 0) is written as -inf.
__device__ inline double finish_logz(double lz) { return (lz > -INFINITY && lz < INFINITY) ? lz : -INFINITY; }

// After the four cosets of an item (one thread): dead = cosets written as
// -inf.  Under a strictly positive model every coset has Z > 0, so these are
// precision losses: all four lose log P(s) (ST_NUMERIC); fewer are cosets
// below the resolution of the form (ST_UNRESOLVED, counted).
__device__ inline void report_dead(int dead, const ItemCheck& ck, const JobDev& job) {
  if (!ck.positive || dead == 0 || !job.status) return;
  if (dead >= 4) {
    atomicOr(job.status, ST_NUMERIC);
  } else {
    atomicOr(job.status, ST_UNRESOLVED);
    atomicAdd(reinterpret_cast<unsigned long long*>(job.status + 2), (unsigned long long)dead);
  }
}

// Forward contraction of one item; returns log Z (FP64).  Writes the class
// index of the coset into *label.  Collective over the work-group.
// Real: type of the MPS in HBM, of the MPO values and of the GEMM operands;
// Fac: type of the LQ / SVD factorisations (LDS);
// GM: how the two contraction GEMMs run: GEMM_VALU (Real arithmetic),
// GEMM_BF16 (bf16 MFMA, FP32 accumulation), GEMM_BF16X3 (split bf16),
// GEMM_F32 (FP32 MFMA: FP32 products, FP32 accumulation) or GEMM_F64 (FP64
// MFMA, for FP64 data).
enum { GEMM_VALU = 0, GEMM_BF16 = 1, GEMM_BF16X3 = 2, GEMM_F32 = 3, GEMM_F64 = 4 };

template <int GM, typename Real, typename AL, typename BL, typename ST>
__device__ inline void contract_gemm(int M, int N, int K, const Real* A, int lda, const Real* B, int ldb, AL, BL,
                                     ST store) {
  if constexpr (GM == GEMM_VALU) {
    gemm_lds<Real>(M, N, K, A, lda, B, ldb, store);
  } else if constexpr (GM == GEMM_F32) {
#ifndef TNMLD_EMU
    gemm_mfma_f32(
        1, M, N, K, [&](int, int i, int k) { return (float)A[i * lda + k]; },
        [&](int, int k, int j) { return (float)B[k * ldb + j]; }, [&](int, int i, int j, float v) { store(i, j, Real(v)); });
#else
    gemm_lds<Real>(M, N, K, A, lda, B, ldb, store);
#endif
  } else if constexpr (GM == GEMM_F64) {
#ifndef TNMLD_EMU
    gemm_mfma_f64(
        1, M, N, K, [&](int, int i, int k) { return (double)A[i * lda + k]; },
        [&](int, int k, int j) { return (double)B[k * ldb + j]; }, [&](int, int i, int j, double v) { store(i, j, Real(v)); });
#else
    gemm_lds<Real>(M, N, K, A, lda, B, ldb, store);
#endif
  } else {
#ifndef TNMLD_EMU
    gemm_mfma_bf16<GM == GEMM_BF16X3>(
        M, N, K, [&](int i, int k) { return (float)A[i * lda + k]; }, [&](int k, int j) { return (float)B[k * ldb + j]; },
        store);
#endif
  }
}

// LDS work areas of the sweep, carved from the dynamic shared memory.
template <typename Real, typename Fac>
struct Work {
  uint8_t* fbits;
  uint8_t* syn;
  int* perm;
  double* dred;
  double* nrm;
  Real *Wv, *Aj, *T, *T2, *L, *C;
  Fac *X, *tau, *diag, *vtmp, *Mm, *Vv, *Lt, *sig;
  int* s_flag;
  int* s_dead;
  // repeated rounds (rounds > 1): the item's syndromes (round-major) and its
  // model's measurement flip probabilities
  int rounds, msyn;
  const uint8_t* syn_rounds;
  const double* meas;
};

// XG: the LQ matrix X is in the work-group's global scratch, lay.xg bytes from
// gbase (a layout with lay.X < 0); else in LDS.  A compile-time choice, so that
// the accesses of either kind keep their address space.
template <typename Real, typename Fac, bool XG = false>
__device__ inline Work<Real, Fac> carve(uint8_t* smem, const LdsLayout& lay, int* flags, uint8_t* gbase = nullptr) {
  Work<Real, Fac> w;
  w.fbits = smem + lay.fbits;
  w.syn = smem + lay.syn;
  w.perm = reinterpret_cast<int*>(smem + lay.perm);
  w.dred = reinterpret_cast<double*>(smem + lay.red);
  w.nrm = reinterpret_cast<double*>(smem + lay.nrm);
  w.Wv = reinterpret_cast<Real*>(smem + lay.W);
  w.Aj = lay.Aj < 0 ? nullptr : reinterpret_cast<Real*>(smem + lay.Aj);
  w.T = reinterpret_cast<Real*>(smem + lay.T);
  w.T2 = (XG && lay.T2 >= 0) ? reinterpret_cast<Real*>(smem + lay.T2) : nullptr;
  w.L = reinterpret_cast<Real*>(smem + lay.L);
  w.C = reinterpret_cast<Real*>(smem + lay.C);
  if constexpr (XG) w.X = reinterpret_cast<Fac*>(gbase + lay.xg);
  else w.X = reinterpret_cast<Fac*>(smem + lay.X);
  w.tau = reinterpret_cast<Fac*>(smem + lay.tau);
  w.diag = reinterpret_cast<Fac*>(smem + lay.diag);
  w.vtmp = reinterpret_cast<Fac*>(smem + lay.v);
  w.Mm = reinterpret_cast<Fac*>(smem + lay.M);
  w.Vv = reinterpret_cast<Fac*>(smem + lay.V);
  w.Lt = reinterpret_cast<Fac*>(smem + lay.Lt);
  w.sig = reinterpret_cast<Fac*>(smem + lay.sig);
  w.s_flag = flags;
  w.s_dead = flags + 1;
  w.rounds = 1;
  w.msyn = 0;
  w.syn_rounds = nullptr;
  w.meas = nullptr;
  return w;
}

// Reference error of coset mlog (paper Sec. 3.2.1: the representative
// E_{l,s} whose stabiliser multiples are summed): fbits[q] = (x | z << 1) of
// R(s) * L_m.  Returns the class index the result belongs to.  Collective.
__device__ inline int prep_reference(const PlanHeader* H, const CheckDesc* checks, const uint8_t* syn_g, int mlog,
                                     uint8_t* syn, uint8_t* fbits, int* s_label) {
  const int d = H->d, n = H->n, m = H->m, tid = threadIdx.x;
  for (int j = tid; j < m; j += NT) syn[j] = syn_g[j];
  __syncthreads();
  for (int q = tid; q < n; q += NT) {
    const int r = q / d, c = q % d;
    int x = 0, z = 0;
    for (int j = 0; j < m; ++j) {
      if (!syn[j]) continue;
      const CheckDesc cd = checks[j];
      if (cd.type == 1) {
        if (c == cd.line && r >= cd.from && r <= cd.to) x ^= 1;
      } else {
        if (r == cd.line && c >= cd.from && c <= cd.to) z ^= 1;
      }
    }
    fbits[q] = (uint8_t)(x | (z << 1));
  }
  __syncthreads();
  if (tid == 0) {
    int a = 0, bb = 0;  // class of R: x-parity on row 0, z-parity on column 0
    for (int c = 0; c < d; ++c) a ^= fbits[c] & 1;
    for (int r = 0; r < d; ++r) bb ^= fbits[r * d] >> 1;
    // logical representatives: X on column lx_col has class X (it crosses row 0
    // once), Z on row lz_row has class Z (it crosses column 0 once)
    const int lx = (mlog == 1 || mlog == 2), lz = (mlog == 2 || mlog == 3);
    *s_label = pauli_code(a ^ lx, bb ^ lz);
  }
  __syncthreads();
  for (int q = tid; q < n; q += NT) {
    const int r = q / d, c = q % d;
    int fb = fbits[q];
    if ((mlog == 1 || mlog == 2) && c == H->lx_col) fb ^= 1;
    if ((mlog == 2 || mlog == 3) && r == H->lz_row) fb ^= 2;
    fbits[q] = (uint8_t)fb;
  }
  __syncthreads();
  return *s_label;
}

// All-ones product state: site J is 1 x dims[J] x 1.  Collective.
template <typename Real>
__device__ inline void mps_ones(Real* scr, const int64_t* region, const uint8_t* dims, int nsite) {
  for (int J = 0; J < nsite; ++J)
    for (int e = threadIdx.x; e < dims[J]; e += NT) scr[region[J] + e] = Real(1);
  __syncthreads();
}

// One row of the boundary-MPS sweep on the MPS stored at scr + region[J]:
// apply the row MPO (transposed when row[J].tr), bring the product to
// right-canonical form (right-to-left LQ), then move the centre back
// left-to-right by QR, truncating the bonds the plan cuts by SVD.  The MPS is
// left normalised; log-norms go to `logscale`.  Returns false when the state
// vanished (the coset has probability zero).  XG: the LQ matrix is in global
// scratch (carve<..., true>).  Collective.
template <typename Real, typename Fac, int GM, bool XG = false>
__device__ bool row_step(const SiteStep* row, int nsite, const uint8_t* codes, const double* rates, Real* scr,
                         const int64_t* region, Work<Real, Fac>& w, double& logscale) {
  const int tid = threadIdx.x;
  // the work areas are LDS (X global scratch when XG): said explicitly, so that
  // an out-of-line copy (the adjoint's) keeps DS instructions for them
  uint8_t* fbits = in_lds(w.fbits);
  int* perm = in_lds(w.perm);
  double* dred = in_lds(w.dred);
  Real *Wv = in_lds(w.Wv), *Aj = w.Aj ? in_lds(w.Aj) : nullptr, *T = in_lds(w.T), *L = in_lds(w.L),
       *C = in_lds(w.C), *T2 = (XG && w.T2) ? in_lds(w.T2) : nullptr;
  Fac *X = XG ? in_global(w.X) : in_lds(w.X), *tau = in_lds(w.tau), *diag = in_lds(w.diag), *vtmp = in_lds(w.vtmp),
      *Mm = in_lds(w.Mm), *Vv = in_lds(w.Vv), *Lt = in_lds(w.Lt), *sig = in_lds(w.sig);
  int* s_dead = in_lds(w.s_dead);
  // BF16 forms: T and L reach the T.L GEMM as bf16 planes, rounded (and, for
  // the split form, split into hi/lo) once when they are written (T row-major,
  // L transposed; rows padded to 8)
#ifndef TNMLD_EMU
  constexpr bool PL = (GM == GEMM_BF16 || GM == GEMM_BF16X3) && sizeof(Real) == 4;
#else
  constexpr bool PL = false;
#endif
  constexpr bool SPL = GM == GEMM_BF16X3;  // the low planes are written and read
  if (tid == 0) s_dead[0] = 0;
  __syncthreads();
  do {
    // --- right-to-left: MPO apply + LQ --------------------------------------
    if constexpr (PL) {  // 1 x 1 carry = 1: one row of 8 (bf16 one = 0x3f80)
      uint16_t* Lh = reinterpret_cast<uint16_t*>(L);
      if (tid < 16) Lh[tid] = tid == 0 ? uint16_t(0x3f80) : uint16_t(0);
    } else {
      if (tid == 0) L[0] = Real(1);
    }
    __syncthreads();
    for (int J = nsite - 1; J >= 0; --J) {
      const SiteStep st = row[J];
      const int A = st.A, B = st.B, qi = st.qi, qo = st.qo;
      const int Dl = st.Dl_old, Dr = st.Dr_old, mJ = st.m, k = st.k, kr = st.kr;
      const int RB = Dr * B, nn = qo * kr;
      const int ncode = A * qi * qo * B;
      const uint8_t* cd = codes + st.wofs;
      for (int e = tid; e < ncode; e += NT) {
        // plan order [a][si][so][b]; a transposed row reads the forward code [a][so][si][b]
        int ci = e;
        if (st.tr) {
          const int bb = e % B, so = (e / B) % qo, si = (e / (B * qo)) % qi, a = e / (B * qo * qi);
          ci = ((a * qo + so) * qi + si) * B + bb;
        }
        const int c = cd[ci];
        Real v = Real(0);
        if (w.rounds <= 1) {
          if (c == W_ONE) v = Real(1);
          else if (c >= W_PAULI) v = pauli_weight<Real>(rates + 3 * st.q, fbits[st.q], c - W_PAULI);
        } else if (c != W_ZERO) {
          // forward rows only (the gradient takes one round)
          const int so = (e / B) % qo, si = (e / (B * qo)) % qi;
          double x = c == W_ONE ? 1.0 : rounds_tensor(rates + 3 * st.q, fbits[st.q], c - W_PAULI, w.rounds);
          if (st.wnew >= 0) x *= rounds_check_weight(w.meas, w.syn_rounds, w.msyn, st.wnew, so, w.rounds);
          if (st.wold >= 0) x *= rounds_check_weight(w.meas, w.syn_rounds, w.msyn, st.wold, si, w.rounds);
          v = Real(x);
        }
        Wv[e] = v;
      }
      Real* g = scr + region[J];
      const Real* As = Aj ? Aj : g;  // LDS copy, or the site region itself (its L2 lines)
      if (Aj)
        for (int e = tid; e < Dl * qi * Dr; e += NT) Aj[e] = g[e];
      __syncthreads();
      const int ldp = (RB + 7) & ~7;  // plane row length (BF16 form)
      const int sA = A == 4 ? 2 : (A == 2 ? 1 : 0), sB = B == 4 ? 2 : (B == 2 ? 1 : 0);
      for (int so = 0; so < qo;) {
        // T[(l,a)][(r,b)] = sum_si Aj[l][si][r] W[a][si][so][b]
        // (A and B, the MPO bonds, are 1, 2 or 4); with a second T slice in
        // LDS (the layouts with the LQ matrix in scratch have room for one),
        // slices so and so + 1 in one pass, sharing the loads of Aj (each
        // slice's sum is formed as when built alone)
        const bool two = XG && T2 && so + 1 < qo;
        auto tval = [&](int la, int rb, int s) {
          const int l = la >> sA, a = la & (A - 1), r = rb >> sB, bb = rb & (B - 1);
          Real acc = 0;
          for (int si = 0; si < qi; ++si)
            acc += As[(l * qi + si) * Dr + r] * Wv[((a * qi + si) * qo + s) * B + bb];
          return acc;
        };
        auto tval2 = [&](int la, int rb, Real& v0, Real& v1) {
          const int l = la >> sA, a = la & (A - 1), r = rb >> sB, bb = rb & (B - 1);
          Real acc0 = 0, acc1 = 0;
          for (int si = 0; si < qi; ++si) {
            const Real x = As[(l * qi + si) * Dr + r];
            acc0 += x * Wv[((a * qi + si) * qo + so) * B + bb];
            acc1 += x * Wv[((a * qi + si) * qo + so + 1) * B + bb];
          }
          v0 = acc0;
          v1 = acc1;
        };
        if constexpr (PL) {
#ifndef TNMLD_EMU
          uint16_t* Th = reinterpret_cast<uint16_t*>(T);
          uint16_t* Tl = Th + mJ * ldp;
          uint16_t* Th2 = reinterpret_cast<uint16_t*>(T2);
          uint16_t* Tl2 = Th2 + mJ * ldp;
          if (two) {
            for_2d(mJ, ldp, [&](int la, int rb) {
              Real v0 = Real(0), v1 = Real(0);
              if (rb < RB) tval2(la, rb, v0, v1);
              uint16_t h, l;
              split_bf16(float(v0), h, l);
              Th[la * ldp + rb] = h;
              if constexpr (SPL) Tl[la * ldp + rb] = l;
              split_bf16(float(v1), h, l);
              Th2[la * ldp + rb] = h;
              if constexpr (SPL) Tl2[la * ldp + rb] = l;
            });
          } else {
            for_2d(mJ, ldp, [&](int la, int rb) {
              uint16_t h, l;
              split_bf16(rb < RB ? float(tval(la, rb, so)) : 0.0f, h, l);
              Th[la * ldp + rb] = h;
              if constexpr (SPL) Tl[la * ldp + rb] = l;
            });
          }
          __syncthreads();
          // X[:, so*kr + c] = T . L
          const uint16_t* Lh = reinterpret_cast<const uint16_t*>(L);
          gemm_mfma_planes<GM == GEMM_BF16X3>(mJ, kr, RB, Th, Tl, ldp, Lh, Lh + kr * ldp, ldp,
                           [&](int i, int j, float v) { X[i * nn + so * kr + j] = Fac(v); });
          if (two)
            gemm_mfma_planes<GM == GEMM_BF16X3>(mJ, kr, RB, Th2, Tl2, ldp, Lh, Lh + kr * ldp, ldp,
                             [&](int i, int j, float v) { X[i * nn + (so + 1) * kr + j] = Fac(v); });
#endif
        } else {
          if (two) {
            for_2d(mJ, RB, [&](int la, int rb) { tval2(la, rb, T[la * RB + rb], T2[la * RB + rb]); });
          } else {
            for_2d(mJ, RB, [&](int la, int rb) { T[la * RB + rb] = tval(la, rb, so); });
          }
          __syncthreads();
          // X[:, so*kr + c] = T . L
          contract_gemm<GM, Real>(mJ, kr, RB, T, RB, L, kr, 0, 0,
                                  [&](int i, int j, Real v) { X[i * nn + so * kr + j] = Fac(v); });
          if (two)
            contract_gemm<GM, Real>(mJ, kr, RB, T2, RB, L, kr, 0, 0,
                                    [&](int i, int j, Real v) { X[i * nn + (so + 1) * kr + j] = Fac(v); });
        }
        __syncthreads();
        so += two ? 2 : 1;
      }
      lq_factor_any<Fac, XG>(X, mJ, nn, nn, tau, diag, dred, vtmp);
      // L (mJ x k) for the site to the left
      auto lval = [&](int r, int c) { return c < r ? X[r * nn + c] : (c == r ? diag[r] : Fac(0)); };
      if (PL && J > 0) {
#ifndef TNMLD_EMU
        // as the left site's B operand: transposed, k rows of pad8(mJ)
        const int ldw = (mJ + 7) & ~7;
        uint16_t* Lh = reinterpret_cast<uint16_t*>(L);
        for_2d(k, ldw, [&](int c, int r) {
          uint16_t h, l;
          split_bf16(r < mJ ? float(lval(r, c)) : 0.0f, h, l);
          Lh[c * ldw + r] = h;
          if constexpr (SPL) Lh[k * ldw + c * ldw + r] = l;
        });
#endif
      } else {
        for_2d(mJ, k, [&](int r, int c) { L[r * k + c] = Real(lval(r, c)); });
      }
      __syncthreads();
      bool staged = false;
      if constexpr (XG && sizeof(Fac) == 4) {
        // X in global scratch (FP32 factorisations: the plans that need it):
        // the reflectors are staged through LDS in chunks and the rows of Q
        // written straight to the site region.  The chunks use the LDS of the
        // input site's copy and of T, both dead by now (L, the next site's
        // carry, comes after them); at least the two rows of vtmp.
        if (lq_regs_fit<Fac>(mJ, nn)) {
          const int W = nn <= 128 ? 128 : 256;
          uint8_t* b0 = reinterpret_cast<uint8_t*>(Aj ? Aj : T);
          Fac* buf = reinterpret_cast<Fac*>(b0);
          int cap = (int)((reinterpret_cast<uint8_t*>(L) - b0) / (W * (int)sizeof(Fac)));
          if (cap < 2) {
            buf = vtmp;
            cap = 2;
          }
          if (nn <= 128)
            lq_form_q_staged<Fac, Real, 8>((const glb_t<Fac>*)X, mJ, nn, nn, (const lds_t<Fac>*)tau,
                                           (lds_t<Fac>*)buf, cap, (glb_t<Real>*)g, nn);
          else if constexpr (kMaxNpl >= 16)
            lq_form_q_staged<Fac, Real, 16>((const glb_t<Fac>*)X, mJ, nn, nn, (const lds_t<Fac>*)tau,
                                            (lds_t<Fac>*)buf, cap, (glb_t<Real>*)g, nn);
          staged = true;
        }
      }
      if (!staged) {
        lq_form_q_any<Fac>(X, mJ, nn, nn, tau, vtmp);
        for (int e = tid; e < k * nn; e += NT) g[e] = Real(X[e]);
      }
      __syncthreads();
    }
    // L is 1x1: the norm of the MPO-applied state
    {
      const Real l0 = L[0];
      __syncthreads();
      if (!(fabs((double)l0) > 0.0)) {
        if (tid == 0) s_dead[0] = 1;
      } else {
        logscale += log(fabs((double)l0));
        if (tid == 0) C[0] = l0 > Real(0) ? Real(1) : Real(-1);
      }
      __syncthreads();
      if (s_dead[0]) break;
    }
    // --- left-to-right: QR of every site matrix, SVD where the bond is cut ----
    for (int J = 0; J < nsite; ++J) {
      const SiteStep st = row[J];
      const int qo = st.qo, k = st.k, kr = st.kr, Dl = st.Dl_new, Dn = st.Dr_new;
      const int nn = qo * kr, R = Dl * qo;
      const int ldm = R + 1, ldl = kr + 1;
      const int k2 = R < kr ? R : kr;  // rank of the site matrix
      const bool cut = Dn < k2;
      Real* g = scr + region[J];
      // M[(l,so)][c] = sum_k C[l][k] Q[k][so][c] (Q read from the site region),
      // stored as M^T rows: Mm[c*ldm + (l,so)]
      contract_gemm<GM, Real>(Dl, nn, k, C, k, g, nn, 0, 0, [&](int i, int j, Real v) {
        int so = 0, c = j;  // j = so * kr + c with so < qo <= 4
        while (c >= kr) {
          c -= kr;
          ++so;
        }
        Mm[c * ldm + i * qo + so] = Fac(v);
      });
      __syncthreads();
      // M^T = Lf Qf (LQ), i.e. M = Qf^T Lf^T: a QR factorisation of M
      lq_factor_any<Fac>(Mm, kr, R, ldm, tau, diag, dred, vtmp);
      // Lf (kr x k2) -> Lt, column-major (column j at Lt + j*ldl)
      for_2d(kr, k2, [&](int r, int c) { Lt[c * ldl + r] = c < r ? Mm[r * ldm + c] : (c == r ? diag[r] : Fac(0)); });
      __syncthreads();
      lq_form_q_any<Fac>(Mm, kr, R, ldm, tau, vtmp);  // rows 0..k2-1 of Mm: Qf (k2 x R)
      if (!cut) {
        // A[(l,so)][r] = Qf[r][(l,so)], carry C[r][c] = Lf[c][r]
        for_2d(R, Dn, [&](int lso, int r) { g[lso * Dn + r] = Real(Mm[r * ldm + lso]); });
        for_2d(Dn, kr, [&](int r, int c) { C[r * kr + c] = Real(Lt[r * ldl + c]); });
        __syncthreads();
        if (J == nsite - 1) {
          // last site: 1x1 carry = remaining norm (sign folded into the site)
          const double l0 = (double)Lt[0];
          if (!(fabs(l0) > TinyNorm<Fac>::v)) {
            if (tid == 0) s_dead[0] = 1;
          } else {
            logscale += log(fabs(l0));
            if (l0 < 0.0)
              for (int e = tid; e < R; e += NT) g[e] = -g[e];
          }
          __syncthreads();
        }
      } else {
        // one-sided Jacobi on the columns of Lf: Lf W = U' S, so that
        // M = (Qf^T W) S U'^T; keep the Dn largest singular values
        for_2d(k2, k2, [&](int r, int c) { Vv[r * ldl + c] = r == c ? Fac(1) : Fac(0); });
        __syncthreads();
        // the data carry the rounding of the storage type Real, whatever Fac is
        jacobi_svd<Fac>(Lt, kr, k2, ldl, Vv, ldl, SplitTol<Fac>::v, (double)Eps<Real>::v, in_lds(w.s_flag), dred,
                        in_lds(w.nrm), perm);
        for (int c = tid; c < k2; c += NT) {
          double s2 = 0;
          for (int r = 0; r < kr; ++r) s2 += (double)Lt[c * ldl + r] * (double)Lt[c * ldl + r];
          sig[c] = Fac(sqrt(s2));
        }
        __syncthreads();
        for (int c = tid; c < k2; c += NT) {
          const Fac sc = sig[c];
          int rank = 0;
          for (int c2 = 0; c2 < k2; ++c2) {
            const Fac s2 = sig[c2];
            rank += (s2 > sc) || (s2 == sc && c2 < c);
          }
          perm[rank] = c;
        }
        __syncthreads();
        // A[(l,so)][r] = sum_c Qf[c][(l,so)] W[c][perm r];  C[r][c'] = (Lf W)[c'][perm r]
#ifndef TNMLD_EMU
        if constexpr (GM == GEMM_BF16 || GM == GEMM_BF16X3) {
          // a GEMM (R x k2) . (k2 x Dn): on the bf16 matrix cores like the other contractions of this form
          gemm_mfma_bf16<GM == GEMM_BF16X3>(
              R, Dn, k2, [&](int lso, int c) { return (float)Mm[c * ldm + lso]; },
              [&](int c, int r) { return (float)Vv[perm[r] * ldl + c]; },
              [&](int lso, int r, float v) { g[lso * Dn + r] = Real(v); });
        } else if constexpr (GM == GEMM_F64 && sizeof(Fac) == 8) {
          gemm_mfma_f64(
              1, R, Dn, k2, [&](int, int lso, int c) { return (double)Mm[c * ldm + lso]; },
              [&](int, int c, int r) { return (double)Vv[perm[r] * ldl + c]; },
              [&](int, int lso, int r, double v) { g[lso * Dn + r] = Real(v); });
        } else if constexpr (GM == GEMM_F32 && sizeof(Fac) == 4) {
          // FP32 factorisations: the FP32 matrix cores (with FP64 ones this
          // product belongs to the FP64 truncation and stays below)
          gemm_mfma_f32(
              1, R, Dn, k2, [&](int, int lso, int c) { return (float)Mm[c * ldm + lso]; },
              [&](int, int c, int r) { return (float)Vv[perm[r] * ldl + c]; },
              [&](int, int lso, int r, float v) { g[lso * Dn + r] = Real(v); });
        } else
#endif
        {
          for_2d(R, Dn, [&](int lso, int r) {
            const Fac* w = Vv + perm[r] * ldl;
            Fac acc = 0;
            for (int c = 0; c < k2; ++c) acc += Mm[c * ldm + lso] * w[c];
            g[lso * Dn + r] = Real(acc);
          });
        }
        for_2d(Dn, kr, [&](int r, int c) { C[r * kr + c] = Real(Lt[perm[r] * ldl + c]); });
        __syncthreads();
      }
      if (s_dead[0]) break;
    }
  } while (0);
  const bool alive = !s_dead[0];
  __syncthreads();
  return alive;
}

// Out-of-line copy of row_step for callers that run it from several places
// (the adjoint): one body instead of three inlined ones keeps register
// pressure, and with it spilling, down.
template <typename Real, typename Fac, int GM>
__device__ __attribute__((noinline)) bool row_step_outlined(const SiteStep* row, int nsite, const uint8_t* codes,
                                                            const double* rates, Real* scr, const int64_t* region,
                                                            Work<Real, Fac>& w, double& logscale) {
  return row_step<Real, Fac, GM>(row, nsite, codes, rates, scr, region, w, logscale);
}

// Sum of the MPS over every physical index (the closing all-ones boundary);
// returns log of it (FP64), -inf when not positive.  Collective.
template <typename Real, typename Fac>
__device__ inline double mps_close(const Real* scr, const int64_t* region, const int16_t* dims, int nsite, Fac* vacc) {
  const int tid = threadIdx.x;
  if (tid == 0) vacc[0] = Fac(1);
  __syncthreads();
  for (int J = 0; J < nsite; ++J) {
    const int Dl = dims[3 * J], qo = dims[3 * J + 1], Dr = dims[3 * J + 2];
    const Real* g = scr + region[J];
    Fac acc = 0;
    if (tid < Dr)
      for (int l = 0; l < Dl; ++l) {
        Fac s = 0;
        for (int so = 0; so < qo; ++so) s += Fac(g[(l * qo + so) * Dr + tid]);
        acc += vacc[l] * s;
      }
    __syncthreads();
    if (tid < Dr) vacc[tid] = acc;
    __syncthreads();
  }
  const double tot = (double)vacc[0];
  __syncthreads();
  return tot > 0.0 ? log(tot) : -INFINITY;
}

// Copy an MPS between the site regions and a compact buffer (sites back to
// back, Dl*q*Dr elements each).  dims(J) -> (Dl, q, Dr).  Collective.
template <typename Real, typename Dims>
__device__ inline void mps_pack(const Real* scr, const int64_t* region, int nsite, Dims dims, Real* out, bool to_regions,
                                Real* regions_out) {
  int64_t off = 0;
  for (int J = 0; J < nsite; ++J) {
    int Dl, q, Dr;
    dims(J, Dl, q, Dr);
    const int sz = Dl * q * Dr;
    if (to_regions)
      for (int e = threadIdx.x; e < sz; e += NT) regions_out[region[J] + e] = out[off + e];
    else
      for (int e = threadIdx.x; e < sz; e += NT) out[off + e] = scr[region[J] + e];
    off += sz;
  }
  __syncthreads();
}

// Forward contraction of the four cosets of syndrome b.  The rows before
// H->shared_rows touch no qubit of the logical representatives, so they are
// contracted once; the MPS after them is saved to snap (mps_elems) and each
// coset continues from it.  Writes logz[b][label] for the four cosets; a
// prefix that vanishes makes all four -inf.  XG: the layout keeps the LQ matrix
// in global scratch (lay.X < 0, lay.xg bytes from scr).  Collective.
template <typename Real, typename Fac, int GM = GEMM_VALU, bool XG = false>
__device__ void contract_syndrome(const JobDev& job, int64_t b, uint8_t* smem, const LdsLayout& lay, Real* scr,
                                  Real* snap) {
  const uint8_t* plan = job.plan;
  const PlanHeader* H = reinterpret_cast<const PlanHeader*>(plan);
  const int n = H->n, m = H->m, nsite = H->nsite, nstep = H->nstep;
  const int ushare = H->shared_rows < nstep ? H->shared_rows : nstep;
  const SiteStep* steps = reinterpret_cast<const SiteStep*>(plan + H->steps_ofs);
  const uint8_t* codes = plan + H->codes_ofs;
  const CheckDesc* checks = reinterpret_cast<const CheckDesc*>(plan + H->checks_ofs);
  const int64_t* region = reinterpret_cast<const int64_t*>(plan + H->region_ofs);
  const int16_t* fin = reinterpret_cast<const int16_t*>(plan + H->final_ofs);
  __shared__ int s_flags[2];
  __shared__ int s_label;
  Work<Real, Fac> w = carve<Real, Fac, XG>(smem, lay, s_flags, reinterpret_cast<uint8_t*>(scr));
  const ItemCheck ck = check_item(job, b, n, m);
  if (!ck.valid) {  // defined outputs (Z = 0 for every coset) and the status bit
    if (threadIdx.x < 4) job.logz[b * 4 + threadIdx.x] = -INFINITY;
    __syncthreads();
    return;
  }
  const double* rates = job.rates + (int64_t)ck.model * n * 3;
  // the reference error comes from the last (perfect) round's syndrome
  const int R = job_rounds(job);
  const uint8_t* syn_b = job.syn + b * (int64_t)m * R;
  const uint8_t* syn_last = syn_b + (int64_t)(R - 1) * m;
  if (R > 1) {
    w.rounds = R;
    w.msyn = m;
    w.syn_rounds = syn_b;
    w.meas = job.meas + (int64_t)ck.model * m;
  }
  const SiteStep* rowS = steps + (int64_t)ushare * nsite;
  auto dims = [rowS](int J, int& Dl, int& q, int& Dr) {
    Dl = rowS[J].Dl_old;
    q = rowS[J].qi;
    Dr = rowS[J].Dr_old;
  };
  // common prefix (coset 0's reference error; the others differ only later)
  prep_reference(H, checks, syn_last, 0, w.syn, w.fbits, &s_label);
  mps_ones(scr, region, plan + H->init_qi_ofs, nsite);
  double base = 0.0;
  bool alive = true;
  for (int u = 0; u < ushare && alive; ++u)
    alive = row_step<Real, Fac, GM, XG>(steps + (int64_t)u * nsite, nsite, codes, rates, scr, region, w, base);
  if (!alive) {
    for (int mlog = 0; mlog < 4; ++mlog) {
      const int label = prep_reference(H, checks, syn_last, mlog, w.syn, w.fbits, &s_label);
      if (threadIdx.x == 0) job.logz[b * 4 + label] = -INFINITY;
      __syncthreads();
    }
    if (threadIdx.x == 0) report_dead(4, ck, job);
    return;
  }
  if (ushare < nstep) mps_pack(scr, region, nsite, dims, snap, false, scr);
  int dead = 0;  // thread 0: cosets written as -inf
  for (int mlog = 0; mlog < 4; ++mlog) {
    if (mlog > 0) mps_pack(scr, region, nsite, dims, snap, true, scr);
    const int label = prep_reference(H, checks, syn_last, mlog, w.syn, w.fbits, &s_label);
    double logscale = base;
    bool ok = true;
    for (int u = ushare; u < nstep && ok; ++u)
      ok = row_step<Real, Fac, GM, XG>(steps + (int64_t)u * nsite, nsite, codes, rates, scr, region, w, logscale);
    const double lz = finish_logz(ok ? logscale + mps_close<Real, Fac>(scr, region, fin, nsite, w.sig) : -INFINITY);
    if (threadIdx.x == 0) {
      job.logz[b * 4 + label] = lz;
      dead += lz == -INFINITY;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) report_dead(dead, ck, job);
}


}  // namespace tnmld
