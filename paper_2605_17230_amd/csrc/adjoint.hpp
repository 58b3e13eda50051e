// Gradient of log Z_l(s) with respect to the per-qubit Pauli rates, by
// environments of the boundary-MPS contraction (paper Sec. 3.2.4: the
// contraction is differentiable in the local error probabilities).  With FP32
// data the GEMM-shaped environment contractions (top site with the left
// environment, bottom site with the right one, and the new environments) run
// on the FP32 matrix cores; the small ones (through the MPO values, inner
// size <= 8) and the derivative fold stay on the vector units.
//
// Z is linear in every qubit tensor, so d log Z / d w_q = Env_q / Z where
// Env_q is the network with the tensor of qubit q removed.  For the row u that
// holds qubit q:  Z ~ <Phi_u| T_u |Psi_{u-1}>, with Psi_{u-1} the top boundary
// MPS before row u, Phi_u the bottom boundary MPS contracted upwards through
// rows u+1.. with transposed row MPOs, and T_u the row MPO.  Left and right
// environments along the row give every site's derivative tensor; the overall
// scale cancels in the ratio.  The top sweep keeps Psi_{u-1} for every row
// (the rows common to the four cosets once), so the bottom MPS climbs back up
// with no recomputation of the top states.
#pragma once
#include "contract.hpp"

namespace tnmld {

// Environments of row u and the derivative of log Z with respect to the
// weights of every qubit on it.  top: compact Psi_{u-1} (dims of the forward
// row's input), bot: Phi_u in site regions (dims of the bottom-up row's
// input).  Accumulates weight * d log Z / d theta into part[q*3 + k].
// Returns false when the sandwich value <Phi_u| T_u |Psi_{u-1}> vanished
// (nothing is added).  The contraction temporaries, the two site tensors
// and the environment bonds of the current site are staged in LDS when the
// layout has room for them (lay.gP, gA, gF, gE, gR >= 0: the storage of the
// row steps, idle between them), else they live in the global P1..P3.
template <typename Real>
__device__ bool row_gradient(const SiteStep* frow, const SiteStep* brow, int nsite, const uint8_t* codes,
                             const double* rates, const uint8_t* fbits, const Real* top, const Real* bot,
                             const int64_t* region, Real* env, Real* P1g, Real* P2g, Real* P3g, Real* Wv,
                             double weight, double* part, uint8_t* smem, const LdsLayout& lay,
                             int64_t tmp_elems) {
  const int tid = threadIdx.x;
  // FP32 data: the GEMM-shaped contractions run on the matrix cores
#ifndef TNMLD_EMU
  constexpr bool MF = sizeof(Real) == 4;
#else
  constexpr bool MF = false;
#endif
  Real* P1 = lay.gP >= 0 ? reinterpret_cast<Real*>(smem + lay.gP) : P1g;
  Real* P2 = lay.gP >= 0 ? P1 + tmp_elems : P2g;
  Real* P3 = lay.gP >= 0 ? P2 + tmp_elems : P3g;
  const bool stage = lay.gA >= 0;
  Real* sA = stage ? reinterpret_cast<Real*>(smem + lay.gA) : nullptr;
  Real* sF = stage ? reinterpret_cast<Real*>(smem + lay.gF) : nullptr;
  Real* sE = stage ? reinterpret_cast<Real*>(smem + lay.gE) : nullptr;
  Real* sR = stage ? reinterpret_cast<Real*>(smem + lay.gR) : nullptr;
  auto copy_in = [&](Real* dst, const Real* src, int cnt) {
    for (int e = tid; e < cnt; e += NT) dst[e] = src[e];
  };
  // offsets: top sites (compact), left environments E_J (J = 0..nsite), right R_J
  __shared__ int64_t s_toff[64], s_eoff[65], s_roff[65];
  __shared__ double s_dw[64];
  if (tid == 0) {
    int64_t o = 0, e = 0;
    for (int J = 0; J < nsite; ++J) {
      s_toff[J] = o;
      o += (int64_t)frow[J].Dl_old * frow[J].qi * frow[J].Dr_old;
    }
    for (int J = 0; J <= nsite; ++J) {
      s_eoff[J] = e;
      const int dt = J < nsite ? frow[J].Dl_old : 1, a = J < nsite ? frow[J].A : 1, db = J < nsite ? brow[J].Dl_old : 1;
      e += (int64_t)dt * a * db;
    }
    for (int J = 0; J <= nsite; ++J) {
      s_roff[J] = e;
      const int dt = J < nsite ? frow[J].Dl_old : 1, a = J < nsite ? frow[J].A : 1, db = J < nsite ? brow[J].Dl_old : 1;
      e += (int64_t)dt * a * db;
    }
  }
  __syncthreads();
  // W of site J in plan order [a][si][so][b]
  auto load_w = [&](const SiteStep& st) {
    const int ncode = st.A * st.qi * st.qo * st.B;
    if (tid < ncode) {
      const int c = codes[st.wofs + tid];
      Real v = Real(0);
      if (c == W_ONE) v = Real(1);
      else if (c >= W_PAULI) v = pauli_weight<Real>(rates + 3 * st.q, fbits[st.q], c - W_PAULI);
      Wv[tid] = v;
    }
  };
  // physical dimensions are 1, 2 or 4 and MPO bonds 1 or 2: index splits are shifts
  auto lg = [](int x) { return x == 4 ? 2 : (x == 2 ? 1 : 0); };
  // P[a][lF][si][rA] = sum_lA E[lA][a][lF] A[lA][si][rA] (E of DlA x (Aa DlF), A of DlA x qi x DrA)
  auto contract_ea = [&](const Real* E, const Real* Aj, Real* P, int Aa, int DlF, int qi, int DlA, int DrA, int lqi) {
    if constexpr (MF) {
      const int me = Aa * DlF;
      gemm_mfma_f32(
          qi, me, DrA, DlA, [&](int, int i, int k) { return (float)E[k * me + i]; },
          [&](int si, int k, int j) { return (float)Aj[(k * qi + si) * DrA + j]; },
          [&](int si, int i, int j, float v) { P[(i * qi + si) * DrA + j] = Real(v); });
    } else {
      for_2d(Aa * DlF * qi, DrA, [&](int row, int rA) {
        const int si = row & (qi - 1), t = row >> lqi, a = t >= DlF ? 1 : 0, lF = t - a * DlF;
        Real acc = 0;
        for (int lA = 0; lA < DlA; ++lA) acc += E[(lA * Aa + a) * DlF + lF] * Aj[(lA * qi + si) * DrA + rA];
        P[row * DrA + rA] = acc;
      });
    }
  };
  // bond sizes of the environment at bond J (left of site J)
  auto envb = [&](int J) {
    const int dt = J < nsite ? frow[J].Dl_old : 1, a = J < nsite ? frow[J].A : 1, db = J < nsite ? brow[J].Dl_old : 1;
    return dt * a * db;
  };
  // --- left environments ---------------------------------------------------
  if (tid == 0) env[s_eoff[0]] = Real(1);
  __syncthreads();
  for (int J = 0; J < nsite; ++J) {
    const SiteStep st = frow[J];
    const int Aa = st.A, B = st.B, qi = st.qi, qo = st.qo;
    const int DlA = st.Dl_old, DrA = st.Dr_old, DlF = brow[J].Dl_old, DrF = brow[J].Dr_old;
    const Real* Aj = top + s_toff[J];
    const Real* Fj = bot + region[J];
    const Real* E = env + s_eoff[J];
    Real* En = env + s_eoff[J + 1];
    load_w(st);
    if (stage) {
      copy_in(sA, Aj, DlA * qi * DrA);
      copy_in(sF, Fj, DlF * qo * DrF);
      copy_in(sE, E, envb(J));
      Aj = sA;
      Fj = sF;
      E = sE;
    }
    __syncthreads();
    const int lqi = lg(qi), lqo = lg(qo), lB = lg(B);
    // P1[a][lF][si][rA] = sum_lA E[lA][a][lF] A[lA][si][rA]
    contract_ea(E, Aj, P1, Aa, DlF, qi, DlA, DrA, lqi);
    __syncthreads();
    // P2[lF][so][b][rA] = sum_{a,si} P1[a][lF][si][rA] W[a][si][so][b]
    for_2d(DlF * qo * B, DrA, [&](int row, int rA) {
      const int b = row & (B - 1), t = row >> lB, so = t & (qo - 1), lF = t >> lqo;
      Real acc = 0;
      for (int a = 0; a < Aa; ++a)
        for (int si = 0; si < qi; ++si)
          acc += P1[((a * DlF + lF) * qi + si) * DrA + rA] * Wv[((a * qi + si) * qo + so) * B + b];
      P2[row * DrA + rA] = acc;
    });
    __syncthreads();
    // En[rA][b][rF] = sum_{lF,so} P2[lF][so][b][rA] F[lF][so][rF]
    if constexpr (MF) {
      gemm_mfma_f32(
          B, DrA, DrF, DlF * qo, [&](int b, int i, int k) { return (float)P2[(k * B + b) * DrA + i]; },
          [&](int, int k, int j) { return (float)Fj[k * DrF + j]; },
          [&](int b, int i, int j, float v) { En[(i * B + b) * DrF + j] = Real(v); });
    } else {
      for_2d(DrA * B, DrF, [&](int row, int rF) {
        const int b = row & (B - 1), rA = row >> lB;
        Real acc = 0;
        for (int lF = 0; lF < DlF; ++lF)
          for (int so = 0; so < qo; ++so) acc += P2[((lF * qo + so) * B + b) * DrA + rA] * Fj[(lF * qo + so) * DrF + rF];
        En[row * DrF + rF] = acc;
      });
    }
    __syncthreads();
  }
  const double S = (double)env[s_eoff[nsite]];
  if (!(fabs(S) > 0.0)) return false;  // uniform: every thread read the same value
  // --- right environments and the derivative tensor of each site -----------
  if (tid == 0) env[s_roff[nsite]] = Real(1);
  __syncthreads();
  for (int J = nsite - 1; J >= 0; --J) {
    const SiteStep st = frow[J];
    const int Aa = st.A, B = st.B, qi = st.qi, qo = st.qo;
    const int DlA = st.Dl_old, DrA = st.Dr_old, DlF = brow[J].Dl_old, DrF = brow[J].Dr_old;
    const Real* Aj = top + s_toff[J];
    const Real* Fj = bot + region[J];
    const Real* R = env + s_roff[J + 1];
    const Real* E = env + s_eoff[J];
    Real* Rn = env + s_roff[J];
    load_w(st);
    if (stage) {
      copy_in(sA, Aj, DlA * qi * DrA);
      copy_in(sF, Fj, DlF * qo * DrF);
      copy_in(sR, R, envb(J + 1));
      copy_in(sE, E, envb(J));
      Aj = sA;
      Fj = sF;
      R = sR;
      E = sE;
    }
    __syncthreads();
    const int lqi = lg(qi), lqo = lg(qo), lB = lg(B), lA_ = lg(Aa);
    // P1r[lF][so][rA][b] = sum_rF F[lF][so][rF] R[rA][b][rF]
    if constexpr (MF) {
      const int nc = DrA * B;
      gemm_mfma_f32(
          1, DlF * qo, nc, DrF, [&](int, int i, int k) { return (float)Fj[i * DrF + k]; },
          [&](int, int k, int j) { return (float)R[j * DrF + k]; },
          [&](int, int i, int j, float v) { P1[i * nc + j] = Real(v); });
    } else {
      for_2d(DlF * qo, DrA * B, [&](int row, int col) {
        const int b = col & (B - 1), rA = col >> lB;
        Real acc = 0;
        for (int rF = 0; rF < DrF; ++rF) acc += Fj[row * DrF + rF] * R[(rA * B + b) * DrF + rF];
        P1[row * (DrA * B) + col] = acc;
      });
    }
    __syncthreads();
    if (st.q >= 0) {
      // P3[a][lF][si][rA] = sum_lA E[lA][a][lF] A[lA][si][rA]
      contract_ea(E, Aj, P3, Aa, DlF, qi, DlA, DrA, lqi);
      __syncthreads();
      // G[a][si][so][b] = sum_{lF,rA} P3[a][lF][si][rA] P1r[lF][so][rA][b] / (sandwich value):
      // 8 lanes per entry split the (lF, rA) sum and add their parts in a fixed order
      const int ng = Aa * qi * qo * B;
      const int len = DlF * DrA;
      for (int e0 = 0; e0 < ng; e0 += NT / 8) {
        const int e = e0 + tid / 8, sub = tid & 7;
        double acc = 0;
        if (e < ng) {
          const int b = e & (B - 1), so = (e >> lB) & (qo - 1), si = (e >> (lB + lqo)) & (qi - 1),
                    a = e >> (lB + lqo + lqi);
          for (int x = sub; x < len; x += 8) {
            const int lF = x / DrA, rA = x - lF * DrA;
            acc += (double)P3[((a * DlF + lF) * qi + si) * DrA + rA] * (double)P1[((lF * qo + so) * DrA + rA) * B + b];
          }
        }
        acc = group_sum(acc, 8);
        if (e < ng && sub == 0) s_dw[e] = acc / S;
      }
      __syncthreads();
      if (tid == 0) {
        // d log Z / d wtab[P] = sum of G over the entries whose code is P
        double dw[4] = {0, 0, 0, 0};
        for (int e = 0; e < ng; ++e) {
          const int c = codes[st.wofs + e];
          if (c >= W_PAULI) dw[c - W_PAULI] += s_dw[e];
        }
        // wtab[P] = p(f xor P): d/dp[E] = d/dwtab[E xor f]
        const int fb = fbits[st.q];
        double dp[4];
        for (int E2 = 0; E2 < 4; ++E2) {
          const int x = pauli_x(E2) ^ (fb & 1), z = pauli_z(E2) ^ (fb >> 1);
          dp[E2] = dw[pauli_code(x, z)];
        }
        const double* rq = rates + 3 * st.q;
        for (int k = 0; k < 3; ++k) part[3 * st.q + k] += weight * rq[k] * (dp[k + 1] - dp[0]);
      }
      __syncthreads();
    }
    // P2r[a][lF][si][rA] = sum_{so,b} P1r[lF][so][rA][b] W[a][si][so][b]
    for_2d(Aa * DlF * qi, DrA, [&](int row, int rA) {
      const int si = row & (qi - 1), t = row >> lqi, a = t >= DlF ? 1 : 0, lF = t - a * DlF;
      Real acc = 0;
      for (int so = 0; so < qo; ++so)
        for (int b = 0; b < B; ++b) acc += P1[((lF * qo + so) * DrA + rA) * B + b] * Wv[((a * qi + si) * qo + so) * B + b];
      P2[row * DrA + rA] = acc;
    });
    __syncthreads();
    // Rn[lA][a][lF] = sum_{si,rA} A[lA][si][rA] P2r[a][lF][si][rA]
    if constexpr (MF) {
      const int kq = qi * DrA;
      gemm_mfma_f32(
          Aa, DlA, DlF, kq, [&](int, int i, int k) { return (float)Aj[i * kq + k]; },
          [&](int a, int k, int j) { return (float)P2[(a * DlF + j) * kq + k]; },
          [&](int a, int i, int j, float v) { Rn[(i * Aa + a) * DlF + j] = Real(v); });
    } else {
      for_2d(DlA * Aa, DlF, [&](int row, int lF) {
        const int a = row & (Aa - 1), lA = row >> lA_;
        Real acc = 0;
        for (int si = 0; si < qi; ++si)
          for (int rA = 0; rA < DrA; ++rA) acc += Aj[(lA * qi + si) * DrA + rA] * P2[((a * DlF + lF) * qi + si) * DrA + rA];
        Rn[row * DlF + lF] = acc;
      });
    }
    __syncthreads();
  }
  return true;
}

// Backward of syndrome b over its four cosets.  The top-down sweep runs here
// (the rows before H->shared_rows once, as in the forward pass, then each
// coset from the state after them), storing the MPS before every row; its log
// Z values give the coset weights grad_logp[b] * P(l|s).  Then each coset
// with a non-zero weight sweeps a second MPS up from the bottom with
// transposed row MPOs and contracts the environments of every row against
// the stored top state: nothing is recomputed.  Scratch layout (Real
// elements): top regions | bottom regions | stored states (the shared rows
// once, then nstep - S per coset; mps_elems each) | environments | three
// temporaries.  write_fwd: also write log Z and log P(s) of the item.
// mode: ADJ_FUSED both sweeps in this call; ADJ_TOP the top sweep only,
// its states stored in job.states (the caller's memory, states_stride
// elements per syndrome) and log Z / log P(s) written; ADJ_BOTTOM the bottom
// sweeps only, against the states and log Z / log P(s) an ADJ_TOP call left.
// Collective.
enum { ADJ_FUSED = 0, ADJ_TOP = 1, ADJ_BOTTOM = 2 };
template <typename Real, typename Fac, int GM>
__device__ void adjoint_syndrome(const JobDev& job, int64_t b, uint8_t* smem, const LdsLayout& lay, Real* scr,
                                 int write_fwd, double* part, int mode = ADJ_FUSED) {
  const uint8_t* plan = job.plan;
  const PlanHeader* H = reinterpret_cast<const PlanHeader*>(plan);
  const int n = H->n, m = H->m, nsite = H->nsite, nstep = H->nstep;
  const int S = H->shared_rows < nstep ? H->shared_rows : nstep;
  const SiteStep* steps = reinterpret_cast<const SiteStep*>(plan + H->steps_ofs);
  const SiteStep* bsteps = reinterpret_cast<const SiteStep*>(plan + H->bu_steps_ofs);
  const uint8_t* codes = plan + H->codes_ofs;
  const CheckDesc* checks = reinterpret_cast<const CheckDesc*>(plan + H->checks_ofs);
  const int64_t* region = reinterpret_cast<const int64_t*>(plan + H->region_ofs);
  const int16_t* fin = reinterpret_cast<const int16_t*>(plan + H->final_ofs);
  __shared__ int s_flags[2];
  __shared__ int s_label;
  __shared__ int s_lab[4];
  __shared__ double s_lz[4];
  __shared__ double s_weight[4];
  Work<Real, Fac> w = carve<Real, Fac>(smem, lay, s_flags);
  const ItemCheck ck = check_item(job, b, n, m);
  if (!ck.valid) {  // no contribution; the status word says why
    if (write_fwd && threadIdx.x < 4) job.logz[b * 4 + threadIdx.x] = -INFINITY;
    if (write_fwd && threadIdx.x == 0) const_cast<double*>(job.logp)[b] = -INFINITY;
    __syncthreads();
    return;
  }
  const int model = ck.model;
  const double* rates = job.rates + (int64_t)model * n * 3;
  const uint8_t* syn = job.syn + b * m;
  const int64_t se = H->scratch_elems, me = H->mps_elems;
  Real* top = scr;
  Real* bot = scr + se;
  Real* env = scr + 2 * se + (int64_t)(S + 4 * (nstep - S)) * me;
  Real* states = mode == ADJ_FUSED ? scr + 2 * se : reinterpret_cast<Real*>(job.states) + b * job.states_stride;
  Real* P1 = env + H->env_elems;
  Real* P2 = P1 + H->tmp_elems;
  Real* P3 = P2 + H->tmp_elems;
  auto state_of = [&](int mlog, int u) -> Real* {
    return states + (u < S ? (int64_t)u : (int64_t)S + (int64_t)mlog * (nstep - S) + (u - S)) * me;
  };
  auto in_dims = [&](const SiteStep* row) {
    return [row](int J, int& Dl, int& q, int& Dr) {
      Dl = row[J].Dl_old;
      q = row[J].qi;
      Dr = row[J].Dr_old;
    };
  };
  int dead = 0;  // thread 0: cosets with Z = 0
  if (mode != ADJ_BOTTOM) {
    // --- top-down: the shared rows once (the reference error of any coset
    // agrees on them), then each coset, storing the state before every row ---
    prep_reference(H, checks, syn, 0, w.syn, w.fbits, &s_label);
    mps_ones(top, region, plan + H->init_qi_ofs, nsite);
    double base = 0.0;
    bool alive = true;
    for (int u = 0; u < S && alive; ++u) {
      const SiteStep* row = steps + (int64_t)u * nsite;
      mps_pack(top, region, nsite, in_dims(row), state_of(0, u), false, top);
      alive = row_step_outlined<Real, Fac, GM>(row, nsite, codes, rates, top, region, w, base);
    }
    for (int mlog = 0; mlog < 4; ++mlog) {
      const int label = prep_reference(H, checks, syn, mlog, w.syn, w.fbits, &s_label);
      double logscale = base;
      bool ok = alive;
      if (ok && mlog > 0 && S < nstep)  // restart from the state after the shared rows
        mps_pack(top, region, nsite, in_dims(steps + (int64_t)S * nsite), state_of(0, S), true, top);
      for (int u = S; u < nstep && ok; ++u) {
        const SiteStep* row = steps + (int64_t)u * nsite;
        mps_pack(top, region, nsite, in_dims(row), state_of(mlog, u), false, top);
        ok = row_step_outlined<Real, Fac, GM>(row, nsite, codes, rates, top, region, w, logscale);
      }
      const double lz = finish_logz(ok ? logscale + mps_close<Real, Fac>(top, region, fin, nsite, w.sig) : -INFINITY);
      if (threadIdx.x == 0) {
        s_lz[mlog] = lz;
        s_lab[mlog] = label;
        dead += lz == -INFINITY;
      }
      __syncthreads();
    }
  } else {
    // log Z of the cosets from the call that stored the states
    for (int mlog = 0; mlog < 4; ++mlog) {
      const int label = prep_reference(H, checks, syn, mlog, w.syn, w.fbits, &s_label);
      if (threadIdx.x == 0) {
        s_lz[mlog] = job.logz[b * 4 + label];
        s_lab[mlog] = label;
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    double mx = -INFINITY;
    for (int k = 0; k < 4; ++k) mx = s_lz[k] > mx ? s_lz[k] : mx;
    double lp = -INFINITY;
    if (mx > -INFINITY) {
      double sum = 0.0;
      for (int k = 0; k < 4; ++k) sum += exp(s_lz[k] - mx);
      lp = mx + log(sum);
    }
    const double gp = mode == ADJ_TOP ? 0.0 : job.gradp[b];
    for (int k = 0; k < 4; ++k)
      s_weight[k] = (s_lz[k] > -INFINITY && lp > -INFINITY && gp != 0.0) ? gp * exp(s_lz[k] - lp) : 0.0;
    if (write_fwd) {
      for (int k = 0; k < 4; ++k) job.logz[b * 4 + s_lab[k]] = s_lz[k];
      const_cast<double*>(job.logp)[b] = lp;
      report_dead(dead, ck, job);
    }
  }
  __syncthreads();
  if (mode == ADJ_TOP) return;
  double* pm = part + (int64_t)model * n * 3;
  // --- bottom-up per coset, against the stored top states ------------------
  for (int mlog = 0; mlog < 4; ++mlog) {
    const double weight = s_weight[mlog];
    if (weight == 0.0) continue;
    prep_reference(H, checks, syn, mlog, w.syn, w.fbits, &s_label);
    for (int J = 0; J < nsite; ++J)  // all-ones over the final frontier
      for (int e = threadIdx.x; e < fin[3 * J + 1]; e += NT) bot[region[J] + e] = Real(1);
    __syncthreads();
    double bscale = 0.0;
    bool ok = true;
    for (int u = nstep - 1; u >= 0 && ok; --u) {
      const SiteStep* frow = steps + (int64_t)u * nsite;
      const SiteStep* brow = bsteps + (int64_t)(nstep - 1 - u) * nsite;
      if (!row_gradient<Real>(frow, brow, nsite, codes, rates, w.fbits, state_of(mlog, u), bot, region, env, P1, P2,
                              P3, w.Wv, weight, pm, smem, lay, H->tmp_elems) &&
          ck.positive && threadIdx.x == 0 && job.status)
        atomicOr(job.status, ST_NUMERIC);
      if (u > 0) ok = row_step_outlined<Real, Fac, GM>(brow, nsite, codes, rates, bot, region, w, bscale);
    }
  }
}

}  // namespace tnmld
