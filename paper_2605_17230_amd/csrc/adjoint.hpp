// Gradient of log Z_l(s) with respect to the per-qubit Pauli rates, by
// environments of the boundary-MPS contraction (paper Sec. 3.2.4: the
// contraction is differentiable in the local error probabilities).
//
// Z is linear in every qubit tensor, so d log Z / d w_q = Env_q / Z where
// Env_q is the network with the tensor of qubit q removed.  For the row u that
// holds qubit q:  Z ~ <Phi_u| T_u |Psi_{u-1}>, with Psi_{u-1} the top boundary
// MPS before row u, Phi_u the bottom boundary MPS contracted upwards through
// rows u+1.. with transposed row MPOs, and T_u the row MPO.  Left and right
// environments along the row give every site's derivative tensor; the overall
// scale cancels in the ratio.  Psi is checkpointed every K rows on the way
// down and each segment of K rows is recomputed from its checkpoint while the
// bottom MPS climbs back up.
#pragma once
#include "contract.hpp"

namespace tnmld {

// Environments of row u and the derivative of log Z with respect to the
// weights of every qubit on it.  top: compact Psi_{u-1} (dims of the forward
// row's input), bot: Phi_u in site regions (dims of the bottom-up row's
// input).  Accumulates weight * d log Z / d theta into part[q*3 + k].
// Returns false when the sandwich value <Phi_u| T_u |Psi_{u-1}> vanished
// (nothing is added).
template <typename Real>
__device__ bool row_gradient(const SiteStep* frow, const SiteStep* brow, int nsite, const uint8_t* codes,
                             const double* rates, const uint8_t* fbits, const Real* top, const Real* bot,
                             const int64_t* region, Real* env, Real* P1, Real* P2, Real* P3, Real* Wv,
                             double weight, double* part) {
  const int tid = threadIdx.x;
  // offsets: top sites (compact), left environments E_J (J = 0..nsite), right R_J
  __shared__ int64_t s_toff[64], s_eoff[65], s_roff[65];
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
    __syncthreads();
  };
  // physical dimensions are 1, 2 or 4 and MPO bonds 1 or 2: index splits are shifts
  auto lg = [](int x) { return x == 4 ? 2 : (x == 2 ? 1 : 0); };
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
    const int lqi = lg(qi), lqo = lg(qo), lB = lg(B);
    // P1[a][lF][si][rA] = sum_lA E[lA][a][lF] A[lA][si][rA]
    for_2d(Aa * DlF * qi, DrA, [&](int row, int rA) {
      const int si = row & (qi - 1), t = row >> lqi, a = t >= DlF ? 1 : 0, lF = t - a * DlF;
      Real acc = 0;
      for (int lA = 0; lA < DlA; ++lA) acc += E[(lA * Aa + a) * DlF + lF] * Aj[(lA * qi + si) * DrA + rA];
      P1[row * DrA + rA] = acc;
    });
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
    for_2d(DrA * B, DrF, [&](int row, int rF) {
      const int b = row & (B - 1), rA = row >> lB;
      Real acc = 0;
      for (int lF = 0; lF < DlF; ++lF)
        for (int so = 0; so < qo; ++so) acc += P2[((lF * qo + so) * B + b) * DrA + rA] * Fj[(lF * qo + so) * DrF + rF];
      En[row * DrF + rF] = acc;
    });
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
    const int lqi = lg(qi), lqo = lg(qo), lB = lg(B), lA_ = lg(Aa);
    // P1r[lF][so][rA][b] = sum_rF F[lF][so][rF] R[rA][b][rF]
    for_2d(DlF * qo, DrA * B, [&](int row, int col) {
      const int b = col & (B - 1), rA = col >> lB;
      Real acc = 0;
      for (int rF = 0; rF < DrF; ++rF) acc += Fj[row * DrF + rF] * R[(rA * B + b) * DrF + rF];
      P1[row * (DrA * B) + col] = acc;
    });
    __syncthreads();
    if (st.q >= 0) {
      // P3[a][lF][si][rA] = sum_lA E[lA][a][lF] A[lA][si][rA]
      for_2d(Aa * DlF * qi, DrA, [&](int row, int rA) {
        const int si = row & (qi - 1), t = row >> lqi, a = t >= DlF ? 1 : 0, lF = t - a * DlF;
        Real acc = 0;
        for (int lA = 0; lA < DlA; ++lA) acc += E[(lA * Aa + a) * DlF + lF] * Aj[(lA * qi + si) * DrA + rA];
        P3[row * DrA + rA] = acc;
      });
      __syncthreads();
      // G[a][si][so][b] = sum_{lF,rA} P3[a][lF][si][rA] P1r[lF][so][rA][b], divided by the sandwich value
      const int ng = Aa * qi * qo * B;
      for (int e = tid; e < ng; e += NT) {
        const int b = e & (B - 1), so = (e >> lB) & (qo - 1), si = (e >> (lB + lqo)) & (qi - 1), a = e >> (lB + lqo + lqi);
        double acc = 0;
        for (int lF = 0; lF < DlF; ++lF)
          for (int rA = 0; rA < DrA; ++rA)
            acc += (double)P3[((a * DlF + lF) * qi + si) * DrA + rA] * (double)P1[((lF * qo + so) * DrA + rA) * B + b];
        P2[e] = Real(acc / S);
      }
      __syncthreads();
      if (tid == 0) {
        // d log Z / d wtab[P] = sum of G over the entries whose code is P
        double dw[4] = {0, 0, 0, 0};
        for (int e = 0; e < ng; ++e) {
          const int c = codes[st.wofs + e];
          if (c >= W_PAULI) dw[c - W_PAULI] += (double)P2[e];
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
    // P2r[lF][si][a][rA] = sum_{so,b} P1r[lF][so][rA][b] W[a][si][so][b]
    for_2d(DlF * qi * Aa, DrA, [&](int row, int rA) {
      const int a = row & (Aa - 1), t = row >> lA_, si = t & (qi - 1), lF = t >> lqi;
      Real acc = 0;
      for (int so = 0; so < qo; ++so)
        for (int b = 0; b < B; ++b) acc += P1[((lF * qo + so) * DrA + rA) * B + b] * Wv[((a * qi + si) * qo + so) * B + b];
      P2[row * DrA + rA] = acc;
    });
    __syncthreads();
    // Rn[lA][a][lF] = sum_{si,rA} A[lA][si][rA] P2r[lF][si][a][rA]
    for_2d(DlA * Aa, DlF, [&](int row, int lF) {
      const int a = row & (Aa - 1), lA = row >> lA_;
      Real acc = 0;
      for (int si = 0; si < qi; ++si)
        for (int rA = 0; rA < DrA; ++rA) acc += Aj[(lA * qi + si) * DrA + rA] * P2[((lF * qi + si) * Aa + a) * DrA + rA];
      Rn[row * DlF + lF] = acc;
    });
    __syncthreads();
  }
  return true;
}

// Backward of syndrome b over its four cosets: adds, for each coset mlog,
// weight_mlog * d log Z_mlog / d theta to part (FP64, [n][3]) where
// weight = grad_logp[b] * P(l|s).  The rows before H->shared_rows are the same
// for the four cosets (as in the forward pass), so the top-down sweep over them
// and its checkpoints are computed once and the MPS after them is kept in
// snap; each coset continues from it.  Segments of kseg rows that lie within
// the shared rows recompute the same top states for every coset: they are
// kept from the first coset that needs them.  Scratch layout (in Real
// elements): top regions | bottom regions | K-row checkpoints | segment
// states | environments | three temporaries | snapshot | shared segment
// states (S / kseg segments of kseg states).  Collective.
template <typename Real, typename Fac, int GM>
__device__ void adjoint_syndrome(const JobDev& job, int64_t b, uint8_t* smem, const LdsLayout& lay, Real* scr,
                                 int kseg, double* part) {
  const uint8_t* plan = job.plan;
  const PlanHeader* H = reinterpret_cast<const PlanHeader*>(plan);
  const int n = H->n, m = H->m, nsite = H->nsite, nstep = H->nstep;
  const int S = H->shared_rows;
  const SiteStep* steps = reinterpret_cast<const SiteStep*>(plan + H->steps_ofs);
  const SiteStep* bsteps = reinterpret_cast<const SiteStep*>(plan + H->bu_steps_ofs);
  const uint8_t* codes = plan + H->codes_ofs;
  const CheckDesc* checks = reinterpret_cast<const CheckDesc*>(plan + H->checks_ofs);
  const int64_t* region = reinterpret_cast<const int64_t*>(plan + H->region_ofs);
  const int16_t* fin = reinterpret_cast<const int16_t*>(plan + H->final_ofs);
  __shared__ int s_flags[2];
  __shared__ int s_label;
  __shared__ double s_weight[4];
  Work<Real, Fac> w = carve<Real, Fac>(smem, lay, s_flags);
  const ItemCheck ck = check_item(job, b, n, m);
  if (!ck.valid) return;  // no contribution; the status word says why
  const int model = ck.model;
  const double* rates = job.rates + (int64_t)model * n * 3;
  const uint8_t* syn = job.syn + b * m;
  int first = -1;
  for (int mlog = 0; mlog < 4; ++mlog) {
    const int label = prep_reference(H, checks, syn, mlog, w.syn, w.fbits, &s_label);
    if (threadIdx.x == 0) {
      const double lz = job.logz[b * 4 + label], lp = job.logp[b], gp = job.gradp[b];
      s_weight[mlog] = (lz > -INFINITY && lp > -INFINITY && gp != 0.0) ? gp * exp(lz - lp) : 0.0;
    }
    __syncthreads();
    if (first < 0 && s_weight[mlog] != 0.0) first = mlog;
  }
  if (first < 0) return;

  const int64_t se = H->scratch_elems, me = H->mps_elems;
  const int ncp = (nstep + kseg - 1) / kseg;
  Real* top = scr;
  Real* bot = scr + se;
  Real* cps = scr + 2 * se;
  Real* seg = cps + (int64_t)ncp * me;
  Real* env = seg + (int64_t)kseg * me;
  Real* P1 = env + H->env_elems;
  Real* P2 = P1 + H->tmp_elems;
  Real* P3 = P2 + H->tmp_elems;
  Real* snap = P3 + H->tmp_elems;
  Real* shseg = snap + me;
  const int nshc = S / kseg;  // segments entirely within the shared rows
  unsigned shdone = 0;        // bit c: shared segment c recomputed
  double* pm = part + (int64_t)model * n * 3;
  auto in_dims = [&](const SiteStep* row) {
    return [row](int J, int& Dl, int& q, int& Dr) {
      Dl = row[J].Dl_old;
      q = row[J].qi;
      Dr = row[J].Dr_old;
    };
  };
  // --- shared rows: top-down once, with their checkpoints ------------------
  // (the reference error of any coset agrees on these rows)
  prep_reference(H, checks, syn, first, w.syn, w.fbits, &s_label);
  mps_ones(top, region, plan + H->init_qi_ofs, nsite);
  double logscale = 0.0;
  for (int u = 0; u < S; ++u) {
    const SiteStep* row = steps + (int64_t)u * nsite;
    if (u % kseg == 0) mps_pack(top, region, nsite, in_dims(row), cps + (int64_t)(u / kseg) * me, false, top);
    if (!row_step_outlined<Real, Fac, GM>(row, nsite, codes, rates, top, region, w, logscale)) return;
  }
  if (S > 0) mps_pack(top, region, nsite, in_dims(steps + (int64_t)S * nsite), snap, false, top);
  const double logscale_s = logscale;

  for (int mlog = first; mlog < 4; ++mlog) {
    const double weight = s_weight[mlog];
    if (weight == 0.0) continue;
    prep_reference(H, checks, syn, mlog, w.syn, w.fbits, &s_label);
    // --- the coset's own rows: top-down with checkpoints every kseg rows ----
    if (S > 0) mps_pack(top, region, nsite, in_dims(steps + (int64_t)S * nsite), snap, true, top);
    else mps_ones(top, region, plan + H->init_qi_ofs, nsite);
    logscale = logscale_s;
    bool alive = true;
    for (int u = S; u < nstep && alive; ++u) {
      const SiteStep* row = steps + (int64_t)u * nsite;
      if (u % kseg == 0) mps_pack(top, region, nsite, in_dims(row), cps + (int64_t)(u / kseg) * me, false, top);
      alive = row_step_outlined<Real, Fac, GM>(row, nsite, codes, rates, top, region, w, logscale);
    }
    if (!alive) continue;
    // --- bottom-up, recomputing each segment of top states -----------------
    for (int J = 0; J < nsite; ++J)  // all-ones over the final frontier
      for (int e = threadIdx.x; e < fin[3 * J + 1]; e += NT) bot[region[J] + e] = Real(1);
    __syncthreads();
    int cur = -1;
    double bscale = 0.0;
    Real* sbase = seg;
    for (int u = nstep - 1; u >= 0 && alive; --u) {
      const int c = u / kseg;
      if (c != cur) {
        const bool shared = c < nshc;
        sbase = shared ? shseg + (int64_t)c * kseg * me : seg;
        if (!(shared && (shdone >> c & 1u))) {
          const int t0 = c * kseg, t1 = (t0 + kseg < nstep ? t0 + kseg : nstep);
          mps_pack(top, region, nsite, in_dims(steps + (int64_t)t0 * nsite), cps + (int64_t)c * me, true, top);
          mps_pack(top, region, nsite, in_dims(steps + (int64_t)t0 * nsite), sbase, false, top);
          for (int t = t0; t + 1 < t1 && alive; ++t) {
            alive = row_step_outlined<Real, Fac, GM>(steps + (int64_t)t * nsite, nsite, codes, rates, top, region, w,
                                                     logscale);
            if (alive)
              mps_pack(top, region, nsite, in_dims(steps + (int64_t)(t + 1) * nsite),
                       sbase + (int64_t)(t + 1 - t0) * me, false, top);
          }
          if (shared && alive) shdone |= 1u << c;
        }
        cur = c;
      }
      if (!alive) break;
      const SiteStep* frow = steps + (int64_t)u * nsite;
      const SiteStep* brow = bsteps + (int64_t)(nstep - 1 - u) * nsite;
      if (!row_gradient<Real>(frow, brow, nsite, codes, rates, w.fbits, sbase + (int64_t)(u - c * kseg) * me, bot,
                              region, env, P1, P2, P3, w.Wv, weight, pm) &&
          ck.positive && threadIdx.x == 0 && job.status)
        atomicOr(job.status, ST_NUMERIC);
      if (u > 0) alive = row_step_outlined<Real, Fac, GM>(brow, nsite, codes, rates, bot, region, w, bscale);
    }
  }
}

}  // namespace tnmld
