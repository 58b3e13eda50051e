// Contraction plan builder (host only).  See plan.hpp for the lattice and the
// sweep; this file fixes every index map the device kernel relies on.
#include "plan.hpp"

#include <algorithm>
#include <cstring>

namespace tnmld {

namespace {

struct Layout {
  int d;
  // generator with corner (r,c): exists? type (0 = X, 1 = Z)
  bool exists(int r, int c) const {
    if (r < -1 || c < -1 || r > d - 1 || c > d - 1) return false;
    bool is_x = ((r + c) & 1) == 0;
    bool bulk = r >= 0 && c >= 0 && r <= d - 2 && c <= d - 2;
    bool tb = (r == -1 || r == d - 1) && is_x && c >= 0 && c <= d - 2;
    bool lr = (c == -1 || c == d - 1) && !is_x && r >= 0 && r <= d - 2;
    return bulk || tb || lr;
  }
  // generator whose corner sum is s at column w
  bool var(int s, int w) const {
    if (((s - w) & 1) != 0) return false;
    int r = (s - w) / 2, c = (s + w) / 2;  // exact: s - w even
    return exists(r, c);
  }
  bool qubit(int u, int w, int* q) const {
    if (((u - w) & 1) != 0) return false;
    int r = (u - w) / 2, c = (u + w) / 2;
    if (r < 0 || c < 0 || r >= d || c >= d) return false;
    *q = r * d + c;
    return true;
  }
};

inline int pauli_of(int x, int z) { return x ? (z ? 2 : 1) : (z ? 3 : 0); }
inline int pad8(int x) { return (x + 7) / 8 * 8; }

inline double qr_flops(double M, double N) {  // Householder factorisation, M >= N
  if (M < N) std::swap(M, N);
  return 2.0 * M * N * N - 2.0 / 3.0 * N * N * N;
}
inline double orgq_flops(double M, double N) {  // explicit thin Q from N reflectors
  if (M < N) std::swap(M, N);
  return 4.0 * M * N * N - 4.0 / 3.0 * N * N * N;
}
inline double svd_flops(double M, double N) {  // dense SVD model 6 M N^2 + 20 N^3
  if (M < N) std::swap(M, N);
  return 6.0 * M * N * N + 20.0 * N * N * N;
}

// Counted work of one site step of the implemented algorithm (standard dense
// counts); *gemm gets its GEMM-class part.
double site_flops(const SiteStep& S, double* gemm) {
  const double m = S.m, nn = (double)S.qo * S.kr, rB = (double)S.Dr_old * S.B;
  const double R = (double)S.Dl_new * S.qo, k2 = std::min(R, (double)S.kr);
  double f = 2.0 * S.Dl_old * S.qi * S.Dr_old * S.A * S.qo * S.B;  // MPO apply
  const double tl = 2.0 * m * S.qo * rB * S.kr;                      // (W A) . L
  f += qr_flops(m, nn) + orgq_flops(nn, S.k);                        // LQ + explicit Q
  const double cq = 2.0 * S.Dl_new * S.k * nn;                        // C . Q
  f += qr_flops(R, S.kr) + orgq_flops(R, k2);                        // QR of the site matrix + Q
  double qw = 0.0;
  if (S.Dr_new < k2) {                                                // bond truncated:
    f += svd_flops(S.kr, k2);                                         //   SVD of the R factor
    qw = 2.0 * R * k2 * S.Dr_new;                                     //   A = Q W
  }
  *gemm = tl + cq + qw;
  return f + tl + cq + qw;
}

// Counted work of the row environments at one site (adjoint): the left
// environment step (three contractions), the right one (three) and, for a site
// with a qubit, the derivative tensor (the top site with the left environment,
// then the fold with the bottom side).  T: forward step of the row, Bv: the
// bottom-up step whose input is the bottom MPS of that row.
double env_flops(const SiteStep& T, const SiteStep& Bv) {
  const double Aa = T.A, B = T.B, qi = T.qi, qo = T.qo, DlA = T.Dl_old, DrA = T.Dr_old, DlF = Bv.Dl_old,
               DrF = Bv.Dr_old;
  const double ea = 2.0 * Aa * DlF * qi * DrA * DlA;  // E . A
  double f = ea + 2.0 * DlF * qo * B * DrA * Aa * qi + 2.0 * DrA * B * DrF * DlF * qo;   // left
  f += 2.0 * DlF * qo * DrA * B * DrF + 2.0 * DlF * qi * Aa * DrA * qo * B + 2.0 * DlA * Aa * DlF * qi * DrA;  // right
  if (T.q >= 0) f += ea + 2.0 * Aa * qi * qo * B * DlF * DrA;  // derivative tensor
  return f;
}

}  // namespace

std::string build_plan(int d, int chi, int group, Plan* out, int rounds) {
  if (d < 3 || d > 31 || (d % 2) == 0) return "d must be odd, 3 <= d <= 31";
  if (chi < 0 || chi > 4096) return "chi out of range";
  if (group < 1 || group > 2) return "group must be 1 or 2";
  if (rounds < 1 || rounds > 2) return "rounds must be 1 or 2";
  if (rounds > 1 && group != 1) return "repeated rounds need one column per site";
  Layout L{d};
  const int V = 1 << rounds;  // values of one column variable (a bit per round)
  const int P = 2 * d - 1;  // columns
  const int nsite = (P + group - 1) / group;
  const int nstep = 2 * d - 1;
  const int n = d * d;
  auto wcol = [&](int i) { return i - (d - 1); };
  auto site_lo = [&](int J) { return J * group; };
  auto site_hi = [&](int J) { return std::min((J + 1) * group, P); };

  std::vector<SiteStep> steps((size_t)nstep * nsite);
  std::vector<uint8_t> codes;
  std::vector<int> Dold(nsite + 1, 1), Dnew(nsite + 1, 1);  // Dold[J] = bond between J and J+1
  std::vector<uint8_t> init_qi(nsite, 1);
  std::vector<int64_t> region(nsite, 1);
  double flops = 0.0;
  double gemm = 0.0;  // GEMM-class part
  PlanHeader h{};
  h.d = d;
  h.n = n;
  h.m = n - 1;
  h.nsite = nsite;
  h.nstep = nstep;
  h.chi = chi;
  h.group = group;
  // logical representatives on the last column / row: the anti-diagonal rows
  // u = r + c they touch start at u = d - 1, so the first d - 1 rows of the
  // sweep are common to the four cosets of a syndrome
  h.lx_col = d - 1;
  h.lz_row = d - 1;
  h.shared_rows = std::min(h.lx_col, h.lz_row);
  h.rounds = rounds;
  // syndrome index of the check with corner (r, c): Z-type checks first, then
  // X-type, each by corner (the order of the check descriptors below)
  std::vector<int> check_id((size_t)(d + 1) * (d + 1), -1);
  {
    int j = 0;
    for (int pass = 0; pass < 2; ++pass)
      for (int r = -1; r <= d - 1; ++r)
        for (int c = -1; c <= d - 1; ++c) {
          if (!L.exists(r, c)) continue;
          if ((pass == 0) == (((r + c) & 1) == 0)) continue;
          check_id[(size_t)(r + 1) * (d + 1) + (c + 1)] = j++;
        }
  }
  auto check_of = [&](int sum, int w) {  // check of the variable at corner sum `sum`, column w
    const int r = (sum - w) / 2, c = (sum + w) / 2;
    return check_id[(size_t)(r + 1) * (d + 1) + (c + 1)];
  };

  // variables before step 0: column w holds corner sum -2 (w even) or -1 (w odd)
  for (int J = 0; J < nsite; ++J) {
    int qi = 1;
    for (int i = site_lo(J); i < site_hi(J); ++i) {
      int w = wcol(i);
      bool v = ((w & 1) == 0) ? L.var(-2, w) : L.var(-1, w);
      if (v) qi *= V;
    }
    init_qi[J] = (uint8_t)qi;
  }

  for (int u = 0; u < nstep; ++u) {
    // per-column variable existence before / after and activity
    std::vector<int> vin(P), vout(P), act(P), qub(P, -1);
    for (int i = 0; i < P; ++i) {
      int w = wcol(i);
      act[i] = ((w - u) & 1) == 0;
      if (act[i]) {
        vin[i] = L.var(u - 2, w);
        vout[i] = L.var(u, w);
        int q;
        if (L.qubit(u, w, &q)) qub[i] = q;
      } else {
        vin[i] = vout[i] = L.var(u - 1, w);
      }
    }
    // MPO bonds: bond J|J+1 carries the control variable next to it when the
    // active column on the other side has a qubit that reads it.
    std::vector<int> bond(nsite + 1, 1), owner(nsite + 1, -1);
    for (int J = 0; J + 1 < nsite; ++J) {
      int iL = site_hi(J) - 1, iR = iL + 1;
      if (act[iL] && qub[iL] >= 0 && vin[iR]) {
        bond[J] = V;
        owner[J] = J + 1;
      } else if (act[iR] && qub[iR] >= 0 && vin[iL]) {
        bond[J] = V;
        owner[J] = J;
      }
    }
    // MPO code tables
    for (int J = 0; J < nsite; ++J) {
      SiteStep& S = steps[(size_t)u * nsite + J];
      int lo = site_lo(J), hi = site_hi(J);
      int A = J > 0 ? bond[J - 1] : 1, B = bond[J];
      int qi = 1, qo = 1;
      int bit_in[2] = {-1, -1}, bit_out[2] = {-1, -1};
      for (int i = lo; i < hi; ++i) {
        if (vin[i]) bit_in[i - lo] = __builtin_ctz(qi), qi *= V;
        if (vout[i]) bit_out[i - lo] = __builtin_ctz(qo), qo *= V;
      }
      int ia = -1;
      for (int i = lo; i < hi; ++i)
        if (act[i]) ia = i;
      S.q = (int16_t)(ia >= 0 ? qub[ia] : -1);
      S.A = (uint8_t)A;
      S.B = (uint8_t)B;
      S.qi = (uint8_t)qi;
      S.qo = (uint8_t)qo;
      S.act = (uint8_t)(ia >= 0 ? ia - lo : 0);
      S.wofs = (int32_t)codes.size();
      S.wnew = S.wold = -1;
      if (rounds > 1 && ia >= 0) {
        const int w = wcol(ia);
        if (vout[ia]) S.wnew = (int16_t)check_of(u, w);
        if (vin[ia] && u - 2 < 0) S.wold = (int16_t)check_of(u - 2, w);
      }
      h.max_ncode = std::max(h.max_ncode, A * qi * qo * B);
      for (int a = 0; a < A; ++a)
        for (int si = 0; si < qi; ++si)
          for (int so = 0; so < qo; ++so)
            for (int b = 0; b < B; ++b) {
              auto bin = [&](int i) { int k = bit_in[i - lo]; return k < 0 ? 0 : (si >> k) & (V - 1); };
              auto bout = [&](int i) { int k = bit_out[i - lo]; return k < 0 ? 0 : (so >> k) & (V - 1); };
              bool ok = true;
              for (int i = lo; i < hi; ++i)
                if (!act[i] && bin(i) != bout(i)) ok = false;
              int ext_l = 0, ext_r = 0;
              if (A > 1) {
                if (owner[J - 1] == J) { if (a != bin(lo)) ok = false; }
                else ext_l = a;
              }
              if (B > 1) {
                if (owner[J] == J) { if (b != bin(hi - 1)) ok = false; }
                else ext_r = b;
              }
              uint8_t code = W_ZERO;
              if (ok) {
                if (ia < 0 || qub[ia] < 0) {
                  code = W_ONE;
                } else {
                  auto ctrl = [&](int i) -> int {
                    if (i < 0 || i >= P || !vin[i]) return 0;
                    if (i < lo) return ext_l;
                    if (i >= hi) return ext_r;
                    return bin(i);
                  };
                  int N = bin(ia), Sv = bout(ia);
                  int c2 = ctrl(ia - 1) ^ ctrl(ia + 1);
                  int x, z;
                  if ((u & 1) == 0) { x = N ^ Sv; z = c2; }
                  else { x = c2; z = N ^ Sv; }
                  if (rounds == 1) {
                    code = (uint8_t)(W_PAULI + pauli_of(x, z));
                  } else {
                    int k = 0;  // digit t: (x, z) bits of round t+1
                    for (int t = 0; t < rounds; ++t) k |= ((((x >> t) & 1) | (((z >> t) & 1) << 1)) << (2 * t));
                    code = (uint8_t)(W_PAULI + k);
                  }
                }
              }
              codes.push_back(code);
            }
    }
    // bond dimensions: right-to-left LQ sizes, then left-to-right truncation
    std::vector<int> kk(nsite + 1, 1);
    for (int J = nsite - 1; J >= 0; --J) {
      SiteStep& S = steps[(size_t)u * nsite + J];
      int Dl = J > 0 ? Dold[J - 1] : 1, Dr = J + 1 < nsite ? Dold[J] : 1;
      int mJ = Dl * S.A;
      int kr = kk[J + 1];
      int k = std::min(mJ, (int)S.qo * kr);
      kk[J] = k;
      S.Dl_old = (int16_t)Dl;
      S.Dr_old = (int16_t)Dr;
      S.m = (int16_t)mJ;
      S.kr = (int16_t)kr;
      S.k = (int16_t)k;
    }
    int Dl = 1;
    for (int J = 0; J < nsite; ++J) {
      SiteStep& S = steps[(size_t)u * nsite + J];
      int Dr = std::min(Dl * (int)S.qo, (int)S.kr);
      if (chi > 0) Dr = std::min(Dr, chi);
      if (J == nsite - 1) Dr = 1;
      S.Dl_new = (int16_t)Dl;
      S.Dr_new = (int16_t)Dr;
      Dnew[J] = Dr;
      Dl = Dr;
    }
    for (int J = 0; J < nsite; ++J) Dold[J] = Dnew[J];
    // sizes and flops
    for (int J = 0; J < nsite; ++J) {
      const SiteStep& S = steps[(size_t)u * nsite + J];
      int64_t sz = std::max<int64_t>({(int64_t)S.k * S.qo * S.kr, (int64_t)S.Dl_new * S.qo * S.Dr_new,
                                      (int64_t)S.Dl_old * S.qi * S.Dr_old});
      region[J] = std::max(region[J], sz);
      int rB = S.Dr_old * S.B;
      h.max_Aj = std::max(h.max_Aj, S.Dl_old * S.qi * S.Dr_old);
      h.max_T = std::max(h.max_T, S.m * pad8(rB));  // rows padded for the bf16 planes
      h.max_X = std::max(h.max_X, S.m * S.qo * S.kr);
      h.max_L = std::max({h.max_L, S.m * S.k, pad8(rB) * S.kr, S.k * pad8(S.m)});
      h.max_C = std::max(h.max_C, S.Dl_new * S.k);
      h.max_M = std::max(h.max_M, (S.Dl_new * S.qo + 1) * S.kr);
      h.max_V = std::max(h.max_V, (S.kr + 1) * S.kr);
      h.max_Q = std::max(h.max_Q, S.k * S.qo * S.kr);
      h.max_kr = std::max(h.max_kr, (int)S.kr);
      h.max_n = std::max(h.max_n, S.qo * S.kr);
      h.max_m = std::max(h.max_m, (int)S.m);
      h.max_rows = std::max(h.max_rows, S.Dl_new * S.qo);
      h.max_bond = std::max({h.max_bond, (int)S.Dl_new, (int)S.Dr_new, (int)S.Dl_old, (int)S.Dr_old});
      double g = 0.0;
      flops += site_flops(S, &g);
      gemm += g;
    }
    if (u + 1 == h.shared_rows) {
      h.flops_shared = flops;
      h.flops_gemm_shared = gemm;
    }
  }
  h.flops_fwd = flops;
  h.flops_gemm = gemm;

  // --- bottom-up sweep (adjoint): the transposed row MPOs applied from the
  // last row upwards to the all-ones closing state; same bond bookkeeping ---
  std::vector<SiteStep> bu((size_t)nstep * nsite);
  {
    std::vector<int> Db(nsite + 1, 1);
    for (int s2 = 0; s2 < nstep; ++s2) {
      const int u = nstep - 1 - s2;
      for (int J = 0; J < nsite; ++J) {
        SiteStep S = steps[(size_t)u * nsite + J];
        std::swap(S.qi, S.qo);
        S.tr = 1;
        bu[(size_t)s2 * nsite + J] = S;
      }
      std::vector<int> kk(nsite + 1, 1);
      for (int J = nsite - 1; J >= 0; --J) {
        SiteStep& S = bu[(size_t)s2 * nsite + J];
        int Dl = J > 0 ? Db[J - 1] : 1, Dr = J + 1 < nsite ? Db[J] : 1;
        int mJ = Dl * S.A, kr = kk[J + 1], k = std::min(mJ, (int)S.qo * kr);
        kk[J] = k;
        S.Dl_old = (int16_t)Dl;
        S.Dr_old = (int16_t)Dr;
        S.m = (int16_t)mJ;
        S.kr = (int16_t)kr;
        S.k = (int16_t)k;
      }
      int Dl = 1;
      for (int J = 0; J < nsite; ++J) {
        SiteStep& S = bu[(size_t)s2 * nsite + J];
        int Dr = std::min(Dl * (int)S.qo, (int)S.kr);
        if (chi > 0) Dr = std::min(Dr, chi);
        if (J == nsite - 1) Dr = 1;
        S.Dl_new = (int16_t)Dl;
        S.Dr_new = (int16_t)Dr;
        Db[J] = Dr;
        Dl = Dr;
      }
    }
  }
  std::vector<int16_t> bu_fin((size_t)nsite * 3);
  for (int J = 0; J < nsite; ++J) {
    const SiteStep& S = bu[(size_t)(nstep - 1) * nsite + J];
    bu_fin[3 * J] = S.Dl_new;
    bu_fin[3 * J + 1] = S.qo;
    bu_fin[3 * J + 2] = S.Dr_new;
  }
  // sizes covering both sweeps; truncated-MPS and environment sizes
  int64_t mps_max = 0, env_max = 0;
  for (int pass = 0; pass < 2; ++pass) {
    const std::vector<SiteStep>& V = pass == 0 ? steps : bu;
    for (int u = 0; u < nstep; ++u) {
      int64_t mps = 0;
      for (int J = 0; J < nsite; ++J) {
        const SiteStep& S = V[(size_t)u * nsite + J];
        int64_t sz = std::max<int64_t>({(int64_t)S.k * S.qo * S.kr, (int64_t)S.Dl_new * S.qo * S.Dr_new,
                                        (int64_t)S.Dl_old * S.qi * S.Dr_old});
        region[J] = std::max(region[J], sz);
        mps += std::max<int64_t>((int64_t)S.Dl_new * S.qo * S.Dr_new, (int64_t)S.Dl_old * S.qi * S.Dr_old);
        int rB = S.Dr_old * S.B;
        h.max_Aj = std::max(h.max_Aj, S.Dl_old * S.qi * S.Dr_old);
        h.max_T = std::max(h.max_T, S.m * pad8(rB));  // rows padded for the bf16 planes
        h.max_X = std::max(h.max_X, S.m * S.qo * S.kr);
        h.max_L = std::max({h.max_L, S.m * S.k, pad8(rB) * S.kr, S.k * pad8(S.m)});
        h.max_C = std::max(h.max_C, S.Dl_new * S.k);
        h.max_M = std::max(h.max_M, (S.Dl_new * S.qo + 1) * S.kr);
        h.max_V = std::max(h.max_V, (S.kr + 1) * S.kr);
        h.max_Q = std::max(h.max_Q, S.k * S.qo * S.kr);
        h.max_kr = std::max(h.max_kr, (int)S.kr);
        h.max_n = std::max(h.max_n, S.qo * S.kr);
        h.max_m = std::max(h.max_m, (int)S.m);
        h.max_rows = std::max(h.max_rows, S.Dl_new * S.qo);
        h.max_bond = std::max({h.max_bond, (int)S.Dl_new, (int)S.Dr_new, (int)S.Dl_old, (int)S.Dr_old});
      }
      mps_max = std::max(mps_max, mps);
    }
  }
  // environments of row u: E_J / R_J over (top bond, MPO bond, bottom bond)
  for (int u = 0; u < nstep; ++u) {
    int64_t env = 0;
    for (int J = 0; J <= nsite; ++J) {
      // bond between J-1 and J: top = fwd row u input bonds, bottom = bu row (nstep-1-u) input bonds
      const SiteStep& T = steps[(size_t)u * nsite + std::min(J, nsite - 1)];
      const SiteStep& Bv = bu[(size_t)(nstep - 1 - u) * nsite + std::min(J, nsite - 1)];
      int dt = J == nsite ? 1 : T.Dl_old, db = J == nsite ? 1 : Bv.Dl_old, a = J == nsite ? 1 : T.A;
      env += (int64_t)dt * a * db;
      h.max_envb = std::max(h.max_envb, dt * a * db);
    }
    env_max = std::max(env_max, env);
  }
  // adjoint work per coset: the bottom-up sweep and the row environments
  h.flops_bu = 0.0;
  h.flops_env = 0.0;
  for (int s2 = 0; s2 < nstep; ++s2)
    for (int J = 0; J < nsite; ++J) {
      double g = 0.0;
      h.flops_bu += site_flops(bu[(size_t)s2 * nsite + J], &g);
    }
  for (int u = 0; u < nstep; ++u)
    for (int J = 0; J < nsite; ++J)
      h.flops_env += env_flops(steps[(size_t)u * nsite + J], bu[(size_t)(nstep - 1 - u) * nsite + J]);
  int64_t tmp_max = 64;
  for (int u = 0; u < nstep; ++u)
    for (int J = 0; J < nsite; ++J) {
      const SiteStep& T = steps[(size_t)u * nsite + J];
      const SiteStep& Bv = bu[(size_t)(nstep - 1 - u) * nsite + J];
      const int64_t DlF = Bv.Dl_old;
      tmp_max = std::max<int64_t>({tmp_max, (int64_t)T.A * DlF * T.qi * T.Dr_old, DlF * T.qo * T.B * T.Dr_old,
                                   DlF * T.qi * T.A * T.Dr_old});
    }
  h.tmp_elems = (tmp_max + 63) / 64 * 64;
  h.mps_elems = (mps_max + 63) / 64 * 64;
  h.env_elems = (2 * env_max + 63) / 64 * 64;
  // the truncation SVD keeps a column pair of up to 128 rows in registers
  if (h.max_kr > 128) return "bond dimension above 128 before truncation: lower chi";


  // final MPS shape per site
  std::vector<int16_t> fin((size_t)nsite * 3);
  for (int J = 0; J < nsite; ++J) {
    const SiteStep& S = steps[(size_t)(nstep - 1) * nsite + J];
    fin[3 * J] = S.Dl_new;
    fin[3 * J + 1] = S.qo;
    fin[3 * J + 2] = S.Dr_new;
  }
  // reference-error strings
  std::vector<CheckDesc> checks;
  for (int pass = 0; pass < 2; ++pass)
    for (int r = -1; r <= d - 1; ++r)
      for (int c = -1; c <= d - 1; ++c) {
        if (!L.exists(r, c)) continue;
        bool is_x = ((r + c) & 1) == 0;
        if ((pass == 0) == is_x) continue;  // Z-type checks first
        CheckDesc cd{};
        if (is_x) {
          cd.type = 0;
          cd.line = (int8_t)std::max(r, 0);
          cd.from = 0;
          cd.to = (int8_t)c;
        } else {
          cd.type = 1;
          cd.line = (int8_t)std::max(c, 0);
          cd.from = 0;
          cd.to = (int8_t)r;
        }
        checks.push_back(cd);
      }
  if ((int)checks.size() != n - 1) return "internal: check count";

  // scratch regions (elements), 64-element aligned
  std::vector<int64_t> rofs(nsite);
  int64_t tot = 0;
  for (int J = 0; J < nsite; ++J) {
    rofs[J] = tot;
    tot += (region[J] + 63) / 64 * 64;
  }
  h.scratch_elems = tot;

  // blob
  auto align8 = [](size_t x) { return (x + 7) / 8 * 8; };
  size_t off = align8(sizeof(PlanHeader));
  h.steps_ofs = (int32_t)off;
  off = align8(off + steps.size() * sizeof(SiteStep));
  h.codes_ofs = (int32_t)off;
  off = align8(off + codes.size());
  h.checks_ofs = (int32_t)off;
  off = align8(off + checks.size() * sizeof(CheckDesc));
  h.region_ofs = (int32_t)off;
  off = align8(off + rofs.size() * sizeof(int64_t));
  h.init_qi_ofs = (int32_t)off;
  off = align8(off + init_qi.size());
  h.final_ofs = (int32_t)off;
  off = align8(off + fin.size() * sizeof(int16_t));
  h.bu_steps_ofs = (int32_t)off;
  off = align8(off + bu.size() * sizeof(SiteStep));
  h.bu_final_ofs = (int32_t)off;
  off = align8(off + bu_fin.size() * sizeof(int16_t));
  h.bytes = (int32_t)off;
  out->h = h;
  out->blob.assign(off, 0);
  std::memcpy(out->blob.data(), &h, sizeof(h));
  std::memcpy(out->blob.data() + h.steps_ofs, steps.data(), steps.size() * sizeof(SiteStep));
  std::memcpy(out->blob.data() + h.codes_ofs, codes.data(), codes.size());
  std::memcpy(out->blob.data() + h.checks_ofs, checks.data(), checks.size() * sizeof(CheckDesc));
  std::memcpy(out->blob.data() + h.region_ofs, rofs.data(), rofs.size() * sizeof(int64_t));
  std::memcpy(out->blob.data() + h.init_qi_ofs, init_qi.data(), init_qi.size());
  std::memcpy(out->blob.data() + h.final_ofs, fin.data(), fin.size() * sizeof(int16_t));
  std::memcpy(out->blob.data() + h.bu_steps_ofs, bu.data(), bu.size() * sizeof(SiteStep));
  std::memcpy(out->blob.data() + h.bu_final_ofs, bu_fin.data(), bu_fin.size() * sizeof(int16_t));
  return "";
}

void merge_maxima(PlanHeader* a, const PlanHeader& h) {
  a->max_Aj = std::max(a->max_Aj, h.max_Aj);
  a->max_T = std::max(a->max_T, h.max_T);
  a->max_X = std::max(a->max_X, h.max_X);
  a->max_L = std::max(a->max_L, h.max_L);
  a->max_C = std::max(a->max_C, h.max_C);
  a->max_M = std::max(a->max_M, h.max_M);
  a->max_V = std::max(a->max_V, h.max_V);
  a->max_Q = std::max(a->max_Q, h.max_Q);
  a->max_kr = std::max(a->max_kr, h.max_kr);
  a->max_n = std::max(a->max_n, h.max_n);
  a->max_m = std::max(a->max_m, h.max_m);
  a->max_rows = std::max(a->max_rows, h.max_rows);
  a->max_bond = std::max(a->max_bond, h.max_bond);
  a->max_envb = std::max(a->max_envb, h.max_envb);
  a->max_ncode = std::max(a->max_ncode, h.max_ncode);
  a->tmp_elems = std::max(a->tmp_elems, h.tmp_elems);
  a->n = std::max(a->n, h.n);
  a->m = std::max(a->m, h.m);
}

}  // namespace tnmld
