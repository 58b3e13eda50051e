// Host-side contraction plan for the boundary-MPS coset contraction of the
// rotated surface code (paper Sec. 3.2.1, generator picture + boundary MPS).
//
// Network.  Every stabiliser generator j carries a binary variable alpha_j
// (the generator-picture sum); a qubit tensor weighs its Pauli
// f_q * X^(sum of X-type alpha on q) * Z^(sum of Z-type alpha on q), where f is
// the coset's reference error.  Rotating the patch by 45 degrees puts qubit
// (r,c) at (u,w) = (r+c, c-r) and the plaquette with corner (r,c) at
// (r+c+1, c-r): a square lattice whose vertical neighbours of a qubit are its
// two same-type plaquettes and whose horizontal neighbours are the other two.
//
// Sweep.  The boundary MPS lives on the 2d-1 columns w = -(d-1)..d-1; column
// w holds the generator variable currently "open" there.  Step u (u = 0..2d-2)
// absorbs the qubits on the anti-diagonal r+c = u: on columns w = u (mod 2) the
// qubit maps its upper plaquette variable (corner sum u-2) to its lower one
// (corner sum u), weighted by the two neighbouring columns' variables (corner
// sum u-1), which stay put.  Each step is therefore an MPO of bond dimension 2
// acting on the MPS (the paper's chi -> chi*q with q = 2).  Columns are grouped
// into sites of `group` columns (physical dimension up to 2^group).
//
// The plan fixes, for every step and site, the MPO tensor (as codes resolved on
// the device from per-qubit rates and the reference error), the MPS bond
// dimensions before/after truncation and the scratch / LDS sizes.
#pragma once
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace tnmld {

// Per (step, site) descriptor; POD, copied to the device verbatim.
struct SiteStep {
  int16_t q;       // qubit index of the site's active column, -1 if none
  uint8_t A, B;    // MPO bond dimension on the left / right of the site (1 or 2)
  uint8_t qi, qo;  // physical dimension before / after the step
  uint8_t act;     // position of the active column inside the site
  uint8_t tr;      // 1: transposed MPO (bottom-up sweep), codes indexed [a][so][si][b]
  int16_t Dl_old, Dr_old;  // MPS bonds of the input site tensor
  int16_t m;               // Dl_old * A: rows of the site matrix in the right-to-left sweep
  int16_t k;               // rows kept by its LQ factorisation: min(m, qo * kr)
  int16_t kr;              // k of the site to the right (1 for the last site)
  int16_t Dl_new, Dr_new;  // bonds after truncation
  int16_t wnew;            // repeated rounds: check whose variable this site creates (its measurement
                           // weights multiply the MPO entries through the output index), -1 if none
  int32_t wofs;            // offset of the A*qi*qo*B MPO code table
  int16_t wold;            // repeated rounds: check whose variable existed before row 0 and ends at this
                           // site (weights through the input index), -1 if none
  int16_t pad2;
};
static_assert(sizeof(SiteStep) == 32, "SiteStep layout");

// Code of one MPO entry: 0 -> 0, 1 -> 1, 2 + P -> p_q(f_q xor P), P in {I,X,Y,Z}
// (xor on the (x,z) bit pair).  Entry order: [a][si][so][b].
//
// Repeated rounds (T >= 2).  A column variable is a T-bit tuple, bit t the
// check's variable in round t+1: for t < T-1 the dual variable b of its
// measurement weight, g(b) = 1/2 (b = 0) or (1 - 2 q_j)/2 (-1)^{s_tj} (b = 1),
// so that sum_b g(b) (-1)^{b x} = Pr(s_tj | parity x); for t = T-1 the
// generator variable.  2 + k then codes the qubit's tensor
//   sum over C_1..C_{T-1} of prod_{t=1..T} p_q(C_{t-1} C_t)
//       * prod_{t<T} (-1)^{bX_t z(C_t) + bZ_t x(C_t)},   C_0 = I, C_T = f_q P_T,
// with k = sum_t 4^t (x_t + 2 z_t): digit t < T-1 holds the XORs (bX, bZ) of the
// round's X-type and Z-type neighbour variables, digit T-1 the Pauli P_T.
enum : uint8_t { W_ZERO = 0, W_ONE = 1, W_PAULI = 2 };

// Reference error R(s) = product over fired checks of a string that flips that
// check alone.  The strings run to the boundary the sweep starts from: a Z-type
// check with corner (r,c) gets X on column max(c,0), rows 0..r; an X-type check
// gets Z on row max(r,0), columns 0..c.  Logical representatives: X on column
// 0, Z on row 0.  With every string absorbed in the first rows, later rows
// never have to cancel the bulk of the boundary state, which keeps FP32
// rounding from being amplified on improbable cosets.
struct CheckDesc {
  int8_t type;      // 0 = X-type (string of Z along a row), 1 = Z-type (string of X along a column)
  int8_t line;      // row (X-type) or column (Z-type) of the string
  int8_t from, to;  // the string covers indices from..to along that line
};

struct PlanHeader {  // device-visible, followed by the tables at the offsets below
  int32_t d, n, m, nsite, nstep, chi, group;
  int32_t lx_col, lz_row;  // logical representatives: X on column lx_col, Z on row lz_row (both d-1)
  int32_t steps_ofs;    // SiteStep[nstep][nsite]
  int32_t codes_ofs;    // uint8 codes
  int32_t checks_ofs;   // CheckDesc[m]
  int32_t region_ofs;   // int64 element offset of each site's scratch region [nsite]
  int32_t init_qi_ofs;  // uint8 physical dimension of each site before step 0 [nsite]
  int32_t final_ofs;    // int16 [nsite][3]: Dl, qo, Dr of the final MPS
  int32_t bu_steps_ofs; // SiteStep[nstep][nsite]: bottom-up sweep, row nstep-1 first (transposed MPOs)
  int32_t bu_final_ofs; // int16 [nsite][3]: dims of the bottom-up MPS after its last row
  int32_t bytes;        // total blob size
  int64_t scratch_elems;  // scratch elements of one MPS (site regions)
  int64_t mps_elems;      // elements of one truncated MPS (sum over sites of Dl*q*Dr, max over rows)
  int64_t env_elems;      // elements of the left + right environments of one row (adjoint)
  int64_t tmp_elems;      // elements of one environment temporary (adjoint)
  // maxima used to carve LDS (elements)
  int32_t max_Aj;   // Dl_old * qi * Dr_old           input site tensor
  int32_t max_T;    // m * pad8(Dr_old * B)           one output slice of the MPO-applied site
  int32_t max_X;    // m * qo * kr                    LQ matrix of the right-to-left sweep
  int32_t max_L;    // max(m k, pad8(Dr_old B) kr, k pad8(m))  carry of the right-to-left sweep
  int32_t max_C;    // Dl_new * k                     carry of the left-to-right sweep
  int32_t max_M;    // (Dl_new * qo + 1) * kr         matrix to truncate (padded columns)
  int32_t max_V;    // (kr + 1) * kr                  right rotations
  int32_t max_Q;    // k * qo * kr                    staged orthonormal site
  int32_t max_kr, max_n, max_m, max_rows, max_bond;
  int32_t max_envb;     // one bond of a row environment (adjoint): top bond * MPO bond * bottom bond
  int32_t rounds;       // syndrome rounds T of the network (1: code capacity)
  int32_t shared_rows;  // rows 0..shared_rows-1 touch no qubit of the logical representatives:
                        // their MPOs, hence the MPS after them, are the same for all four cosets
  int32_t max_ncode;    // entries of the largest MPO code table (A*qi*qo*B)
  double flops_fwd;     // counted flops of one coset's contraction (see count in plan.cpp)
  double flops_shared;  // the part of flops_fwd spent in rows 0..shared_rows-1
  double flops_gemm;         // GEMM-class part of flops_fwd (T.L, C.Q, and Q.W on truncated bonds)
  double flops_gemm_shared;  // the part of flops_gemm spent in rows 0..shared_rows-1
  double flops_bu;           // counted flops of one coset's bottom-up sweep (adjoint), as flops_fwd
  double flops_env;          // counted flops of one coset's row environments and derivative tensors (adjoint)
};

struct Plan {
  PlanHeader h;
  std::vector<uint8_t> blob;  // header + tables, as uploaded
};

// Build the plan; returns an empty string on success, else an error message.
// rounds >= 2 (repeated noisy rounds) needs group = 1.
std::string build_plan(int d, int chi, int group, Plan* out, int rounds = 1);

// Element-wise maximum of the LDS maxima of two plans (for one launch that
// serves several plans).
void merge_maxima(PlanHeader* acc, const PlanHeader& h);

// LDS carve-up of the sweep kernel, in bytes from the base.  Storage-type
// buffers (site tensors, carries, GEMM operands) use `rb` bytes per element,
// factorisation buffers (LQ matrix, SVD matrix and rotations) `fb` bytes.  The
// right-to-left phase (Aj, T, X, L, tau/diag/v) and the left-to-right phase
// (C, M, V, Q, sig) are never live together and share storage.
struct LdsLayout {
  int32_t Aj, T, X, L;                // right-to-left phase
  int32_t T2;                         // a second slice of T where the phase has room for it, else -1
  int32_t C, M, V, Lt, Q, sig;        // left-to-right phase
  int32_t tau, diag, v;               // Householder scalars and reflector (both phases)
  int32_t W;                          // MPO values of the current site (<= 64, storage type)
  int32_t red, perm, rank, fbits, syn;  // FP64 reduction scratch, kept columns, column sets, reference-error bits, syndrome
  int32_t nrm;                         // FP64 squared column norms of the truncation SVD
  // adjoint row environments (between row steps, over the storage of the two
  // sweep phases; -1 = kept in the work-group's global scratch instead):
  // three contraction temporaries, the top and bottom site, two bonds of
  // environment
  int32_t gP, gA, gF, gE, gR;
  // X < 0: the LQ matrix of the right-to-left sweep lives in the work-group's
  // global scratch, xg bytes from its base (set by the launch)
  int32_t xg;
  int32_t bytes;
};

inline int32_t pad64b(int64_t x) { return (int32_t)((x + 63) / 64 * 64); }

// Caller workspace header (the first kWorkspaceAlign bytes of every workspace):
// work counters from byte 0, the status word of the last call at
// kStatusOffset (ST_* bits) and its 64-bit count of unresolved cosets 8 bytes on.
constexpr size_t kWorkspaceAlign = 256;
constexpr size_t kStatusOffset = 128;

// aj_global: the MPO step reads the input site tensor from its scratch region
// instead of an LDS copy (o.Aj = -1), to fit two work-groups of the 256-thread
// build in a CU.  x_global: the LQ matrix of the right-to-left sweep (the
// largest buffer, m x qo kr) lives in global scratch too (o.X = -1; the launch
// sets o.xg); its explicit Q then stages one reflector at a time through LDS.
inline LdsLayout lds_layout(const PlanHeader& h, int rb, int fb, bool aj_global = false, bool x_global = false) {
  LdsLayout o{};
  int32_t p = 0;
  o.Aj = aj_global ? -1 : p;
  if (!aj_global) p += pad64b((int64_t)h.max_Aj * rb);
  o.T = p; p += pad64b((int64_t)h.max_T * rb);
  o.X = x_global ? -1 : p;
  if (!x_global) p += pad64b((int64_t)h.max_X * fb);
  o.xg = 0;
  o.L = p; p += pad64b((int64_t)h.max_L * rb);
  const int32_t rl_end = p;
  p = 0;
  o.C = p; p += pad64b((int64_t)h.max_C * rb);
  o.M = p; p += pad64b((int64_t)h.max_M * fb);
  o.V = p; p += pad64b((int64_t)h.max_V * fb);
  o.Lt = p; p += pad64b((int64_t)h.max_V * fb);
  o.sig = p; p += pad64b((int64_t)(h.max_kr > h.max_bond ? h.max_kr : h.max_bond) * fb);
  const int32_t lr_end = p;
  // a second T slice (the MPO step then builds two output slices per pass) where
  // the right-to-left phase has room for it below the left-to-right phase's end
  // (used by the kernels built for an LQ matrix in scratch)
  o.T2 = -1;
  if (rl_end + pad64b((int64_t)h.max_T * rb) <= lr_end) o.T2 = rl_end;
  p = rl_end > lr_end ? rl_end : lr_end;
  const int32_t nh = h.max_m > h.max_kr ? h.max_m : h.max_kr;
  int32_t nv = h.max_n > h.max_rows ? h.max_n : h.max_rows;
  // the register LQ stages each reflector over a whole row of lanes (128 or 256 columns)
  if (nv < (nv <= 128 ? 128 : 256)) nv = nv <= 128 ? 128 : 256;
  o.tau = p; p += pad64b((int64_t)nh * fb);
  o.diag = p; p += pad64b((int64_t)nh * fb);
  o.v = p; p += pad64b((int64_t)2 * nv * fb);
  {
    // the adjoint's environment contractions run between row steps: their
    // buffers reuse the storage of the two sweep phases [0, phase_end)
    const int32_t phase_end = rl_end > lr_end ? rl_end : lr_end;
    const int32_t tP = pad64b((int64_t)h.tmp_elems * rb), tS = pad64b((int64_t)h.max_Aj * rb),
                  tE = pad64b((int64_t)h.max_envb * rb);
    o.gP = o.gA = o.gF = o.gE = o.gR = -1;
    if (3 * tP + 2 * tS + 2 * tE <= phase_end) {
      o.gP = 0;
      o.gA = 3 * tP;
      o.gF = o.gA + tS;
      o.gE = o.gF + tS;
      o.gR = o.gE + tE;
    } else if (3 * tP <= phase_end) {
      o.gP = 0;
    }
  }
  o.W = p; p += pad64b((int64_t)(h.max_ncode > 64 ? h.max_ncode : 64) * rb);
  o.red = p; p += 64 * 8;
  o.nrm = p; p += pad64b((int64_t)(h.max_kr > h.max_bond ? h.max_kr : h.max_bond) * 8);
  o.perm = p; p += pad64b((int64_t)h.max_kr * 4);
  o.fbits = p; p += pad64b(h.n);
  o.syn = p; p += pad64b(h.m);
  o.bytes = p;
  return o;
}

}  // namespace tnmld
