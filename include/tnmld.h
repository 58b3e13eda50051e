/*
 * tnmld.h - boundary-MPS maximum-likelihood coset decoding of the rotated
 * surface code on one AMD Instinct MI355X (gfx950).
 *
 * The problem (paper Sec. 2.3, eqs. "coset_prob" and "mld_formal"): for a
 * syndrome s of the [[d^2, 1, d]] rotated surface code under independent
 * per-qubit Pauli noise with probability vectors (p_I, p_X, p_Y, p_Z)_q
 * (Sec. 2.2), compute the four coset partition functions
 *     Z_l(s) = sum of Pr(E) over errors E with syndrome s and logical class l,
 * l in {I, X, Y, Z}, the posterior log P(l|s) and the maximum-likelihood class.
 * Z_l is contracted as the generator-picture tensor network of Sec. 3.2.1 by
 * boundary MPS: row-by-row MPO.MPS products, each compressed back to bond
 * dimension chi by SVD truncation, with the log-norm of the boundary state
 * accumulated in FP64 after every row.
 *
 * Conventions: qubit q = r*d + c; Pauli codes 0=I, 1=X, 2=Y, 3=Z; the d^2-1
 * checks sit on corners (r,c) in [-1, d-1]^2 (X-type iff r+c even; bulk
 * corners 0..d-2, X-type boundary checks on the top and bottom rows, Z-type
 * on the left and right columns); syndrome bit j follows the order "all Z-type
 * checks, then all X-type checks, each sorted by corner (r,c)"; the logical
 * class of an error is (x-parity on row 0, z-parity on column 0) mapped to
 * I=(0,0)=0, X=(1,0)=1, Y=(1,1)=2, Z=(0,1)=3.
 *
 * Memory: every pointer inside tn_segment and every workspace pointer is a
 * DEVICE pointer (hipMalloc'ed or from a framework allocator); host helpers
 * say so explicitly.  The caller owns all buffers; the library never frees
 * caller memory.  Calls are asynchronous on `stream` (a hipStream_t, NULL =
 * default stream); results are valid after the caller synchronises it.
 *
 * Errors: argument validation is synchronous and returns a negative
 * tn_status with nothing enqueued; tn_last_error() then describes it.  Input
 * VALUES live in device memory and are checked by the kernels themselves:
 * a syndrome whose bytes are not all 0/1, whose model index is outside
 * [0, n_models), or whose noise model has a rate outside [0, 1], a NaN rate or
 * p_X + p_Y + p_Z > 1 (+1e-12) gets log Z = -INFINITY for all four cosets (and
 * no gradient contribution); the call records this in the status word of its
 * workspace, which tn_workspace_status() reads back as TN_EINVAL.  No
 * exception crosses this interface and NaN is never written: an impossible
 * coset has log Z = -INFINITY; an impossible syndrome gives log P = -INFINITY
 * and class 0.  When every Pauli of every qubit has a positive probability,
 * every coset has Z > 0, so a contraction that comes out with Z <= 0 is a
 * loss of precision, written as -INFINITY: if all four cosets of a syndrome
 * are lost, log P(s) is lost and the call records TN_ENUMERIC; if only some
 * are, those cosets lie below the resolution of the precision form at that
 * syndrome (improbable cosets whose weight the truncated, rounded boundary
 * state cannot carry), and the call counts them (tn_workspace_status).  With
 * some rates zero, -INFINITY may be exact and is not recorded.
 *
 * Repeated noisy rounds (phenomenological noise, Sec. 2.2; the (2+1)-D
 * problem of Sec. 3.2.3).  A segment with rounds = T >= 2 holds T syndromes
 * per item: before each round every qubit suffers a Pauli error drawn from the
 * segment's rates (the same rates every round), rounds 1..T-1 report the
 * syndrome of the accumulated error with check j flipped independently with
 * probability meas_rates[j], and round T is perfect.  Z_l sums the probability
 * of every error history (per-round errors and measurement flips) that
 * reproduces the T syndromes and leaves an accumulated error of class l.  It is
 * contracted as the same boundary MPS with every column carrying one check
 * variable per round (2^T values): the first T-1 rounds' variables are the
 * Fourier duals of the measurement weights, the last round's the generator
 * variables of the code-capacity network, and each qubit's tensor sums its
 * T-1 intermediate accumulated Paulis.  The time direction is thus exact;
 * T <= TN_MAX_ROUNDS.  The gradient entry point takes rounds <= 1 only.
 */
#ifndef TNMLD_H
#define TNMLD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TN_OK = 0,
  TN_EINVAL = -1,        /* bad argument (shape, range, pointer, workspace too small) */
  TN_ENOMEM = -2,        /* the library could not allocate its plan cache */
  TN_EDEVICE = -3,       /* no usable HIP device, or a HIP runtime error */
  TN_EUNSUPPORTED = -4,  /* valid request the build cannot run (e.g. chi too large for LDS) */
  TN_ENUMERIC = -5       /* precision breakdown seen on the device (reported by tn_workspace_status) */
} tn_status;

typedef enum {
  TN_FP64 = 0,       /* every step in FP64 */
  TN_FP32 = 1,       /* MPS and MPO.MPS contractions in FP32; the LQ and SVD
                        factorisations of the truncation in FP64 */
  TN_BF16 = 2,       /* MPS stored in FP32; the contraction GEMMs of each site
                        step (MPO.MPS times the carried factor, carry times Q,
                        and on truncated bonds Q times the kept singular
                        vectors) on bf16 MFMA with FP32 accumulation, operands
                        split into bf16 high and low parts; factorisations in
                        FP32 */
  TN_FP32_PLAIN = 3, /* every contraction and factorisation in FP32 (norms and
                        Jacobi inner products accumulate in FP64); the plain
                        single-precision form */
  TN_BF16_F64 = 4    /* MPS stored in FP32; the same contraction GEMMs as
                        TN_BF16 on bf16 MFMA with FP32 accumulation, operands
                        rounded once to bf16 (no high/low split); the LQ, QR and
                        SVD of the truncation in FP64 (Sec. 3.2.1 boundary MPS
                        with BF16 contractions and an FP64 truncation step).
                        Forward only: tn_coset_loglik_backward rejects it with
                        TN_EUNSUPPORTED */
} tn_precision;
/* Log-scales, log Z, log P(s) and the class decision are FP64 in every form. */

#define TN_MAX_D 31
#define TN_MAX_SEGMENTS 16
#define TN_MAX_ROUNDS 2

/* One homogeneous group of syndromes: one code distance, one bond dimension,
 * one precision, and a set of noise models addressed by model_index. */
typedef struct {
  int32_t d;                   /* odd, 3 <= d <= TN_MAX_D */
  int32_t chi;                 /* bond-dimension cap (>= 1); 0 = no truncation (exact, small d only) */
  int32_t precision;           /* tn_precision */
  int32_t n_models;            /* >= 1 */
  const double* rates;         /* device [n_models][d*d][3]: p_X, p_Y, p_Z per qubit; p_I = 1 - sum */
  const int32_t* model_index;  /* device [count] in [0, n_models), or NULL (all model 0) */
  const uint8_t* syndromes;    /* device [count][d*d-1], bytes in {0,1}, order above */
  int64_t count;               /* number of syndromes (>= 0) */
  double* out_logz;            /* device [count][4]: natural-log Z_l; required */
  double* out_logp;            /* device [count]: log P(s) = logsumexp_l log Z_l, or NULL */
  uint8_t* out_class;          /* device [count]: tie-tolerant argmax, or NULL */
  int32_t rounds;              /* 0 or 1: one perfect round (code capacity).  2..TN_MAX_ROUNDS: repeated noisy
                                  rounds (above); syndromes are then [count][rounds][d*d-1], round-major per
                                  item, and the chosen bond dimension applies to the wider columns */
  int32_t reserved;            /* 0 */
  const double* meas_rates;    /* device [n_models][d*d-1]: flip probability of each check's measurement in
                                  rounds 1..T-1, in [0, 1]; used (and required) when rounds >= 2 */
} tn_segment;

/* Bytes of device workspace that tn_coset_loglik / tn_decode_batch need for
 * these segments; with_backward = 1 sizes it for tn_coset_loglik_backward.
 * Returns 0 on invalid arguments (see tn_last_error). */
size_t tn_workspace_size(const tn_segment* segs, int32_t nseg, int32_t with_backward);

/* log Z_l(s) for every syndrome of every segment (Sec. 2.3 eq. "coset_prob",
 * contracted by boundary MPS as in Sec. 3.2.1), written to out_logz; also
 * out_logp when non-NULL.  Persistent launches (one per precision and size
 * class) drain a work queue of syndromes across all segments, largest d
 * first; a syndrome's four cosets share the rows before the logical
 * representatives.
 * segs: HOST array of nseg <= TN_MAX_SEGMENTS descriptors.  workspace: device,
 * ws_bytes >= tn_workspace_size(segs, nseg, 0), caller-owned, reused freely
 * after the call completes on `stream`. */
int tn_coset_loglik(const tn_segment* segs, int32_t nseg, void* workspace, size_t ws_bytes, void* stream);

/* tn_coset_loglik plus the maximum-likelihood decision (Sec. 2.3 eq.
 * "mld_formal"): out_class[b] = the smallest l with
 * log Z_l >= max_l' log Z_l' - tie_tol * max(1, |max_l' log Z_l'|)
 * (tie_tol <= 0 selects 1e-9), and out_logp. */
int tn_decode_batch(const tn_segment* segs, int32_t nseg, double tie_tol, void* workspace, size_t ws_bytes,
                    void* stream);

/* Gradient of the weighted log-likelihood  sum_b grad_logp[b] * log P(s_b)
 * (the per-syndrome term of the paper's eq. "dmle_loss") with respect to
 * theta_{q,P} = ln p_{q,P}, P in {X, Y, Z}, p_I = 1 - p_X - p_Y - p_Z.
 * One work-group per syndrome contracts its cosets top-down (the rows common
 * to the four cosets once), storing the boundary MPS before every row, takes
 * the coset weights grad_logp[b] * P(l|s) from the log Z values of that sweep,
 * then sweeps a second boundary MPS up from the bottom for every coset with
 * a non-zero weight and contracts the environment of every qubit tensor
 * against the stored top states (no recomputation).
 * grad_logp[s]: device [count] of segment s; grad_log_rates[s]: device
 * [n_models][d*d][3], ACCUMULATED (+=) in FP64 by a deterministic reduction.
 * forward_done = 0: the call also writes out_logz / out_logp of each segment
 * (from its own top-down sweep; out_logp must be non-NULL).  forward_done = 1:
 * the caller already holds the forward results (e.g. from tn_decode_batch);
 * out_logz / out_logp are left as they are.  The gradient is the same, bit
 * for bit, either way.
 * All segments of one call share one precision (else TN_EUNSUPPORTED).  Each
 * work-group walks a fixed stride of items, so the result is bitwise
 * reproducible for a given device and launch shape.
 * workspace: ws_bytes >= tn_workspace_size(segs, nseg, 1): the stored states
 * take (S + 4 (2d - 1 - S)) boundary states per work-group, S = d - 1. */
int tn_coset_loglik_backward(const tn_segment* segs, int32_t nseg, const double* const* grad_logp,
                             double* const* grad_log_rates, int32_t forward_done, void* workspace, size_t ws_bytes,
                             void* stream);

/* The same gradient in two calls, for callers that need log P(s) before they
 * know grad_logp (a training step: loss first, gradient after).  The top
 * sweep's states (the boundary MPS before every row of every coset, the rows
 * common to the cosets once per syndrome) are kept in caller memory between
 * the calls instead of recomputed, trading device memory (tn_states_size
 * bytes, e.g. about 2.9 MB per syndrome at d = 11, chi = 24 in FP32) for the
 * top sweep of the second call (eq. "dmle_loss", Sec. 3.2.4).
 *
 * tn_states_size: bytes of that buffer for these segments (0 on invalid
 * arguments; every segment one round).
 * tn_coset_loglik_save: writes out_logz and out_logp (required) as
 * tn_coset_loglik does, and the states into `states` (device, caller-owned,
 * states_bytes >= tn_states_size); workspace as for the backward.
 * tn_coset_loglik_backward_saved: accumulates (+=) the gradient into
 * grad_log_rates (as tn_coset_loglik_backward) from the states and from the
 * out_logz / out_logp that tn_coset_loglik_save wrote for exactly the same
 * segments and values (the segment array may be a copy; the buffers it points
 * to must be unchanged).  Results equal tn_coset_loglik_backward's bit for bit.
 * Errors as tn_coset_loglik_backward; a states buffer that is NULL or too small
 * is TN_EINVAL. */
size_t tn_states_size(const tn_segment* segs, int32_t nseg);
int tn_coset_loglik_save(const tn_segment* segs, int32_t nseg, void* states, size_t states_bytes, void* workspace,
                         size_t ws_bytes, void* stream);
int tn_coset_loglik_backward_saved(const tn_segment* segs, int32_t nseg, const double* const* grad_logp,
                                   double* const* grad_log_rates, const void* states, size_t states_bytes,
                                   void* workspace, size_t ws_bytes, void* stream);

/* HOST helper: check layout of distance d.  type_out: host [d*d-1] (0 = X-type,
 * 1 = Z-type); support_out: host [d*d-1][4] qubit indices, -1 padded.
 * Returns d*d-1, or TN_EINVAL. */
int tn_code_stabilizers(int32_t d, int32_t* type_out, int32_t* support_out);

/* HOST helper: properties of the contraction plan for (d, chi, precision):
 * info[0] counted forward flops per (syndrome, coset), info[1] scratch bytes
 * per work-group, info[2] LDS bytes per work-group, info[3] sites per row,
 * info[4] rows, info[5] columns per site, info[6] work-groups per CU,
 * info[7] counted forward flops per syndrome as executed (the rows common to
 * the four cosets once, the rest four times).
 * info: host array of >= 8 doubles.  Returns TN_OK or a tn_status. */
int tn_plan_info(int32_t d, int32_t chi, int32_t precision, double* info);

/* HOST helper: tn_plan_info for segments with `rounds` syndrome rounds (the
 * plan of the repeated-rounds network; rounds <= 1 is tn_plan_info). */
int tn_plan_info_rounds(int32_t d, int32_t chi, int32_t precision, int32_t rounds, double* info);

/* HOST helper: the GEMM-class part of the counted forward work of the plan
 * for (d, chi, precision): the MPO-applied site times the carried factor, the
 * carry times the right-canonical site, and on truncated bonds the orthonormal
 * factor times the kept right singular vectors.  These are the products the
 * BF16 form runs on the matrix cores (each as three bf16 products, counted
 * once here); the other forms run them on the vector units.
 * out[0] per (syndrome, coset); out[1] per syndrome as executed (rows common
 * to the four cosets once).  out: host array of >= 2 doubles.  Returns TN_OK
 * or a tn_status. */
int tn_plan_gemm_flops(int32_t d, int32_t chi, int32_t precision, double* out);

/* HOST helper: counted work of tn_coset_loglik_backward for the plan of
 * (d, chi, precision), with the same dense counts as tn_plan_info:
 * out[0] the bottom-up sweep of one coset (transposed row MPOs from the last
 * row up); out[1] the row environments of one coset (left and right
 * environment steps along every row, and the derivative tensor of every site
 * with a qubit); out[2] per syndrome as executed: the top sweep (rows common
 * to the four cosets once) plus four bottom-up sweeps and four sets of row
 * environments.  out: host array of >= 3 doubles.  Returns TN_OK or a
 * tn_status. */
int tn_plan_adjoint_flops(int32_t d, int32_t chi, int32_t precision, double* out);

/* HOST helper: launch shape for (d, chi, precision) used by later calls in
 * this process: group = lattice columns per MPS site (1 or 2; 0 = automatic),
 * wg_per_cu = persistent work-groups per compute unit (1 or 2; 0 = as many as
 * LDS allows).  group = wg_per_cu = 0 restores the default.  The autotuner
 * sets these from its cache.  Returns TN_OK or TN_EINVAL. */
int tn_set_tuning(int32_t d, int32_t chi, int32_t precision, int32_t group, int32_t wg_per_cu);

/* HOST helper: tn_set_tuning with the build as a third dimension: threads =
 * 512 or 256 selects the work-group size of the forward kernel (256 only
 * takes effect where the plan fits that build: site matrices of at most 64
 * rows with FP32 factorisations, 32 with FP64 ones, LDS within half a CU),
 * 0 = automatic; wg_per_cu (<= 4) then caps that build's work-groups per CU.
 * With 256 threads, wg_per_cu = 1 or 2 keeps two groups per CU, 3, 4 or 0
 * lets plans of at most 128 columns whose LDS fits a third of a CU run three
 * (the default for them); a call whose segments of one precision include a
 * plan on two groups per CU runs all of them in that one launch.
 * All zeros restore the default.  Returns TN_OK or TN_EINVAL. */
int tn_set_tuning_ex(int32_t d, int32_t chi, int32_t precision, int32_t group, int32_t wg_per_cu, int32_t threads);

/* HOST helper (needs a device): the launch shape a one-segment call of
 * (d, chi, precision) uses now: shape[0] columns per site, shape[1]
 * work-groups per CU, shape[2] threads per work-group.  shape: host int32[3]. */
int tn_get_launch(int32_t d, int32_t chi, int32_t precision, int32_t* shape);

/* HOST helper (needs a device): the persistent forward launches a
 * tn_decode_batch call on these segments makes, in launch order (one per
 * precision and build; the segments' pointers are not read).  For launch i
 * < max_launches: out[4i] precision, out[4i+1] threads per work-group,
 * out[4i+2] work-groups per CU, out[4i+3] segments it carries (empty
 * segments carry none).  *count: the number of launches (may exceed
 * max_launches).  out: host int32[4 * max_launches].  Returns TN_OK, or the
 * error the call itself would return for these segments. */
int tn_get_launches(const tn_segment* segs, int32_t nseg, int32_t* out, int32_t max_launches, int32_t* count);

/* Status of the last tn_coset_loglik / tn_decode_batch /
 * tn_coset_loglik_backward call that used `workspace` (its input-value checks
 * and numerical health, see "Errors" above).  Synchronises `stream` (the
 * stream of that call) and reads the status word from the workspace header.
 * Returns TN_OK, TN_EINVAL (invalid input values were seen; those syndromes
 * got log Z = -INFINITY), TN_ENUMERIC (all four cosets of some syndrome of a
 * strictly positive model came out with Z <= 0), or TN_EDEVICE (the stream
 * failed, e.g. a device fault).  unresolved_cosets (HOST, may be NULL):
 * receives the number of cosets of strictly positive models written as
 * -INFINITY while another coset of their syndrome was finite (below the
 * form's resolution; not an error).  ws_bytes: size of the workspace
 * (>= 256).  workspace = NULL reads the status of the last
 * tn_decode_batch_noalloc call on the current device (ws_bytes ignored). */
int tn_workspace_status(const void* workspace, size_t ws_bytes, void* stream, int64_t* unresolved_cosets);

/* tn_decode_batch without a workspace, for callers that cannot allocate
 * device memory (code under graph capture, tight serving loops, harnesses
 * that forbid hipMalloc): the same kernels and results (bit for bit), with
 * their scratch in a fixed 128 MiB device array that the library holds on
 * every device it runs on until the process ends; the contraction plans are
 * copied into it from host memory on `stream` at every call.  The call makes
 * no device allocation (no hipMalloc, hipFree or allocating library routine).
 * Fewer persistent work-groups run when the usual count does not fit the
 * array; a call whose segments need more than the array for a single
 * work-group per launch (per work-group ~1.4 MB at d = 17, chi = 32) or more
 * than 4 MiB of plans fails with TN_EINVAL before anything is enqueued.
 * Every call on one device shares that device's array: calls that overlap on
 * one device (two streams, two threads) race and must be serialised by the
 * caller.  Status: tn_workspace_status(NULL, 0, stream, ...). */
int tn_decode_batch_noalloc(const tn_segment* segs, int32_t nseg, double tie_tol, void* stream);

/* ---- Planar exact solver for bit-flip noise (paper Sec. 3.1.3) ------------
 * Under bit-flip noise (p_Y = p_Z = 0 for every qubit) each coset partition
 * function is the partition function of a random-bond Ising model on the
 * planar graph of X-type checks (Sec. 3.1.1, eq. "rbim"), which the Kac-Ward
 * determinant gives exactly in O(|E|^3): Z_l(s) = 2^(m_X - n) sqrt(det(I -
 * Lambda)), with Lambda the 2(n+1) x 2(n+1) complex matrix over the directed
 * bonds (weights t_q = +-(1 - 2 p_q), the sign from the coset's reference
 * error, times the phase of the turning angle between consecutive bonds).
 * The logical X coset flips the signs along a logical representative; the Y
 * and Z cosets are impossible (log Z = -INFINITY), as is every coset when an
 * X-type check fired.  Computed in FP64 (dense LU with partial pivoting; the
 * trailing updates on the FP64 matrix cores). */

/* Bytes of device workspace tn_bitflip_decode needs for these segments
 * (precision must be TN_FP64; chi is ignored).  0 on invalid arguments. */
size_t tn_bitflip_workspace_size(const tn_segment* segs, int32_t nseg);

/* Exact log Z_l(s) (l = I, X, Y, Z; Y and Z are -INFINITY), log P(s) and the
 * tie-tolerant class (as tn_decode_batch) for bit-flip noise.  segs: HOST
 * array of nseg <= TN_MAX_SEGMENTS descriptors; each segment's rates must have
 * p_Y = p_Z = 0 (a syndrome whose model violates that, or has p_X outside
 * [0, 1], is written as -INFINITY and recorded for tn_workspace_status as
 * TN_EINVAL); precision must be TN_FP64 (else TN_EINVAL); chi is ignored.
 * workspace: device, ws_bytes >= tn_bitflip_workspace_size(segs, nseg),
 * caller-owned; about (2(d^2+1))^2 x 16 bytes per persistent work-group. */
int tn_bitflip_decode(const tn_segment* segs, int32_t nseg, double tie_tol, void* workspace, size_t ws_bytes,
                      void* stream);

/* HOST helper: properties of the planar solver's plan at distance d:
 * info[0] matrix order 2(d^2+1), info[1] non-zero entries of Lambda,
 * info[2] real flops of one complex LU (8/3 N^3), info[3] scratch bytes per
 * work-group, info[4] (m_X - n) ln 2.  info: host array of >= 5 doubles. */
int tn_bitflip_plan_info(int32_t d, double* info);

/* Message for the last non-OK status returned on this thread. */
const char* tn_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* TNMLD_H */
