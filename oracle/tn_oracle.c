/*
 * FP64 CPU oracle for maximum-likelihood coset decoding of the rotated surface
 * code under independent per-qubit Pauli noise.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links, loads or calls
 * this file; only the test suite, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, table or header with the GPU library.
 *
 * What it computes (paper, Sec. 2.3, eqs. "coset_prob" and "mld_formal"):
 *     Z_l(s) = sum over Pauli errors E with syndrome s and logical class l of
 *              prod_q p_q(E_q),
 * the posterior log P(l|s) = log Z_l - log sum_l' Z_l', and the class.
 *
 * Procedures (each follows one passage of the paper):
 *   O1 orc_enumerate        - every E in {I,X,Y,Z}^n (eq. "mld"), d = 3 only.
 *   O2 orc_generator_sum    - sum over stabiliser products of a representative
 *                             error (Sec. 3.2.1, generator-picture equation).
 *   O3 orc_transfer         - exact (untruncated) contraction of the same
 *                             network, qubit by qubit in row-major order, with
 *                             one binary variable per stabiliser generator
 *                             (Sec. 3.2.1; the boundary-MPS limit chi -> inf).
 *   O4 orc_rbim             - bit-flip noise as a random-bond Ising partition
 *                             function over spins on X-type plaquettes
 *                             (Sec. 3.1.1, eq. "rbim").
 *   O5 orc_grad_logp        - d log P(s) / d log p_{q,P} for P in {X,Y,Z} with
 *                             p_I = 1 - sum, from single-qubit posterior
 *                             marginals obtained by restricting qubit q to one
 *                             Pauli in O3 (the derivative of the likelihood in
 *                             eq. "dmle_loss").
 *   O6 orc_phen_enum2       - phenomenological noise (Sec. 2.2, repeated noisy
 *                             syndrome rounds), T = 2 rounds, d = 3: every
 *                             first-round error, with the second round's
 *                             errors summed through the O1 table.
 *   O7 orc_phen_transfer    - the same distribution for any T (small d): the
 *                             sum over every per-round error consistent with
 *                             the measured syndromes, as a transfer over the
 *                             qubits with the checks' partial parities as the
 *                             state (the (2+1)-D problem of Sec. 3.2.3,
 *                             computed exactly).
 *
 * Phenomenological model (O6, O7).  Rounds t = 1..T.  Before round t every
 * qubit suffers E_t(q) with the code-capacity rates; C_t = E_1 ... E_t is the
 * accumulated error.  Round t < T reports s_t = sigma(C_t) xor m_t, each check
 * j flipped independently with probability meas[j]; round T is perfect,
 * s_T = sigma(C_T).  The class is that of C_T.  With E_t = C_{t-1} C_t:
 *     Z_l(s_1..s_T) = sum over C_1..C_T with sigma(C_T) = s_T and class(C_T) = l
 *         of prod_t prod_q p_q(C_{t-1,q} C_{t,q})
 *            * prod_{t<T} prod_j meas_j^{[s_tj != sigma_j(C_t)]} (1-meas_j)^{[s_tj == sigma_j(C_t)]},
 * C_0 = I.
 *
 * Conventions: qubit q = r*d + c; Pauli 0=I,1=X,2=Y,3=Z (x-bit for X,Y; z-bit
 * for Y,Z); checks at corners (r,c) in [-1,d-1]^2, X-type iff r+c even; bulk
 * corners 0..d-2, X-type boundary checks on top/bottom, Z-type on left/right;
 * syndrome order Z-type checks then X-type checks, each by corner; logical
 * class (x-parity on row 0, z-parity on column 0) -> I=0, X=1, Y=2, Z=3.
 * Representative (pure) errors: a Z-type check at corner (r,c) is flipped
 * alone by X on column max(c,0), rows 0..r; an X-type check by Z on row
 * max(r,0), columns 0..c.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXD 21
#define ORC_MAXN (ORC_MAXD * ORC_MAXD)
#define ORC_MAXM (ORC_MAXN - 1)

typedef struct {
    int d, n, m;
    int type[ORC_MAXM]; /* 0 = X-type, 1 = Z-type */
    int cr[ORC_MAXM], cc[ORC_MAXM];
    int supp[ORC_MAXM][4];
    int ns[ORC_MAXM];
} code_t;

static int build_code(int d, code_t* C) {
    if (d < 3 || d > ORC_MAXD || (d % 2) == 0) return -1;
    C->d = d;
    C->n = d * d;
    C->m = 0;
    for (int pass = 0; pass < 2; ++pass) { /* pass 0: Z-type, pass 1: X-type */
        for (int r = -1; r <= d - 1; ++r) {
            for (int c = -1; c <= d - 1; ++c) {
                int is_x = ((r + c) & 1) == 0;
                int bulk = r >= 0 && c >= 0 && r <= d - 2 && c <= d - 2;
                int tb = (r == -1 || r == d - 1) && is_x && c >= 0 && c <= d - 2;
                int lr = (c == -1 || c == d - 1) && !is_x && r >= 0 && r <= d - 2;
                if (!(bulk || tb || lr)) continue;
                if ((pass == 0) == is_x) continue;
                int j = C->m++;
                C->type[j] = is_x ? 0 : 1;
                C->cr[j] = r;
                C->cc[j] = c;
                C->ns[j] = 0;
                for (int k = 0; k < 4; ++k) C->supp[j][k] = -1;
                for (int dr = 0; dr < 2; ++dr)
                    for (int dc = 0; dc < 2; ++dc) {
                        int rr = r + dr, cq = c + dc;
                        if (rr >= 0 && rr < d && cq >= 0 && cq < d) C->supp[j][C->ns[j]++] = rr * d + cq;
                    }
            }
        }
    }
    return 0;
}

static inline int xbit(int p) { return p == 1 || p == 2; }
static inline int zbit(int p) { return p == 2 || p == 3; }
static inline int pauli_of(int x, int z) { return x ? (z ? 2 : 1) : (z ? 3 : 0); }

/* ---------------------------------------------------------------- helpers */
int orc_layout(int d, int* type_out, int* support_out) {
    code_t C;
    if (build_code(d, &C)) return -1;
    for (int j = 0; j < C.m; ++j) {
        type_out[j] = C.type[j];
        for (int k = 0; k < 4; ++k) support_out[4 * j + k] = C.supp[j][k];
    }
    return C.m;
}

static void syndrome_of(const code_t* C, const uint8_t* e, uint8_t* s) {
    for (int j = 0; j < C->m; ++j) {
        int par = 0;
        for (int k = 0; k < C->ns[j]; ++k) {
            int p = e[C->supp[j][k]];
            par ^= (C->type[j] == 1) ? xbit(p) : zbit(p);
        }
        s[j] = (uint8_t)par;
    }
}

static int class_of(const code_t* C, const uint8_t* e) {
    int a = 0, b = 0;
    for (int c = 0; c < C->d; ++c) a ^= xbit(e[c]);
    for (int r = 0; r < C->d; ++r) b ^= zbit(e[r * C->d]);
    return pauli_of(a, b);
}

int orc_syndrome(int d, const uint8_t* errors, int64_t count, uint8_t* syn_out, uint8_t* class_out) {
    code_t C;
    if (build_code(d, &C)) return -1;
    for (int64_t b = 0; b < count; ++b) {
        syndrome_of(&C, errors + b * C.n, syn_out + b * C.m);
        if (class_out) class_out[b] = (uint8_t)class_of(&C, errors + b * C.n);
    }
    return 0;
}

/* Pauli product of two n-qubit Paulis (phases dropped): XOR of (x,z). */
static void pauli_mul(int n, uint8_t* a, const uint8_t* b) {
    for (int q = 0; q < n; ++q) {
        int x = xbit(a[q]) ^ xbit(b[q]), z = zbit(a[q]) ^ zbit(b[q]);
        a[q] = (uint8_t)pauli_of(x, z);
    }
}

/* Representative error flipping check j alone. */
static void pure_error(const code_t* C, int j, uint8_t* t) {
    int d = C->d;
    memset(t, 0, (size_t)C->n);
    if (C->type[j] == 1) {
        int col = C->cc[j] < 0 ? 0 : C->cc[j];
        for (int r = 0; r <= C->cr[j]; ++r) t[r * d + col] = 1;
    } else {
        int row = C->cr[j] < 0 ? 0 : C->cr[j];
        for (int c = 0; c <= C->cc[j]; ++c) t[row * d + c] = 3;
    }
}

int orc_pure_error(int d, int j, uint8_t* out) {
    code_t C;
    if (build_code(d, &C) || j < 0 || j >= C.m) return -1;
    pure_error(&C, j, out);
    return 0;
}

/* Logical representative of class l (I, X, Y, Z): X on column 0, Z on row 0. */
static void logical_rep(const code_t* C, int l, uint8_t* t) {
    int d = C->d;
    memset(t, 0, (size_t)C->n);
    if (l == 1 || l == 2)
        for (int r = 0; r < d; ++r) t[r * d] = 1;
    if (l == 3 || l == 2) {
        uint8_t z[ORC_MAXN];
        memset(z, 0, (size_t)C->n);
        for (int c = 0; c < d; ++c) z[c] = 3;
        pauli_mul(C->n, t, z);
    }
}

/* Base errors R(s) * L_l for l = 0..3 and the class each one represents. */
static void coset_bases(const code_t* C, const uint8_t* s, uint8_t bases[4][ORC_MAXN], int label[4]) {
    uint8_t R[ORC_MAXN], t[ORC_MAXN];
    memset(R, 0, (size_t)C->n);
    for (int j = 0; j < C->m; ++j)
        if (s[j]) {
            pure_error(C, j, t);
            pauli_mul(C->n, R, t);
        }
    for (int l = 0; l < 4; ++l) {
        logical_rep(C, l, t);
        memcpy(bases[l], R, (size_t)C->n);
        pauli_mul(C->n, bases[l], t);
        label[l] = class_of(C, bases[l]);
    }
}

/* Per-qubit weights w[q][P] = p_q(P), p_I = 1 - p_X - p_Y - p_Z. */
static void weights_from_rates(int n, const double* rates, double* w) {
    for (int q = 0; q < n; ++q) {
        double px = rates[3 * q], py = rates[3 * q + 1], pz = rates[3 * q + 2];
        w[4 * q + 0] = 1.0 - px - py - pz;
        w[4 * q + 1] = px;
        w[4 * q + 2] = py;
        w[4 * q + 3] = pz;
    }
}


/* Neumaier compensated accumulator. */
typedef struct { double s, c; } ksum_t;
static inline void kadd(ksum_t* k, double v) {
    double t = k->s + v;
    if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
    else k->c += (v - t) + k->s;
    k->s = t;
}
static inline double kval(const ksum_t* k) { return k->s + k->c; }

/* ---------------------------------------------------------------- O1
 * table[s_index][l] = Z_l(s) for every syndrome (s_index = sum_j s_j 2^j),
 * by enumerating all 4^n errors.  Optional marg[s_index][q][P] accumulates
 * sum over E with syndrome s and E_q = P of Pr(E).  n <= 12. */
int orc_enumerate(int d, const double* rates, double* table, double* marg) {
    code_t C;
    if (build_code(d, &C) || C.n > 12) return -1;
    int n = C.n, m = C.m;
    double w[4 * ORC_MAXN];
    weights_from_rates(n, rates, w);
    size_t ns = (size_t)1 << m;
    ksum_t* acc = calloc(ns * 4, sizeof(ksum_t));
    ksum_t* macc = marg ? calloc(ns * (size_t)n * 4, sizeof(ksum_t)) : NULL;
    uint8_t e[ORC_MAXN], s[ORC_MAXM];
    uint64_t total = (uint64_t)1 << (2 * n);
    for (uint64_t code = 0; code < total; ++code) {
        double pr = 1.0;
        for (int q = 0; q < n; ++q) {
            e[q] = (uint8_t)((code >> (2 * q)) & 3);
            pr *= w[4 * q + e[q]];
        }
        syndrome_of(&C, e, s);
        size_t si = 0;
        for (int j = 0; j < m; ++j) si |= (size_t)s[j] << j;
        kadd(&acc[si * 4 + class_of(&C, e)], pr);
        if (macc)
            for (int q = 0; q < n; ++q) kadd(&macc[(si * n + q) * 4 + e[q]], pr);
    }
    for (size_t i = 0; i < ns * 4; ++i) table[i] = kval(&acc[i]);
    if (macc)
        for (size_t i = 0; i < ns * (size_t)n * 4; ++i) marg[i] = kval(&macc[i]);
    free(acc);
    free(macc);
    return 0;
}

/* ---------------------------------------------------------------- O2
 * Z[label] = sum over alpha in {0,1}^m of Pr(base * prod_i S_i^alpha_i). m <= 26. */
int orc_generator_sum(int d, const double* rates, const uint8_t* syn, double* Z) {
    code_t C;
    if (build_code(d, &C) || C.m > 26) return -1;
    int n = C.n, m = C.m;
    double w[4 * ORC_MAXN];
    weights_from_rates(n, rates, w);
    uint8_t bases[4][ORC_MAXN];
    int label[4];
    coset_bases(&C, syn, bases, label);
    for (int l = 0; l < 4; ++l) Z[l] = 0.0;
    for (int l = 0; l < 4; ++l) {
        ksum_t acc = {0.0, 0.0};
        uint8_t e[ORC_MAXN];
        uint64_t total = (uint64_t)1 << m;
        /* Gray-code walk: each step multiplies in one generator. */
        memcpy(e, bases[l], (size_t)n);
        for (uint64_t k = 0; k < total; ++k) {
            if (k) { /* multiply generator j into e: flips x (X-type) or z (Z-type) bits */
                int j = __builtin_ctzll(k);
                for (int t = 0; t < C.ns[j]; ++t) {
                    int q = C.supp[j][t];
                    int x = xbit(e[q]) ^ (C.type[j] == 0), z = zbit(e[q]) ^ (C.type[j] == 1);
                    e[q] = (uint8_t)pauli_of(x, z);
                }
            }
            double pr = 1.0;
            for (int q = 0; q < n; ++q) pr *= w[4 * q + e[q]];
            kadd(&acc, pr);
        }
        Z[label[l]] = kval(&acc);
    }
    return 0;
}

/* ---------------------------------------------------------------- O3
 * Exact contraction over stabiliser variables alpha_j.  The state psi is a
 * dense array over 'slots'; a slot holds one open generator variable, and psi
 * does not depend on free slots.  Qubits are visited in row-major order: the
 * generators touching qubit q that have not been seen yet are opened (take a
 * free slot), psi is multiplied by w_q(base_q * X^(sum of X-type alpha)
 * Z^(sum of Z-type alpha)), and generators whose last qubit is q are summed
 * out (slot freed).  psi is rescaled by its maximum after every qubit and the
 * logarithms are accumulated. */
typedef struct {
    int nslot;
    int first[ORC_MAXM], last[ORC_MAXM];
    int qn[ORC_MAXN];       /* number of generators on qubit q */
    int qg[ORC_MAXN][4];    /* generator ids on qubit q */
} plan_t;

static void make_plan(const code_t* C, plan_t* P) {
    for (int q = 0; q < C->n; ++q) P->qn[q] = 0;
    for (int j = 0; j < C->m; ++j) {
        P->first[j] = C->n;
        P->last[j] = -1;
        for (int k = 0; k < C->ns[j]; ++k) {
            int q = C->supp[j][k];
            if (q < P->first[j]) P->first[j] = q;
            if (q > P->last[j]) P->last[j] = q;
            P->qg[q][P->qn[q]++] = j;
        }
    }
    int open = 0, maxopen = 0;
    for (int q = 0; q < C->n; ++q) {
        for (int j = 0; j < C->m; ++j)
            if (P->first[j] == q) ++open;
        if (open > maxopen) maxopen = open;
        for (int j = 0; j < C->m; ++j)
            if (P->last[j] == q) --open;
    }
    P->nslot = maxopen;
}

static double transfer_one(const code_t* C, const plan_t* P, const double* w, const uint8_t* base, double* psi) {
    int n = C->n, m = C->m;
    size_t N = (size_t)1 << P->nslot;
    int slot_of[ORC_MAXM];
    int slot_used[32] = {0};
    for (size_t i = 0; i < N; ++i) psi[i] = 1.0;
    double logscale = 0.0;
    for (int q = 0; q < n; ++q) {
        for (int k = 0; k < P->qn[q]; ++k) {
            int j = P->qg[q][k];
            if (P->first[j] == q) {
                int s = 0;
                while (slot_used[s]) ++s;
                slot_used[s] = 1;
                slot_of[j] = s;
            }
        }
        size_t mx = 0, mz = 0;
        for (int k = 0; k < P->qn[q]; ++k) {
            int j = P->qg[q][k];
            if (C->type[j] == 0) mx |= (size_t)1 << slot_of[j];
            else mz |= (size_t)1 << slot_of[j];
        }
        int bx = xbit(base[q]), bz = zbit(base[q]);
        double wq[4];
        for (int k = 0; k < 4; ++k) wq[k] = w[4 * q + k];
        double mxv = 0.0;
        for (size_t i = 0; i < N; ++i) {
            int x = bx ^ (__builtin_popcountll(i & mx) & 1);
            int z = bz ^ (__builtin_popcountll(i & mz) & 1);
            psi[i] *= wq[pauli_of(x, z)];
        }
        for (int k = 0; k < P->qn[q]; ++k) {
            int j = P->qg[q][k];
            if (P->last[j] == q) {
                size_t b = (size_t)1 << slot_of[j];
                for (size_t i = 0; i < N; ++i)
                    if (!(i & b)) {
                        double v = psi[i] + psi[i | b];
                        psi[i] = v;
                        psi[i | b] = v;
                    }
                slot_used[slot_of[j]] = 0;
            }
        }
        for (size_t i = 0; i < N; ++i)
            if (psi[i] > mxv) mxv = psi[i];
        if (!(mxv > 0.0)) return -INFINITY;
        for (size_t i = 0; i < N; ++i) psi[i] /= mxv;
        logscale += log(mxv);
    }
    (void)m;
    return logscale + log(psi[0]);
}

/* logZ[l] for one syndrome with explicit per-qubit weight table w[n][4]. */
int orc_transfer_w(int d, const double* w, const uint8_t* syn, double* logZ) {
    code_t C;
    if (build_code(d, &C)) return -1;
    plan_t P;
    make_plan(&C, &P);
    uint8_t bases[4][ORC_MAXN];
    int label[4];
    coset_bases(&C, syn, bases, label);
    double* psi = malloc(sizeof(double) << P.nslot);
    if (!psi) return -2;
    for (int l = 0; l < 4; ++l) logZ[label[l]] = transfer_one(&C, &P, w, bases[l], psi);
    free(psi);
    return 0;
}

int orc_max_slots(int d) {
    code_t C;
    if (build_code(d, &C)) return -1;
    plan_t P;
    make_plan(&C, &P);
    return P.nslot;
}

/* Batched O3 over syndromes: rates [n_models][n][3], model_index [count] or
 * NULL, syndromes [count][m] -> logZ [count][4].  OpenMP over syndromes. */
int orc_transfer(int d, const double* rates, int n_models, const int32_t* model_index, const uint8_t* syn,
                 int64_t count, double* logZ, int nthreads) {
    code_t C;
    if (build_code(d, &C)) return -1;
    int n = C.n, m = C.m;
    double* w = malloc(sizeof(double) * 4 * (size_t)n * (size_t)n_models);
    for (int k = 0; k < n_models; ++k) weights_from_rates(n, rates + (size_t)k * n * 3, w + (size_t)k * n * 4);
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t b = 0; b < count; ++b) {
        int mi = model_index ? model_index[b] : 0;
        if (orc_transfer_w(d, w + (size_t)mi * n * 4, syn + b * m, logZ + 4 * b)) err = -2;
    }
    (void)nthreads;
    free(w);
    return err;
}

/* ---------------------------------------------------------------- O4
 * Bit-flip noise only (p_Y = p_Z = 0, p_X = p on every qubit).  Spins tau = +-1
 * on the X-type plaquettes; a missing plaquette is a fixed +1.  With
 * K = ln((1-p)/p) / 2 and eta_q = (-1)^(x-bit of the base error on q),
 *   Z = (p(1-p))^(n/2) sum_tau exp(K sum_q eta_q prod_{X-plaquettes P on q} tau_P).
 * Cosets whose base carries a z-bit (and any syndrome with an X-type check
 * fired) have probability zero. */
int orc_rbim(int d, double p, const uint8_t* syn, double* logZ) {
    code_t C;
    if (build_code(d, &C)) return -1;
    int n = C.n;
    int xs[ORC_MAXM], nx = 0;
    for (int j = 0; j < C.m; ++j)
        if (C.type[j] == 0) xs[nx++] = j;
    if (nx > 26) return -1;
    /* per qubit: which X-plaquette spins sit on it */
    int qn[ORC_MAXN], qs[ORC_MAXN][2];
    for (int q = 0; q < n; ++q) qn[q] = 0;
    for (int k = 0; k < nx; ++k) {
        int j = xs[k];
        for (int t = 0; t < C.ns[j]; ++t) {
            int q = C.supp[j][t];
            qs[q][qn[q]++] = k;
        }
    }
    uint8_t bases[4][ORC_MAXN];
    int label[4];
    coset_bases(&C, syn, bases, label);
    double K = 0.5 * log((1.0 - p) / p);
    double pref = 0.5 * n * log(p * (1.0 - p));
    for (int l = 0; l < 4; ++l) {
        int has_z = 0;
        for (int q = 0; q < n; ++q) has_z |= zbit(bases[l][q]);
        if (has_z) {
            logZ[label[l]] = -INFINITY;
            continue;
        }
        int eta[ORC_MAXN];
        for (int q = 0; q < n; ++q) eta[q] = xbit(bases[l][q]) ? -1 : 1;
        /* log-sum-exp over spin configurations */
        uint64_t total = (uint64_t)1 << nx;
        double emax = -INFINITY;
        for (int pass = 0; pass < 2; ++pass) {
            ksum_t acc = {0.0, 0.0};
            for (uint64_t cfg = 0; cfg < total; ++cfg) {
                int e = 0;
                for (int q = 0; q < n; ++q) {
                    int prod = eta[q];
                    for (int t = 0; t < qn[q]; ++t)
                        if ((cfg >> qs[q][t]) & 1) prod = -prod;
                    e += prod;
                }
                double E = K * e;
                if (pass == 0) {
                    if (E > emax) emax = E;
                } else {
                    kadd(&acc, exp(E - emax));
                }
            }
            if (pass == 1) logZ[label[l]] = pref + emax + log(kval(&acc));
        }
    }
    return 0;
}

/* ---------------------------------------------------------------- O5
 * grad[q][k] = d log P(s) / d log p_{q,k+1}, k = 0,1,2 (X, Y, Z), with
 * p_I = 1 - sum.  Posterior marginals pi_q(P|s) come from O3 with qubit q
 * restricted to Pauli P:  pi_q(P|s) = sum_l Z_l^{(q,P)} / sum_l Z_l.
 * Then grad = pi_q(P|s) - (p_P / p_I) pi_q(I|s).  Also returns log P(s). */
static double lse4(const double* v) {
    double mx = -INFINITY;
    for (int k = 0; k < 4; ++k)
        if (v[k] > mx) mx = v[k];
    if (mx == -INFINITY) return -INFINITY;
    double s = 0.0;
    for (int k = 0; k < 4; ++k) s += exp(v[k] - mx);
    return mx + log(s);
}

int orc_grad_logp(int d, const double* rates, const uint8_t* syn, double* grad, double* logp_out) {
    code_t C;
    if (build_code(d, &C)) return -1;
    int n = C.n;
    double* w = malloc(sizeof(double) * 4 * (size_t)n);
    weights_from_rates(n, rates, w);
    double lz[4];
    if (orc_transfer_w(d, w, syn, lz)) {
        free(w);
        return -2;
    }
    double logp = lse4(lz);
    if (logp_out) *logp_out = logp;
    for (int q = 0; q < n; ++q) {
        double pi[4];
        double keep[4];
        for (int k = 0; k < 4; ++k) keep[k] = w[4 * q + k];
        for (int P = 0; P < 4; ++P) {
            for (int k = 0; k < 4; ++k) w[4 * q + k] = (k == P) ? keep[k] : 0.0;
            double lzm[4];
            orc_transfer_w(d, w, syn, lzm);
            pi[P] = exp(lse4(lzm) - logp);
        }
        for (int k = 0; k < 4; ++k) w[4 * q + k] = keep[k];
        for (int k = 0; k < 3; ++k) {
            double pP = keep[k + 1], pI = keep[0];
            grad[3 * q + k] = pi[k + 1] - (pP / pI) * pi[0];
        }
    }
    free(w);
    return 0;
}

/* ---------------------------------------------------------------- O6
 * T = 2, d = 3.  Z_l = sum_{C_1} Pr(E_1 = C_1) Pr(m_1) * sum_{E_2} Pr(E_2)
 * [sigma(C_1 E_2) = s_2, class(C_1 E_2) = l].  The inner sum is the O1 table
 * entry of syndrome s_2 xor sigma(C_1) and class l xor class(C_1) (both are
 * linear in the error).  syn: [2][m]; logZ[4]. */
int orc_phen_enum2(int d, const double* rates, const double* meas, const uint8_t* syn, int64_t count, double* logZ) {
    code_t C;
    if (build_code(d, &C) || C.n > 12) return -1;
    int n = C.n, m = C.m;
    double w[4 * ORC_MAXN];
    weights_from_rates(n, rates, w);
    double* table = malloc(sizeof(double) * ((size_t)4 << m));
    if (!table || orc_enumerate(d, rates, table, NULL)) {
        free(table);
        return -2;
    }
    uint8_t e[ORC_MAXN], s1[ORC_MAXM];
    uint64_t total = (uint64_t)1 << (2 * n);
    for (int64_t b = 0; b < count; ++b) {
        const uint8_t* sy1 = syn + b * 2 * m;
        const uint8_t* sy2 = sy1 + m;
        size_t si2 = 0;
        for (int j = 0; j < m; ++j) si2 |= (size_t)sy2[j] << j;
        ksum_t acc[4] = {{0, 0}, {0, 0}, {0, 0}, {0, 0}};
        for (uint64_t code = 0; code < total; ++code) {
            double pr = 1.0;
            for (int q = 0; q < n; ++q) {
                e[q] = (uint8_t)((code >> (2 * q)) & 3);
                pr *= w[4 * q + e[q]];
            }
            syndrome_of(&C, e, s1);
            size_t si = 0;
            for (int j = 0; j < m; ++j) {
                pr *= (s1[j] != sy1[j]) ? meas[j] : 1.0 - meas[j];
                si |= (size_t)s1[j] << j;
            }
            const int c1 = class_of(&C, e);
            for (int l = 0; l < 4; ++l) {
                const int l2 = pauli_of(xbit(l) ^ xbit(c1), zbit(l) ^ zbit(c1));
                kadd(&acc[l], pr * table[(si2 ^ si) * 4 + l2]);
            }
        }
        for (int l = 0; l < 4; ++l) {
            double v = kval(&acc[l]);
            logZ[4 * b + l] = v > 0.0 ? log(v) : -INFINITY;
        }
    }
    free(table);
    return 0;
}

/* ---------------------------------------------------------------- O7
 * Any T (1 <= T <= 4), small d.  Qubits in row-major order; each qubit takes
 * all 4^T histories (C_{1,q}..C_{T,q}) with weight prod_t p_q(C_{t-1,q} C_{t,q}).
 * The state holds, for every open check (the slots of O3) and every round,
 * the parity of sigma_j(C_t) over the qubits seen so far, plus the two class
 * parities of C_T; a history XORs its contributions into the state.  When a
 * check's last qubit is done, round t < T multiplies by the measurement
 * probability of s_tj given the parity and round T keeps parity == s_Tj; the
 * slot is then free (its bits back to 0).  psi is rescaled after every qubit.
 * syn: [count][T][m]; meas: [m]; logZ: [count][4]. */
static int phen_one(const code_t* C, const plan_t* P, int T, const double* w, const double* meas,
                    const uint8_t* syn, double* psi, double* tmp, double* logZ) {
    const int n = C->n, d = C->d;
    const int sb = P->nslot * T, cb = sb;  /* class bits at cb (x, row 0) and cb + 1 (z, column 0) */
    const size_t N = (size_t)1 << (sb + 2);
    int slot_of[ORC_MAXM];
    int slot_used[32] = {0};
    for (size_t i = 0; i < N; ++i) psi[i] = 0.0;
    psi[0] = 1.0;
    double logscale = 0.0;
    const int nh = 1 << (2 * T);
    for (int q = 0; q < n; ++q) {
        for (int k = 0; k < P->qn[q]; ++k) {
            int j = P->qg[q][k];
            if (P->first[j] == q) {
                int s = 0;
                while (slot_used[s]) ++s;
                slot_used[s] = 1;
                slot_of[j] = s;
            }
        }
        for (size_t i = 0; i < N; ++i) tmp[i] = 0.0;
        for (int h = 0; h < nh; ++h) {
            /* history h: C_t = (h >> 2(t-1)) & 3 as a Pauli code, t = 1..T */
            double wt = 1.0;
            int prev = 0;
            size_t mask = 0;
            for (int t = 0; t < T; ++t) {
                const int c = (h >> (2 * t)) & 3;
                const int e = pauli_of(xbit(prev) ^ xbit(c), zbit(prev) ^ zbit(c));
                wt *= w[4 * q + e];
                prev = c;
                for (int k = 0; k < P->qn[q]; ++k) {
                    const int j = P->qg[q][k];
                    const int flip = C->type[j] == 1 ? xbit(c) : zbit(c);
                    if (flip) mask ^= (size_t)1 << (slot_of[j] * T + t);
                }
                if (t == T - 1) {
                    if (q < d && xbit(c)) mask ^= (size_t)1 << cb;
                    if (q % d == 0 && zbit(c)) mask ^= (size_t)1 << (cb + 1);
                }
            }
            if (wt == 0.0) continue;
            for (size_t i = 0; i < N; ++i)
                if (psi[i] != 0.0) tmp[i ^ mask] += wt * psi[i];
        }
        for (size_t i = 0; i < N; ++i) psi[i] = tmp[i];
        for (int k = 0; k < P->qn[q]; ++k) {
            const int j = P->qg[q][k];
            if (P->last[j] != q) continue;
            const int s = slot_of[j];
            const size_t smask = (((size_t)1 << T) - 1) << (s * T);
            for (size_t i = 0; i < N; ++i) {
                if (i & smask) continue;
                double acc = 0.0;
                for (int bits = 0; bits < (1 << T); ++bits) {
                    const size_t ii = i | ((size_t)bits << (s * T));
                    double g = 1.0;
                    for (int t = 0; t < T; ++t) {
                        const int par = (bits >> t) & 1, obs = syn[t * C->m + j];
                        if (t < T - 1) g *= par != obs ? meas[j] : 1.0 - meas[j];
                        else if (par != obs) g = 0.0;
                    }
                    acc += g * psi[ii];
                }
                for (int bits = 1; bits < (1 << T); ++bits) psi[i | ((size_t)bits << (s * T))] = 0.0;
                psi[i] = acc;
            }
            slot_used[s] = 0;
        }
        double mx = 0.0;
        for (size_t i = 0; i < N; ++i)
            if (fabs(psi[i]) > mx) mx = fabs(psi[i]);
        if (!(mx > 0.0)) {
            for (int l = 0; l < 4; ++l) logZ[l] = -INFINITY;
            return 0;
        }
        for (size_t i = 0; i < N; ++i) psi[i] /= mx;
        logscale += log(mx);
    }
    for (int a = 0; a < 2; ++a)
        for (int b2 = 0; b2 < 2; ++b2) {
            const double v = psi[((size_t)a << cb) | ((size_t)b2 << (cb + 1))];
            logZ[pauli_of(a, b2)] = v > 0.0 ? logscale + log(v) : -INFINITY;
        }
    return 0;
}

int orc_phen_max_bits(int d, int T) {
    code_t C;
    if (build_code(d, &C)) return -1;
    plan_t P;
    make_plan(&C, &P);
    return P.nslot * T + 2;
}

int orc_phen_transfer(int d, int T, const double* rates, const double* meas, const uint8_t* syn, int64_t count,
                      double* logZ, int nthreads) {
    code_t C;
    if (build_code(d, &C) || T < 1 || T > 4) return -1;
    plan_t P;
    make_plan(&C, &P);
    if (P.nslot * T + 2 > 26) return -1;
    int n = C.n, m = C.m;
    double w[4 * ORC_MAXN];
    weights_from_rates(n, rates, w);
    const size_t N = (size_t)1 << (P.nslot * T + 2);
    int err = 0;
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
#endif
    for (int64_t b = 0; b < count; ++b) {
        double* psi = malloc(sizeof(double) * N);
        double* tmp = malloc(sizeof(double) * N);
        if (!psi || !tmp) err = -2;
        else phen_one(&C, &P, T, w, meas, syn + b * (int64_t)T * m, psi, tmp, logZ + 4 * b);
        free(psi);
        free(tmp);
    }
    (void)nthreads;
    return err;
}

/* ---------------------------------------------------------------- decisions
 * Tie rule: the class is the smallest l with logZ_l >= max - tau, where
 * tau = tie_tol * max(1, |max|).  All -inf gives class 0 and log P = -inf. */
int orc_decide(const double* logZ, int64_t count, double tie_tol, double* logp, uint8_t* cls) {
    for (int64_t b = 0; b < count; ++b) {
        const double* z = logZ + 4 * b;
        double mx = -INFINITY;
        for (int k = 0; k < 4; ++k)
            if (z[k] > mx) mx = z[k];
        if (logp) logp[b] = lse4(z);
        if (cls) {
            int c = 0;
            if (mx > -INFINITY) {
                double tau = tie_tol * (fabs(mx) > 1.0 ? fabs(mx) : 1.0);
                for (int k = 3; k >= 0; --k)
                    if (z[k] >= mx - tau) c = k;
            }
            cls[b] = (uint8_t)c;
        }
    }
    return 0;
}
