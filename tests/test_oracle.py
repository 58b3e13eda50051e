"""Pins for the FP64 oracle: each test ties it to something other than itself.

* layout invariants of the rotated surface code (Sec. 2.1) and agreement with
  the independently written input generator;
* representative errors flip exactly one check;
* O1 (every error, eq. "mld"): probabilities over all syndromes sum to one;
* O2 (generator sum, Sec. 3.2.1) = O1 and O3 (exact contraction) = O1 on every
  d = 3 syndrome; O2 = O3 at d = 5;
* O4 (textbook random-bond Ising model, eq. "rbim") = O3 under bit-flip noise;
* brute force over errors supported on a few qubits = O3 at d up to 17;
* 180-degree rotation symmetry with inhomogeneous rates;
* O5 (gradient of log P(s), eq. "dmle_loss") = central finite differences of
  O3 and = O1 marginals; the score identity sum_s P(s) grad log P(s) = 0.
"""
import itertools

import numpy as np
import pytest

import oracle
import synth


def gf2_rank(mat):
    a = mat.copy().astype(np.uint8)
    rank = 0
    rows, cols = a.shape
    for c in range(cols):
        piv = None
        for r in range(rank, rows):
            if a[r, c]:
                piv = r
                break
        if piv is None:
            continue
        a[[rank, piv]] = a[[piv, rank]]
        for r in range(rows):
            if r != rank and a[r, c]:
                a[r] ^= a[rank]
        rank += 1
    return rank


def symplectic(d):
    """Checks as binary symplectic rows [x | z] from the oracle layout."""
    types, sup = oracle.layout(d)
    n = d * d
    rows = np.zeros((n - 1, 2 * n), np.uint8)
    for j in range(n - 1):
        for q in sup[j]:
            if q >= 0:
                rows[j, q if types[j] == 0 else n + q] = 1
    return types, sup, rows


def commute(a, b, n):
    return (int(a[:n] @ b[n:] + a[n:] @ b[:n]) & 1) == 0


@pytest.mark.parametrize("d", [3, 5, 7, 9, 17])
def test_layout_invariants(d):
    n = d * d
    types, sup, rows = symplectic(d)
    assert (types == 0).sum() == (n - 1) // 2 and (types == 1).sum() == (n - 1) // 2
    weights = (sup >= 0).sum(1)
    assert set(weights.tolist()) <= {2, 4}
    # all checks commute; they are independent
    x, z = rows[:, :n], rows[:, n:]
    assert not ((x @ z.T + z @ x.T) & 1).any()
    assert gf2_rank(rows) == n - 1
    # canonical logicals: X on column 0, Z on row 0
    xl = np.zeros(2 * n, np.uint8)
    xl[[r * d for r in range(d)]] = 1
    zl = np.zeros(2 * n, np.uint8)
    zl[[n + c for c in range(d)]] = 1
    for r in rows:
        assert commute(r, xl, n) and commute(r, zl, n)
    assert not commute(xl, zl, n)
    # Z-type checks first, then X-type; the input generator agrees
    assert (types[: (n - 1) // 2] == 1).all()
    st, ss = synth.code_checks(d)
    assert np.array_equal(st, types) and np.array_equal(ss, sup)


@pytest.mark.parametrize("d", [3, 5, 9, 13, 17])
def test_pure_errors_flip_one_check(d):
    m = d * d - 1
    errs = np.stack([oracle.pure_error(d, j) for j in range(m)])
    s, _ = oracle.syndromes(d, errs)
    assert np.array_equal(s, np.eye(m, dtype=np.uint8))
    assert np.array_equal(synth.syndromes_of(d, errs), s)


@pytest.mark.parametrize("d", [3, 7, 11])
def test_syndromes_and_classes_match_generator(d):
    smp = synth.sample(d, synth.inhomogeneous(d, 0.01, 0.2, seed=d), 200, seed=1)
    s, c = oracle.syndromes(d, smp["errors"])
    assert np.array_equal(s, smp["syndromes"])
    assert np.array_equal(c, smp["true_class"])


def all_syndromes(d):
    m = d * d - 1
    idx = np.arange(1 << m)
    return ((idx[:, None] >> np.arange(m)) & 1).astype(np.uint8)


@pytest.fixture(scope="module")
def d3_table():
    r = synth.depolarizing(3, 0.10)
    return r, oracle.enumerate_table(3, r)


def test_o1_total_probability(d3_table):
    _, t = d3_table
    assert abs(t.sum() - 1.0) < 1e-14
    assert (t >= 0).all()
    r = synth.inhomogeneous(3, 0.01, 0.3, seed=7)
    t2 = oracle.enumerate_table(3, r)
    assert abs(t2.sum() - 1.0) < 1e-14


def test_o1_matches_sampling_frequencies(d3_table):
    # Pr(s, l) from enumeration against the empirical frequency of sampled errors
    r, t = d3_table
    smp = synth.sample(3, r, 200000, seed=11)
    si = (smp["syndromes"].astype(np.int64) << np.arange(8)).sum(1)
    freq = np.zeros((256, 4))
    np.add.at(freq, (si, smp["true_class"]), 1.0)
    freq /= len(si)
    sd = np.sqrt(t * (1 - t) / len(si)) + 1e-12
    assert np.max(np.abs(freq - t) / sd) < 6.0


def test_o2_and_o3_match_o1_all_d3_syndromes(d3_table):
    r, t = d3_table
    syn = all_syndromes(3)
    z2 = np.stack([oracle.generator_sum(3, r, s) for s in syn])
    assert np.max(np.abs(z2 - t) / t) < 1e-13
    lz = oracle.transfer(3, r, syn)
    assert np.max(np.abs(lz - np.log(t))) < 1e-13


def test_o2_matches_o3_d5():
    r = synth.inhomogeneous(5, 0.02, 0.15, seed=3)
    smp = synth.sample(5, r, 2, seed=4)
    for s in smp["syndromes"]:
        z2 = oracle.generator_sum(5, r, s)
        lz = oracle.transfer(5, r, s[None])[0]
        assert np.max(np.abs(np.log(z2) - lz)) < 1e-12


@pytest.mark.parametrize("d,count", [(3, 256), (5, 6), (7, 1)])
def test_o4_rbim_matches_o3_bitflip(d, count):
    p = 0.12
    r = synth.bitflip(d, p)
    if d == 3:
        syn = all_syndromes(3)
    else:
        syn = synth.sample(d, r, count, seed=21)["syndromes"]
    for s in syn[:count]:
        a = oracle.rbim(d, p, s)
        b = oracle.transfer(d, r, s[None])[0]
        fin = np.isfinite(a)
        assert np.array_equal(fin, np.isfinite(b))
        assert np.max(np.abs(a[fin] - b[fin]), initial=0.0) < 1e-11


def test_rbim_worked_values():
    # d = 3, p = 0.1, trivial syndrome: I and X cosets, Y and Z impossible
    z = oracle.rbim(3, 0.10, np.zeros(8, np.uint8))
    assert np.isneginf(z[2]) and np.isneginf(z[3])
    # direct sum: I coset = no error + every X-stabiliser product
    r = synth.bitflip(3, 0.10)
    t = oracle.enumerate_table(3, r)
    assert abs(z[0] - np.log(t[0, 0])) < 1e-13 and abs(z[1] - np.log(t[0, 1])) < 1e-13


def sparse_bruteforce(d, support, rates, syndrome):
    """Z_l(s) over all errors supported on `support` (rates zero elsewhere)."""
    k = len(support)
    n = d * d
    errs = np.zeros((4 ** k, n), np.uint8)
    for i, combo in enumerate(itertools.product(range(4), repeat=k)):
        errs[i, support] = combo
    syn = synth.syndromes_of(d, errs)
    cls = synth.classes_of(d, errs)
    w = np.concatenate([1 - rates.sum(1, keepdims=True), rates], 1)
    pr = np.prod(w[np.arange(n)[None, :], errs], axis=1)
    ok = (syn == syndrome[None, :]).all(1)
    z = np.zeros(4)
    np.add.at(z, cls[ok], pr[ok])
    return z


@pytest.mark.parametrize("d,k,seed", [(5, 6, 0), (9, 6, 1), (13, 5, 2), (17, 5, 3), (17, 6, 4)])
def test_o3_sparse_support_bruteforce(d, k, seed):
    rng = np.random.default_rng(seed)
    n = d * d
    # a connected-ish cluster so that stabiliser products inside the support occur
    r0, c0 = rng.integers(0, d - 2, size=2)
    cand = [(r0 + i) * d + (c0 + j) for i in range(3) for j in range(3)]
    support = sorted(rng.choice(cand, size=k, replace=False).tolist())
    rates = np.zeros((n, 3))
    rates[support] = rng.uniform(0.02, 0.3, size=(k, 3))
    e0 = np.zeros((1, n), np.uint8)
    e0[0, support] = rng.integers(0, 4, size=k)
    s = synth.syndromes_of(d, e0)[0]
    z = sparse_bruteforce(d, support, rates, s)
    lz = oracle.transfer(d, rates, s[None])[0]
    with np.errstate(divide="ignore"):
        ref = np.log(z)
    assert np.array_equal(np.isfinite(ref), np.isfinite(lz))
    f = np.isfinite(ref)
    assert np.max(np.abs(ref[f] - lz[f])) < 1e-12


def rotate_errors(d, e):
    return e.reshape(-1, d, d)[:, ::-1, ::-1].reshape(-1, d * d)


CLASS_BITS = np.array([[0, 0], [1, 0], [1, 1], [0, 1]])


def class_xor(a, b):
    bits = CLASS_BITS[a] ^ CLASS_BITS[b]
    return np.array([[0, 3], [1, 2]])[bits[..., 0], bits[..., 1]]


@pytest.mark.parametrize("d", [3, 5, 7, 9])
def test_o3_rotation_symmetry(d):
    r = synth.inhomogeneous(d, 0.01, 0.2, seed=40 + d)
    smp = synth.sample(d, r, 4, seed=41)
    e = smp["errors"]
    er = rotate_errors(d, e)
    rr = r.reshape(d, d, 3)[::-1, ::-1].reshape(d * d, 3)
    lz = oracle.transfer(d, r, synth.syndromes_of(d, e))
    lzr = oracle.transfer(d, rr, synth.syndromes_of(d, er))
    c, cr = synth.classes_of(d, e), synth.classes_of(d, er)
    for b in range(len(e)):
        for ell in range(4):
            assert abs(lz[b, class_xor(c[b], ell)] - lzr[b, class_xor(cr[b], ell)]) < 1e-10


def test_o3_degenerate_rates():
    d = 7
    n, m = d * d, d * d - 1
    zero = np.zeros((n, 3))
    lz = oracle.transfer(d, zero, np.zeros((1, m), np.uint8))[0]
    assert lz[0] == 0.0 and np.isneginf(lz[1:]).all()
    s = np.zeros((1, m), np.uint8)
    s[0, 5] = 1
    assert np.isneginf(oracle.transfer(d, zero, s)[0]).all()


def logp_of(d, r, s):
    lz = oracle.transfer(d, r, s[None])[0]
    mx = lz.max()
    return mx + np.log(np.exp(lz - mx).sum())


@pytest.mark.parametrize("d", [3, 5])
def test_o5_matches_central_differences(d):
    r = synth.inhomogeneous(d, 0.01, 0.1, seed=50 + d)
    s = synth.sample(d, r, 1, seed=51)["syndromes"][0]
    g, lp = oracle.grad_logp(d, r, s)
    assert abs(lp - logp_of(d, r, s)) < 1e-12
    h = 1e-5
    rng = np.random.default_rng(d)
    picks = [(q, k) for q in rng.choice(d * d, size=min(6, d * d), replace=False) for k in range(3)]
    for q, k in picks:
        rp, rm = r.copy(), r.copy()
        rp[q, k] *= np.exp(h)
        rm[q, k] *= np.exp(-h)
        fd = (logp_of(d, rp, s) - logp_of(d, rm, s)) / (2 * h)
        assert abs(fd - g[q, k]) < 1e-7 * max(1.0, abs(fd))


def test_o5_matches_o1_marginals_and_score_identity():
    d = 3
    r = synth.inhomogeneous(3, 0.02, 0.2, seed=60)
    t, mg = oracle.enumerate_table(3, r, marginals=True)
    syn = all_syndromes(3)
    ps = t.sum(1)
    w = np.concatenate([1 - r.sum(1, keepdims=True), r], 1)
    score = np.zeros((9, 3))
    for si in range(256):
        g, lp = oracle.grad_logp(3, r, syn[si])
        pi = mg[si] / ps[si]  # [n, 4] posterior marginals by enumeration
        ref = pi[:, 1:] - (w[:, 1:] / w[:, :1]) * pi[:, :1]
        assert np.max(np.abs(g - ref)) < 1e-12
        assert abs(lp - np.log(ps[si])) < 1e-13
        score += ps[si] * g
    assert np.max(np.abs(score)) < 1e-14


def test_decide_tie_rule():
    z = np.array([[-1.0, -1.0, -3.0, -4.0],
                  [-5.0, -1.0, -1.0 + 1e-12, -2.0],
                  [-np.inf] * 4,
                  [-np.inf, -2.0, -np.inf, -2.0 - 0.5e-9 * 2.0],
                  [-10.0, -10.0 + 2e-8, -11.0, -12.0]])
    lp, c = oracle.decide(z, tie_tol=1e-9)
    assert c.tolist() == [0, 1, 0, 1, 1]
    assert np.isneginf(lp[2])
    assert abs(lp[0] - np.log(2 * np.exp(-1) + np.exp(-3) + np.exp(-4))) < 1e-14
