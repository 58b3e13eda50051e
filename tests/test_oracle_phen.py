"""Pins of the phenomenological-noise oracle (repeated noisy syndrome rounds,
paper Sec. 2.2 "Phenomenological noise"; the (2+1)-D problem of Sec. 3.2.3).

O6 (enumeration over every first-round error, T = 2, d = 3) and O7 (exact
transfer over the qubits, any T) are checked against each other and against
facts that do not come from either:
  * the distribution of records (s_1..s_T, class) drawn by the sampler, which
    applies the model directly (per-round Paulis, measurement flips, parities);
  * the probabilities of all d = 3, T = 2 records summing to one;
  * T = 1 (a single perfect round) reducing to the code-capacity oracle O3;
  * measurement flips at rate 1/2, where the noisy rounds carry no
    information: Z_l = 2^{-m (T-1)} times the code-capacity Z_l of the last
    round under the T-fold composed single-qubit channel (O1 / O3);
  * noiseless limits (all rates zero).
"""
import numpy as np
import pytest

import oracle
import synth


def compose(r1, r2):
    """Single-qubit Pauli channel of two independent errors: p(P) = sum over
    A * B = P of p1(A) p2(B) (rates as [n, 3] of X, Y, Z)."""
    def full(r):
        return np.concatenate([1.0 - r.sum(1, keepdims=True), r], 1)
    a, b = full(r1), full(r2)
    lut = np.array([[0, 1, 2, 3], [1, 0, 3, 2], [2, 3, 0, 1], [3, 2, 1, 0]])
    out = np.zeros_like(a)
    for i in range(4):
        for j in range(4):
            out[:, lut[i, j]] += a[:, i] * b[:, j]
    return out[:, 1:]


def test_o6_matches_o7():
    d = 3
    r = synth.inhomogeneous(d, 0.01, 0.12, seed=3)
    q = np.linspace(0.01, 0.2, d * d - 1)
    smp = synth.sample_phenom(d, r, q, 2, 24, seed=4)
    a = oracle.phen_enum2(d, r, q, smp["syndromes"])
    b = oracle.phen_transfer(d, 2, r, q, smp["syndromes"])
    fin = np.isfinite(a)
    assert np.array_equal(fin, np.isfinite(b))
    assert np.max(np.abs(a[fin] - b[fin])) < 1e-11


def all_records_d3_t2():
    m = 8
    idx = np.arange(1 << (2 * m))
    bits = ((idx[:, None] >> np.arange(2 * m)) & 1).astype(np.uint8)
    return bits.reshape(-1, 2, m)


def test_o7_total_probability_d3():
    """Every (s_1, s_2) record of d = 3, T = 2: sum over records and classes of
    Z_l = 1."""
    r = synth.depolarizing(3, 0.15)
    q = np.full(8, 0.1)
    z = oracle.phen_transfer(3, 2, r, q, all_records_d3_t2(), threads=8)
    tot = np.exp(z).sum()
    assert abs(tot - 1.0) < 1e-12


@pytest.mark.parametrize("rounds", [2, 3])
def test_o7_matches_sampling_frequencies(rounds):
    """Probabilities of the 40 most frequent (record, class) outcomes against
    their empirical frequencies over 200,000 sampled histories (6 sigma)."""
    d, m = 3, 8
    r = synth.depolarizing(d, 0.03)
    q = np.full(m, 0.03)
    smp = synth.sample_phenom(d, r, q, rounds, 200000, seed=20 + rounds)
    key = (smp["syndromes"].reshape(len(smp["syndromes"]), -1).astype(np.int64) << np.arange(rounds * m)).sum(1)
    key = key * 4 + smp["true_class"]
    u, cnt = np.unique(key, return_counts=True)
    top = np.argsort(-cnt)[:40]
    recs = u[top] // 4
    cls = (u[top] % 4).astype(int)
    syn = ((recs[:, None] >> np.arange(rounds * m)) & 1).astype(np.uint8).reshape(-1, rounds, m)
    z = oracle.phen_transfer(d, rounds, r, q, syn)
    prob = np.exp(z[np.arange(len(cls)), cls])
    freq = cnt[top] / len(key)
    sig = np.sqrt(prob * (1 - prob) / len(key))
    assert np.all(np.abs(freq - prob) < 6 * sig + 1e-12)
    if rounds == 2:
        z6 = oracle.phen_enum2(d, r, q, syn)
        assert np.max(np.abs(z6 - z)[np.isfinite(z)]) < 1e-11


@pytest.mark.parametrize("d", [3, 5])
def test_o7_single_round_is_code_capacity(d):
    r = synth.inhomogeneous(d, 0.01, 0.15, seed=d)
    smp = synth.sample(d, r, 12, seed=d + 1)
    z1 = oracle.phen_transfer(d, 1, r, np.zeros(d * d - 1), smp["syndromes"][:, None, :])
    z3 = oracle.transfer(d, r, smp["syndromes"])
    fin = np.isfinite(z3)
    assert np.array_equal(fin, np.isfinite(z1))
    assert np.max(np.abs(z1[fin] - z3[fin])) < 1e-11


@pytest.mark.parametrize("d,rounds", [(3, 2), (3, 3), (5, 2)])
def test_o7_uninformative_measurements(d, rounds):
    """meas = 1/2: the noisy rounds say nothing; Z_l(s_1..s_T) =
    2^{-m(T-1)} Z_l^{cc}(s_T) under the T-fold composed channel."""
    m = d * d - 1
    r = synth.inhomogeneous(d, 0.01, 0.1, seed=10 + d)
    rng = np.random.default_rng(rounds)
    syn = rng.integers(0, 2, (6, rounds, m)).astype(np.uint8)
    smp = synth.sample(d, r, 6, seed=3)
    syn[:, -1] = smp["syndromes"]  # likely last-round syndromes
    rc = r
    for _ in range(rounds - 1):
        rc = compose(rc, r)
    z = oracle.phen_transfer(d, rounds, r, np.full(m, 0.5), syn)
    if d == 3:
        t = oracle.enumerate_table(3, rc)
        si = (syn[:, -1].astype(np.int64) << np.arange(m)).sum(1)
        ref = np.log(t[si]) - m * (rounds - 1) * np.log(2.0)
    else:
        ref = oracle.transfer(d, rc, syn[:, -1]) - m * (rounds - 1) * np.log(2.0)
    assert np.max(np.abs(z - ref)) < 1e-10


def test_o7_noiseless_limits():
    d, m = 3, 8
    r = np.zeros((9, 3))
    syn = np.zeros((3, 2, m), np.uint8)
    syn[1, 0, 2] = 1  # a flipped first-round bit with no measurement errors
    syn[2, 1, 0] = 1  # a last-round defect with no data errors
    z = oracle.phen_transfer(d, 2, r, np.zeros(m), syn)
    assert z[0, 0] == 0.0 and np.isneginf(z[0, 1:]).all()
    assert np.isneginf(z[1:]).all()
    # measurement errors only: the first round's bits are pure flips
    q = np.full(m, 0.2)
    z = oracle.phen_transfer(d, 2, r, q, syn[:2])
    assert abs(z[1, 0] - (np.log(0.2) + 7 * np.log(0.8))) < 1e-12
    assert np.isneginf(z[1, 1:]).all()


CLASS_BITS = np.array([[0, 0], [1, 0], [1, 1], [0, 1]])


def class_xor(a, b):
    bits = CLASS_BITS[a] ^ CLASS_BITS[b]
    return np.array([[0, 3], [1, 2]])[bits[..., 0], bits[..., 1]]


@pytest.mark.parametrize("d,rounds", [(3, 3), (5, 2)])
def test_o7_rotation_symmetry(d, rounds):
    """The 180-degree rotation maps the patch onto itself (qubit q -> n-1-q,
    checks permuted): a record and its rotated image, under rotated rates,
    have the same coset weights once classes are aligned through the true
    classes of the two histories."""
    n, m = d * d, d * d - 1
    types, supp = synth.code_checks(d)
    key = {tuple(sorted(x for x in row if x >= 0)): j for j, row in enumerate(supp)}
    perm = np.array([key[tuple(sorted(n - 1 - x for x in row if x >= 0))] for row in supp])
    inv = np.argsort(perm)
    r = synth.inhomogeneous(d, 0.01, 0.15, seed=50 + d)
    rr = r[::-1].copy()
    q = np.full(m, 0.07)
    smp = synth.sample_phenom(d, r, q, rounds, 4, seed=51)
    acc = np.zeros((4, n), np.uint8)
    for t in range(rounds):
        acc = synth._pauli_xor(acc, smp["errors"][:, t])
    c = synth.classes_of(d, acc)
    cr = synth.classes_of(d, acc[:, ::-1])
    syn_r = smp["syndromes"][:, :, inv]
    z = oracle.phen_transfer(d, rounds, r, q, smp["syndromes"])
    zr = oracle.phen_transfer(d, rounds, rr, q, syn_r)
    for b in range(4):
        for ell in range(4):
            assert abs(z[b, class_xor(c[b], ell)] - zr[b, class_xor(cr[b], ell)]) < 1e-10
