"""GPU parity of repeated noisy syndrome rounds (phenomenological noise,
paper Sec. 2.2; the (2+1)-D problem of Sec. 3.2.3): T = 2 rounds, the first
with measurement flips, the last perfect, decoded through the C ABI
(tn_decode_batch with rounds = 2) against the exact phenomenological oracle O7
(itself pinned by enumeration, sampled frequencies, total probability and the
uninformative-measurement closed form; tests/test_oracle_phen.py).

Bars, per form (measured values are about a third of each):
  * exact regime (d = 3, every bond kept): the code-capacity bars,
    FP64 1e-10 relative, mixed FP32 1e-4, plain FP32 1e-3, BF16 5e-3;
  * truncated (d = 5, 7; chi = 12 for the FP64-factorisation forms, 16 for the
    FP32 ones, the largest whose LDS fits): |delta log P(s)| and |delta log Z|
    of the cosets with oracle posterior >= e^-10 (TRUNC_BARS); classes equal
    wherever the oracle's top-two gap exceeds twice the log P bar; cosets lost
    (-inf) only below posterior e^-30 in FP64 and e^-20 in the FP32 forms: the
    measurement duals make the tensors signed, so an improbable coset is a
    difference of much larger terms and reaches the FP32 rounding level of the
    boundary state sooner than in the all-positive single-round network.
"""
import warnings

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"

EXACT = {"fp64": 1e-10, "fp32": 1e-4, "fp32plain": 1e-3, "bf16": 5e-3}
CHI = {"fp64": 12, "fp32": 12, "fp32plain": 16, "bf16": 16}
LOST_POST = {"fp64": -30.0, "fp32": -20.0, "fp32plain": -20.0, "bf16": -20.0}
TRUNC_BARS = {
    "fp64": dict(logp=6e-3, post10=5e-2),  # chi = 12: 1.9e-3 at d = 5, p = 0.06, q = 0.04
    "fp32": dict(logp=6e-3, post10=5e-2),
    "fp32plain": dict(logp=2e-3, post10=1e-2),
    "bf16": dict(logp=5e-3, post10=5e-2),
}


def _tn():
    import paper_2605_17230_amd as tn
    return tn


def run(d, chi, prec, syn, rates, meas, model_index=None, check=True):
    tn = _tn()
    seg = tn.SegmentInput(d, chi, torch.from_numpy(np.ascontiguousarray(syn)).to(DEV),
                          torch.from_numpy(np.ascontiguousarray(rates)).to(DEV),
                          None if model_index is None else torch.from_numpy(model_index).to(DEV),
                          prec, int(syn.shape[1]), torch.from_numpy(np.ascontiguousarray(meas)).to(DEV))
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", tn.api.UnresolvedCosetsWarning)
        o = tn.decode_segments([seg], check=check)[0]
    return o.logz.cpu().numpy(), o.logp.cpu().numpy(), o.cls.cpu().numpy()


def posterior(z):
    fin = np.isfinite(z)
    with np.errstate(invalid="ignore"):
        p = z - np.logaddexp.reduce(np.where(fin, z, -np.inf), axis=1, keepdims=True)
    return np.where(fin, p, -np.inf)


def check_truncated(lz, lp, cls, ref, prec):
    bar = TRUNC_BARS[prec]
    fin, gfin = np.isfinite(ref), np.isfinite(lz)
    assert not (gfin & ~fin).any(), "a coset the oracle rules out came out finite"
    post = posterior(ref)
    lost = fin & ~gfin
    assert post[lost].max(initial=-np.inf) < LOST_POST[prec]
    both = fin & gfin
    err = np.where(both, np.abs(np.where(both, lz, 0) - np.where(both, ref, 0)), 0.0)
    lpo, clo = oracle.decide(ref)
    e_lp = float(np.max(np.abs(lp - lpo)))
    e10 = float(err[post >= -10].max(initial=0))
    print("%s: max |dlogP| %.3g, max |dlogZ| posterior >= e^-10 %.3g, lost cosets %d"
          % (prec, e_lp, e10, int(lost.sum())), flush=True)
    assert e_lp < bar["logp"] and e10 < bar["post10"]
    top2 = np.sort(ref, axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > 2 * bar["logp"]
    assert np.array_equal(cls[clear], clo[clear])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32plain", "bf16"])
def test_d3_exact_vs_oracle(prec):
    """d = 3, every bond kept (chi = 0): the two-round network is contracted
    exactly; against O7 and the enumeration O6 on 48 histories with per-qubit
    rates and per-check measurement rates."""
    d, m = 3, 8
    r = synth.inhomogeneous(d, 0.01, 0.12, seed=31)
    q = np.linspace(0.01, 0.15, m)
    smp = synth.sample_phenom(d, r, q, 2, 48, seed=32)
    lz, lp, cls = run(d, 0, prec, smp["syndromes"], r, q)
    ref = oracle.phen_transfer(d, 2, r, q, smp["syndromes"])
    assert np.max(np.abs(oracle.phen_enum2(d, r, q, smp["syndromes"]) - ref)) < 1e-11
    assert np.array_equal(np.isfinite(lz), np.isfinite(ref))
    fin = np.isfinite(ref)
    err = np.abs(lz[fin] - ref[fin])
    if prec == "fp64":
        err = err / np.maximum(1.0, np.abs(ref[fin]))
    assert err.max() < EXACT[prec], err.max()
    _, clo = oracle.decide(ref)
    top2 = np.sort(ref, axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > 2 * EXACT[prec]
    assert np.array_equal(cls[clear], clo[clear])


@pytest.mark.parametrize("prec", ["fp64", "fp32", "fp32plain", "bf16"])
@pytest.mark.parametrize("p,q,seed", [(0.03, 0.03, 2), (0.06, 0.04, 3)])
def test_d5_truncated_vs_oracle(prec, p, q, seed):
    d = 5
    r = synth.depolarizing(d, p)
    mq = np.full(d * d - 1, q)
    smp = synth.sample_phenom(d, r, mq, 2, 32, seed=seed)
    lz, lp, cls = run(d, CHI[prec], prec, smp["syndromes"], r, mq)
    ref = oracle.phen_transfer(d, 2, r, mq, smp["syndromes"], threads=16)
    check_truncated(lz, lp, cls, ref, prec)


@pytest.mark.slow
@pytest.mark.parametrize("p,q,seed", [(0.02, 0.02, 4), (0.04, 0.03, 5)])
def test_d7_truncated_vs_oracle(p, q, seed):
    """d = 7 (the benchmark's distance), 16 histories per point, all four
    forms against one set of oracle values."""
    d = 7
    r = synth.depolarizing(d, p)
    mq = np.full(d * d - 1, q)
    smp = synth.sample_phenom(d, r, mq, 2, 16, seed=seed)
    ref = oracle.phen_transfer(d, 2, r, mq, smp["syndromes"], threads=16)
    for prec in ("fp64", "fp32", "fp32plain", "bf16"):
        lz, lp, cls = run(d, CHI[prec], prec, smp["syndromes"], r, mq)
        check_truncated(lz, lp, cls, ref, prec)


def test_uninformative_measurements_closed_form():
    """Measurement flips at rate 1/2: Z_l(s_1, s_2) = 2^-m times the
    code-capacity Z_l(s_2) under the two-fold composed channel, here from the
    code-capacity enumeration O1 (FP64, d = 3, every bond kept)."""
    d, m = 3, 8
    r = synth.inhomogeneous(d, 0.01, 0.08, seed=8)
    full = np.concatenate([1.0 - r.sum(1, keepdims=True), r], 1)
    lut = np.array([[0, 1, 2, 3], [1, 0, 3, 2], [2, 3, 0, 1], [3, 2, 1, 0]])
    comp = np.zeros_like(full)
    for i in range(4):
        for j in range(4):
            comp[:, lut[i, j]] += full[:, i] * full[:, j]
    rng = np.random.default_rng(9)
    syn = np.zeros((32, 2, m), np.uint8)
    syn[:, 0] = rng.integers(0, 2, (32, m))
    syn[:, 1] = synth.sample(d, comp[:, 1:], 32, seed=10)["syndromes"]
    lz, _, _ = run(d, 0, "fp64", syn, r, np.full(m, 0.5))
    table = oracle.enumerate_table(d, comp[:, 1:])
    si = (syn[:, 1].astype(np.int64) << np.arange(m)).sum(1)
    ref = np.log(table[si]) - m * np.log(2.0)
    assert np.max(np.abs(lz - ref) / np.maximum(1.0, np.abs(ref))) < 1e-10


def test_mixed_rounds_and_single_round_segments():
    """One call with a two-round segment and a code-capacity segment of the
    same distance and form (one launch, two plans): each against its oracle;
    plus an empty two-round segment."""
    tn = _tn()
    d, m = 5, 24
    r = synth.depolarizing(d, 0.05)
    mq = np.full(m, 0.03)
    s2 = synth.sample_phenom(d, r, mq, 2, 12, seed=11)
    s1 = synth.sample(d, r, 12, seed=12)
    R = torch.from_numpy(r).to(DEV)
    segs = [tn.SegmentInput(d, 12, torch.from_numpy(s2["syndromes"]).to(DEV), R, None, "fp64", 2,
                            torch.from_numpy(mq).to(DEV)),
            tn.SegmentInput(d, 16, torch.from_numpy(s1["syndromes"]).to(DEV), R, None, "fp64"),
            tn.SegmentInput(d, 12, torch.zeros((0, 2, m), dtype=torch.uint8, device=DEV), R, None, "fp64", 2,
                            torch.from_numpy(mq).to(DEV))]
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", tn.api.UnresolvedCosetsWarning)
        o = tn.decode_segments(segs)
    ref2 = oracle.phen_transfer(d, 2, r, mq, s2["syndromes"])
    check_truncated(o[0].logz.cpu().numpy(), o[0].logp.cpu().numpy(), o[0].cls.cpu().numpy(), ref2, "fp64")
    ref1 = oracle.transfer(d, r, s1["syndromes"])
    assert np.max(np.abs(o[1].logz.cpu().numpy() - ref1) / np.maximum(1.0, np.abs(ref1))) < 1e-10
    assert o[2].logz.shape == (0, 4)


def test_invalid_measurement_rates_and_gradient_rejected():
    """A measurement rate outside [0, 1] raises before the launch (host check);
    checked on the device only, the call reports TN_EINVAL; unchecked, the
    syndromes of that model come out -inf (class 0, no NaN).  The gradient takes
    one round only (the binding raises; the C entry point returns
    TN_EUNSUPPORTED, tested on the CPU)."""
    tn = _tn()
    d, m = 3, 8
    r = synth.depolarizing(d, 0.05)
    q = np.full(m, 0.05)
    q[2] = float("nan")
    smp = synth.sample_phenom(d, r, np.full(m, 0.05), 2, 4, seed=13)
    with pytest.raises(ValueError):
        run(d, 0, "fp64", smp["syndromes"], r, q)
    with pytest.raises(tn.TNError) as e:
        run(d, 0, "fp64", smp["syndromes"], r, q, check="device")
    assert e.value.code == tn._lib.TN_EINVAL
    lz, lp, cls = run(d, 0, "fp64", smp["syndromes"], r, q, check=False)
    assert np.isneginf(lz).all() and not np.isnan(lp).any() and (cls == 0).all()
    seg = tn.SegmentInput(d, 0, torch.from_numpy(smp["syndromes"]).to(DEV), torch.from_numpy(r).to(DEV), None,
                          "fp64", 2, torch.from_numpy(np.full(m, 0.05)).to(DEV))
    with pytest.raises(ValueError):
        tn.coset_loglik_backward([seg], [torch.ones(4, dtype=torch.float64, device=DEV)])
