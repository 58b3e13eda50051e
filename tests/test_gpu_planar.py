"""The planar exact solver for bit-flip noise (Kac-Ward determinant, paper
Sec. 3.1.3) against the FP64 oracle: the textbook random-bond Ising brute
force O4 at d = 3, 5, 7 and the exact transfer-matrix contraction O3 up to
d = 17, then against the boundary-MPS path at d = 17 (GPU)."""
import warnings

import numpy as np
import pytest

import oracle
import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _tn():
    import paper_2605_17230_amd as tn
    return tn


def kw(d, syn, rates, mi=None):
    tn = _tn()
    print("planar d=%d B=%d" % (d, len(syn)), flush=True)
    s = torch.from_numpy(np.ascontiguousarray(syn)).to(DEV)
    r = torch.from_numpy(np.ascontiguousarray(rates)).to(DEV)
    m = None if mi is None else torch.from_numpy(np.asarray(mi, np.int32)).to(DEV)
    lz, lp, cls = tn.decode_bitflip(s, r, d, model_index=m)
    torch.cuda.synchronize()
    return lz.cpu().numpy(), lp.cpu().numpy(), cls.cpu().numpy()


def rel(got, ref):
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin), "finite pattern differs"
    return float(np.max(np.abs(got[fin] - ref[fin]) / np.maximum(1.0, np.abs(ref[fin])), initial=0.0))


def check_exact(got, ref):
    """Bars of the planar solver (FP64): log Z within 1e-10 relative for every
    coset whose posterior is >= e^-5, 1e-7 for >= e^-20, 1e-5 for all.  The
    loop sum of an improbable coset has signed terms (the flipped bonds) that
    nearly cancel, so its value is ill-conditioned in the inputs themselves:
    a relative perturbation eps of the bond weights moves it by about
    eps n / posterior.  log P(s) stays within 1e-10."""
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin), "finite pattern differs"
    with np.errstate(invalid="ignore"):
        post = np.where(fin, ref - np.logaddexp.reduce(ref, axis=1, keepdims=True), -np.inf)
    r = np.where(fin, np.abs(np.where(fin, got, 0) - np.where(fin, ref, 0)) / np.maximum(1.0, np.abs(np.where(fin, ref, 1))),
                 0.0)
    b5, b20, ball = (float(r[post >= -5].max(initial=0)), float(r[post >= -20].max(initial=0)), float(r.max(initial=0)))
    print("max rel |dlogZ|: posterior >= e^-5 %.3g, >= e^-20 %.3g, all %.3g" % (b5, b20, ball), flush=True)
    assert b5 < 1e-10 and b20 < 1e-7 and ball < 1e-5
    lp, lpr = np.logaddexp.reduce(got, 1), np.logaddexp.reduce(ref, 1)
    ok = np.isfinite(lpr)
    assert np.max(np.abs(lp[ok] - lpr[ok]) / np.maximum(1.0, np.abs(lpr[ok])), initial=0) < 1e-10


@pytest.mark.parametrize("d", [3, 5, 7])
@pytest.mark.parametrize("p", [0.02, 0.1, 0.3])
def test_vs_ising_brute_force(d, p):
    """Exact against the random-bond Ising partition function summed over all
    spin configurations (oracle O4), cosets I and X; Y and Z are -inf."""
    rates = synth.bitflip(d, p)
    smp = synth.sample(d, rates, 24, seed=100 + d)
    ref = np.stack([oracle.rbim(d, p, s) for s in smp["syndromes"]])
    got, lp, cls = kw(d, smp["syndromes"], rates)
    check_exact(got, ref)
    _, rcls = oracle.decide(ref)
    assert np.array_equal(cls, rcls)


@pytest.mark.parametrize("d", [9, 13])
def test_inhomogeneous_vs_transfer(d):
    """Per-qubit bit-flip rates log-uniform in [0.005, 0.2], two noise models
    selected per syndrome: exact against the transfer-matrix oracle O3."""
    r0 = synth.inhomogeneous(d, 0.005, 0.2, seed=d)
    models = np.zeros((2, d * d, 3))
    models[0, :, 0] = r0[:, 0]
    models[1, :, 0] = r0[::-1, 1]
    mi = np.arange(16) % 2
    smp = synth.sample(d, models, 16, seed=7 * d, model_index=mi)
    ref = np.concatenate([oracle.transfer(d, models[k], smp["syndromes"][mi == k], threads=8) for k in range(2)])
    order = np.concatenate([np.nonzero(mi == k)[0] for k in range(2)])
    got, _, _ = kw(d, smp["syndromes"], models, mi)
    check_exact(got[order], ref)


@pytest.mark.slow
def test_d17_vs_transfer_and_boundary_mps():
    """d = 17 (a 580 x 580 complex determinant per coset): exact against O3 on
    8 syndromes; the boundary-MPS path (FP64, chi = 32) on 256 syndromes
    agrees within its truncation error."""
    tn = _tn()
    d, p = 17, 0.1
    rates = synth.bitflip(d, p)
    smp = synth.sample(d, rates, 256, seed=17)
    got, lp, cls = kw(d, smp["syndromes"], rates)
    ref = oracle.transfer(d, rates, smp["syndromes"][:8], threads=16)
    check_exact(got[:8], ref)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", tn.api.UnresolvedCosetsWarning)
        mz, mlp, mcls = tn.decode(torch.from_numpy(smp["syndromes"]).to(DEV), torch.from_numpy(rates).to(DEV), d, 32,
                                  "fp64")
    mlp = mlp.cpu().numpy()
    err = float(np.max(np.abs(mlp - lp)))
    print("d=17 bit-flip: boundary MPS chi=32 vs planar exact, max |dlogP| %.3g" % err, flush=True)
    assert err < 1e-6
    assert (mcls.cpu().numpy() == cls).mean() >= 0.99


def test_edge_cases_and_invalid_rates():
    """An X-type check fired (needs a Z error): every coset -inf, class 0.
    Zero rates: the trivial syndrome has log Z_I = 0 and the others -inf.
    Rates with a Y or Z part are refused (host check) and flagged by the
    kernel's own check (TN_EINVAL) with -inf outputs, never NaN."""
    tn = _tn()
    d = 5
    m = d * d - 1
    rates = synth.bitflip(d, 0.1)
    syn = np.zeros((3, m), np.uint8)
    syn[1, m - 1] = 1  # an X-type check
    got, lp, cls = kw(d, syn, rates)
    assert np.isneginf(got[1]).all() and np.isneginf(lp[1]) and cls[1] == 0
    assert np.isfinite(got[0, :2]).all() and np.isneginf(got[0, 2:]).all()
    zero = np.zeros((d * d, 3))
    got, _, _ = kw(d, syn[:1], zero)
    assert abs(got[0, 0]) < 1e-12 and np.isneginf(got[0, 1:]).all()
    dep = synth.depolarizing(d, 0.1)
    seg = tn.SegmentInput(d, 0, torch.from_numpy(syn).to(DEV), torch.from_numpy(dep).to(DEV), None, "fp64")
    with pytest.raises(ValueError):
        tn.decode_bitflip_segments([seg])
    with pytest.raises(tn.TNError) as e:
        tn.decode_bitflip_segments([seg], check="device")
    assert e.value.code == tn._lib.TN_EINVAL
    out = tn.decode_bitflip_segments([seg], check=False)[0]
    torch.cuda.synchronize()
    lz = out.logz.cpu().numpy()
    assert np.isneginf(lz).all() and not np.isnan(lz).any()


def test_mixed_segments_equal_single_calls():
    tn = _tn()
    segs, ins = [], []
    for d in (13, 5, 9):
        r = synth.bitflip(d, 0.08)
        smp = synth.sample(d, r, 20, seed=d)
        ins.append((d, smp["syndromes"], r))
        segs.append(tn.SegmentInput(d, 0, torch.from_numpy(smp["syndromes"]).to(DEV), torch.from_numpy(r).to(DEV),
                                    None, "fp64"))
    outs = tn.decode_bitflip_segments(segs)
    for (d, syn, r), o in zip(ins, outs):
        a, _, _ = kw(d, syn, r)
        assert np.array_equal(a, o.logz.cpu().numpy())
