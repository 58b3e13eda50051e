"""Input-value checks, the numeric status, per-stream workspaces and graph
replay after a larger eager call (GPU).  Invalid values must never reach an
output as NaN: the host check raises before any launch, and the kernels' own
check (exercised here with the host check switched off) writes -inf and
reports TN_EINVAL through the workspace status word."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _tn():
    import paper_2605_17230_amd as tn
    return tn


def _seg(d, chi, syn, rates, prec="fp32", mi=None):
    tn = _tn()
    return tn.SegmentInput(d, chi, torch.from_numpy(np.ascontiguousarray(syn)).to(DEV),
                           torch.from_numpy(np.ascontiguousarray(rates)).to(DEV),
                           None if mi is None else torch.from_numpy(np.asarray(mi, np.int32)).to(DEV), prec)


def _inputs():
    d = 5
    rates = np.stack([synth.depolarizing(d, 0.1), synth.biased(d, 0.1, 10.0)])
    smp = synth.sample(d, rates[0], 12, seed=5)
    return d, rates, smp["syndromes"], np.zeros(12, np.int32)


@pytest.mark.parametrize("case", ["byte", "index", "nan", "over"])
def test_invalid_values_raise_before_launch_and_on_device(case):
    tn = _tn()
    d, rates, syn, mi = _inputs()
    print("case", case, flush=True)
    clean = tn.decode_segments([_seg(d, 8, syn, rates, mi=mi)])[0]
    syn2, rates2, mi2 = syn.copy(), rates.copy(), mi.copy()
    bad_rows = [4]
    if case == "byte":
        syn2[4, 10] = 7
    elif case == "index":
        mi2[4] = 5
    elif case == "nan":
        rates2[1, 3, 1] = np.nan
        mi2[[4, 9]] = 1
        bad_rows = [4, 9]
    else:
        rates2[1, 0] = [0.5, 0.5, 0.5]
        mi2[[4, 9]] = 1
        bad_rows = [4, 9]
    seg = _seg(d, 8, syn2, rates2, mi=mi2)
    with pytest.raises(ValueError):
        tn.decode_segments([seg])
    with pytest.raises(tn.TNError) as e:
        tn.decode_segments([seg], check="device")
    assert e.value.code == tn._lib.TN_EINVAL
    out = tn.decode_segments([seg], check=False)[0]
    torch.cuda.synchronize()
    lz = out.logz.cpu().numpy()
    assert not np.isnan(lz).any()
    assert np.isneginf(lz[bad_rows]).all()
    assert (out.cls.cpu().numpy()[bad_rows] == 0).all()
    keep = np.setdiff1d(np.arange(12), bad_rows)
    if case in ("byte", "index"):
        assert np.array_equal(lz[keep], clean.logz.cpu().numpy()[keep])


def test_backward_skips_invalid_syndromes():
    """The adjoint's own check: an invalid syndrome adds nothing to the
    gradient, and the call reports TN_EINVAL."""
    tn = _tn()
    d, rates, syn, mi = _inputs()
    gw = torch.ones(12, dtype=torch.float64, device=DEV)
    _, g_valid = tn.coset_loglik_backward([_seg(d, 0, syn[:11], rates, "fp64", mi[:11])], [gw[:11]])
    syn2 = syn.copy()
    syn2[11, 0] = 3
    seg = _seg(d, 0, syn2, rates, "fp64", mi)
    with pytest.raises(tn.TNError) as e:
        tn.coset_loglik_backward([seg], [gw], check="device")
    assert e.value.code == tn._lib.TN_EINVAL
    _, g_bad = tn.coset_loglik_backward([seg], [gw], check=False)
    torch.cuda.synchronize()
    a, b = g_bad[0].cpu().numpy(), g_valid[0].cpu().numpy()
    assert np.allclose(a, b, rtol=1e-12, atol=1e-14 * np.abs(b).max())


def test_numeric_breakdown_is_reported():
    """Every rate 1e-46: positive in FP64, zero in FP32.  The FP32 form cannot
    represent the weights, so the syndrome that needs an error comes out with
    Z = 0 in all four cosets; the model is strictly positive, so that is
    reported as TN_ENUMERIC (outputs -inf, never NaN) instead of an
    impossible syndrome.  The FP64 form decodes log P(s) of both syndromes."""
    tn = _tn()
    d = 3
    rates = np.full((d * d, 3), 1e-46)
    syn = np.zeros((2, d * d - 1), np.uint8)
    syn[1, 2] = 1
    with pytest.raises(tn.TNError) as e:
        tn.decode_segments([_seg(d, 0, syn, rates, "fp32plain")])
    assert e.value.code == tn._lib.TN_ENUMERIC
    out = tn.decode_segments([_seg(d, 0, syn, rates, "fp32plain")], check=False)[0]
    torch.cuda.synchronize()
    assert not np.isnan(out.logz.cpu().numpy()).any()
    import warnings
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", tn.api.UnresolvedCosetsWarning)  # cosets near 1e-300 underflow FP64 too
        out = tn.decode_segments([_seg(d, 0, syn, rates, "fp64")])[0]
    assert np.isfinite(out.logp.cpu().numpy()).all()


def test_graph_replay_after_larger_eager_call():
    """Capture a call at size X, then run an eager call at 2X on the same
    stream (which outgrows the workspace the graph captured), then replay:
    the replay still equals an eager call on the captured inputs, because a
    workspace a graph captured is never freed."""
    tn = _tn()
    d, chi = 7, 12
    rates = synth.depolarizing(d, 0.1)
    small = synth.sample(d, rates, 64, seed=1)["syndromes"]
    big = synth.sample(d, rates, 4096, seed=2)["syndromes"]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        seg = _seg(d, chi, small, rates)
        tn.decode_segments([seg])  # plans uploaded, workspace sized
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=s):
            cap = tn.decode_segments([seg])[0]
        torch.cuda.synchronize()
        eager_big = tn.decode_segments([_seg(d, chi, big, rates)])[0]
        torch.cuda.synchronize()
        for rep in range(3):
            cap.logz.fill_(float("nan"))
            torch.cuda.synchronize()
            g.replay()
            torch.cuda.synchronize()
            ref = tn.decode_segments([seg])[0]
            torch.cuda.synchronize()
            assert torch.equal(cap.logz, ref.logz) and torch.equal(cap.cls, ref.cls)
    assert torch.isfinite(eager_big.logp).all()


def test_side_stream_and_caller_workspace():
    """A call on a side stream (temporaries recorded on it) and a call with a
    caller-owned workspace give the same results as the default call."""
    tn = _tn()
    d, rates, syn, mi = _inputs()
    seg = _seg(d, 8, syn, rates, mi=mi)
    ref = tn.decode_segments([seg])[0]
    s = torch.cuda.Stream()
    out = tn.decode_segments([seg], stream=s)[0]
    s.synchronize()
    assert torch.equal(out.logz, ref.logz)
    buf = torch.empty(tn.workspace_bytes([seg]), dtype=torch.uint8, device=DEV)
    out2 = tn.decode_segments([seg], workspace_buf=buf)[0]
    assert torch.equal(out2.logz, ref.logz)
    with pytest.raises(ValueError):
        tn.decode_segments([seg], workspace_buf=buf[:16])
