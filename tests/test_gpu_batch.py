"""Mixed batches in one persistent launch (distances 5..15, three Z-biases per
distance, chi by distance) and replay of a captured launch, against the FP64
oracle and against single-segment launches."""
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


def _inputs(segs, prec="fp32"):
    tn = _tn()
    return [tn.SegmentInput(s["d"], s["chi"], torch.from_numpy(s["syndromes"]).to(DEV),
                            torch.from_numpy(s["rates"]).to(DEV), torch.from_numpy(s["model_index"]).to(DEV), prec)
            for s in segs]


def _oracle_logz(s, idx):
    out = np.zeros((len(idx), 4))
    for m in range(s["rates"].shape[0]):
        sel = [i for i, b in enumerate(idx) if s["model_index"][b] == m]
        if sel:
            out[sel] = oracle.transfer(s["d"], s["rates"][m], s["syndromes"][[idx[i] for i in sel]])
    return out


# Bars against the exact oracle at the C4 bond dimensions (truncation plus
# precision error), per form: |delta log P(s)|, and |delta log Z| of every
# coset whose oracle posterior is >= e^-10.  A reduced-precision form may
# report a coset far below its syndrome's probable ones as -inf (below the
# form's resolution, counted by the library); that is accepted only for
# oracle posteriors below e^-30.
C4_BARS = {"fp32": dict(logp=1e-4, logz=5e-4), "bf16": dict(logp=2e-3, logz=2e-2)}
UNRESOLVED_POST = -30.0


def _check_vs_oracle(s, o, idx, prec="fp32"):
    ref = _oracle_logz(s, idx)
    lz = o.logz.cpu().numpy()[idx]
    cls = o.cls.cpu().numpy()[idx]
    lp_ref, cls_ref = oracle.decide(ref)
    lp = o.logp.cpu().numpy()[idx]
    bar = C4_BARS[prec]
    dlp = float(np.max(np.abs(lp - lp_ref)))
    assert dlp < bar["logp"], (s["d"], dlp)
    fin, gfin = np.isfinite(ref), np.isfinite(lz)
    assert not (gfin & ~fin).any(), "finite where the oracle says impossible"
    with np.errstate(invalid="ignore"):
        post = np.where(fin, ref - lp_ref[:, None], -np.inf)
    unres = fin & ~gfin
    assert post[unres].max(initial=-np.inf) < UNRESOLVED_POST, (s["d"], post[unres].max())
    both = fin & gfin
    err = np.where(both, np.abs(np.where(both, lz, 0) - np.where(both, ref, 0)), 0.0)
    dz = float(err[post >= -10].max(initial=0))
    assert dz < bar["logz"], (s["d"], dz)
    top2 = np.sort(ref, axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > 2e-2
    assert np.all(cls[clear] == cls_ref[clear])
    print("C4 %s d=%d: max |dlogP| %.3g, max |dlogZ| (post >= e^-10) %.3g, unresolved %d"
          % (prec, s["d"], dlp, dz, int(unres.sum())), flush=True)
    return dz


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_c4_mixed_launch_small(prec):
    """Every C4 segment at 1/256 of its count in one call: each against the
    exact oracle under the form's bars, and bitwise against the segment
    decoded alone."""
    tn = _tn()
    segs = synth.config_inputs("C4", scale=1 / 256)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", tn.api.UnresolvedCosetsWarning)
        outs = tn.decode_segments(_inputs(segs, prec))
        for s, o in zip(segs, outs):
            _check_vs_oracle(s, o, list(range(len(s["syndromes"]))), prec)
            alone = tn.decode_segments(_inputs([s], prec))[0]
            assert torch.equal(alone.logz, o.logz)
            assert torch.equal(alone.cls, o.cls)


@pytest.mark.slow
@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_c4_full_mixed_launch_sampled(prec):
    """The whole C4 batch (63,488 syndromes, six distances) in one call (one
    persistent launch per size class); 12 syndromes of every segment against
    the exact oracle under the form's bars."""
    tn = _tn()
    segs = synth.config_inputs("C4")
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", tn.api.UnresolvedCosetsWarning)
        outs = tn.decode_segments(_inputs(segs, prec))
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    for s, o in zip(segs, outs):
        n = len(s["syndromes"])
        idx = sorted(rng.choice(n, 12, replace=False).tolist())
        _check_vs_oracle(s, o, idx, prec)
        assert np.all(np.isfinite(o.logp.cpu().numpy()))


def test_graph_capture_replay():
    """A warm mixed-batch call captured into a graph and replayed with new
    syndromes copied into the captured inputs: each replay equals an eager
    call on the same inputs."""
    tn = _tn()
    segs = synth.config_inputs("C4", scale=1 / 512)
    inp = _inputs(segs)
    eager = tn.decode_segments(inp)  # uploads plans and sizes the workspace
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        captured = tn.decode_segments(inp)
    torch.cuda.synchronize()
    for rep in range(3):
        if rep > 0:
            for k, (s, x) in enumerate(zip(segs, inp)):
                new = synth.sample(s["d"], s["rates"], len(s["syndromes"]), 9000 + 17 * rep + k, s["model_index"])
                x.syndromes.copy_(torch.from_numpy(new["syndromes"]).to(DEV))
        for o in captured:
            o.logz.fill_(float("nan"))
            o.cls.fill_(255)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        ref = tn.decode_segments(inp)
        torch.cuda.synchronize()
        for a, b in zip(captured, ref):
            assert torch.equal(a.logz, b.logz)
            assert torch.equal(a.logp, b.logp)
            assert torch.equal(a.cls, b.cls)
    del eager


def test_launch_plan_one_launch_per_precision_and_build():
    """The mixed batch stays one persistent launch per form: d = 5..9 alone
    would run three 256-thread groups per CU and d = 11..15 need two, so the
    whole C4 batch runs on two.  The p-sweep (d = 9 only) runs on three; a
    call with two forms makes one launch for each."""
    tn = _tn()
    c4 = synth.config_inputs("C4", scale=1 / 1024)
    plan = tn.api.launch_plan(_inputs(c4, "bf16"))
    print("C4 bf16:", plan, flush=True)
    assert plan == [dict(precision="bf16", threads=256, wg_per_cu=2, segments=len(c4))]
    small = [s for s in c4 if s["d"] <= 9]
    plan = tn.api.launch_plan(_inputs(small, "bf16"))
    print("C4 d <= 9, bf16:", plan, flush=True)
    assert plan == [dict(precision="bf16", threads=256, wg_per_cu=3, segments=len(small))]
    c2 = synth.config_inputs("C2", scale=1 / 4096)
    plan = tn.api.launch_plan(_inputs(c2, "fp32plain"))
    print("C2 fp32plain:", plan, flush=True)
    assert plan == [dict(precision="fp32plain", threads=256, wg_per_cu=3, segments=len(c2))]
    mixed = _inputs(small, "bf16") + _inputs(small, "fp32plain")
    plan = tn.api.launch_plan(mixed)
    print("two forms:", plan, flush=True)
    assert len(plan) == 2 and {p["precision"] for p in plan} == {"bf16", "fp32plain"}
    assert all(p["wg_per_cu"] == 3 and p["segments"] == len(small) for p in plan)
