"""Mixed batches in one persistent launch (distances 5..15, three Z-biases per
distance, chi by distance) and replay of a captured launch, against the FP64
oracle and against single-segment launches."""
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


def _check_vs_oracle(s, o, idx):
    ref = _oracle_logz(s, idx)
    lz = o.logz.cpu().numpy()[idx]
    cls = o.cls.cpu().numpy()[idx]
    lp_ref, cls_ref = oracle.decide(ref)
    lp = o.logp.cpu().numpy()[idx]
    # truncation error at these chi: log P(s) to 1e-2, classes equal unless the
    # oracle's top-two gap is inside the error
    assert np.max(np.abs(lp - lp_ref)) < 1e-2, (s["d"], np.max(np.abs(lp - lp_ref)))
    top2 = np.sort(ref, axis=1)[:, -2:]
    clear = (top2[:, 1] - top2[:, 0]) > 2e-2
    assert np.all(cls[clear] == cls_ref[clear])
    return float(np.max(np.abs(np.where(np.isfinite(ref), lz - ref, 0.0))))


def test_c4_mixed_launch_small():
    """Every C4 segment at 1/256 of its count in one call: each against the
    exact oracle and bitwise against the segment decoded alone."""
    tn = _tn()
    segs = synth.config_inputs("C4", scale=1 / 256)
    outs = tn.decode_segments(_inputs(segs))
    for s, o in zip(segs, outs):
        _check_vs_oracle(s, o, list(range(len(s["syndromes"]))))
        alone = tn.decode_segments(_inputs([s]))[0]
        assert torch.equal(alone.logz, o.logz)
        assert torch.equal(alone.cls, o.cls)


@pytest.mark.slow
def test_c4_full_mixed_launch_sampled():
    """The whole C4 batch (63,488 syndromes, six distances) in one persistent
    launch; 12 syndromes of every segment against the exact oracle."""
    tn = _tn()
    segs = synth.config_inputs("C4")
    outs = tn.decode_segments(_inputs(segs))
    torch.cuda.synchronize()
    rng = np.random.default_rng(4)
    for s, o in zip(segs, outs):
        n = len(s["syndromes"])
        idx = sorted(rng.choice(n, 12, replace=False).tolist())
        _check_vs_oracle(s, o, idx)
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
