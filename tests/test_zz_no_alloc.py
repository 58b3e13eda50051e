"""The allocation-free entry point (tn_decode_batch_noalloc) against
tn_decode_batch through the C ABI: the same kernels on the same inputs, so
log Z, log P and the class must be equal bit for bit.  Two calls in a row, the
second smaller, reuse the fixed device array; a third call at the benchmark's
size (d = 17, chi = 32) runs with fewer persistent work-groups than usual."""
import ctypes
import warnings

import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def _segments(specs, prec):
    import paper_2605_17230_amd as tn
    segs = []
    for d, chi, count, seed in specs:
        r = synth.depolarizing(d, 0.1)
        smp = synth.sample(d, r, count, seed)
        segs.append(tn.SegmentInput(d, chi, torch.from_numpy(smp["syndromes"]).to(DEV), torch.from_numpy(r).to(DEV),
                                    None, prec))
    return segs


def _noalloc(segs):
    import paper_2605_17230_amd as tn
    from paper_2605_17230_amd import api
    arr, outs, keep = api._prepare(segs, check=True)
    for o in outs:  # poison the outputs: every element must be written
        o.logz.fill_(float("nan"))
        o.cls.fill_(77)
    L = tn.lib()
    st = torch.cuda.current_stream().cuda_stream
    tn._lib.check(L.tn_decode_batch_noalloc(arr, len(segs), 1e-9, ctypes.c_void_p(st)))
    cnt = ctypes.c_int64(0)
    tn._lib.check(L.tn_workspace_status(None, 0, ctypes.c_void_p(st), ctypes.byref(cnt)))
    torch.cuda.synchronize()
    del keep
    return outs


@pytest.mark.parametrize("prec", ["fp32", "bf16"])
def test_noalloc_matches_workspace_entry_point(prec):
    import paper_2605_17230_amd as tn
    big = _segments([(5, 8, 300, 1), (9, 16, 200, 2), (13, 24, 40, 3)], prec)
    small = _segments([(7, 12, 17, 4)], prec)
    for segs in (big, small):  # second call smaller than the first
        print("noalloc %s: %s" % (prec, [(s.d, s.chi, s.syndromes.shape[0]) for s in segs]), flush=True)
        with warnings.catch_warnings():
            warnings.simplefilter("ignore", tn.api.UnresolvedCosetsWarning)
            ref = tn.decode_segments(segs)
            got = _noalloc(segs)
        for a, b in zip(got, ref):
            assert torch.equal(a.logz, b.logz)
            assert torch.equal(a.logp, b.logp)
            assert torch.equal(a.cls, b.cls)


def test_noalloc_at_the_benchmark_size():
    """d = 17, chi = 32: one work-group needs about 1.4 MB, so the fixed array
    holds fewer persistent groups than the 256 of the usual launch; the
    results are still bitwise those of tn_decode_batch."""
    import paper_2605_17230_amd as tn
    segs = _segments([(17, 32, 512, 3000)], "bf16")
    print("noalloc d=17 chi=32 bf16, 512 syndromes", flush=True)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore", tn.api.UnresolvedCosetsWarning)
        ref = tn.decode_segments(segs)
        got = _noalloc(segs)
    assert torch.equal(got[0].logz, ref[0].logz) and torch.equal(got[0].cls, ref[0].cls)
