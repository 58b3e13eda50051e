"""The gradient in two calls (tn_coset_loglik_save, then
tn_coset_loglik_backward_saved): the top sweep's states kept in device memory
between the calls give the same log Z, log P(s) and gradient, bit for bit,
as the one-call backward (tn_coset_loglik_backward), which recomputes them;
the autograd binding uses the two calls."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def _tn():
    import paper_2605_17230_amd as tn
    return tn


@pytest.mark.parametrize("d,chi,prec", [(5, 8, "fp64"), (9, 16, "fp32"), (11, 24, "fp32plain"), (9, 16, "bf16")])
def test_two_calls_equal_one_call(d, chi, prec):
    tn = _tn()
    r = np.stack([synth.inhomogeneous(d, 0.01, 0.1, seed=d), synth.depolarizing(d, 0.08)])
    mi = (np.arange(40) % 2).astype(np.int32)
    smp = synth.sample(d, r, 40, seed=d + 1, model_index=mi)
    seg = tn.SegmentInput(d, chi, torch.from_numpy(smp["syndromes"]).to(DEV), torch.from_numpy(r).to(DEV),
                          torch.from_numpy(mi).to(DEV), prec)
    g = torch.from_numpy(np.random.default_rng(d).normal(size=40)).to(DEV)
    o1, g1 = tn.coset_loglik_backward([seg], [g])
    o2, states = tn.coset_loglik_save([seg])
    assert states.numel() >= tn.states_bytes([seg])
    g2 = tn.coset_loglik_backward_saved([seg], [g], o2, states)
    torch.cuda.synchronize()
    assert torch.equal(o1[0].logz, o2[0].logz) and torch.equal(o1[0].logp, o2[0].logp)
    assert torch.equal(g1[0], g2[0])
    # a second backward from the same states (another weight vector) accumulates the same way
    g3 = tn.coset_loglik_backward_saved([seg], [2.0 * g], o2, states)
    _, g4 = tn.coset_loglik_backward([seg], [2.0 * g], outputs=o1)
    assert torch.equal(g3[0], g4[0])


def test_autograd_uses_saved_states():
    """log_posterior keeps the states in its forward; its gradient equals the
    one-call backward's."""
    tn = _tn()
    d, chi = 7, 12
    r = synth.inhomogeneous(d, 0.01, 0.1, seed=3)
    smp = synth.sample(d, r, 24, seed=4)
    syn = torch.from_numpy(smp["syndromes"]).to(DEV)
    theta = torch.from_numpy(np.log(r)).to(DEV).requires_grad_()
    logp, _ = tn.log_posterior(theta, syn, d, chi, "fp32")
    logp.sum().backward()
    # the same rates the forward used: exp(ln r), which may differ from r in the last bit
    seg = tn.SegmentInput(d, chi, syn, theta.detach().exp(), None, "fp32")
    _, g = tn.coset_loglik_backward([seg], [torch.ones(24, dtype=torch.float64, device=DEV)])
    assert torch.equal(theta.grad, g[0][0])


def test_no_states_kept_without_gradient():
    """Under torch.no_grad (or for rates that need no gradient) log_posterior
    runs the plain forward pass: same log P(s), and no state buffer is
    allocated."""
    tn = _tn()
    d, chi = 7, 12
    r = synth.inhomogeneous(d, 0.01, 0.1, seed=5)
    smp = synth.sample(d, r, 24, seed=6)
    syn = torch.from_numpy(smp["syndromes"]).to(DEV)
    theta = torch.from_numpy(np.log(r)).to(DEV)
    seg = tn.SegmentInput(d, chi, syn, theta.exp(), None, "fp32")
    ref = tn.decode_segments([seg])[0].logp  # the workspace of this shape now exists
    need = tn.states_bytes([seg])
    torch.cuda.synchronize()
    for grad_on, th in ((False, theta.clone().requires_grad_()), (True, theta)):
        torch.cuda.reset_peak_memory_stats()
        base = torch.cuda.memory_allocated()
        with torch.set_grad_enabled(grad_on):
            logp, _ = tn.log_posterior(th, syn, d, chi, "fp32")
        torch.cuda.synchronize()
        assert torch.cuda.max_memory_allocated() - base < need // 2
        assert torch.equal(logp.detach(), ref)


def test_saved_call_argument_errors():
    tn = _tn()
    d = 5
    r = torch.from_numpy(synth.depolarizing(d, 0.05)).to(DEV)
    syn = torch.from_numpy(synth.sample(d, synth.depolarizing(d, 0.05), 4, seed=1)["syndromes"]).to(DEV)
    seg = tn.SegmentInput(d, 8, syn, r, None, "fp32")
    need = tn.states_bytes([seg])
    with pytest.raises(ValueError):
        tn.coset_loglik_save([seg], states=torch.empty(need - 1, dtype=torch.uint8, device=DEV))
    o, states = tn.coset_loglik_save([seg])
    with pytest.raises(tn.TNError) as e:
        tn.coset_loglik_backward_saved([seg], [torch.ones(4, dtype=torch.float64, device=DEV)], o, states[:need - 1])
    assert e.value.code == tn._lib.TN_EINVAL
