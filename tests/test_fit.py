"""Noise-model fitting (paper Sec. 3.2.4, eq. "dmle_loss"): Adam on the per-qubit
log rates, minimising the mean negative log-likelihood of observed syndromes.

CPU: driven by the oracle's exact log P(s) and gradient (O5), the fit must reach
the likelihood of the model that generated the data (the maximum-likelihood
estimate can only be better on its own data) and end at a stationary point.
GPU: the library-driven fit (FP64 path) must follow the oracle-driven one step
for step, and a d = 5 fit in the FP32 form must reach the true model's
likelihood as judged by the oracle."""
import numpy as np
import pytest
import torch

import oracle
import synth
from paper_2605_17230_amd.fit import fit_log_rates


class OracleLogP(torch.autograd.Function):
    """log P(s) [B] from the oracle, with its exact gradient in ln rates."""

    @staticmethod
    def forward(ctx, theta, syn, d):
        rates = theta.detach().exp().numpy()
        out = [oracle.grad_logp(d, rates, s) for s in syn.cpu().numpy()]
        ctx.save_for_backward(torch.from_numpy(np.stack([g for g, _ in out])))
        return torch.tensor([lp for _, lp in out], dtype=torch.float64)

    @staticmethod
    def backward(ctx, go):
        (g,) = ctx.saved_tensors
        return (go[:, None, None] * g).sum(0), None, None


def oracle_loglik(d):
    return lambda theta, syn: OracleLogP.apply(theta, syn, d)


def oracle_loss(d, rates, uniq, counts):
    logz = oracle.transfer(d, rates, uniq)
    logp = np.logaddexp.reduce(logz, axis=1)
    return -float((counts * logp).sum() / counts.sum())


def data(d, n, seed):
    true = synth.inhomogeneous(d, 0.02, 0.12, seed=seed)
    syn = synth.sample(d, true, n, seed=seed + 1)["syndromes"]
    uniq, counts = np.unique(syn, axis=0, return_counts=True)
    return true, uniq, counts.astype(np.float64)


def test_oracle_driven_fit_reaches_true_likelihood():
    d = 3
    true, uniq, counts = data(d, 20000, seed=11)
    theta0 = torch.full((d * d, 3), np.log(0.05), dtype=torch.float64)
    theta, hist = fit_log_rates(torch.from_numpy(uniq), d, 0, theta0, steps=150, lr=0.05,
                                weights=torch.from_numpy(counts), loglik=oracle_loglik(d))
    fitted = oracle_loss(d, theta.exp().numpy(), uniq, counts)
    assert hist[-1] < hist[0]
    assert fitted <= oracle_loss(d, true, uniq, counts) + 1e-4
    # stationary: the weighted score is small next to its value at the start
    g0 = sum(c * oracle.grad_logp(d, np.exp(theta0.numpy()), s)[0] for s, c in zip(uniq, counts)) / counts.sum()
    g1 = sum(c * oracle.grad_logp(d, theta.exp().numpy(), s)[0] for s, c in zip(uniq, counts)) / counts.sum()
    assert np.abs(g1).max() < 0.05 * np.abs(g0).max()


@pytest.mark.gpu
def test_library_fit_follows_oracle_fit():
    d = 3
    _, uniq, counts = data(d, 4000, seed=21)
    theta0 = torch.full((d * d, 3), np.log(0.04), dtype=torch.float64)
    syn = torch.from_numpy(uniq)
    w = torch.from_numpy(counts)
    th_o, h_o = fit_log_rates(syn, d, 0, theta0, steps=30, lr=0.05, weights=w, loglik=oracle_loglik(d))
    th_g, h_g = fit_log_rates(syn.cuda(), d, 0, theta0.cuda(), steps=30, lr=0.05, precision="fp64", weights=w.cuda())
    assert np.allclose(h_g, h_o, rtol=1e-9, atol=0)
    assert torch.max(torch.abs(th_g.cpu() - th_o)) < 1e-7


@pytest.mark.gpu
def test_fp32_fit_d5_reaches_true_likelihood():
    d = 5
    true, uniq, counts = data(d, 8192, seed=31)
    theta0 = torch.full((d * d, 3), np.log(0.05), dtype=torch.float64, device="cuda")
    theta, hist = fit_log_rates(torch.from_numpy(uniq).cuda(), d, 16, theta0, steps=120, lr=0.05,
                                precision="fp32", weights=torch.from_numpy(counts).cuda())
    assert hist[-1] < hist[0]
    fitted = oracle_loss(d, theta.cpu().exp().numpy(), uniq, counts)
    assert fitted <= oracle_loss(d, true, uniq, counts) + 1e-3
