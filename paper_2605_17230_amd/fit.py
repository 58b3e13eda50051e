"""Noise-model fitting from syndromes alone (paper Sec. 3.2.4, eq. "dmle_loss").

The per-qubit Pauli rates theta = ln p_{q,X|Y|Z} (p_I = 1 - sum) are fitted by
minimising the mean negative log-likelihood of the observed syndromes,

    L(theta) = -(1 / |D|) sum_{s in D} log P_theta(s),

with Adam.  log P_theta(s) and its gradient come from the library's boundary-MPS
contraction and its adjoint (``log_posterior``); nothing here is specific to
the GPU beyond that call, so another log-likelihood with the same signature
can be passed in.
"""
import math

import torch

from .api import log_posterior


def fit_log_rates(syndromes, d, chi, log_rates0, steps=50, lr=0.05, precision="fp32", weights=None, batch=0,
                  seed=0, pmax=0.3, loglik=None):
    """Adam on theta; returns (theta [.., d*d, 3] float64, per-step losses).

    syndromes  uint8 [B, d*d-1] (device tensor for the library path)
    log_rates0 float64 [d*d, 3] or [M, d*d, 3]: starting point
    weights    optional float64 [B]: multiplicities (loss = weighted mean)
    batch      syndromes per step drawn without replacement (0: all)
    pmax       each rate is kept <= pmax after every step, so p_I >= 1 - 3 pmax > 0
    loglik     f(theta, syndromes) -> log P [B] with autograd; default: the library
    """
    if loglik is None:
        def loglik(th, syn):
            return log_posterior(th, syn, d, chi, precision)[0]
    if not 0.0 < pmax < 1.0 / 3.0:
        raise ValueError("pmax must lie in (0, 1/3)")
    theta = log_rates0.detach().clone().to(torch.float64).requires_grad_(True)
    opt = torch.optim.Adam([theta], lr=lr)
    gen = torch.Generator().manual_seed(seed)
    nb = syndromes.shape[0]
    hist = []
    for _ in range(steps):
        syn, w = syndromes, weights
        if 0 < batch < nb:
            idx = torch.randperm(nb, generator=gen)[:batch].to(syndromes.device)
            syn = syndromes[idx]
            w = None if weights is None else weights[idx]
        logp = loglik(theta, syn)
        loss = -(logp.mean() if w is None else (w * logp).sum() / w.sum())
        opt.zero_grad()
        loss.backward()
        opt.step()
        with torch.no_grad():
            theta.clamp_(max=math.log(pmax))
        hist.append(float(loss.detach()))
    return theta.detach(), hist
