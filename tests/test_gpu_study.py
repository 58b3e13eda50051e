"""Decoder sanity on the same kernels: the truncation error against chi
converges to the exact contraction (oracle O3), and the logical error rate
falls with the distance below the depolarizing threshold and rises with it
above (paper Sec. 3.1.2, table "thresholds": about 18.9 % for MLD of
depolarizing code-capacity noise on the surface code)."""
import numpy as np
import pytest
import torch

import oracle
import synth
import paper_2605_17230_amd as tn

pytestmark = pytest.mark.gpu


def test_chi_convergence_d9_vs_exact():
    d, p = 9, 0.17
    rates = synth.depolarizing(d, p)
    smp = synth.sample(d, rates, 128, seed=6950)
    ref = np.logaddexp.reduce(oracle.transfer(d, rates, smp["syndromes"]), axis=1)
    syn, rt = torch.from_numpy(smp["syndromes"]).cuda(), torch.from_numpy(rates).cuda()
    err = []
    for chi in (4, 8, 16, 32):
        lp = tn.decode(syn, rt, d, chi, "fp64")[1].cpu().numpy()
        err.append(float(np.mean(np.abs(lp - ref))))
    assert err[0] > 1e-3
    assert all(a > 10 * b for a, b in zip(err, err[1:])), err
    assert err[-1] < 1e-6, err


def test_logical_error_rate_crosses_with_distance():
    n = 16384

    def ler(d, p, seed):
        rates = synth.depolarizing(d, p)
        smp = synth.sample(d, rates, n, seed=seed)
        cls = tn.decode(torch.from_numpy(smp["syndromes"]).cuda(), torch.from_numpy(rates).cuda(), d, 16,
                        "fp32plain")[2].cpu().numpy()
        return float((cls != smp["true_class"]).mean())

    def sigma(a, b):  # standard error of the difference of two independent rates
        return np.sqrt((a * (1 - a) + b * (1 - b)) / n)

    lo5, lo9 = ler(5, 0.12, 7001), ler(9, 0.12, 7002)
    hi5, hi9 = ler(5, 0.23, 7003), ler(9, 0.23, 7004)
    assert lo9 < lo5 - 5 * sigma(lo5, lo9), (lo5, lo9)
    assert hi9 > hi5 + 5 * sigma(hi5, hi9), (hi5, hi9)
