"""Host-side checks of the C-ABI library that need no GPU."""
import ctypes
import os

import numpy as np
import pytest

import oracle

_lib = pytest.importorskip("paper_2605_17230_amd._lib")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libtnmld.so not built (run __graft_entry__.build())")
    return _lib.lib()


def test_exports_every_declared_symbol(L):
    names = _lib.header_functions()
    assert {"tn_workspace_size", "tn_coset_loglik", "tn_decode_batch", "tn_coset_loglik_backward",
            "tn_code_stabilizers", "tn_plan_info", "tn_last_error"} <= set(names)
    for nm in names:
        assert hasattr(L, nm), nm


@pytest.mark.parametrize("d", [3, 5, 9, 17, 21])
def test_code_stabilizers_match_oracle_layout(d):
    import paper_2605_17230_amd as tn
    t, s = tn.code_stabilizers(d)
    ot, os_ = oracle.layout(d)
    assert np.array_equal(t, ot) and np.array_equal(s, os_)


def _seg(**kw):
    base = dict(d=5, chi=8, precision=1, n_models=1, rates=1, model_index=None, syndromes=1, count=4,
                out_logz=1, out_logp=None, out_class=None)
    base.update(kw)
    return _lib.Segment(**base)


@pytest.mark.parametrize("bad", [dict(d=4), dict(d=1), dict(d=33), dict(chi=-1), dict(precision=7),
                                 dict(n_models=0), dict(count=-2), dict(syndromes=None), dict(out_logz=None),
                                 dict(rounds=3), dict(rounds=-1), dict(rounds=2, meas_rates=None)])
def test_invalid_arguments_rejected_before_device(L, bad):
    arr = (_lib.Segment * 1)(_seg(**bad))
    rc = L.tn_coset_loglik(arr, 1, None, 0, None)
    assert rc == _lib.TN_EINVAL
    assert L.tn_last_error()
    assert L.tn_workspace_size(arr, 1, 0) == 0


def test_segment_count_limits(L):
    arr = (_lib.Segment * 17)(*[_seg() for _ in range(17)])
    assert L.tn_coset_loglik(arr, 17, None, 0, None) == _lib.TN_EINVAL
    assert L.tn_coset_loglik(arr, 0, None, 0, None) == _lib.TN_EINVAL


def test_no_device_reports_edevice(L):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    arr = (_lib.Segment * 1)(_seg())
    assert L.tn_coset_loglik(arr, 1, None, 0, None) == _lib.TN_EDEVICE


def test_plan_info_counts():
    import paper_2605_17230_amd as tn
    a = tn.plan_info(17, 32, "fp32")
    b = tn.plan_info(17, 16, "fp32")
    assert a["rows"] == 33 and a["flops"] > b["flops"] > 0
    assert a["lds_bytes"] <= 160 * 1024
    with pytest.raises(tn.TNError):
        tn.plan_info(4, 8, "fp32")


@pytest.mark.parametrize("d,chi", [(3, 0), (9, 16), (17, 32)])
def test_gemm_flops_are_part_of_the_counted_work(L, d, chi):
    """tn_plan_gemm_flops: the GEMM-class part of the counted forward work, per
    coset and per syndrome as executed (shared rows once, as for the total)."""
    import paper_2605_17230_amd as tn
    i = tn.plan_info(d, chi, "bf16")
    assert 0 < i["gemm_flops"] < i["flops"]
    assert i["gemm_flops"] <= i["gemm_flops_syndrome"] <= 4 * i["gemm_flops"]
    assert i["gemm_flops_syndrome"] < i["flops_syndrome"]


def test_status_entry_point_rejects_small_workspace(L):
    """tn_workspace_status needs a workspace of at least one header block
    (a NULL workspace names the allocation-free entry point's array, which
    needs a device)."""
    buf = ctypes.create_string_buffer(64)
    assert L.tn_workspace_status(buf, 64, None, None) == _lib.TN_EINVAL
    assert L.tn_last_error()
    import torch
    if not torch.cuda.is_available():
        assert L.tn_workspace_status(None, 0, None, None) == _lib.TN_EDEVICE


@pytest.mark.parametrize("case", ["byte", "neg", "nan", "over", "index", "index_neg"])
def test_input_value_checks_raise_before_launch(case):
    """The host-side value check that runs before every checked launch: each
    kind of invalid input raises ValueError (no kernel is launched); valid
    inputs pass.  Runs on CPU tensors."""
    import torch
    import paper_2605_17230_amd as tn
    import synth
    d = 5
    rates = torch.from_numpy(np.stack([synth.depolarizing(d, 0.1), synth.biased(d, 0.1, 10.0)]))
    syn = torch.from_numpy(synth.sample(d, synth.depolarizing(d, 0.1), 8, seed=1)["syndromes"])
    mi = torch.zeros(8, dtype=torch.int32)
    tn.check_input_values(syn, rates, mi)
    tn.check_input_values(syn, rates[0], None)
    if case == "byte":
        syn = syn.clone()
        syn[3, 7] = 2
    elif case == "neg":
        rates = rates.clone()
        rates[1, 4, 0] = -1e-9
    elif case == "nan":
        rates = rates.clone()
        rates[0, 0, 2] = float("nan")
    elif case == "over":
        rates = rates.clone()
        rates[0, 3] = torch.tensor([0.4, 0.4, 0.3], dtype=torch.float64)
    elif case == "index":
        mi = mi.clone()
        mi[5] = 2
    else:
        mi = mi.clone()
        mi[0] = -1
    with pytest.raises(ValueError):
        tn.check_input_values(syn, rates, mi)


@pytest.mark.parametrize("d", [3, 5, 9, 17, 31])
def test_planar_plan_counts(d):
    """The Kac-Ward plan: matrix order 2(n + 1) (a bond per qubit and the ghost
    bond, both directions); the entries of Lambda are the pairs of bonds
    meeting at a vertex, sum over vertices of deg (deg - 1), with the degrees
    counted here from the check layout (an X-type check has one bond per qubit
    of its support; each ghost has the d qubits of its side plus the ghost
    bond); the prefactor (m_X - n) ln 2."""
    import paper_2605_17230_amd as tn
    import synth
    info = tn.bitflip_plan_info(d)
    n = d * d
    types, sup = synth.code_checks(d)
    deg = [int((s >= 0).sum()) for t, s in zip(types, sup) if t == 0]
    deg += [d + 1, d + 1]
    assert info["order"] == 2 * (n + 1)
    assert info["nnz"] == sum(k * (k - 1) for k in deg)
    assert abs(info["log_pref"] - ((n - 1) // 2 - n) * np.log(2.0)) < 1e-12
    with pytest.raises(tn.TNError):
        tn.bitflip_plan_info(4)


def test_tune_cache_entries_are_their_fastest_candidates():
    """Every autotuner cache entry stores the launch shape of its fastest
    timed candidate (the cache is the tuner's output, not edited by hand)."""
    import json
    from paper_2605_17230_amd import tune
    with open(tune.DEFAULT_CACHE) as f:
        cache = json.load(f)
    assert cache["entries"]
    for key, e in cache["entries"].items():
        best = max(e["candidates"], key=lambda c: c["syndromes_per_s"])
        assert (e["group"], e["wg_per_cu"], e["threads"]) == (best["group"], best["wg_per_cu"], best["threads"]), key
        assert e["syndromes_per_s"] == best["syndromes_per_s"]


def test_rounds_plans():
    """Plans of the repeated-rounds network (T = 2): one column per site, more
    counted work than one round at the same chi, and the LDS limits of each
    form (the FP64 factorisations of chi = 16 do not fit a CU)."""
    import paper_2605_17230_amd as tn
    for d, chi in [(3, 0), (5, 12), (9, 12)]:
        one = tn.plan_info(d, chi, "fp64")
        two = tn.plan_info(d, chi, "fp64", rounds=2)
        assert two["group"] == 1 and two["flops"] > one["flops"] and two["rows"] == one["rows"]
    assert tn.plan_info(17, 16, "fp32plain", rounds=2)["lds_bytes"] <= 160 * 1024
    with pytest.raises(tn.TNError):
        tn.plan_info(9, 16, "fp64", rounds=2)
    with pytest.raises(tn.TNError):
        tn.plan_info(9, 8, "fp64", rounds=3)


def test_rounds_input_checks():
    import torch
    import paper_2605_17230_amd as tn
    import synth
    d = 5
    r = torch.from_numpy(synth.depolarizing(d, 0.05))
    q = torch.full((d * d - 1,), 0.05, dtype=torch.float64)
    smp = synth.sample_phenom(d, r.numpy(), q.numpy(), 2, 4, seed=1)
    syn = torch.from_numpy(smp["syndromes"].reshape(4, -1))
    tn.check_input_values(syn, r, None, q)
    bad = q.clone()
    bad[3] = float("nan")
    with pytest.raises(ValueError):
        tn.check_input_values(syn, r, None, bad)
    bad[3] = 1.5
    with pytest.raises(ValueError):
        tn.check_input_values(syn, r, None, bad)


def test_gradient_rejects_repeated_rounds(L):
    """tn_coset_loglik_backward takes one syndrome round: a two-round segment
    is refused with TN_EUNSUPPORTED before any device call."""
    arr = (_lib.Segment * 1)(_seg(rounds=2, meas_rates=1))
    g = (ctypes.c_void_p * 1)(1)
    rc = L.tn_coset_loglik_backward(arr, 1, g, g, 0, None, 0, None)
    assert rc == _lib.TN_EUNSUPPORTED


def test_bf16_fp64_truncation_form(L):
    """TN_BF16_F64 (single-rounded bf16 contraction GEMMs, FP64 truncation) is a
    forward form: its plans build like the TN_FP32 form's (same storage and
    factorisation types), and the gradient refuses it with TN_EUNSUPPORTED
    before any device call."""
    import paper_2605_17230_amd as tn
    a, b = tn.plan_info(17, 32, "bf16f64"), tn.plan_info(17, 32, "fp32")
    assert a["lds_bytes"] == b["lds_bytes"] and a["flops_syndrome"] == b["flops_syndrome"]
    arr = (_lib.Segment * 1)(_seg(precision=_lib.TN_BF16_F64))
    g = (ctypes.c_void_p * 1)(1)
    assert L.tn_coset_loglik_backward(arr, 1, g, g, 0, None, 0, None) == _lib.TN_EUNSUPPORTED
    arr = (_lib.Segment * 1)(_seg(precision=5))
    assert L.tn_coset_loglik(arr, 1, None, 0, None) == _lib.TN_EINVAL


@pytest.mark.parametrize("d,chi", [(5, 8), (11, 24), (17, 32)])
def test_adjoint_flop_counts(d, chi):
    """tn_plan_adjoint_flops: the bottom-up sweep of a coset crosses the same
    rows as the top-down one (comparable counts; the bond dimensions differ
    with the direction: 0.65 of it at d = 5, chi = 8, 1.00 at d = 17,
    chi = 32), the row environments add work, and the per-syndrome total is
    the top sweep as executed plus four bottom sweeps and four sets of
    environments."""
    import paper_2605_17230_amd as tn
    i = tn.plan_info(d, chi, "fp32")
    assert 0.5 < i["bottom_sweep_flops"] / i["flops"] < 1.5
    assert 0 < i["environment_flops"] < i["flops"]
    tot = i["flops_syndrome"] + 4.0 * (i["bottom_sweep_flops"] + i["environment_flops"])
    assert abs(i["adjoint_flops_syndrome"] - tot) <= 1e-9 * tot


def test_saved_state_entry_points_reject_bad_arguments(L):
    """The two-call gradient's entry points check their arguments before any
    device call: invalid segments give size 0 and TN_EINVAL."""
    arr = (_lib.Segment * 1)(_seg(d=4))
    assert L.tn_states_size(arr, 1) == 0
    assert L.tn_coset_loglik_save(arr, 1, None, 0, None, 0, None) == _lib.TN_EINVAL
    g = (ctypes.c_void_p * 1)(1)
    assert L.tn_coset_loglik_backward_saved(arr, 1, g, g, None, 0, None, 0, None) == _lib.TN_EINVAL
