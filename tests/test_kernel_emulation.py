"""The sweep kernels' own source, run on the host: tests/emu maps one
work-group onto 512 std::threads (barriers for __syncthreads and the lane
exchanges), so the forward contraction and the adjoint of
paper_2605_17230_amd/csrc can be checked against the FP64 oracle without a
GPU.  DPP lane moves are the one device feature replaced (by the same
exchange through memory), so these tests pin the algorithm and its
synchronisation, the GPU tests the lane layout."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EMU = os.path.join(ROOT, "tests", "emu")
CSRC = os.path.join(ROOT, "paper_2605_17230_amd", "csrc")
LIB = os.path.join(EMU, "_build", "libemu.so")


@pytest.fixture(scope="module")
def emu():
    os.makedirs(os.path.dirname(LIB), exist_ok=True)
    subprocess.check_call(["g++", "-O2", "-std=c++20", "-shared", "-fPIC", "-I", CSRC, "-I", EMU,
                           os.path.join(EMU, "emu_main.cpp"), os.path.join(CSRC, "plan.cpp"), "-o", LIB,
                           "-lpthread"])
    L = ctypes.CDLL(LIB)
    P = ctypes.c_void_p
    L.emu_forward.argtypes = [ctypes.c_int] * 4 + [P, P, ctypes.c_int, P]
    L.emu_gradient.argtypes = [ctypes.c_int] * 4 + [P, P, ctypes.c_int, P, P, P, P]
    L.emu_forward_models.argtypes = [ctypes.c_int] * 4 + [P, ctypes.c_int, P, P, ctypes.c_int, P, P]
    L.emu_forward_rounds.argtypes = [ctypes.c_int] * 4 + [P, P, P, ctypes.c_int, P, P]
    return L


@pytest.fixture(scope="module")
def emu256():
    """The same sources built for 256-thread work-groups (the second build of
    the forward kernel: four rows per lane group in the register LQ)."""
    lib = os.path.join(EMU, "_build", "libemu256.so")
    os.makedirs(os.path.dirname(lib), exist_ok=True)
    subprocess.check_call(["g++", "-O2", "-std=c++20", "-shared", "-fPIC", "-DTNMLD_NT=256", "-I", CSRC, "-I", EMU,
                           os.path.join(EMU, "emu_main.cpp"), os.path.join(CSRC, "plan.cpp"), "-o", lib,
                           "-lpthread"])
    L = ctypes.CDLL(lib)
    P = ctypes.c_void_p
    L.emu_forward.argtypes = [ctypes.c_int] * 4 + [P, P, ctypes.c_int, P]
    L.emu_forward_xg.argtypes = [ctypes.c_int] * 4 + [P, P, ctypes.c_int, P]
    return L


def forward(L, d, chi, prec, group, rates, syn):
    rates = np.ascontiguousarray(rates, np.float64)
    syn = np.ascontiguousarray(syn, np.uint8)
    out = np.full((len(syn), 4), np.nan)
    assert L.emu_forward(d, chi, prec, group, rates.ctypes.data, syn.ctypes.data, len(syn), out.ctypes.data) == 0
    return out


@pytest.mark.parametrize("prec,group,tol", [(0, 1, 1e-12), (3, 2, 1e-4)])
def test_d3_exact_forward(emu, prec, group, tol):
    rates = synth.inhomogeneous(3, 0.01, 0.15, seed=1)
    syn = synth.sample(3, rates, 1, seed=2)["syndromes"]
    got = forward(emu, 3, 0, prec, group, rates, syn)
    ref = oracle.transfer(3, rates, syn)
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(got), fin)
    assert np.max(np.abs(got[fin] - ref[fin])) < tol


def test_d3_truncated_forward_is_deterministic(emu):
    """chi = 2 truncates every inner bond (Jacobi on every cut): two runs of
    512 racing threads must agree bit for bit, and stay near the exact value."""
    rates = synth.depolarizing(3, 0.1)
    syn = synth.sample(3, rates, 1, seed=4)["syndromes"]
    a = forward(emu, 3, 2, 0, 1, rates, syn)
    b = forward(emu, 3, 2, 0, 1, rates, syn)
    assert np.array_equal(a, b)
    ref = oracle.transfer(3, rates, syn)
    assert np.max(np.abs(np.logaddexp.reduce(a, 1) - np.logaddexp.reduce(ref, 1))) < 0.5


def test_d3_gradient(emu):
    rates = synth.inhomogeneous(3, 0.01, 0.15, seed=5)
    syn = synth.sample(3, rates, 1, seed=6)["syndromes"]
    logz = forward(emu, 3, 0, 0, 2, rates, syn)
    logp = np.logaddexp.reduce(logz, 1)
    gw = np.array([-0.7])
    out = np.zeros((9, 3))
    assert emu.emu_gradient(3, 0, 0, 2, np.ascontiguousarray(rates).ctypes.data,
                            np.ascontiguousarray(syn, np.uint8).ctypes.data, len(syn), logz.ctypes.data,
                            logp.ctypes.data, gw.ctypes.data, out.ctypes.data) == 0
    ref = sum(w * oracle.grad_logp(3, rates, s)[0] for s, w in zip(syn, gw))
    assert np.max(np.abs(out - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


def forward_models(L, d, chi, prec, rates, model_index, syn):
    """Forward with per-syndrome models; returns (log Z, status word)."""
    rates = np.ascontiguousarray(rates, np.float64)
    if rates.ndim == 2:
        rates = rates[None]
    mi = np.ascontiguousarray(model_index, np.int32)
    syn = np.ascontiguousarray(syn, np.uint8)
    out = np.full((len(syn), 4), np.nan)
    st = np.zeros(4, np.uint32)  # status word, then the 64-bit count of unresolved cosets
    assert L.emu_forward_models(d, chi, prec, 1, rates.ctypes.data, rates.shape[0], mi.ctypes.data, syn.ctypes.data,
                                len(syn), out.ctypes.data, st.ctypes.data) == 0
    return out, int(st[0])


ST_BAD_INPUT, ST_NUMERIC, ST_UNRESOLVED = 1, 2, 4


def test_device_input_checks(emu):
    """The kernels' own input check, one call: a syndrome byte above 1, a model
    with a negative, a NaN or an over-unity rate, and model indices out of
    range each give log Z = -inf for that syndrome only (never NaN) and raise
    the status bit the host reads back as TN_EINVAL; the valid syndrome is
    decoded exactly."""
    d = 3
    good = synth.depolarizing(d, 0.1)
    neg, nan, over = good.copy(), good.copy(), good.copy()
    neg[4, 1] = -1e-3
    nan[7, 2] = np.nan
    over[2] = [0.5, 0.4, 0.2]
    rates = np.stack([good, neg, nan, over])
    syn = np.repeat(synth.sample(d, good, 1, seed=3)["syndromes"], 7, axis=0)
    syn[0, 3] = 2
    mi = np.array([0, 1, 2, 3, 4, -1, 0], np.int32)
    out, st = forward_models(emu, d, 0, 0, rates, mi, syn)
    assert st == ST_BAD_INPUT
    assert np.isneginf(out[:6]).all() and not np.isnan(out).any()
    ref = oracle.transfer(d, good, syn[6:])
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(out[6:]), fin)
    assert np.max(np.abs(out[6:] - ref)[fin]) < 1e-12


def test_numeric_status_only_for_positive_models(emu):
    """A coset whose contraction vanishes is impossible when some rates are
    zero (log Z = -inf, no status), but a precision loss when every Pauli has
    a positive probability: with rates so small that FP32 underflows them to
    zero, a syndrome that needs an error loses all four cosets (ST_NUMERIC)
    and the trivial syndrome keeps coset I and loses the other three
    (ST_UNRESOLVED, counted), instead of silently reporting impossible
    cosets."""
    d = 3
    zero = np.zeros((d * d, 3))
    syn = np.zeros((1, d * d - 1), np.uint8)
    syn[0, 0] = 1
    out, st = forward_models(emu, d, 0, 3, zero, np.zeros(1), syn)
    assert st == 0 and np.isneginf(out).all()
    tiny = np.full((d * d, 3), 1e-46)  # positive in FP64, zero once rounded to FP32
    out, st = forward_models(emu, d, 0, 3, tiny, np.zeros(1), syn)
    assert st == ST_NUMERIC and not np.isnan(out).any()
    out, st = forward_models(emu, d, 0, 3, tiny, np.zeros(1), np.zeros_like(syn))
    assert st == ST_UNRESOLVED and np.isfinite(out[0, 0]) and np.isneginf(out[0, 1:]).all()
    out64, st64 = forward_models(emu, d, 0, 0, tiny, np.zeros(1), syn)  # FP64 keeps log P(s)
    assert not (st64 & ST_NUMERIC) and np.isfinite(np.logaddexp.reduce(out64, 1)).all()


def test_d3_two_rounds_exact(emu):
    """Repeated noisy rounds (T = 2, last round perfect): the kernel source's
    column variables with one bit per round, the measurement weights as
    Fourier duals and the qubit tensors summed over the intermediate
    accumulated Pauli, untruncated at d = 3 in FP64, against the exact
    phenomenological oracle O7 (itself pinned by enumeration, sampled
    frequencies and total probability)."""
    d, m = 3, 8
    r = synth.inhomogeneous(d, 0.01, 0.1, seed=1)
    q = np.linspace(0.02, 0.12, m)
    smp = synth.sample_phenom(d, r, q, 2, 2, seed=2)
    syn = np.ascontiguousarray(smp["syndromes"], np.uint8)
    out = np.zeros((2, 4))
    st = np.zeros(4, np.uint32)
    assert emu.emu_forward_rounds(d, 0, 0, 2, r.ctypes.data, q.ctypes.data, syn.ctypes.data, 2, out.ctypes.data,
                                  st.ctypes.data) == 0
    ref = oracle.phen_transfer(d, 2, r, q, syn)
    assert st[0] == 0
    assert np.max(np.abs(out - ref) / np.maximum(1.0, np.abs(ref))) < 1e-12


@pytest.mark.parametrize("chi,prec,group", [(0, 3, 2)])
def test_lq_matrix_in_global_scratch(emu256, chi, prec, group):
    """The layout of the 256-thread launches whose LQ matrix does not fit LDS
    (the LQ matrix in the work-group's scratch; with FP32 factorisations the
    explicit Q stages one reflector at a time through LDS)
    gives the same log Z, bit for bit, as the LDS layout: the same operations in
    the same order per row.  d = 3, exact, two columns per site (the layout is
    used with FP32 factorisations only)."""
    d = 3
    rates = synth.inhomogeneous(d, 0.01, 0.15, seed=11)
    syn = np.ascontiguousarray(synth.sample(d, rates, 1, seed=12)["syndromes"])
    r = np.ascontiguousarray(rates)
    a = np.full((1, 4), np.nan)
    b = np.full((1, 4), np.nan)
    assert emu256.emu_forward(d, chi, prec, group, r.ctypes.data, syn.ctypes.data, 1, a.ctypes.data) == 0
    assert emu256.emu_forward_xg(d, chi, prec, group, r.ctypes.data, syn.ctypes.data, 1, b.ctypes.data) == 0
    assert np.array_equal(a, b)
    ref = oracle.transfer(d, rates, syn)
    fin = np.isfinite(ref)
    assert np.max(np.abs(b[fin] - ref[fin])) < (1e-4 if prec == 3 else 1e-3)
