"""FP64 CPU oracle (test infrastructure only).

Python bindings (ctypes) for ``tn_oracle.c``.  Only the test suite, the smoke
check and the CPU-baseline leg of the benchmark import this package; the GPU
library neither links nor calls it, and this package imports nothing from it.

Procedures (see the C file header for the passages they follow):
  enumerate_table  O1, every Pauli error, d = 3
  generator_sum    O2, sum over stabiliser products of a representative error
  transfer         O3, exact contraction over stabiliser variables
  rbim             O4, bit-flip noise as a random-bond Ising model
  grad_logp        O5, d log P(s) / d log p_{q,P}
  phen_enum2       O6, phenomenological noise, T = 2 rounds, d = 3 (enumeration)
  phen_transfer    O7, phenomenological noise, any T (exact transfer, small d)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "tn_oracle.c")
_LIB = os.path.join(_HERE, "libtnoracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, FP64 only)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        I = ctypes.c_int
        L = ctypes.c_int64
        D = ctypes.c_double
        sigs = {
            "orc_layout": (I, [I, P, P]),
            "orc_syndrome": (I, [I, P, L, P, P]),
            "orc_pure_error": (I, [I, I, P]),
            "orc_enumerate": (I, [I, P, P, P]),
            "orc_generator_sum": (I, [I, P, P, P]),
            "orc_transfer_w": (I, [I, P, P, P]),
            "orc_transfer": (I, [I, P, I, P, P, L, P, I]),
            "orc_max_slots": (I, [I]),
            "orc_rbim": (I, [I, D, P, P]),
            "orc_grad_logp": (I, [I, P, P, P, P]),
            "orc_decide": (I, [P, L, D, P, P]),
            "orc_phen_enum2": (I, [I, P, P, P, L, P]),
            "orc_phen_transfer": (I, [I, I, P, P, P, L, P, I]),
            "orc_phen_max_bits": (I, [I, I]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(lib, name)
            f.restype = res
            f.argtypes = args
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _chk(rc, what):
    if rc < 0:
        raise RuntimeError("oracle %s failed (%d)" % (what, rc))
    return rc


def layout(d: int):
    n = d * d
    t = np.zeros(n - 1, np.int32)
    s = np.zeros((n - 1, 4), np.int32)
    _chk(_load().orc_layout(d, _p(t), _p(s)), "layout")
    return t, s


def syndromes(d: int, errors: np.ndarray):
    e = np.ascontiguousarray(errors, np.uint8)
    b = e.shape[0]
    s = np.zeros((b, d * d - 1), np.uint8)
    c = np.zeros(b, np.uint8)
    _chk(_load().orc_syndrome(d, _p(e), b, _p(s), _p(c)), "syndrome")
    return s, c


def pure_error(d: int, j: int) -> np.ndarray:
    out = np.zeros(d * d, np.uint8)
    _chk(_load().orc_pure_error(d, j, _p(out)), "pure_error")
    return out


def _rates1(rates, n):
    r = np.ascontiguousarray(rates, np.float64)
    if r.shape != (n, 3):
        raise ValueError("rates must be [n,3]")
    return r


def enumerate_table(d: int, rates, marginals: bool = False):
    """O1: Z[s_index, l] for all 2^m syndromes (s_index = sum s_j 2^j)."""
    n, m = d * d, d * d - 1
    r = _rates1(rates, n)
    t = np.zeros((1 << m, 4), np.float64)
    mg = np.zeros((1 << m, n, 4), np.float64) if marginals else None
    _chk(_load().orc_enumerate(d, _p(r), _p(t), _p(mg) if marginals else None), "enumerate")
    return (t, mg) if marginals else t


def generator_sum(d: int, rates, syndrome) -> np.ndarray:
    """O2: Z_l(s), linear scale."""
    r = _rates1(rates, d * d)
    s = np.ascontiguousarray(syndrome, np.uint8)
    z = np.zeros(4, np.float64)
    _chk(_load().orc_generator_sum(d, _p(r), _p(s), _p(z)), "generator_sum")
    return z


def transfer_w(d: int, weights, syndrome) -> np.ndarray:
    """O3 with an explicit [n,4] per-qubit weight table; returns logZ[4]."""
    w = np.ascontiguousarray(weights, np.float64)
    s = np.ascontiguousarray(syndrome, np.uint8)
    z = np.zeros(4, np.float64)
    _chk(_load().orc_transfer_w(d, _p(w), _p(s), _p(z)), "transfer_w")
    return z


def transfer(d: int, rates, syndromes, model_index=None, threads: int = 0) -> np.ndarray:
    """O3 batched: rates [n,3] or [M,n,3], syndromes [B,m] -> logZ [B,4]."""
    r = np.ascontiguousarray(rates, np.float64)
    if r.ndim == 2:
        r = r[None]
    s = np.ascontiguousarray(syndromes, np.uint8)
    if s.ndim == 1:
        s = s[None]
    b = s.shape[0]
    mi = None if model_index is None else np.ascontiguousarray(model_index, np.int32)
    out = np.zeros((b, 4), np.float64)
    _chk(_load().orc_transfer(d, _p(r), r.shape[0], _p(mi) if mi is not None else None, _p(s), b,
                              _p(out), int(threads)), "transfer")
    return out


def max_slots(d: int) -> int:
    return _chk(_load().orc_max_slots(d), "max_slots")


def rbim(d: int, p: float, syndrome) -> np.ndarray:
    """O4: logZ[4] for bit-flip noise with rate p."""
    s = np.ascontiguousarray(syndrome, np.uint8)
    z = np.zeros(4, np.float64)
    _chk(_load().orc_rbim(d, float(p), _p(s), _p(z)), "rbim")
    return z


def grad_logp(d: int, rates, syndrome):
    """O5: (grad [n,3] = d log P(s) / d log p_{q,P}, log P(s))."""
    r = _rates1(rates, d * d)
    s = np.ascontiguousarray(syndrome, np.uint8)
    g = np.zeros((d * d, 3), np.float64)
    lp = np.zeros(1, np.float64)
    _chk(_load().orc_grad_logp(d, _p(r), _p(s), _p(g), _p(lp)), "grad_logp")
    return g, float(lp[0])


def decide(logz, tie_tol: float = 1e-9):
    """(log P(s), class) with the tie rule: smallest l within tau of the max."""
    z = np.ascontiguousarray(logz, np.float64).reshape(-1, 4)
    b = z.shape[0]
    lp = np.zeros(b, np.float64)
    c = np.zeros(b, np.uint8)
    _load().orc_decide(_p(z), b, float(tie_tol), _p(lp), _p(c))
    return lp, c


def _phen_inputs(d, rounds, rates, meas, syndromes):
    n, m = d * d, d * d - 1
    r = _rates1(rates, n)
    q = np.ascontiguousarray(meas, np.float64)
    if q.shape != (m,):
        raise ValueError("meas must be [m]")
    s = np.ascontiguousarray(syndromes, np.uint8)
    if s.ndim == 2:
        s = s[None]
    if s.shape[1:] != (rounds, m):
        raise ValueError("syndromes must be [B, T, m]")
    return r, q, s


def phen_enum2(d: int, rates, meas, syndromes) -> np.ndarray:
    """O6: logZ [B,4] under phenomenological noise with T = 2 rounds (d = 3);
    syndromes [B, 2, m] (round 1 noisy, round 2 perfect), meas [m]."""
    r, q, s = _phen_inputs(d, 2, rates, meas, syndromes)
    out = np.zeros((s.shape[0], 4), np.float64)
    _chk(_load().orc_phen_enum2(d, _p(r), _p(q), _p(s), s.shape[0], _p(out)), "phen_enum2")
    return out


def phen_transfer(d: int, rounds: int, rates, meas, syndromes, threads: int = 0) -> np.ndarray:
    """O7: logZ [B,4] under phenomenological noise with T rounds; syndromes
    [B, T, m] (rounds 1..T-1 noisy, round T perfect), meas [m]."""
    r, q, s = _phen_inputs(d, rounds, rates, meas, syndromes)
    out = np.zeros((s.shape[0], 4), np.float64)
    _chk(_load().orc_phen_transfer(d, int(rounds), _p(r), _p(q), _p(s), s.shape[0], _p(out), int(threads)),
         "phen_transfer")
    return out


def phen_state_bits(d: int, rounds: int) -> int:
    """log2 of the O7 state size (its cost is 4^T times that per qubit)."""
    return _chk(_load().orc_phen_max_bits(d, int(rounds)), "phen_max_bits")
