"""Seeded synthetic inputs for boundary-MPS coset decoding.

This module only draws inputs: per-qubit Pauli rates for the noise models the
paper lists for code capacity (bit-flip, phase-flip, depolarizing; Sec. 2.2
"Noise models"), plus the biased and inhomogeneous families used by the
workloads, and i.i.d. Pauli errors on the rotated surface code (Sec. 2.1) with
their syndromes.  It performs none of the decoding arithmetic (no coset sums,
no tensor contraction).  Both the FP64 oracle and the GPU path consume what it
returns; neither is imported here.

Conventions (shared by every independent implementation in this repository):
  * qubit q = r*d + c, 0 <= r, c < d;
  * Pauli code 0=I, 1=X, 2=Y, 3=Z; x-bit set for X and Y, z-bit for Y and Z;
  * checks sit at corners (r, c) in [-1, d-1]^2 and cover the existing qubits of
    (r,c), (r,c+1), (r+1,c), (r+1,c+1); X-type iff r+c is even; bulk corners
    0 <= r,c <= d-2, X-type boundary checks on the top/bottom rows, Z-type on
    the left/right columns;
  * syndrome order: all Z-type checks, then all X-type, each sorted by corner;
    a Z-type check fires on odd x-parity of its support, an X-type on z-parity;
  * logical label of an error: (x-parity on row 0, z-parity on column 0),
    class index I=(0,0)->0, X=(1,0)->1, Y=(1,1)->2, Z=(0,1)->3.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "code_checks", "depolarizing", "bitflip", "phaseflip", "biased",
    "inhomogeneous", "sample_errors", "syndromes_of", "classes_of", "sample",
    "sample_phenom", "CONFIGS", "config_inputs",
]


def code_checks(d: int):
    """Return (types, supports) for the rotated d x d patch.

    types: int8 [m], 0 = X-type, 1 = Z-type.  supports: int32 [m, 4], -1 pad.
    """
    if d < 3 or d % 2 == 0:
        raise ValueError("d must be odd and >= 3")
    rows = {0: [], 1: []}  # keyed by type: 1 = Z first in the syndrome order
    for r in range(-1, d):
        for c in range(-1, d):
            is_x = ((r + c) & 1) == 0
            bulk = 0 <= r <= d - 2 and 0 <= c <= d - 2
            tb = (r == -1 or r == d - 1) and is_x and 0 <= c <= d - 2
            lr = (c == -1 or c == d - 1) and not is_x and 0 <= r <= d - 2
            if not (bulk or tb or lr):
                continue
            sup = [rr * d + cc for rr in (r, r + 1) for cc in (c, c + 1)
                   if 0 <= rr < d and 0 <= cc < d]
            rows[0 if is_x else 1].append(sup + [-1] * (4 - len(sup)))
    types = np.array([1] * len(rows[1]) + [0] * len(rows[0]), dtype=np.int8)
    supports = np.array(rows[1] + rows[0], dtype=np.int32)
    return types, supports


# ----------------------------------------------------------------- noise models
def depolarizing(d: int, p: float) -> np.ndarray:
    """Rates [n,3] = (p_X, p_Y, p_Z), each p/3."""
    return np.full((d * d, 3), p / 3.0, dtype=np.float64)


def bitflip(d: int, p: float) -> np.ndarray:
    r = np.zeros((d * d, 3), dtype=np.float64)
    r[:, 0] = p
    return r


def phaseflip(d: int, p: float) -> np.ndarray:
    r = np.zeros((d * d, 3), dtype=np.float64)
    r[:, 2] = p
    return r


def biased(d: int, p: float, eta: float) -> np.ndarray:
    """Z-biased Pauli noise with eta = p_Z / p_X and p_X = p_Y."""
    r = np.empty((d * d, 3), dtype=np.float64)
    r[:, 0] = r[:, 1] = p / (eta + 2.0)
    r[:, 2] = eta * p / (eta + 2.0)
    return r


def inhomogeneous(d: int, lo: float, hi: float, seed: int) -> np.ndarray:
    """Independent per-qubit, per-Pauli rates, log-uniform in [lo, hi]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random((d * d, 3))
    return np.exp(np.log(lo) + u * (np.log(hi) - np.log(lo)))


# ----------------------------------------------------------------- sampling
def sample_errors(rates: np.ndarray, count: int, seed: int,
                  model_index: np.ndarray | None = None) -> np.ndarray:
    """Draw i.i.d. Pauli errors by inverse CDF.  rates: [n,3] or [M,n,3]."""
    rates = np.asarray(rates, dtype=np.float64)
    if rates.ndim == 2:
        rates = rates[None]
    m_count, n, _ = rates.shape
    if model_index is None:
        model_index = np.zeros(count, dtype=np.int32)
    rng = np.random.Generator(np.random.PCG64(seed))
    u = rng.random((count, n))
    cum = np.cumsum(np.concatenate([1.0 - rates.sum(-1, keepdims=True), rates], -1), -1)
    cum = cum[model_index]  # [count, n, 4]
    err = (u[..., None] >= cum[..., :3]).sum(-1).astype(np.uint8)
    return err


def syndromes_of(d: int, errors: np.ndarray) -> np.ndarray:
    types, supports = code_checks(d)
    errors = np.asarray(errors, dtype=np.uint8)
    xbit = ((errors == 1) | (errors == 2)).astype(np.uint8)
    zbit = ((errors == 2) | (errors == 3)).astype(np.uint8)
    pad = np.zeros((errors.shape[0], 1), dtype=np.uint8)
    xb = np.concatenate([xbit, pad], 1)
    zb = np.concatenate([zbit, pad], 1)
    sup = np.where(supports < 0, d * d, supports)
    sx = np.bitwise_xor.reduce(xb[:, sup], axis=2)
    sz = np.bitwise_xor.reduce(zb[:, sup], axis=2)
    return np.where(types[None, :] == 1, sx, sz).astype(np.uint8)


def classes_of(d: int, errors: np.ndarray) -> np.ndarray:
    errors = np.asarray(errors, dtype=np.uint8)
    xbit = ((errors == 1) | (errors == 2)).astype(np.uint8)
    zbit = ((errors == 2) | (errors == 3)).astype(np.uint8)
    a = np.bitwise_xor.reduce(xbit[:, :d], axis=1)          # row 0
    b = np.bitwise_xor.reduce(zbit[:, ::d], axis=1)         # column 0
    lut = np.array([[0, 3], [1, 2]], dtype=np.uint8)
    return lut[a, b]


def sample(d: int, rates: np.ndarray, count: int, seed: int,
           model_index: np.ndarray | None = None):
    """Return dict(errors, syndromes, true_class, model_index, rates)."""
    rates = np.asarray(rates, dtype=np.float64)
    if rates.ndim == 2:
        rates = rates[None]
    if model_index is None:
        model_index = np.zeros(count, dtype=np.int32)
    err = sample_errors(rates, count, seed, model_index)
    return dict(errors=err, syndromes=syndromes_of(d, err), true_class=classes_of(d, err),
                model_index=np.ascontiguousarray(model_index, dtype=np.int32),
                rates=np.ascontiguousarray(rates))


def _pauli_xor(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Product of Pauli codes (phases dropped) as codes."""
    lut = np.array([[0, 1, 2, 3], [1, 0, 3, 2], [2, 3, 0, 1], [3, 2, 1, 0]], dtype=np.uint8)
    return lut[a, b]


def sample_phenom(d: int, rates: np.ndarray, meas: np.ndarray, rounds: int, count: int, seed: int):
    """Phenomenological noise (repeated noisy syndrome rounds): before each of
    the T rounds every qubit draws a Pauli with the code-capacity rates; rounds
    1..T-1 report the syndrome of the accumulated error with each check flipped
    independently with probability meas[j]; round T is perfect.  Returns
    dict(syndromes [B, T, m], true_class [B] of the accumulated error,
    errors [B, T, n] per round, flips [B, T-1, m])."""
    rates = np.asarray(rates, dtype=np.float64)
    meas = np.asarray(meas, dtype=np.float64)
    n, m = d * d, d * d - 1
    rng = np.random.Generator(np.random.PCG64(seed))
    cum = np.cumsum(np.concatenate([1.0 - rates.sum(-1, keepdims=True), rates], -1), -1)  # [n, 4]
    u = rng.random((count, rounds, n))
    err = (u[..., None] >= cum[None, None, :, :3]).sum(-1).astype(np.uint8)
    flips = (rng.random((count, max(rounds - 1, 0), m)) < meas[None, None, :]).astype(np.uint8)
    syn = np.zeros((count, rounds, m), np.uint8)
    acc = np.zeros((count, n), np.uint8)
    for t in range(rounds):
        acc = _pauli_xor(acc, err[:, t])
        syn[:, t] = syndromes_of(d, acc)
        if t < rounds - 1:
            syn[:, t] ^= flips[:, t]
    return dict(syndromes=syn, true_class=classes_of(d, acc), errors=err, flips=flips)


# ----------------------------------------------------------------- workloads
CONFIGS = {
    "C1": dict(d=3, p=0.10, count=1024, seed=0, chi=0, precision="fp64"),
    "C2": dict(d=9, ps=(0.05, 0.08, 0.11, 0.14, 0.17), count=65536, seed=2000,
               chi=16, precision="fp32"),
    "C3": dict(d=17, p=0.12, count=16384, seed=3000, chi=32, precision="bf16"),
    "C4": dict(ds=(5, 7, 9, 11, 13, 15), counts=(32768, 16384, 8192, 4096, 2048, 1024),
               chis=(8, 12, 16, 20, 24, 28), p=0.08, etas=(1.0, 10.0, 100.0), seed=4000),
    "C5": dict(d=11, lo=1e-3, hi=5e-2, rate_seed=5000, count=8192, seed=5001, chi=24,
               precision="fp32"),
}


def config_inputs(name: str, scale: float = 1.0):
    """Inputs of a named workload as a list of segments (dicts).

    scale < 1 keeps the first fraction of each segment's syndromes (same seeds,
    so a scaled run is a prefix of the full one).
    """
    cfg = CONFIGS[name]
    segs = []

    def take(n):
        return max(1, int(round(n * scale)))

    if name in ("C1", "C3"):
        r = depolarizing(cfg["d"], cfg["p"])
        s = sample(cfg["d"], r, take(cfg["count"]), cfg["seed"])
        segs.append(dict(d=cfg["d"], chi=cfg["chi"], **s))
    elif name == "C2":
        for i, p in enumerate(cfg["ps"]):
            r = depolarizing(cfg["d"], p)
            s = sample(cfg["d"], r, take(cfg["count"]), cfg["seed"] + i)
            segs.append(dict(d=cfg["d"], chi=cfg["chi"], p=p, **s))
    elif name == "C4":
        for d, n, chi in zip(cfg["ds"], cfg["counts"], cfg["chis"]):
            r = np.stack([biased(d, cfg["p"], eta) for eta in cfg["etas"]])
            n = take(n)
            mi = (np.arange(n) % len(cfg["etas"])).astype(np.int32)
            s = sample(d, r, n, cfg["seed"] + d, mi)
            segs.append(dict(d=d, chi=chi, **s))
    elif name == "C5":
        r = inhomogeneous(cfg["d"], cfg["lo"], cfg["hi"], cfg["rate_seed"])
        s = sample(cfg["d"], r, take(cfg["count"]), cfg["seed"])
        segs.append(dict(d=cfg["d"], chi=cfg["chi"], **s))
    else:
        raise KeyError(name)
    return segs
