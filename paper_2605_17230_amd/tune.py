"""Autotuner for the launch shape of the boundary-MPS kernels.

For each (d, chi, precision) bucket it times every valid candidate
(columns per MPS site in {1, 2}) x (persistent work-groups per CU in {1, 2})
on a seeded sample batch and keeps the fastest.  Results live in a JSON cache
(``tune_cache.json`` beside this file, or $TNMLD_TUNE_CACHE) that the package
applies at import through ``tn_set_tuning``.

    python -m paper_2605_17230_amd.tune --bucket 17:32:fp32plain --bucket 9:16:fp32
"""
from __future__ import annotations

import argparse
import json
import os
import time

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "tune_cache.json")


def cache_path():
    return os.environ.get("TNMLD_TUNE_CACHE", DEFAULT_CACHE)


def load(apply: bool = True) -> dict:
    """Read the cache and push every entry into the library."""
    path = cache_path()
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        cache = json.load(f)
    if apply:
        from .api import set_tuning
        for key, v in cache.get("entries", {}).items():
            d, chi, prec = key.split(":")
            try:
                set_tuning(int(d), int(chi), prec, int(v["group"]), int(v["wg_per_cu"]))
            except Exception:
                pass
    return cache


def tune_bucket(d: int, chi: int, prec: str, count: int = 512, p: float = 0.12, seed: int = 7):
    import torch

    import synth
    from .api import decode, plan_info, set_tuning
    rates = synth.depolarizing(d, p)
    smp = synth.sample(d, rates, count, seed)
    dev = torch.device("cuda:0")
    syn = torch.from_numpy(smp["syndromes"]).to(dev)
    rt = torch.from_numpy(rates).to(dev)
    results = []
    for g in (1, 2):
        for w in (1, 2):
            try:
                set_tuning(d, chi, prec, g, w)
                info = plan_info(d, chi, prec)
            except Exception:
                continue
            if info["group"] != g or info["wg_per_cu"] != w:
                continue
            decode(syn[: min(64, count)], rt, d, chi, prec)
            torch.cuda.synchronize()
            t0 = time.time()
            decode(syn, rt, d, chi, prec)
            torch.cuda.synchronize()
            dt = time.time() - t0
            results.append(dict(group=g, wg_per_cu=w, seconds=dt, syndromes_per_s=count / dt))
            print("tune d=%d chi=%d %s group=%d wg/cu=%d: %.1f syn/s" % (d, chi, prec, g, w, count / dt),
                  flush=True)
    set_tuning(d, chi, prec, 0, 0)
    if not results:
        return None
    best = max(results, key=lambda r: r["syndromes_per_s"])
    return dict(best=best, candidates=results)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--bucket", action="append", required=True, help="d:chi:precision")
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--out", default=None)
    a = ap.parse_args()
    path = a.out or cache_path()
    cache = {"entries": {}, "device": None}
    if os.path.exists(path):
        with open(path) as f:
            cache = json.load(f)
    import torch
    cache["device"] = torch.cuda.get_device_name(0)
    for b in a.bucket:
        d, chi, prec = b.split(":")
        r = tune_bucket(int(d), int(chi), prec, a.count)
        if r:
            cache["entries"][b] = dict(group=r["best"]["group"], wg_per_cu=r["best"]["wg_per_cu"],
                                       syndromes_per_s=r["best"]["syndromes_per_s"], candidates=r["candidates"])
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    print("wrote", path)


if __name__ == "__main__":
    main()
