"""Autotuner for the launch shape of the boundary-MPS kernels.

For each (d, chi, precision) bucket it times every valid candidate
(columns per MPS site in {1, 2}) x (work-group size 512 or 256 threads) x
(persistent work-groups per CU: 1 or 2 for 512 threads, 2 to 4 for 256) on a
seeded sample batch and keeps the fastest.  A candidate the library cannot
run (the 256-thread build needs the plan to fit it) is skipped: the launch
shape is read back after it is set.  Results live in a JSON cache
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
                set_tuning(int(d), int(chi), prec, int(v["group"]), int(v["wg_per_cu"]), int(v.get("threads", 0)))
            except Exception:
                pass
    return cache


def default_count(d: int) -> int:
    """Syndromes per timing: enough persistent items to fill every CU."""
    return 16384 if d <= 7 else 8192 if d <= 11 else 4096 if d <= 15 else 2048


def tune_bucket(d: int, chi: int, prec: str, count: int = 0, p: float = 0.12, seed: int = 7, reps: int = 2):
    import torch

    import synth
    from .api import decode, launch_shape, set_tuning
    count = count or default_count(d)
    rates = synth.depolarizing(d, p)
    smp = synth.sample(d, rates, count, seed)
    dev = torch.device("cuda:0")
    syn = torch.from_numpy(smp["syndromes"]).to(dev)
    rt = torch.from_numpy(rates).to(dev)
    results = []
    for g in (1, 2):
        for threads, wgs in ((512, (1, 2)), (256, (2, 3, 4))):
            for w in wgs:
                try:
                    set_tuning(d, chi, prec, g, w, threads)
                    shape = launch_shape(d, chi, prec)
                except Exception:
                    continue
                if shape[0] != g or shape[2] != threads or shape[1] != w:
                    continue
                decode(syn[: min(64, count)], rt, d, chi, prec)
                torch.cuda.synchronize()
                best = None
                for _ in range(reps):
                    t0 = time.time()
                    decode(syn, rt, d, chi, prec)
                    torch.cuda.synchronize()
                    dt = time.time() - t0
                    best = dt if best is None else min(best, dt)
                results.append(dict(group=g, threads=threads, wg_per_cu=w, seconds=best, syndromes_per_s=count / best))
                print("tune d=%d chi=%d %s group=%d threads=%d wg/cu=%d: %.1f syn/s"
                      % (d, chi, prec, g, threads, w, count / best), flush=True)
    set_tuning(d, chi, prec, 0, 0, 0)
    if not results:
        return None
    best = max(results, key=lambda r: r["syndromes_per_s"])
    return dict(best=best, candidates=results)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--bucket", action="append", required=True, help="d:chi:precision")
    ap.add_argument("--count", type=int, default=0, help="syndromes per timing (0: by distance)")
    ap.add_argument("--out", default=None)
    ap.add_argument("--fresh", action="store_true", help="start a new cache instead of updating the file")
    a = ap.parse_args()
    path = a.out or cache_path()
    cache = {"entries": {}, "device": None}
    if os.path.exists(path) and not a.fresh:
        with open(path) as f:
            cache = json.load(f)
    import torch
    props = torch.cuda.get_device_properties(0)
    cache["device"] = "%s (%s, %d CUs)" % (props.name, props.gcnArchName, props.multi_processor_count)
    for b in a.bucket:
        d, chi, prec = b.split(":")
        r = tune_bucket(int(d), int(chi), prec, a.count)
        if r:
            cache["entries"][b] = dict(group=r["best"]["group"], wg_per_cu=r["best"]["wg_per_cu"],
                                       threads=r["best"]["threads"], syndromes_per_s=r["best"]["syndromes_per_s"],
                                       candidates=r["candidates"])
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    print("wrote", path)


if __name__ == "__main__":
    main()
