"""Throughput of batched boundary-MPS coset decoding on one MI355X.

Workload: rotated surface code d = 17 under depolarizing noise p = 0.12,
16,384 seeded synthetic syndromes, bond dimension chi = 32, four cosets per
syndrome.  One step = decode the whole batch (every row MPO, LQ sweep and
truncation sweep of all 65,536 contractions, then the per-syndrome decision),
inputs already resident in HBM.  Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--precision fp32plain|fp32|fp64]
                  [--compare fp32plain] [--cpu-seconds S] [--no-cpu]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

D, CHI, P, COUNT, SEED = 17, 32, 0.12, 16384, 3000
PEAK_ALU_TFLOPS = 78.6  # MI355X: 256 CU x 4 SIMD x 16 lanes x 2 flop x 2.4 GHz (FP64 / non-packed FP32 FMA)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default="fp32plain")
    ap.add_argument("--compare", default="")
    ap.add_argument("--count", type=int, default=COUNT)
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy (reference kernel for HBM byte counters)")
    return ap.parse_args()


def copy_calibration():
    """A plain copy of known size: 1 GiB read + 1 GiB written, for scaling the
    FETCH_SIZE / WRITE_SIZE counters of the decoding kernel."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4}), flush=True)


def cpu_baseline(syn, rates, target_s):
    """FP64 oracle (exact transfer-matrix contraction) on a bounded prefix."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n = max(threads, 1)
    t0 = time.time()
    ref = oracle.transfer(D, rates, syn[:n], threads=threads)
    dt = time.time() - t0
    per = dt / n * threads  # seconds per syndrome per thread
    more = int(max(0, target_s - dt) / max(per, 1e-9) * threads) // threads * threads
    if more > 0:
        t1 = time.time()
        ref2 = oracle.transfer(D, rates, syn[n:n + more], threads=threads)
        dt += time.time() - t1
        ref = np.concatenate([ref, ref2])
        n += more
    return ref, n, dt, threads


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(syndromes would shard across GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)
    if a.copy_calibration:
        copy_calibration()
        return
    import torch

    import paper_2605_17230_amd as tn
    import synth

    dev = torch.device("cuda:0")
    rates = synth.depolarizing(D, P)
    smp = synth.sample(D, rates, a.count, SEED)
    syn_h = smp["syndromes"]
    syn = torch.from_numpy(syn_h).to(dev)
    rt = torch.from_numpy(rates).to(dev)
    info = tn.plan_info(D, CHI, a.precision)
    flops_per_step = 4.0 * a.count * info["flops"]
    stream = torch.cuda.current_stream(dev)

    def step(prec):
        return tn.decode(syn, rt, D, CHI, prec)

    print("bench: d=%d chi=%d %s, %d syndromes, %d warmup + %d timed steps"
          % (D, CHI, a.precision, a.count, a.warmup, a.steps), file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        step(a.precision)
    torch.cuda.synchronize()
    ev = []
    t0 = time.time()
    for i in range(a.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        logz, logp, cls = step(a.precision)
        e1.record(stream)
        ev.append((e0, e1))
        print("bench: step %d enqueued" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.time() - t0
    ms = [e0.elapsed_time(e1) for e0, e1 in ev]
    ms_step = float(np.mean(ms))
    value = a.count / (ms_step / 1e3)
    achieved = flops_per_step / (ms_step / 1e3) / 1e12
    out = {
        "metric": "syndromes/s at d=17 chi=32 (boundary-MPS coset decoding)",
        "value": value,
        "unit": "syndromes/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32plain": "f32", "fp32": "f32+f64", "fp64": "f64", "bf16": "bf16+f64"}[a.precision],
        "data": "synthetic",
        "config": {"workload": "rotated surface code d=17, depolarizing p=0.12, 16384 seeded syndromes, chi=32",
                   "d": D, "chi": CHI, "p": P, "syndromes": a.count, "cosets": 4, "precision": a.precision},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_ALU_TFLOPS, "traffic": None,
                     "flops_per_launch": flops_per_step, "kernel": "fwd_kernel"},
        "wall_s": wall,
    }
    logz_h = logz.cpu().numpy()
    cls_h = cls.cpu().numpy()
    if a.compare:
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lz2, _, c2 = step(a.compare)
        e1.record(stream)
        torch.cuda.synchronize()
        ms2 = e0.elapsed_time(e1)
        out["compare"] = {"precision": a.compare, "value": a.count / (ms2 / 1e3), "ms_per_step": ms2,
                          "speedup": ms2 / ms_step,
                          "max_abs_dlogz_vs_primary": float(np.max(np.abs(lz2.cpu().numpy() - logz_h))),
                          "class_agreement": float((c2.cpu().numpy() == cls_h).mean())}
    if not a.no_cpu:
        import oracle
        ref, n, dt, threads = cpu_baseline(syn_h, rates, a.cpu_seconds)
        _, rcls = oracle.decide(ref)
        err = np.abs(logz_h[:n] - ref)
        out["cpu_baseline"] = {"value": n / dt, "unit": "syndromes/s", "cores": threads, "kind": "oracle",
                               "sample": "first %d syndromes of the batch, exact FP64 transfer-matrix "
                                         "contraction (4 cosets each), %.1f s" % (n, dt)}
        out["parity_vs_oracle"] = {"syndromes": n, "max_abs_dlogz": float(err.max()),
                                   "max_abs_dlogp": float(np.max(np.abs(
                                       np.logaddexp.reduce(logz_h[:n], 1) - np.logaddexp.reduce(ref, 1)))),
                                   "class_agreement": float((cls_h[:n] == rcls).mean())}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
