"""Throughput of batched boundary-MPS coset decoding on one MI355X.

Default workload: rotated surface code d = 17 under depolarizing noise
p = 0.12, 16,384 seeded synthetic syndromes, bond dimension chi = 32, four
cosets per syndrome.  One step = decode the whole batch (row MPOs, LQ sweeps
and truncation sweeps of all 65,536 contractions, then the per-syndrome
decision) with inputs already resident in HBM.  The timed form is the BF16
form (bf16 MFMA contractions, FP32 factorisations); the plain FP32 form is
timed once beside it, and both are compared with the FP64 form on a sample.
Prints one JSON line.

  python bench.py [--steps K] [--warmup W] [--precision bf16|fp32plain|fp32|fp64]
                  [--compare fp32plain] [--workload c2|c3|c4|c5|fit|study|planar]
                  [--cpu-seconds S] [--cpu-min N] [--no-cpu]

--workload c2 decodes the d = 9 p-sweep (five noise levels, 65,536 syndromes
each) in one call in the plain FP32 form and reports the logical error rate
per p; c4 decodes the mixed batch (distances 5..15) in one call; c5 times the
adjoint (forward + backward) on the gradient workload (d = 11, per-qubit
log-uniform rates, 8,192 syndromes, chi = 24, FP32 unless --precision says
otherwise); fit runs the noise-model fit; study the logical-error and chi
sweeps; planar the exact bit-flip solver at d = 17.
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
# MI355X non-packed VALU peak: 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz;
# FP64 runs at the same rate.
PEAK_ALU_TFLOPS = 78.6
PEAK_MFMA_BF16_TFLOPS = 2500.0  # dense bf16 matrix peak of the MI355X


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", default=None,
                    help="form timed (default: bf16; fp32plain for c2, as that workload names; fp32 for c5 and fit)")
    ap.add_argument("--compare", default="fp32plain", help="second form timed once ('' to skip)")
    ap.add_argument("--workload", default="c3", choices=["c2", "c3", "c4", "c5", "fit", "study", "planar", "rounds"])
    ap.add_argument("--study-count", type=int, default=4096, help="syndromes per (d, p) point of the study")
    ap.add_argument("--fit-steps", type=int, default=60, help="Adam steps of the fit workload")
    ap.add_argument("--fit-batch", type=int, default=1024, help="syndromes per step of the fit workload")
    ap.add_argument("--fit-ns", default="1024,2048,4096,8192", help="data sizes N of the fit workload")
    ap.add_argument("--count", type=int, default=COUNT)
    ap.add_argument("--fp64-sample", type=int, default=16384,
                    help="syndromes decoded in FP64 at the same chi for the precision-error report (0: none)")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--cpu-min", type=int, default=256, help="fewest syndromes the oracle baseline times")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device-to-device copy (reference kernel for HBM byte counters)")
    a = ap.parse_args()
    if a.precision is None:
        a.precision = {"c2": "fp32plain", "c5": "fp32", "fit": "fp32"}.get(a.workload, "bf16")
    return a


def copy_calibration():
    """A plain copy of known size: 1 GiB read + 1 GiB written, for scaling the
    FETCH_SIZE / WRITE_SIZE counters of the decoding kernel."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4}), flush=True)


def environment():
    """Hardware and software the line was measured on."""
    import platform
    import torch
    cpu = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    props = torch.cuda.get_device_properties(0)
    return {"gpu": "%s (%s, %d CUs)" % (props.name, props.gcnArchName, props.multi_processor_count),
            "rocm_hip": torch.version.hip, "torch": torch.__version__,
            "cpu": cpu, "nproc": os.cpu_count(),
            "omp_threads": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))}


def cpu_baseline(d, rates, syn, target_s, min_count=256):
    """FP64 oracle (exact transfer-matrix contraction) on a bounded prefix of
    at least min_count syndromes (more while under target_s seconds)."""
    import oracle
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    n = max(threads, min(min_count, len(syn)))
    t0 = time.time()
    ref = oracle.transfer(d, rates, syn[:n], threads=threads)
    dt = time.time() - t0
    per = dt / n * threads  # seconds per syndrome per thread
    more = int(max(0, target_s - dt) / max(per, 1e-9) * threads) // threads * threads
    more = min(more, len(syn) - n)
    if more > 0:
        t1 = time.time()
        ref2 = oracle.transfer(d, rates, syn[n:n + more], threads=threads)
        dt += time.time() - t1
        ref = np.concatenate([ref, ref2])
        n += more
    return ref, n, dt, threads


DTYPE = {"fp32plain": "f32", "fp32": "f32+f64", "fp64": "f64", "bf16": "bf16+f32", "bf16f64": "bf16+f64"}


def max_finite_diff(a, b):
    """Largest |a - b| over the cosets finite in both (lists of [B, 4] arrays);
    cosets -inf in one form only are counted separately by the caller."""
    m = 0.0
    for x, y in zip(a, b):
        both = np.isfinite(x) & np.isfinite(y)
        if both.any():
            m = max(m, float(np.max(np.abs(x[both] - y[both]))))
    return m


# Sources the boundary-MPS kernels (fwd_kernel, its two 256-thread builds, bwd_kernel)
# are compiled from; the planar solver's files are not among them.
FWD_SOURCES = ("adjoint.hpp", "contract.hpp", "plan.cpp", "plan.hpp", "sweep.hpp", "tnmld.hip", "tnmld_small.hip",
               "tnmld_small3.hip")


def kernel_name(shape):
    """Forward kernel a launch shape (columns per site, groups per CU, threads) runs."""
    if shape[2] != 256:
        return "fwd_kernel"
    return "fwd_kernel_small3" if shape[1] >= 3 else "fwd_kernel_small"


def kernel_sources_sha256():
    """sha256 over the names and contents of the boundary-MPS kernel sources
    and the C header, in sorted order."""
    import hashlib
    h = hashlib.sha256()
    files = [os.path.join(ROOT, "paper_2605_17230_amd", "csrc", f) for f in FWD_SOURCES]
    files.append(os.path.join(ROOT, "include", "tnmld.h"))
    for f in sorted(files, key=os.path.basename):
        h.update(os.path.basename(f).encode())
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(precision, count, workload):
    """HBM bytes per launch from the committed counter runs, only when they were
    taken on these exact kernel sources, precision and batch; else None."""
    import glob
    if workload != "c3":
        return None
    sha = kernel_sources_sha256()
    for f in glob.glob(os.path.join(ROOT, "profiles", "*_traffic.json")):
        with open(f) as fh:
            r = json.load(fh)
        if r.get("sources_sha256") == sha and r.get("precision") == precision and r.get("count") == count:
            return float(r["traffic_bytes_per_launch"])
    return None


def bench_adjoint(a, torch, tn, synth, dev, stream):
    """Forward + backward of sum_b log P(s_b) over the gradient workload."""
    s = synth.config_inputs("C5")[0]
    prec = "fp32" if a.precision in ("bf16", "bf16f64") else a.precision  # the adjoint's forms
    n = len(s["syndromes"])
    seg = tn.SegmentInput(s["d"], s["chi"], torch.from_numpy(s["syndromes"]).to(dev),
                          torch.from_numpy(s["rates"]).to(dev), None, prec)
    gw = torch.ones(n, dtype=torch.float64, device=dev)
    info = tn.plan_info(s["d"], s["chi"], prec)
    print("bench: adjoint d=%d chi=%d %s, %d syndromes" % (s["d"], s["chi"], prec, n), file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        tn.coset_loglik_backward([seg], [gw])
    torch.cuda.synchronize()
    ev = []
    for i in range(a.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        _, grads = tn.coset_loglik_backward([seg], [gw])
        e1.record(stream)
        ev.append((e0, e1))
    torch.cuda.synchronize()
    ms_step = float(np.mean([e0.elapsed_time(e1) for e0, e1 in ev]))
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    tn.decode_segments([seg])
    e1.record(stream)
    torch.cuda.synchronize()
    ms_fwd = e0.elapsed_time(e1)
    # counted work: the top-down sweep (one forward pass as executed: shared
    # rows once per syndrome), the transposed bottom-up sweep of every coset and
    # its row environments (tn_plan_adjoint_flops)
    flops = n * info["adjoint_flops_syndrome"]
    achieved = flops / (ms_step / 1e3) / 1e12
    g = grads[0].cpu().numpy()
    out = {
        "metric": "syndromes/s of the adjoint d sum log P(s) / d ln p at d=11 chi=24 (gradient workload)",
        "value": n / (ms_step / 1e3), "unit": "syndromes/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[prec], "data": "synthetic",
        "config": {"workload": "d=11, per-qubit log-uniform rates in [1e-3, 5e-2], %d syndromes, chi=24" % n,
                   "precision": prec, "parameters": int(g.size)},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_ALU_TFLOPS, "traffic": None, "flops_per_launch": flops,
                     "kernel": "bwd_kernel"},
        "counted_flops_per_syndrome": {"top_sweep": info["flops_syndrome"],
                                       "bottom_sweeps": 4.0 * info["bottom_sweep_flops"],
                                       "environments": 4.0 * info["environment_flops"]},
        "forward_only": {"ms": ms_fwd, "value": n / (ms_fwd / 1e3), "backward_over_forward": ms_step / ms_fwd},
        "grad_abs_sum": float(np.abs(g).sum()),
    }
    print(json.dumps(out), flush=True)


def bench_fit(a, torch, tn, synth, dev):
    """Noise-model fitting on the gradient workload: Adam on the per-qubit log
    rates from a uniform start, one forward + backward per step on a random
    mini-batch, with the first N of its syndromes for each N of --fit-ns.
    Reports the rate error against the generating rates per N and the logical
    error rate of decoding fresh syndromes of the same model with the true,
    the refitted (largest N) and the starting prior."""
    s = synth.config_inputs("C5")[0]
    prec = "fp32" if a.precision in ("bf16", "bf16f64") else a.precision  # the adjoint's forms
    d, chi = s["d"], s["chi"]
    syn_all = torch.from_numpy(s["syndromes"]).to(dev)
    true_rates = s["rates"][0]
    true = torch.from_numpy(np.log(true_rates)).to(dev)
    theta0 = torch.full_like(true, float(np.log(true_rates.mean())))
    ns = [int(x) for x in a.fit_ns.split(",")]
    print("bench: fit d=%d chi=%d %s, N in %s, %d steps" % (d, chi, prec, ns, a.fit_steps), file=sys.stderr,
          flush=True)
    tn.fit_log_rates(syn_all[:256], d, chi, theta0, steps=1, batch=256, precision=prec)  # warm-up
    torch.cuda.synchronize()

    def loss(th, syn):
        with torch.no_grad():
            return float(-tn.log_posterior(th, syn, d, chi, prec)[0].mean())

    per_n = {}
    theta_last, rate = None, None
    for n in ns:
        syn = syn_all[:n]
        batch = min(a.fit_batch, n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        theta, hist = tn.fit_log_rates(syn, d, chi, theta0, steps=a.fit_steps, lr=0.05, batch=batch, precision=prec)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        err = (theta - true).abs()
        per_n[str(n)] = {"mean_abs_log_rate_error": float(err.mean()), "median_abs_log_rate_error": float(err.median()),
                         "loss_end": loss(theta, syn), "loss_true_rates": loss(true, syn), "seconds": dt}
        print("bench: fit N=%d done: mean |d ln p| %.3f" % (n, float(err.mean())), file=sys.stderr, flush=True)
        theta_last, rate = theta, a.fit_steps * batch / dt
    # logical error rate on fresh syndromes of the generating model
    test = synth.sample(d, true_rates, 8192, 5002)
    tsyn = torch.from_numpy(test["syndromes"]).to(dev)
    ler, held = {}, {}
    for name, th in (("true_prior", true), ("refit_prior_N=%d" % ns[-1], theta_last), ("start_prior", theta0)):
        _, lp, cls = tn.decode(tsyn, th.exp(), d, chi, prec)
        ler[name] = float((cls.cpu().numpy() != test["true_class"]).mean())
        held[name] = float(-lp.mean())
    out = {
        "metric": "syndromes/s through the noise fit (forward + adjoint + Adam step) at d=11 chi=24",
        "value": rate, "unit": "syndromes/s", "n_gpus": 1, "steps": a.fit_steps,
        "warmup": 1, "ms_per_step": per_n[str(ns[-1])]["seconds"] / a.fit_steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": DTYPE[prec], "data": "synthetic",
        "config": {"workload": "fit of 363 log rates to the first N syndromes of the d=11 gradient model, chi=24, "
                               "mini-batch %d, Adam lr 0.05, %d steps" % (a.fit_batch, a.fit_steps),
                   "precision": prec},
        "start": {"mean_abs_log_rate_error": float((theta0 - true).abs().mean())},
        "rate_error_vs_N": per_n,
        "logical_error_rate_fresh_8192": ler,
        "mean_neg_log_p_fresh_8192": held,
        "environment": environment(),
    }
    print(json.dumps(out), flush=True)


def bench_study(a, torch, tn, synth, dev):
    """Decoder sanity on the same kernels: logical error rate against p and d
    at chi = 32 (the curves should cross near the depolarizing MLD threshold,
    about 18.9 %, paper Sec. 3.1.2), and the truncation error against chi at
    d = 9 (FP64, relative to chi = 32)."""
    prec = a.precision
    ds, ps, n = (5, 9, 13, 17), (0.12, 0.15, 0.17, 0.19, 0.21, 0.23), a.study_count
    print("bench: study, %s, %d syndromes per point" % (prec, n), file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    table = {}
    for d in ds:
        row = {}
        for i, p in enumerate(ps):
            rates = synth.depolarizing(d, p)
            smp = synth.sample(d, rates, n, seed=6000 + 100 * d + i)
            _, _, cls = tn.decode(torch.from_numpy(smp["syndromes"]).to(dev), torch.from_numpy(rates).to(dev), d,
                                  32, prec)
            e = float((cls.cpu().numpy() != smp["true_class"]).mean())
            row["%.2f" % p] = {"ler": e, "stderr": float(np.sqrt(max(e * (1 - e), 1e-12) / n))}
        table["d=%d" % d] = row
        print("bench: d=%d done" % d, file=sys.stderr, flush=True)
    t_ler = time.perf_counter() - t0
    d, p, m = 9, 0.17, 1024
    rates = synth.depolarizing(d, p)
    smp = synth.sample(d, rates, m, seed=6900)
    syn, rt = torch.from_numpy(smp["syndromes"]).to(dev), torch.from_numpy(rates).to(dev)
    ref_logp = tn.decode(syn, rt, d, 32, "fp64")[1].cpu().numpy()
    conv = {}
    for chi in (2, 4, 8, 16):
        _, lp, cls = tn.decode(syn, rt, d, chi, "fp64")
        dl = np.abs(lp.cpu().numpy() - ref_logp)
        conv["chi=%d" % chi] = {"mean_abs_dlogp": float(dl.mean()), "max_abs_dlogp": float(dl.max()),
                                "ler": float((cls.cpu().numpy() != smp["true_class"]).mean())}
    out = {
        "metric": "logical error rate vs p and d (chi=32), truncation error vs chi at d=9",
        "value": sum(len(ps) * n for _ in ds) / t_ler, "unit": "syndromes/s", "n_gpus": 1, "steps": 1,
        "warmup": 0, "ms_per_step": t_ler * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE[prec], "data": "synthetic",
        "config": {"workload": "depolarizing p in %s, d in %s, %d syndromes per point, chi=32; chi sweep at d=9 "
                               "p=0.17 on %d syndromes" % (list(ps), list(ds), n, m), "precision": prec},
        "logical_error_rate": table,
        "chi_convergence_vs_chi32_fp64": conv,
    }
    print(json.dumps(out), flush=True)


PEAK_MFMA_FP64_TFLOPS = 78.6  # dense FP64 matrix peak of the MI355X (equal to the FP64 vector peak)


def bench_planar(a, torch, tn, synth, dev, stream):
    """Planar exact solver under bit-flip noise: d = 17, p = 0.10, 16,384
    seeded syndromes (two 580 x 580 complex LU factorisations per syndrome),
    against the boundary-MPS path on the same syndromes and the oracle."""
    import oracle
    d, p, n = 17, 0.10, a.count
    rates = synth.bitflip(d, p)
    smp = synth.sample(d, rates, n, 3100)
    syn, rt = torch.from_numpy(smp["syndromes"]).to(dev), torch.from_numpy(rates).to(dev)
    info = tn.bitflip_plan_info(d)
    print("bench: planar exact solver d=%d bit-flip p=%.2f, %d syndromes" % (d, p, n), file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        tn.decode_bitflip(syn, rt, d)
    torch.cuda.synchronize()
    ev = []
    for _ in range(a.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        lz, lp, cls = tn.decode_bitflip(syn, rt, d)
        e1.record(stream)
        ev.append((e0, e1))
    torch.cuda.synchronize()
    ms = float(np.mean([x.elapsed_time(y) for x, y in ev]))
    flops = 2.0 * n * info["lu_flops"]  # two cosets; complex LU, leading term (8/3) N^3
    ach = flops / (ms / 1e3) / 1e12
    lp = lp.cpu().numpy()
    cls = cls.cpu().numpy()
    out = {
        "metric": "syndromes/s of exact decoding under bit-flip noise at d=17 (planar Kac-Ward solver)",
        "value": n / (ms / 1e3), "unit": "syndromes/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "rotated surface code d=17, bit-flip p=0.10, %d seeded syndromes, exact" % n},
        "roofline": {"bound": "mfma", "achieved": ach, "peak": PEAK_MFMA_FP64_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach / PEAK_MFMA_FP64_TFLOPS, "traffic": None, "flops_per_launch": flops,
                     "kernel": "kw_kernel"},
        "logical_error_rate": float((cls != smp["true_class"]).mean()),
    }
    ns = min(512, n)
    with __import__("warnings").catch_warnings():
        __import__("warnings").simplefilter("ignore")
        _, mlp, mcls = tn.decode(syn[:ns], rt, d, 32, "bf16")
    out["vs_boundary_mps_bf16_chi32"] = {"syndromes": ns,
                                         "max_abs_dlogp": float(np.max(np.abs(mlp.cpu().numpy() - lp[:ns]))),
                                         "class_agreement": float((mcls.cpu().numpy() == cls[:ns]).mean())}
    if not a.no_cpu:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        k = max(threads, 1)
        t0 = time.time()
        ref = oracle.transfer(d, rates, smp["syndromes"][:k], threads=threads)
        dt = time.time() - t0
        out["cpu_baseline"] = {"value": k / dt, "unit": "syndromes/s", "cores": threads, "kind": "oracle",
                               "sample": "first %d syndromes, exact FP64 transfer-matrix contraction, %.1f s" % (k, dt)}
        out["parity_vs_oracle"] = {"syndromes": k, "max_abs_dlogp": float(np.max(np.abs(
            np.logaddexp.reduce(ref, 1) - lp[:k])))}
    print(json.dumps(out), flush=True)


def bench_rounds(a, torch, tn, synth, dev, stream):
    """Repeated noisy rounds (phenomenological noise): d = 7, T = 2 rounds
    (the first with measurement flips at q = 0.02, the last perfect),
    depolarizing p = 0.02 per round, 16,384 seeded histories, chi = 16 (12 in
    the FP64-factorisation forms); against the exact phenomenological oracle
    on a sample."""
    import oracle
    d, p, q, T, n = 7, 0.02, 0.02, 2, a.count
    chi = 12 if a.precision in ("fp64", "fp32", "bf16f64") else 16
    rates = synth.depolarizing(d, p)
    meas = np.full(d * d - 1, q)
    smp = synth.sample_phenom(d, rates, meas, T, n, 7000)
    syn, rt, mq = (torch.from_numpy(smp["syndromes"]).to(dev), torch.from_numpy(rates).to(dev),
                   torch.from_numpy(meas).to(dev))
    info = tn.plan_info(d, chi, a.precision, rounds=T)
    print("bench: two-round decoding d=%d T=%d p=q=%.2f chi=%d %s, %d histories" % (d, T, p, chi, a.precision, n),
          file=sys.stderr, flush=True)
    W = __import__("warnings")
    with W.catch_warnings():
        W.simplefilter("ignore", tn.api.UnresolvedCosetsWarning)
        for _ in range(a.warmup):
            tn.decode_rounds(syn, rt, mq, d, chi, a.precision)
        torch.cuda.synchronize()
        ev = []
        for _ in range(a.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            lz, lp, cls = tn.decode_rounds(syn, rt, mq, d, chi, a.precision)
            e1.record(stream)
            ev.append((e0, e1))
        torch.cuda.synchronize()
    ms = float(np.mean([x.elapsed_time(y) for x, y in ev]))
    flops = n * info["flops_syndrome"]
    ach = flops / (ms / 1e3) / 1e12
    lz, lp, cls = lz.cpu().numpy(), lp.cpu().numpy(), cls.cpu().numpy()
    out = {
        "metric": "histories/s of two-round (phenomenological) decoding at d=7",
        "value": n / (ms / 1e3), "unit": "histories/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": DTYPE[a.precision], "data": "synthetic",
        "config": {"workload": "rotated surface code d=7, 2 syndrome rounds (first with check flips q=0.02, last "
                               "perfect), depolarizing p=0.02 per round, %d seeded histories, chi=%d" % (n, chi),
                   "precision": a.precision},
        "roofline": {"bound": "alu", "achieved": ach, "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach / PEAK_ALU_TFLOPS, "traffic": None, "flops_per_launch": flops,
                     # the two-round plan's 64-row site matrices fit the 256-thread build with FP32
                     # factorisations only (LQ matrix in scratch); with FP64 ones the 512-thread build runs
                     "kernel": "fwd_kernel_small" if a.precision in ("bf16", "fp32plain") else "fwd_kernel"},
        "logical_error_rate": float((cls != smp["true_class"]).mean()),
        "environment": environment(),
    }
    if not a.no_cpu:
        threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
        k = min(4 * max(threads, 1), n)  # about 10 s of oracle work on 16 cores
        t0 = time.time()
        ref = oracle.phen_transfer(d, T, rates, meas, smp["syndromes"][:k], threads=threads)
        dt = time.time() - t0
        out["cpu_baseline"] = {"value": k / dt, "unit": "histories/s", "cores": threads, "kind": "oracle",
                               "sample": "first %d histories, exact FP64 transfer over the qubits, %.1f s" % (k, dt)}
        lpo, clo = oracle.decide(ref)
        out["parity_vs_oracle"] = {"histories": k, "max_abs_dlogp": float(np.max(np.abs(lpo - lp[:k]))),
                                   "class_agreement": float((clo == cls[:k]).mean())}
    print(json.dumps(out), flush=True)


def main():
    a = parse()
    if a.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(syndromes would shard across GPUs with no exchange)", file=sys.stderr)
        sys.exit(2)
    if a.copy_calibration:
        copy_calibration()
        return
    import torch

    import paper_2605_17230_amd as tn
    import synth

    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream(dev)
    if a.workload == "c5":
        bench_adjoint(a, torch, tn, synth, dev, stream)
        return
    if a.workload == "fit":
        bench_fit(a, torch, tn, synth, dev)
        return
    if a.workload == "study":
        bench_study(a, torch, tn, synth, dev)
        return
    if a.workload == "planar":
        bench_planar(a, torch, tn, synth, dev, stream)
        return
    if a.workload == "rounds":
        bench_rounds(a, torch, tn, synth, dev, stream)
        return
    if a.workload == "c3":
        rates = synth.depolarizing(D, P)
        smp = synth.sample(D, rates, a.count, SEED)
        segs_h = [dict(d=D, chi=CHI, syndromes=smp["syndromes"], rates=rates,
                       model_index=np.zeros(a.count, np.int32), true_class=smp["true_class"])]
        workload = "rotated surface code d=17, depolarizing p=0.12, %d seeded syndromes, chi=32" % a.count
    elif a.workload == "c2":
        segs_h = synth.config_inputs("C2")
        workload = ("p-sweep at d=9, chi=16: depolarizing p in {0.05, 0.08, 0.11, 0.14, 0.17}, 65,536 seeded "
                    "syndromes per p, one call")
    else:
        segs_h = synth.config_inputs("C4")
        workload = ("mixed batch in one launch: d=5..15 with 32768..1024 syndromes, biased p=0.08, "
                    "eta in {1,10,100}, chi=8..28")
    n_syn = sum(len(s["syndromes"]) for s in segs_h)
    dev_in = [(torch.from_numpy(s["syndromes"]).to(dev), torch.from_numpy(s["rates"]).to(dev),
               torch.from_numpy(s["model_index"]).to(dev)) for s in segs_h]

    def inputs(prec, limit=None):
        out = []
        for s, (sy, rt, mi) in zip(segs_h, dev_in):
            if limit is not None:
                sy, mi = sy[:limit], mi[:limit]
            out.append(tn.SegmentInput(s["d"], s["chi"], sy, rt, mi, prec))
        return out

    # counted work as executed: per syndrome, the rows common to its four cosets once, the rest four times
    flops_per_step = sum(len(s["syndromes"]) * tn.plan_info(s["d"], s["chi"], a.precision)["flops_syndrome"]
                         for s in segs_h)
    gemm_per_step = sum(len(s["syndromes"]) * tn.plan_info(s["d"], s["chi"], a.precision)["gemm_flops_syndrome"]
                        for s in segs_h)
    segs = inputs(a.precision)
    # the forward kernel build each distinct (d, chi) of the batch runs on
    shapes = {(s["d"], s["chi"]): tuple(tn.api.launch_shape(s["d"], s["chi"], a.precision)) for s in segs_h}
    # one persistent launch per build: a call with plans on two 256-thread
    # groups per CU runs its three-group plans there as well
    if any(sh[2] == 256 and sh[1] < 3 for sh in shapes.values()):
        shapes = {k: (sh[0], 2, 256) if sh[2] == 256 else sh for k, sh in shapes.items()}
    kernels = sorted({kernel_name(sh) for sh in shapes.values()})
    print("bench: %s, %s, %d warmup + %d timed steps" % (workload, a.precision, a.warmup, a.steps),
          file=sys.stderr, flush=True)
    for _ in range(a.warmup):
        tn.decode_segments(segs)
    torch.cuda.synchronize()
    ev = []
    t0 = time.time()
    outs = None
    for i in range(a.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        outs = tn.decode_segments(segs)
        e1.record(stream)
        ev.append((e0, e1))
        print("bench: step %d enqueued" % i, file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    wall = time.time() - t0
    ms = [e0.elapsed_time(e1) for e0, e1 in ev]
    ms_step = float(np.mean(ms))
    value = n_syn / (ms_step / 1e3)
    achieved = flops_per_step / (ms_step / 1e3) / 1e12
    metric = {"c3": "syndromes/s at d=17 chi=32 (boundary-MPS coset decoding), BF16 form vs FP32 plain; "
                    "coset log-likelihood error vs FP64",
              "c2": "syndromes/s of the d=9 chi=16 p-sweep (boundary-MPS coset decoding, plain FP32)",
              "c4": "syndromes/s of the mixed-distance batch d=5..15 (boundary-MPS coset decoding)"}[a.workload]
    out = {
        "metric": metric,
        "value": value,
        "unit": "syndromes/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[a.precision],
        "data": "synthetic",
        "config": {"workload": workload, "syndromes": n_syn, "cosets": 4, "precision": a.precision,
                   "segments": [{"d": s["d"], "chi": s["chi"], "count": len(s["syndromes"])} for s in segs_h]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_ALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / PEAK_ALU_TFLOPS,
                     "traffic": measured_traffic(a.precision, a.count, a.workload),
                     "flops_per_launch": flops_per_step, "kernel": " + ".join(kernels)},
        "launch": {"%d:%d" % k: {"group": v[0], "wg_per_cu": v[1], "threads": v[2]} for k, v in shapes.items()},
        "wall_s": wall,
    }
    if a.precision in ("bf16", "bf16f64"):
        # the GEMM-class part on the matrix cores, counted once: in the split
        # form each product runs as three bf16 MFMA products (hi/lo), in the
        # single-rounded form as one
        mf = gemm_per_step / (ms_step / 1e3) / 1e12
        out["mfma"] = {"gemm_flops_per_launch": gemm_per_step, "gemm_share_of_counted": gemm_per_step / flops_per_step,
                       "achieved": mf, "peak": PEAK_MFMA_BF16_TFLOPS, "unit": "TFLOP/s",
                       "frac": mf / PEAK_MFMA_BF16_TFLOPS,
                       "bf16_products_per_gemm_flop": 3 if a.precision == "bf16" else 1}
    print("bench: timed %.1f ms per step" % ms_step, file=sys.stderr, flush=True)
    out["environment"] = environment()
    if a.workload == "c2":
        out["logical_error_rate"] = {
            "p=%.2f" % sg["p"]: float((o.cls.cpu().numpy() != sg["true_class"]).mean()) for sg, o in zip(segs_h, outs)}
    lz = [o.logz.cpu().numpy() for o in outs]
    cls = [o.cls.cpu().numpy() for o in outs]
    o2 = None
    if a.compare and a.compare != a.precision:
        s2 = inputs(a.compare)
        tn.decode_segments(s2)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        o2 = tn.decode_segments(s2)
        e1.record(stream)
        torch.cuda.synchronize()
        ms2 = e0.elapsed_time(e1)
        out["compare"] = {"precision": a.compare, "value": n_syn / (ms2 / 1e3), "ms_per_step": ms2,
                          "speedup_of_primary": ms2 / ms_step,
                          "max_abs_dlogz_vs_primary": max_finite_diff([x.logz.cpu().numpy() for x in o2], lz),
                          "cosets_finite_in_one_form_only": int(sum(
                              int((np.isfinite(x.logz.cpu().numpy()) != np.isfinite(y)).sum()) for x, y in zip(o2, lz))),
                          "class_agreement_with_primary": float(np.mean(np.concatenate(
                              [x.cls.cpu().numpy() == y for x, y in zip(o2, cls)])))}
        print("bench: compare %s %.1f ms" % (a.compare, ms2), file=sys.stderr, flush=True)
    if a.fp64_sample > 0 and a.workload == "c3":
        ns = min(a.fp64_sample, n_syn)
        with __import__("warnings").catch_warnings():
            __import__("warnings").simplefilter("ignore")
            o64 = tn.decode_segments(inputs("fp64", ns))[0]
        ref64 = o64.logz.cpu().numpy()
        c64 = o64.cls.cpu().numpy()
        err = {"syndromes": ns, "chi": CHI}
        forms = [(a.precision, lz[0][:ns], cls[0][:ns])]
        if o2 is not None:
            forms.append((a.compare, o2[0].logz.cpu().numpy()[:ns], o2[0].cls.cpu().numpy()[:ns]))
        with np.errstate(invalid="ignore"):
            post = ref64 - np.logaddexp.reduce(ref64, 1)[:, None]
        for name, z, c in forms:
            fin = np.isfinite(ref64) & np.isfinite(z)
            dz = np.abs(np.where(fin, z - ref64, 0.0))
            err[name] = {"max_abs_dlogz": float(dz.max()),
                         "max_abs_dlogz_posterior_ge_e-10": float(dz[post >= -10].max(initial=0)),
                         "max_abs_dlogz_posterior_ge_e-20": float(dz[post >= -20].max(initial=0)),
                         "unresolved_cosets": int((np.isfinite(ref64) & ~np.isfinite(z)).sum()),
                         "max_abs_dlogp": float(np.max(np.abs(np.logaddexp.reduce(z, 1)
                                                              - np.logaddexp.reduce(ref64, 1)))),
                         "class_agreement": float(np.mean(c == c64))}
        out["error_vs_fp64_same_chi"] = err
        print("bench: fp64 comparison done", file=sys.stderr, flush=True)
    if not a.no_cpu and a.workload == "c3":
        import oracle
        s0 = segs_h[0]
        ref, n, dt, threads = cpu_baseline(D, s0["rates"], s0["syndromes"], a.cpu_seconds, a.cpu_min)
        _, rcls = oracle.decide(ref)
        fin = np.isfinite(ref)
        out["cpu_baseline"] = {"value": n / dt, "unit": "syndromes/s", "cores": threads, "kind": "oracle",
                               "sample": "first %d syndromes of the batch, exact FP64 transfer-matrix "
                                         "contraction (4 cosets each), %.1f s" % (n, dt)}
        out["parity_vs_oracle"] = {"syndromes": n,
                                   "max_abs_dlogz": float(np.max(np.where(fin, np.abs(lz[0][:n] - ref), 0.0))),
                                   "max_abs_dlogp": float(np.max(np.abs(
                                       np.logaddexp.reduce(lz[0][:n], 1) - np.logaddexp.reduce(ref, 1)))),
                                   "class_agreement": float((cls[0][:n] == rcls).mean())}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
