#!/usr/bin/env python3
"""Throughput of the MI355X sparse FFT on its headline workload.

Workload (one step): a batch of 512 independent exactly-sparse signals,
n = 2^22, k = 256, complex64 storage, log-uniform |coefficient| in [0.1, 10],
uniform phases, each signal with its own seed, through the batched path: one
HashToBins launch for the first round group of every signal, the device decode
loop, HashToBins of later round groups for the signals still decoding, FP64
re-estimation; replayed from hipGraphs.  Inputs are resident in HBM before the
timed region.

Printed: ONE JSON line with the batched sFFTs/s as `value`, plus the plain
one-signal-at-a-time path, a dense full-length FFT + top-k on the same GPU
(the crossover reference), per-step latency percentiles, the roofline of the
dominant kernel (HashToBins, HBM bound; achieved = algorithmic bytes / its
event-timed duration), parity of every signal against the FP64 oracle, and the
oracle itself timed on the host (cpu_baseline: a process pool over the host's
cores, with the one-process rate beside it).  `--workload c4` (the general-mode
precision split) and `--workload section5` (k-point DFTs through the n-point
sFFT of the periodic extension) print their own line instead.
"""
import argparse
import json
import math
import os
import sys
import tempfile
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# The serving runtime runs one stream per resident plan instance; with HIP's
# default of 4 hardware queues per process, batches of different shapes
# serialise behind each other's launch chains (measured at half load: p50
# 18.9 ms with 4 queues, 3.9 ms with 16).  Must be set before HIP starts.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4") or 4) < 16:
    os.environ["GPU_MAX_HW_QUEUES"] = "16"

from paper_1201_2501_amd.prof import kernel_source_hash  # noqa: E402

METRIC = "sFFTs/s at n=2^22,k=256 (batched vs plain), HBM GB/s, p50/p99 latency"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "h2b_pair_c3_traffic.json")
TUNE_FILE = os.path.join(ROOT, "paper_1201_2501_amd", "tuned.json")


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def percentile(vals, q):
    return float(np.percentile(np.asarray(vals, dtype=np.float64), q))


def load_traffic(signals, cfg_key):
    """Counter-measured HBM bytes per HashToBins launch, if recorded for the
    current kernel source and this configuration; else None."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    try:
        rec = json.load(open(TRAFFIC_FILE))
    except ValueError:
        return None
    if rec.get("source_hash") != kernel_source_hash() or rec.get("config") != cfg_key:
        return None
    per_signal = rec.get("bytes_per_signal")
    return None if per_signal is None else float(per_signal) * signals


def host_cores():
    """Cores this process may use, at most 16 (the host share of one GPU)."""
    try:
        c = len(os.sched_getaffinity(0))
    except AttributeError:
        c = os.cpu_count() or 1
    return max(1, min(16, c))


def _oracle_worker(job):
    """One oracle run on signal `s` of the memory-mapped batch (pool worker;
    imports no GPU library)."""
    path, count, n, fields, seed, s = job
    from oracle.exact import noiseless_sparse_fft
    from oracle.params import SfftParams
    x = np.array(np.memmap(path, dtype=np.complex64, mode="r", shape=(count, n))[s])
    t = time.perf_counter()
    noiseless_sparse_fft(x, SfftParams(**{**fields, "seed": seed}))
    return time.perf_counter() - t


def oracle_pool_rate(path, count, n, desc, seeds, procs):
    """sFFTs/s of the oracle over `count` signals spread over `procs` spawned
    processes (one numpy thread each); the pool is started and warmed before
    the clock starts.  Returns (rate, wall seconds)."""
    import multiprocessing as mp
    fields = oracle_params(desc, 0).__dict__.copy()
    env_keep = {k: os.environ.get(k) for k in ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")}
    for k in env_keep:
        os.environ[k] = "1"
    try:
        ctx = mp.get_context("spawn")
        with ctx.Pool(procs) as pool:
            pool.map(_oracle_worker, [(path, count, n, fields, seeds[0], 0)] * procs)   # warm-up
            t = time.perf_counter()
            pool.map(_oracle_worker, [(path, count, n, fields, seeds[s], s) for s in range(count)], chunksize=1)
            wall = time.perf_counter() - t
    finally:
        for k, v in env_keep.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v
    return count / wall, wall


def serving_bench(args, torch, dev, sfft):
    """Mixed request stream through the serving runtime: n log-uniform over
    2^16..2^24, k uniform in [8, 1024], half exactly sparse (unit magnitudes)
    and half noisy (tail/head 0.05), per-request seeds.  Signals come from a
    pool of 4 planted signals per (n, mode), each with its own k.  Phases:
    warm-up (every shape once, plans made resident), saturated (all requests
    submitted at once: capacity), Poisson arrivals at each of serve_loads x
    capacity (latency).  Recovery is checked per request against the planted spectra."""
    import siggen

    rng = np.random.Generator(np.random.PCG64(20241203))
    sizes = [1 << e for e in range(16, 25)]
    pool = {}
    t = time.time()
    for n in sizes:
        for mode in (sfft.SFFT_MODE_EXACT, sfft.SFFT_MODE_GENERAL):
            for j in range(4):
                kk = int(rng.integers(8, 1025))
                gseed = 7_000_000 + (n.bit_length() << 8) + (mode << 4) + j
                x, sups, vals = siggen.torch_planted_batch(n, kk, [gseed], dev, magnitude="unit",
                                                           noise_ratio=0.05 if mode else 0.0)
                order = np.argsort(sups[0])
                pool.setdefault((n, mode), []).append((x[0].contiguous(), sups[0][order], vals[0][order], kk))
    torch.cuda.synchronize()
    log("serving: signal pool of %d signals in %.1fs" % (sum(len(v) for v in pool.values()), time.time() - t))

    def draw(count):
        out = []
        for _ in range(count):
            n = sizes[int(rng.integers(0, len(sizes)))]
            mode = int(rng.integers(0, 2))
            out.append((n, mode, int(rng.integers(0, 4)), int(rng.integers(1, 1 << 62))))
        return out

    srv = sfft.Server(budget_bytes=64 << 30, slots=args.serve_slots, instances=args.serve_instances)

    def run(reqs, arrivals=None):
        tickets = []
        lag = 0.0
        t0 = time.perf_counter()
        for q, (n, mode, j, seed) in enumerate(reqs):
            if arrivals is not None:
                due = t0 + arrivals[q]
                while time.perf_counter() < due:
                    pass
                lag = max(lag, time.perf_counter() - due)
            x, _, _, kk = pool[(n, mode)][j]
            tickets.append(srv.submit(x, kk, mode, seed))
        outs = [srv.wait(tk) for tk in tickets]
        return outs, lag

    misses, worst = [], []

    def recovery(reqs, outs):
        exact_ok, exact_n, noisy_err = 0, 0, []
        for (n, mode, j, seed), (idx, val, res) in zip(reqs, outs):
            _, sup, vals, kk = pool[(n, mode)][j]
            tag = {"n": n, "k": kk, "seed": seed, "path": "dense" if res.path else "sparse", "rounds": res.rounds,
                   "count": res.count}
            if mode == sfft.SFFT_MODE_EXACT:
                exact_n += 1
                good = bool(np.array_equal(idx, sup))
                exact_ok += int(good)
                if not good and len(misses) < 8:
                    misses.append(dict(tag, missing=len(set(sup.tolist()) - set(idx.tolist())),
                                       extra=len(set(idx.tolist()) - set(sup.tolist()))))
            else:
                est = dict(zip(idx.tolist(), val))
                err2 = sum(abs(est.pop(int(i), 0) - v) ** 2 for i, v in zip(sup, vals)) + \
                    sum(abs(v) ** 2 for v in est.values())
                e = math.sqrt(err2) / float(np.linalg.norm(vals))
                noisy_err.append(e)
                worst.append(dict(tag, err=round(e, 5)))
                worst.sort(key=lambda r: -r["err"])
                del worst[4:]
        return exact_ok, exact_n, noisy_err

    def tail_classes(reqs, outs):
        """The slowest 1% of a phase's requests, by (n, mode, path): count,
        mean service and queue time, mean k."""
        lat = np.array([res.latency_ms for (_, _, res) in outs])
        cut = percentile(lat.tolist(), 99)
        groups = {}
        for (n, mode, j, seed), (_, _, res) in zip(reqs, outs):
            if res.latency_ms < cut:
                continue
            key = "2^%d %s %s" % (n.bit_length() - 1, "exact" if mode == sfft.SFFT_MODE_EXACT else "general",
                                  "dense" if res.path else "sparse")
            g = groups.setdefault(key, [0, 0.0, 0.0, 0])
            g[0] += 1
            g[1] += res.service_ms
            g[2] += res.queue_ms
            g[3] += pool[(n, mode)][j][3]
        rows = [{"class": key, "count": c, "service_ms": round(sv / c, 3), "queue_ms": round(qu / c, 3),
                 "mean_k": round(kk / c)} for key, (c, sv, qu, kk) in groups.items()]
        return sorted(rows, key=lambda r: -r["count"])[:6]

    # warm-up: every (n, mode, pool entry) once, so every shape's plans are resident
    warm = [(n, mode, j, 1 + j) for (n, mode) in pool for j in range(4)]
    run(warm)
    warm_instances = int(srv.stats().instances)
    log("serving: warm-up left %d resident instances for %d pool signals" % (warm_instances, len(warm)))
    srv.reset_stats()
    # saturated: capacity
    reqs = draw(args.serve_requests)
    outs, _ = run(reqs)
    st = srv.stats()
    capacity = st.rate
    ok_s, n_s, err_s = recovery(reqs, outs)
    log("serving: capacity %.0f requests/s (mean batch %.2f, %d dense)" % (capacity, st.mean_batch, st.dense))
    # Poisson arrivals at each load
    sweep, ok_p, n_p, err_p, peak, evict, failed = [], 0, 0, [], 0, 0, 0
    for load in [float(v) for v in args.serve_loads.split(",")]:
        srv.reset_stats()
        rate = load * capacity
        reqs = draw(args.serve_requests)
        arrivals = np.cumsum(rng.exponential(1.0 / rate, size=len(reqs)))
        outs, lag = run(reqs, arrivals)
        st = srv.stats()
        o, nn, e = recovery(reqs, outs)
        tail = tail_classes(reqs, outs)
        ok_p, n_p, err_p = ok_p + o, n_p + nn, err_p + e
        peak, evict, failed = max(peak, int(st.peak_bytes)), evict + int(st.evictions), failed + int(st.failed)
        by_path = {}
        for name, want in (("sparse", 0), ("dense", 1)):
            lat = [res.latency_ms for (_, _, res) in outs if res.path == want]
            by_path[name] = {"requests": len(lat), "share": round(len(lat) / len(outs), 4),
                             "p50_ms": round(percentile(lat, 50), 3) if lat else None,
                             "p99_ms": round(percentile(lat, 99), 3) if lat else None}
        sweep.append({"load": load, "arrival_rate_per_s": round(rate, 1), "sFFTs_per_s": round(st.rate, 1),
                      "p50_ms": round(st.p50_ms, 3), "p99_ms": round(st.p99_ms, 3), "by_path": by_path,
                      "queue_p50_ms": round(st.queue_p50_ms, 3), "service_p50_ms": round(st.service_p50_ms, 3),
                      "mean_batch": round(st.mean_batch, 2), "dense_fallback": int(st.dense),
                      "max_submit_lag_ms": round(lag * 1e3, 3), "slowest_1pct": tail})
        log("serving: Poisson %.0f/s (%.2f x capacity) -> p50 %.3f ms p99 %.3f ms, %.0f sFFTs/s; sparse %.0f%% "
            "(p50 %s p99 %s ms), dense p50 %s p99 %s ms"
            % (rate, load, st.p50_ms, st.p99_ms, st.rate, 100 * by_path["sparse"]["share"],
               by_path["sparse"]["p50_ms"], by_path["sparse"]["p99_ms"], by_path["dense"]["p50_ms"],
               by_path["dense"]["p99_ms"]))
    srv.close()
    err_all = err_s + err_p
    mid = sweep[len(sweep) // 2]
    return {"requests_per_phase": len(reqs), "slots": args.serve_slots, "instances": args.serve_instances,
            "resident_instances_after_warmup": warm_instances,
            "hw_queues": os.environ.get("GPU_MAX_HW_QUEUES", "default"),
            "capacity_sFFTs_per_s": round(capacity, 1),
            "value": mid["sFFTs_per_s"], "unit": "sFFTs/s", "load": mid["load"],
            "p50_ms": mid["p50_ms"], "p99_ms": mid["p99_ms"], "by_path": mid["by_path"], "sweep": sweep,
            "failed": failed, "evictions": evict, "peak_device_bytes": peak,
            "exact_recovered": "%d/%d" % (ok_s + ok_p, n_s + n_p),
            "exact_misses": misses,
            "noisy_l2_rel_err_vs_planted": {"median": round(float(np.median(err_all)), 5) if err_all else None,
                                            "max": round(float(np.max(err_all)), 5) if err_all else None,
                                            "worst": worst},
            "what": "Poisson stream, n in 2^16..2^24 log-uniform, k in [8,1024], 50/50 exact/noisy(0.05), "
                    "complex64, per-request seeds; latency = submit -> results on the host"}


def precision_split_bench(args, torch, dev, sfft, siggen):
    """The precision split on the general-mode workload: 16 signals of
    n = 2^26, k = 1024, unit magnitudes, tail/head noise 0.01, complex64,
    B = 4096, delta = 1e-7.  Variants (Kaiser-Bessel window): FP32 location
    and estimation hashings; FP64 location pairs (the default at this n);
    FP64 throughout; and FP64 location pairs with the Gaussian window.
    Each reports its batch rate, supports equal to the planted ones and the
    l2/l2 ratio ||xhat - x'|| / Err(xhat, k), with Err from a full FP64 FFT
    of the same input bytes (torch.fft on the device, a measurement only)."""
    from paper_1201_2501_amd.sfft import Plan
    n, k, B, S = 1 << 26, 1024, 4096, 16
    t = time.time()
    X, sups, vals = siggen.torch_planted_batch(n, k, [90_000 + s for s in range(S)], dev, magnitude="unit",
                                               noise_ratio=0.01, chunk=4)
    seeds = torch.arange(S, dtype=torch.int64, device=dev) * 31 + 5
    torch.cuda.synchronize()
    log("c4: inputs ready in %.1fs" % (time.time() - t))
    errk = []
    for s in range(S):
        F = torch.fft.fft(X[s].to(torch.complex128), norm="ortho").abs().pow(2)
        top = torch.topk(F, k).values.sum()
        errk.append(math.sqrt(max(float(F.sum() - top), 0.0)))
        del F
    variants = []
    # the precision variants with the Kaiser-Bessel window (half the
    # Gaussian construction's samples), and FP64 location with the Gaussian
    # window for comparison
    for name, lp, ep, win in (("fp32", sfft.SFFT_F32, sfft.SFFT_F32, 1),
                              ("fp64_location", sfft.SFFT_F64, sfft.SFFT_F32, 1),
                              ("fp64_all", sfft.SFFT_F64, sfft.SFFT_F64, 1),
                              ("fp64_location_gaussian", sfft.SFFT_F64, sfft.SFFT_F32, 0)):
        wk = sfft.sfft_window_w(n, B, 0.5, 1e-7, win)
        plan = Plan(n, k, B, wk, 0, mode=sfft.SFFT_MODE_GENERAL, delta=1e-7, loc_prec=lp, est_prec=ep, max_batch=S,
                    flags=sfft.SFFT_FLAG_TIMING, window=win)
        bufs = plan.execute_batch(X, seeds)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            plan.execute_batch(X, seeds, bufs=bufs)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        tm = plan.timings()
        counts = bufs["counts"].cpu().numpy()
        idx = bufs["idx"].cpu().numpy()
        val = bufs["val"].cpu().numpy()
        exact, ratios = 0, []
        Xh = None
        for s in range(S):
            c = int(counts[s])
            exact += int(np.array_equal(idx[s, :c], np.sort(sups[s])))
            Xh = torch.fft.fft(X[s].to(torch.complex128), norm="ortho")
            est = torch.zeros_like(Xh)
            est[torch.from_numpy(idx[s, :c]).to(dev)] = torch.from_numpy(val[s, :c]).to(dev)
            ratios.append(float((Xh - est).abs().pow(2).sum().sqrt()) / errk[s])
        del Xh
        variants.append({"variant": name, "loc_prec": "f64" if lp else "f32", "est_prec": "f64" if ep else "f32",
                         "ms_per_batch": round(ms, 3), "sFFTs_per_s": round(S / (ms * 1e-3), 1),
                         "hash_ms": round(float(tm[0]), 3), "supports_equal_planted": "%d/%d" % (exact, S),
                         "l2l2_ratio_max": round(max(ratios), 4), "l2l2_ratio_median": round(float(np.median(ratios)), 4),
                         "w": int(plan.desc.w), "rounds": int(plan.desc.rounds),
                         "window": ["gaussian", "kaiser-bessel"][plan.desc.window]})
        log("c4 %s: %.3f ms/batch, supports %d/%d, l2/l2 max %.4f" % (name, ms, exact, S, max(ratios)))
        plan.close()
    best = min(variants, key=lambda v: v["ms_per_batch"])
    return {"metric": "sFFTs/s at n=2^26,k=1024 (precision split)", "value": best["sFFTs_per_s"], "unit": "sFFTs/s",
            "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": best["ms_per_batch"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": best["loc_prec"],
            "data": "synthetic",
            "config": {"workload": "general-mode sFFT: 16 signals, n=2^26, k=1024, complex64, unit magnitudes, "
                                   "tail/head noise 0.01, B=4096, delta=1e-7", "signals": S, "n": n, "k": k, "B": B},
            "variants": variants}


def general_schedule_bench(args, torch, dev, sfft, siggen):
    """The general-case round schedule against fixed B and w (SparseFFT,
    Algorithm 2): the practical schedule (k_r = k / 4^r, B_r halving down to
    4 k_r, w_r = w B_r / B) and the same plan with b_min = B (B and w fixed
    in every round), on two workloads: 64 signals of n = 2^20, k = 64,
    tail/head 0.05, B = 1024, delta = 1e-6; and 16 signals of n = 2^26,
    k = 1024, tail/head 0.01, B = 4096, delta = 1e-7 (unit magnitudes,
    complex64).  Each variant reports the samples one signal gathers and their
    algorithmic bytes, the batch time, the planted heads found, supports
    equal to the planted ones, and the l2/l2 ratio against Err(xhat, k) from
    a full FP64 FFT of the same input bytes."""
    from paper_1201_2501_amd.sfft import Plan
    out = []
    for name, n, k, B, S, noise, delta, gen0 in (("c2", 1 << 20, 64, 1024, 64, 0.05, 1e-6, 95_000),
                                                 ("c4", 1 << 26, 1024, 4096, 16, 0.01, 1e-7, 90_000)):
        X, sups, vals = siggen.torch_planted_batch(n, k, [gen0 + s for s in range(S)], dev, magnitude="unit",
                                                   noise_ratio=noise, chunk=4)
        seeds = torch.arange(S, dtype=torch.int64, device=dev) * 37 + 11
        errk = []
        for s in range(S):
            F = torch.fft.fft(X[s].to(torch.complex128), norm="ortho").abs().pow(2)
            errk.append(math.sqrt(max(float(F.sum() - torch.topk(F, k).values.sum()), 0.0)))
            del F
        for sched, b_min in (("practical", 0), ("fixed_B_w", B)):
            plan = Plan(n, k, B, 0, 0, mode=sfft.SFFT_MODE_GENERAL, delta=delta, b_min=b_min, max_batch=S)
            samples = sfft.sfft_plan_samples(plan.desc)
            bufs = plan.execute_batch(X, seeds)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                plan.execute_batch(X, seeds, bufs=bufs)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            counts, idx, val = bufs["counts"].cpu().numpy(), bufs["idx"].cpu().numpy(), bufs["val"].cpu().numpy()
            found = exact = 0
            ratios = []
            for s in range(S):
                c = int(counts[s])
                found += len(np.intersect1d(idx[s, :c], sups[s]))
                exact += int(np.array_equal(idx[s, :c], np.sort(sups[s])))
                Xh = torch.fft.fft(X[s].to(torch.complex128), norm="ortho")
                est = torch.zeros_like(Xh)
                est[torch.from_numpy(idx[s, :c]).to(dev)] = torch.from_numpy(val[s, :c]).to(dev)
                ratios.append(float((Xh - est).abs().pow(2).sum().sqrt()) / errk[s])
                del Xh, est
            rec = {"workload": name, "schedule": sched, "n": n, "k": k, "B": B, "signals": S, "noise": noise,
                   "w": int(plan.desc.w), "rounds": int(plan.desc.rounds), "samples_per_signal": samples,
                   "alg_bytes_per_signal": samples * 8, "ms_per_batch": round(ms, 3),
                   "sFFTs_per_s": round(S / (ms * 1e-3), 1), "heads_found": "%d/%d" % (found, S * k),
                   "supports_equal_planted": "%d/%d" % (exact, S), "l2l2_ratio_max": round(max(ratios), 4),
                   "l2l2_ratio_median": round(float(np.median(ratios)), 4)}
            log("gsched %s %s: %d samples/signal, %.3f ms/batch, heads %s, supports %s, l2/l2 max %.4f" % (
                name, sched, samples, ms, rec["heads_found"], rec["supports_equal_planted"], max(ratios)))
            out.append(rec)
            plan.close()
        del X
        torch.cuda.empty_cache()
    head = next(r for r in out if r["workload"] == "c2" and r["schedule"] == "practical")
    return {"metric": "general-mode schedule: samples and sFFTs/s, practical vs fixed B and w",
            "value": head["sFFTs_per_s"], "unit": "sFFTs/s", "n_gpus": 1, "steps": args.steps, "warmup": 1,
            "ms_per_step": head["ms_per_batch"], "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
            "dtype": "f64", "data": "synthetic",
            "config": {"workload": "general-mode sFFT, practical schedule vs b_min = B: 64 x 2^20 (k=64, 5% noise) "
                                   "and 16 x 2^26 (k=1024, 1% noise)"},
            "variants": out}


def stream_mode_bench(args, torch, dev, sfft, siggen):
    """Stream-mode HashToBins against the gather, batched exact mode, 512
    signals per shape, unit magnitudes, complex64, delta = 1e-9, b_min 32,
    24 rounds, patience 5 (the served exact schedule): hash_mode 0 (gather
    every round), 1 (stream the rounds whose window covers n/8 or more), 2
    (stream every round).  Reports the batch time, the samples one signal
    reads in round group 0 (streamed rounds count n) and the supports
    recovered."""
    from paper_1201_2501_amd.sfft import Plan
    out = []
    S = 512
    for n, k, B in ((1 << 16, 16, 64), (1 << 16, 64, 256), (1 << 18, 100, 512), (1 << 20, 256, 1024)):
        X, sups, _ = siggen.torch_planted_batch(n, k, [60_000 + s for s in range(S)], dev, magnitude="unit")
        seeds = torch.arange(S, dtype=torch.int64, device=dev) * 13 + 1
        for mode in (0, 1, 2):
            plan = Plan(n, k, B, 0, 0, delta=1e-9, b_min=32, rounds=24, patience=5, hash_mode=mode, max_batch=S,
                        flags=sfft.SFFT_FLAG_TIMING)
            bufs = plan.execute_batch(X, seeds)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                plan.execute_batch(X, seeds, bufs=bufs)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            tm = plan.timings()
            counts, idx = bufs["counts"].cpu().numpy(), bufs["idx"].cpu().numpy()
            ok = sum(int(np.array_equal(idx[s, :int(counts[s])], np.sort(sups[s]))) for s in range(S))
            rec = {"n": n, "k": k, "B": B, "w": int(plan.desc.w), "hash_mode": mode,
                   "stream_rounds": sfft.sfft_plan_stream_rounds(plan.desc),
                   "samples_per_signal": sfft.sfft_plan_samples(plan.desc), "ms_per_batch": round(ms, 3),
                   "hash_ms": round(float(tm[0]), 3), "sFFTs_per_s": round(S / (ms * 1e-3), 1),
                   "supports": "%d/%d" % (ok, S)}
            log("stream n=2^%d k=%d B=%d mode %d: %.3f ms/batch (hash %.3f), %d stream rounds, supports %d/%d" % (
                n.bit_length() - 1, k, B, mode, ms, tm[0], rec["stream_rounds"], ok, S))
            out.append(rec)
            plan.close()
        del X
        torch.cuda.empty_cache()
    head = out[0]
    return {"metric": "batched exact sFFTs/s, stream-mode vs gathered HashToBins", "value": head["sFFTs_per_s"],
            "unit": "sFFTs/s", "n_gpus": 1, "steps": args.steps, "warmup": 1, "ms_per_step": head["ms_per_batch"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
            "config": {"workload": "512 exactly sparse signals per shape, n = 2^16..2^20, hash_mode 0/1/2"},
            "variants": out}


def section5_bench(args, torch, dev, sfft):
    """The Section 5 reduction as a workload: the k-point DFT of x_k computed
    through the n-point exactly sparse sFFT of its periodic extension
    y_t = x_{t mod k}, whose unitary spectrum is sqrt(n/k) times the unitary
    k-point DFT of x_k on the multiples of n/k and zero elsewhere.  512
    signals, n = 2^22, k = 256, complex64; each k-point spectrum has
    log-uniform magnitudes (scaled so the n-point coefficients lie in
    [0.1, 10]) and uniform phases.  The lattice support never collides at
    B = 4k bins, and every coefficient of a round shares one offset within
    its bin, so the plan keeps B fixed (b_min = B) and stops once all k are
    found and a round comes back empty.  Timed against a direct k-point FFT
    of the same batch (torch.fft, rocFFT).  Checked against the definition:
    supports equal to the lattice, values against an FP64 k-point DFT."""
    from paper_1201_2501_amd.sfft import Plan
    n, k, S = 1 << 22, 256, 512
    B = 4 * k
    rng = np.random.Generator(np.random.PCG64(20260501))
    mags = np.exp(rng.uniform(math.log(0.1), math.log(10.0), size=(S, k)))
    spec = mags * np.exp(2j * math.pi * rng.uniform(0.0, 1.0, size=(S, k))) / math.sqrt(n / k)
    xk = torch.fft.ifft(torch.from_numpy(spec).to(dev), dim=-1, norm="ortho")      # FP64, [S, k]
    Y = xk.to(torch.complex64).repeat(1, n // k)                                       # [S, n], 16 GiB
    xk64 = xk.to(torch.complex64).contiguous()
    # expected: the FP64 k-point DFT of the stored (complex64) x_k, on the lattice
    expect = (torch.fft.fft(xk64.to(torch.complex128), dim=-1, norm="ortho") * math.sqrt(n / k)).cpu().numpy()
    seeds = torch.arange(S, dtype=torch.int64, device=dev) * 4099 + 11
    torch.cuda.synchronize()
    plan = Plan(n, k, B, 0, 0, alpha=0.5, delta=1e-9, theta=0.01, g_min=0.25, rounds=16, b_min=B, patience=8,
                stop_count=k, stop_patience=1, group0=2, loc_prec=sfft.SFFT_F64, max_batch=S,
                flags=sfft.SFFT_FLAG_TIMING)
    bufs = plan.execute_batch(Y, seeds)
    for _ in range(args.warmup):
        plan.execute_batch(Y, seeds, bufs=bufs)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        plan.execute_batch(Y, seeds, bufs=bufs)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    counts = bufs["counts"].cpu().numpy()
    idx = bufs["idx"].cpu().numpy()
    val = bufs["val"].cpu().numpy()
    rounds = bufs["info"][:, 0].cpu().numpy()          # rounds each signal used
    lattice = np.arange(k, dtype=np.int64) * (n // k)
    ok, rel = 0, 0.0
    for s in range(S):
        c = int(counts[s])
        good = c == k and np.array_equal(idx[s, :c], lattice)
        ok += int(good)
        if good:
            rel = max(rel, float(np.max(np.abs(val[s, :c] - expect[s]) / np.abs(expect[s]))))
    # direct k-point FFT of the same batch
    out = torch.fft.fft(xk64, dim=-1)
    for _ in range(args.warmup):
        torch.fft.fft(xk64, dim=-1, out=out)
    torch.cuda.synchronize()
    reps = max(args.steps, 50)
    e0.record()
    for _ in range(reps):
        torch.fft.fft(xk64, dim=-1, out=out)
    e1.record()
    torch.cuda.synchronize()
    ms_direct = e0.elapsed_time(e1) / reps
    log("section5: sFFT %.3f ms/batch, supports %d/%d, max rel err %.2e; direct %d-point FFT %.4f ms/batch"
        % (ms, ok, S, rel, k, ms_direct))
    rec = {"metric": "k-point DFTs/s through the n-point sFFT (Section 5 reduction)",
           "value": round(S / (ms * 1e-3), 1), "unit": "k-point DFTs/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 4), "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "Section 5 reduction: 512 periodic signals y_t = x_{t mod k}, n=2^22, k=256, "
                                  "complex64, log-uniform k-point spectra", "signals": S, "n": n, "k": k, "B": B,
                      "w": int(plan.desc.w), "alpha": 0.5, "delta": 1e-9, "theta": 0.01,
                      "round_groups": list(plan.round_groups())},
           "supports_equal_lattice": "%d/%d" % (ok, S), "max_rel_err_vs_fp64_dft": float("%.3g" % rel),
           "mean_rounds": round(float(np.mean(rounds)), 2), "max_rounds": int(np.max(rounds)),
           "direct_k_point_fft": {"ms_per_batch": round(ms_direct, 5),
                                  "DFTs_per_s": round(S / (ms_direct * 1e-3), 1),
                                  "what": "torch.fft.fft over [512, 256] complex64 (rocFFT)"},
           "sfft_over_direct_time": round(ms / ms_direct, 1)}
    plan.close()
    return rec


def oracle_params(desc, seed):
    from oracle.params import SfftParams
    return SfftParams(n=desc.n, k=desc.k, B=desc.B, w=desc.w, seed=seed, alpha=desc.alpha, delta=desc.delta,
                      theta=desc.theta, g_min=desc.g_min, rounds=desc.rounds, b_min=desc.b_min,
                      patience=desc.patience, stop_count=desc.stop_count,
                      stop_patience=desc.stop_patience, ratio_tol=desc.ratio_tol, cap=desc.cap,
                      alpha_decay=desc.alpha_decay, refine_shift=desc.refine_shift,
                      refine_window=desc.refine_window or 16, window=desc.window)


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--inflight", type=int, default=4,
                    help="batches in flight in the throughput measurement (one plan instance and stream each)")
    ap.add_argument("--signals", type=int, default=512)
    ap.add_argument("--log2n", type=int, default=22)
    ap.add_argument("--k", type=int, default=256)
    ap.add_argument("--B", type=int, default=1024)
    ap.add_argument("--b-min", type=int, default=32,
                    help="smallest bin count of the shrinking schedule (tuned on the oracle: 512/512 "
                         "recovered with 7%% fewer samples than B/16)")
    ap.add_argument("--rounds", type=int, default=24, help="most exact-mode rounds")
    ap.add_argument("--delta", type=float, default=1e-9, help="window accuracy (with --tune off)")
    ap.add_argument("--patience", type=int, default=3, help="empty rounds before a signal stops (with --tune off)")
    ap.add_argument("--hash-threads", type=int, default=256, help="HashToBins workgroup size (with --tune off)")
    ap.add_argument("--hash-order", type=int, default=None,
                    help="HashToBins workgroup order over (signal, round): 0 round-major, 1 signal-major, "
                         "2 signal-major per XCD (default: the plan's)")
    ap.add_argument("--alpha", type=float, default=0.5, help="window transition fraction (with --tune off)")
    ap.add_argument("--stop-count", type=int, default=0,
                    help="stop after --stop-patience empty rounds once this many entries are found (with --tune "
                         "off; 0 = off)")
    ap.add_argument("--stop-patience", type=int, default=2)
    ap.add_argument("--extra-batches", type=int, default=0,
                    help="also run the plan on this many fresh batches (generator seeds 5000003 + 512 i + s) "
                         "and report exact recovery over them")
    ap.add_argument("--alpha-decay", type=float, default=0.0,
                    help="alpha_t schedule on top of the chosen plan: alpha shrinks by this factor per round "
                         "while B shrinks (0: fixed alpha)")
    ap.add_argument("--loc-prec", choices=["f32", "f64"], default=None,
                    help="arithmetic of the location pair's fold and FFT, over the chosen plan's (default FP64: "
                         "the phase step 2 pi / n at n = 2^22 is near FP32 resolution)")
    ap.add_argument("--hash-split", type=int, default=None,
                    help="exact mode: workgroups per (signal, round) of the HashToBins pair launches (over the "
                         "chosen plan's)")
    ap.add_argument("--window", type=int, default=None,
                    help="flat window over the chosen plan's: 0 Gaussian (Section 7 construction), 1 Kaiser-Bessel "
                         "(the window length then follows Kaiser's rule unless --w is given)")
    ap.add_argument("--refine-shift", type=int, default=0,
                    help="exact mode: shift A of the multi-shift phase refinement (a third hashing per round; "
                         "0: off)")
    ap.add_argument("--refine-window", type=int, default=0,
                    help="half-width E of the refinement's candidate window (0: the library default)")
    ap.add_argument("--w", type=int, default=0)
    ap.add_argument("--plain-signals", type=int, default=8)
    ap.add_argument("--parity-signals", type=int, default=0,
                    help="signals the oracle runs and checks (0: every signal of the batch)")
    ap.add_argument("--cpu-procs", type=int, default=0,
                    help="oracle process pool size for the multi-core CPU baseline (0: the host's cores, at "
                         "most 16; 1: one process only)")
    ap.add_argument("--no-dense", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run one 1 GiB device-to-device tensor copy first (counter calibration)")
    ap.add_argument("--serve-requests", type=int, default=10000,
                    help="requests per serving phase (0: skip the serving measurement)")
    ap.add_argument("--serve-slots", type=int, default=32, help="signals per served batch")
    ap.add_argument("--serve-instances", type=int, default=2, help="resident plan instances per request shape")
    ap.add_argument("--serve-loads", default="0.25,0.5,0.75",
                    help="Poisson arrival rates as fractions of the measured serving capacity; the p50/p99 "
                         "reported at top level are the middle one's")
    ap.add_argument("--tune", choices=["off", "cache", "run"], default="cache",
                    help="plan parameters: off = the flags above; cache = the autotuner's stored choice for this "
                         "device and shape (from this library build if stored, else from another), measured now "
                         "when none is stored; run = measure now")
    ap.add_argument("--tune-budget", type=float, default=300.0, help="seconds of autotuner measurement at most")
    ap.add_argument("--tune-out", default="", help="also store the autotuner's choice in this JSON file")
    ap.add_argument("--tune-confirm", type=int, default=6,
                    help="fresh batches the fastest accepted candidates must also pass")
    ap.add_argument("--workload", choices=["c3", "c4", "section5", "gsched", "stream"], default="c3",
                    help="c3: the batched exactly-sparse headline; c4: the general-mode precision split; "
                         "section5: k-point DFTs through the n-point sFFT against a direct k-point FFT; "
                         "gsched: the general-mode round schedule against fixed B and w; stream: stream-mode "
                         "HashToBins against the gather at small n")
    ap.add_argument("--config-key", action="store_true",
                    help="print the key that names this configuration in the traffic record, then exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py: runs on one GPU only (--gpus 1); sharding over several GPUs is not built",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import siggen
    from paper_1201_2501_amd import sfft
    from paper_1201_2501_amd.sfft import Plan

    from paper_1201_2501_amd import autotune

    sfft.load()
    dev = torch.device("cuda:0")
    if args.workload == "c4":
        print(json.dumps(precision_split_bench(args, torch, dev, sfft, siggen)), flush=True)
        return
    if args.workload == "section5":
        print(json.dumps(section5_bench(args, torch, dev, sfft)), flush=True)
        return
    if args.workload == "gsched":
        print(json.dumps(general_schedule_bench(args, torch, dev, sfft, siggen)), flush=True)
        return
    if args.workload == "stream":
        print(json.dumps(stream_mode_bench(args, torch, dev, sfft, siggen)), flush=True)
        return
    n, k, S = 1 << args.log2n, args.k, args.signals
    loc_prec = sfft.SFFT_F32 if args.loc_prec == "f32" else sfft.SFFT_F64
    base_kw = dict(theta=0.02, loc_prec=loc_prec, rounds=args.rounds)

    # ---------------------------------------------------------- plan choice
    B, tuned, tune_rec = args.B, dict(delta=args.delta, b_min=args.b_min, patience=args.patience,
                                      hash_threads=args.hash_threads, alpha=args.alpha,
                                      stop_count=args.stop_count, stop_patience=args.stop_patience), None
    if args.tune != "off" and not args.w:
        res = None
        if args.tune == "cache":
            res = autotune.lookup(TUNE_FILE, n, k, sfft.SFFT_MODE_EXACT, S, sfft.SFFT_C64, autotune.device_tag(dev),
                                  any_build=True)
        if res is None and not args.config_key:
            t = time.time()
            cal_seeds = [2_000_003 + s for s in range(S)]
            Xc, sup_c, _ = siggen.torch_planted_batch(n, k, cal_seeds, dev, magnitude="loguniform")
            seeds_c = torch.arange(S, dtype=torch.int64, device=dev) * 104729 + 777
            torch.cuda.synchronize()
            log("autotune: calibration batch of %d signals (seeds 2000003..) ready in %.1fs" % (S, time.time() - t))
            confirm_batches = {}

            def confirm(i):
                # fresh batches of the same workload, kept in HBM while tuning
                if i not in confirm_batches:
                    gs = [3_000_003 + i * S + s for s in range(S)]
                    xb, sb, _ = siggen.torch_planted_batch(n, k, gs, dev, magnitude="loguniform")
                    confirm_batches[i] = (xb, torch.arange(S, dtype=torch.int64, device=dev) * 65537 +
                                          99991 * (i + 1), sb)
                return confirm_batches[i]

            # the stored choice for this device and shape (any build) joins
            # the search as an incumbent
            prev = autotune.lookup(TUNE_FILE, n, k, sfft.SFFT_MODE_EXACT, S, sfft.SFFT_C64,
                                   autotune.device_tag(dev), any_build=True)
            incumbents = [dict(prev.fields, B=prev.B)] if prev is not None else []
            if incumbents:
                log("autotune: incumbent %s" % ", ".join("%s=%s" % kv for kv in sorted(incumbents[0].items())))
            res = autotune.tune(Xc, k, sfft.SFFT_MODE_EXACT, seeds=seeds_c, truth=sup_c, base=base_kw,
                                budget_s=args.tune_budget, cache=args.tune_out or None, log=log, force=True,
                                confirm=confirm, confirm_batches=args.tune_confirm, incumbents=incumbents)
            del Xc
            confirm_batches.clear()
            torch.cuda.empty_cache()
            log("autotune: %d candidates in %.1fs" % (len(res.table), time.time() - t))
        if res is not None:
            B = res.B
            tuned = {f: v for f, v in res.fields.items() if f != "mode"}
            tune_rec = res.as_dict()
    window = args.window if args.window is not None else tuned.get("window", 0)
    w = args.w or sfft.sfft_window_w(n, B, tuned.get("alpha", 0.5), tuned.get("delta", 1e-9), window)
    plan_kw = dict(base_kw, **tuned, max_batch=S, flags=sfft.SFFT_FLAG_TIMING)
    if args.alpha_decay:
        plan_kw["alpha_decay"] = args.alpha_decay
    if args.hash_order is not None:
        plan_kw["hash_order"] = args.hash_order
    if args.loc_prec is not None:
        plan_kw["loc_prec"] = loc_prec
    if args.hash_split is not None:
        plan_kw["hash_split"] = args.hash_split
    plan_kw["window"] = window
    if args.refine_shift:
        plan_kw.update(refine_shift=args.refine_shift, refine_window=args.refine_window)
    log("plan: B=%d w=%d %s" % (B, w, ", ".join("%s=%s" % kv for kv in sorted(tuned.items()))))
    plan = Plan(n, k, B, w, 0, **plan_kw)
    desc = plan.desc
    # names the dominant launch for the counter record: its rounds (group 0)
    # and workgroup size set the gathered samples and the dispatch
    cfg_key = "n=2^%d,k=%d,B=%d,w=%d,b_min=%d,g0=%d,threads=%d,signals=%d" % (
        args.log2n, k, B, w, desc.b_min, plan.round_groups()[0], desc.hash_threads, S)
    if desc.alpha_decay:
        cfg_key += ",alpha_decay=%g" % desc.alpha_decay
    if desc.hash_order:
        cfg_key += ",order=%d" % desc.hash_order
    if desc.refine_shift:
        cfg_key += ",refine=%d" % desc.refine_shift
    if desc.hash_split > 1:
        cfg_key += ",split=%d" % desc.hash_split
    if desc.window:
        cfg_key += ",window=%d" % desc.window
    if desc.loc_prec == sfft.SFFT_F32:
        cfg_key += ",f32"
    if args.config_key:
        print(cfg_key)
        plan.close()
        return

    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)      # 1 GiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("copy calibration: 1073741824 bytes read and written")
        del src, dst

    # ---------------------------------------------------------------- inputs
    t = time.time()
    gen_seeds = [1_000_003 + s for s in range(S)]
    X, supports, values = siggen.torch_planted_batch(n, k, gen_seeds, dev, magnitude="loguniform")
    seeds = torch.arange(S, dtype=torch.int64, device=dev) * 7919 + 12345
    torch.cuda.synchronize()
    log("inputs ready: %d x 2^%d complex64 (%.1f GiB) in %.1fs" % (S, args.log2n, X.numel() * 8 / 2**30, time.time() - t))

    bufs = plan.batch_buffers(S, dev)
    # throughput plans: the same description without phase events (a
    # one-chunk step replays as one graph), one plan instance and stream per
    # batch in flight; step i runs on instance i mod inflight, so the
    # latency-bound decode of one batch overlaps the gathers of the next
    inflight = max(1, args.inflight)
    tplans = [Plan(n, k, B, w, 0, **dict(plan_kw, flags=0)) for _ in range(inflight)]
    tbufs = [tp.batch_buffers(S, dev) for tp in tplans]
    tstreams = [torch.cuda.Stream() for _ in range(inflight)]

    def throughput(m):
        """ms per step over K steps with m batches in flight, bracketed by a
        synchronisation on each side (GPU events on the current stream; with
        m > 1 the instance streams join it, with m = 1 the steps run on it)."""
        cur = torch.cuda.current_stream()
        streams = [cur] if m == 1 else tstreams[:m]
        for i in range(max(args.warmup, m)):
            tplans[i % m].execute_batch(X, seeds, stream=streams[i % m], bufs=tbufs[i % m])
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(cur)
        for st in streams:
            if st is not cur:
                st.wait_stream(cur)
        for i in range(args.steps):
            tplans[i % m].execute_batch(X, seeds, stream=streams[i % m], bufs=tbufs[i % m])
        for st in streams:
            if st is not cur:
                cur.wait_stream(st)
        e1.record(cur)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / args.steps

    # ---------------------------------------------------------------- batched
    by_inflight = {}
    for m in sorted({1, inflight}):
        by_inflight[m] = throughput(m)
        log("throughput with %d batch(es) in flight: %.3f ms/step, %.0f sFFTs/s"
            % (m, by_inflight[m], S / by_inflight[m] * 1e3))
    ms_per_step = by_inflight[inflight]
    elapsed_ms = ms_per_step * args.steps
    value = S * args.steps / (elapsed_ms / 1e3)
    # phases and per-step latency: K more steps on the plan with phase
    # events, each step waited for
    for _ in range(args.warmup):
        plan.execute_batch(X, seeds, bufs=bufs)
    torch.cuda.synchronize()
    h2b_ms, dec_ms, tail_ms, step_ms = [], [], [], []
    for _ in range(args.steps):
        plan.execute_batch(X, seeds, bufs=bufs)
        torch.cuda.synchronize()
        tm = plan.timings()
        h2b_ms.append(tm[0])
        dec_ms.append(tm[1])
        tail_ms.append(tm[2])
        step_ms.append(tm[3])
        chunks = int(tm[4])
    log("batched: %.3f ms/step, %.0f sFFTs/s; steps waited for one by one: %.3f ms (hash %.3f ms, decode %.3f ms "
        "overlapped, tail %.3f ms, %d chunks)" % (ms_per_step, value, np.mean(step_ms), np.mean(h2b_ms),
                                                   np.mean(dec_ms), np.mean(tail_ms), chunks))
    same = all(torch.equal(tb[f], bufs[f]) for tb in tbufs for f in ("idx", "val", "counts"))
    log("throughput and phase plans give identical outputs: %s" % same)
    if not same:
        raise SystemExit("the throughput plans' outputs differ from the phase plan's")
    for tp in tplans:
        tp.close()
    del tbufs, tplans

    counts = bufs["counts"].cpu().numpy()
    info = bufs["info"].cpu().numpy()
    idx_all = bufs["idx"].cpu().numpy()
    val_all = bufs["val"].cpu().numpy()
    exact_vs_planted = int(sum(np.array_equal(idx_all[s, :counts[s]], supports[s]) for s in range(S)))

    # recovery over fresh batches of the same workload (untimed)
    extra = None
    if args.extra_batches > 0:
        ok_x, n_x, miss_x = 0, 0, []
        for i in range(args.extra_batches):
            gs = [5_000_003 + i * S + s for s in range(S)]
            Xe, sup_e, _ = siggen.torch_planted_batch(n, k, gs, dev, magnitude="loguniform")
            seeds_e = torch.arange(S, dtype=torch.int64, device=dev) * 6151 + 4099 * (i + 1)
            be = plan.execute_batch(Xe, seeds_e, bufs=bufs)
            torch.cuda.synchronize()
            ce = be["counts"].cpu().numpy()
            ie = be["idx"].cpu().numpy()
            for s in range(S):
                good = np.array_equal(ie[s, :ce[s]], sup_e[s])
                ok_x += int(good)
                if not good and len(miss_x) < 8:
                    miss_x.append({"batch": i, "signal": s, "count": int(ce[s]),
                                   "missing": len(set(sup_e[s].tolist()) - set(ie[s, :ce[s]].tolist()))})
            n_x += S
            del Xe
        torch.cuda.empty_cache()
        extra = {"batches": args.extra_batches, "recovered_exactly_vs_planted": "%d/%d" % (ok_x, n_x),
                 "misses": miss_x, "generator_seeds": "5000003 + %d i + s" % S}
        log("extra batches: %d/%d supports exact" % (ok_x, n_x))

    # roofline of the dominant kernel: the first HashToBins pair launch of a
    # chunk (round group 0, hashed for every signal; later groups only for
    # signals still decoding)
    groups = plan.round_groups()
    rounds_used = info[:, 0].astype(np.int64)
    hashed = np.array([next(e for e in groups if e >= max(int(r), 1)) for r in rounds_used])
    per_launch = S // chunks
    alg_bytes = plan.h2b_bytes(per_launch)
    h2b_avg = float(np.mean(h2b_ms)) / chunks
    achieved = alg_bytes / (h2b_avg * 1e-3) / 1e9
    traffic = load_traffic(per_launch, cfg_key)
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                "kernel": "k_h2b_pair", "launch": "rounds 0..%d of every signal" % (groups[0] - 1),
                "signals_per_launch": per_launch, "alg_bytes_per_launch": alg_bytes,
                "avg_launch_ms": round(h2b_avg, 4)}
    hbm = {"algorithmic_GBps": round(achieved, 1),
           "counter_GBps": None if traffic is None else round(traffic / (h2b_avg * 1e-3) / 1e9, 1)}
    phases = {"hash_ms": round(float(np.mean(h2b_ms)), 4), "decode_ms_overlapped": round(float(np.mean(dec_ms)), 4),
              "tail_ms": round(float(np.mean(tail_ms)), 4), "chunks": chunks}

    # ---------------------------------------------------------------- plain
    plain = None
    if args.plain_signals > 0 and not desc.refine_shift:   # the plain path has no refinement hashing
        pplan = Plan(n, k, B, w, int(seeds[0].item()), **{**plan_kw, "max_batch": 1})
        pplan.execute(X[0])                       # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        for s in range(args.plain_signals):
            pidx, pval, pinfo, _ = pplan.execute(X[s])
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        pidx0, pval0, _, _ = pplan.execute(X[0])
        same = bool(np.array_equal(pidx0, idx_all[0, :counts[0]]) and
                    np.allclose(pval0, val_all[0, :counts[0]], rtol=1e-9, atol=1e-12))
        plain = {"value": round(args.plain_signals / dt, 1), "unit": "sFFTs/s", "signals": args.plain_signals,
                 "ms_per_signal": round(1e3 * dt / args.plain_signals, 3), "matches_batched_signal0": same}
        pplan.close()
        log("plain: %.1f sFFTs/s" % plain["value"])

    # ---------------------------------------------------------------- dense
    dense = None
    if not args.no_dense:
        chunk = 64
        def dense_pass():
            for c0 in range(0, S, chunk):
                F = torch.fft.fft(X[c0:c0 + chunk], dim=-1, norm="ortho")
                torch.topk(F.abs(), k, dim=-1)
        dense_pass()
        torch.cuda.synchronize()
        d0, d1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        d0.record()
        dense_pass()
        d1.record()
        torch.cuda.synchronize()
        dms = d0.elapsed_time(d1)
        dense = {"value": round(S / (dms / 1e3), 1), "unit": "sFFTs/s", "ms_per_batch": round(dms, 3),
                 "what": "torch.fft.fft (rocFFT) full length + torch.topk, complex64, same batch"}
        log("dense: %.1f signals/s" % dense["value"])

    # -------------------------------------------- oracle: parity + cpu baseline
    parity, cpu_baseline = None, None
    if not args.no_cpu:
        from oracle.exact import noiseless_sparse_fft
        nchk = S if args.parity_signals <= 0 else min(S, args.parity_signals)
        shm = None
        if args.cpu_procs != 1:
            shm = tempfile.NamedTemporaryFile(prefix="sfft_oracle_", suffix=".c64", dir="/dev/shm"
                                              if os.path.isdir("/dev/shm") else None, delete=False)
            shm.close()
            mm = np.memmap(shm.name, dtype=np.complex64, mode="w+", shape=(nchk, n))
        try:
            mism, max_rel, l2, t_cpu = 0, 0.0, [], 0.0
            seed_list = [int(seeds[s].item()) for s in range(nchk)]
            for s in range(nchk):
                x = X[s].cpu().numpy()
                if shm is not None:
                    mm[s] = x
                t = time.perf_counter()
                ref = noiseless_sparse_fft(x, oracle_params(desc, seed_list[s]))
                t_cpu += time.perf_counter() - t
                c = counts[s]
                if not np.array_equal(idx_all[s, :c], ref.indices):
                    mism += 1
                else:
                    rel = np.abs(val_all[s, :c] - ref.values) / np.maximum(np.abs(ref.values), 1e-300)
                    max_rel = max(max_rel, float(rel.max()) if c else 0.0)
                est = dict(zip(idx_all[s, :c].tolist(), val_all[s, :c]))
                sup_set = set(supports[s].tolist())
                err = math.sqrt(sum(abs(est.get(int(i), 0) - v) ** 2 for i, v in zip(supports[s], values[s])) +
                                sum(abs(v) ** 2 for i, v in est.items() if i not in sup_set))
                l2.append(err / float(np.linalg.norm(values[s])))
                if (s + 1) % 128 == 0:
                    log("oracle: %d of %d signals checked, %d mismatches" % (s + 1, nchk, mism))
            # FP64 bins match the FP64 oracle to rounding; FP32 bins (loc_prec f32)
            # carry their own rounding into the values
            parity = {"signals_checked": nchk, "support_mismatches": mism, "max_rel_err": max_rel,
                      "tolerance": 1e-10 if desc.loc_prec == sfft.SFFT_F64 else 1e-4,
                      "l2_rel_err_vs_planted_max": max(l2)}
            one = {"value": round(nchk / t_cpu, 3), "unit": "sFFTs/s", "cores": 1, "seconds": round(t_cpu, 2)}
            log("oracle: %d signals in %.1fs on one core, parity mismatches %d of %d" % (nchk, t_cpu, mism, nchk))
            cpu_baseline = {**one, "kind": "oracle",
                            "sample": "%d signals of the same workload, FP64 numpy oracle, one process" % nchk}
            if shm is not None:
                mm.flush()
                procs = args.cpu_procs if args.cpu_procs > 0 else host_cores()
                rate, wall = oracle_pool_rate(shm.name, nchk, n, desc, seed_list, procs)
                log("oracle: %d signals in %.1fs on %d processes" % (nchk, wall, procs))
                cpu_baseline = {"value": round(rate, 3), "unit": "sFFTs/s", "cores": procs, "kind": "oracle",
                                "sample": "%d signals of the same workload, FP64 numpy oracle, a pool of %d "
                                          "processes (one thread each)" % (nchk, procs),
                                "single_core": one}
        finally:
            if shm is not None:
                del mm
                os.unlink(shm.name)

    # ---------------------------------------------------------------- serving
    serving = None
    if args.serve_requests > 0:
        plan.close()
        del X, bufs
        torch.cuda.empty_cache()
        serving = serving_bench(args, torch, dev, sfft)

    out = {
        "metric": METRIC,
        "value": round(value, 1),
        "unit": "sFFTs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if desc.loc_prec == sfft.SFFT_F64 else "f32",
        "data": "synthetic",
        "config": {"workload": "batched exactly-sparse sFFT: %d signals, n=2^%d, k=%d, complex64, log-uniform "
                               "|c| in [0.1,10], per-signal seeds" % (S, args.log2n, k),
                   "signals": S, "n": n, "k": k, "B": B, "w": w, "rounds": desc.rounds,
                   "b_min": desc.b_min or max(2, B >> 4), "patience": desc.patience, "delta": desc.delta,
                   "alpha": desc.alpha, "theta": desc.theta, "g_min": desc.g_min,
                   "stop_count": desc.stop_count, "stop_patience": desc.stop_patience, "ratio_tol": desc.ratio_tol,
                   "alpha_decay": desc.alpha_decay, "samples_per_signal_group0": sfft.sfft_plan_samples(desc),
                   "hash_threads": desc.hash_threads, "hash_order": desc.hash_order,
                   "hash_split": desc.hash_split, "window": ["gaussian", "kaiser-bessel"][desc.window],
                   "inflight": inflight,
                   "chunks": chunks,
                   "loc_prec": "f64" if desc.loc_prec == sfft.SFFT_F64 else "f32",
                   "refine_shift": desc.refine_shift, "refine_window": desc.refine_window,
                   "input": "complex64"},
        "autotune": tune_rec,
        "throughput_by_inflight": {str(m): {"ms_per_step": round(t, 4), "sFFTs_per_s": round(S / t * 1e3, 1)}
                                   for m, t in by_inflight.items()},
        "latency_ms": {"p10": round(percentile(step_ms, 10), 4), "p50": round(percentile(step_ms, 50), 4),
                       "p90": round(percentile(step_ms, 90), 4), "p99": round(percentile(step_ms, 99), 4),
                       "steps": len(step_ms),
                       "what": "per batch step waited for alone (graph replays with phase events), HIP events"},
        "phases": phases,
        "plain": plain,
        "dense": dense,
        "hbm": hbm,
        "recovered_exactly_vs_planted": "%d/%d" % (exact_vs_planted, S),
        "fresh_batches": extra,
        "rounds_used_max": int(info[:, 0].max()),
        "rounds": {"groups": groups, "used_p50": float(np.median(rounds_used)),
                   "used_hist": {int(r): int(c) for r, c in zip(*np.unique(rounds_used, return_counts=True))},
                   "hashed_mean": round(float(hashed.mean()), 3)},
        "parity": parity,
        "roofline": roofline,
        "cpu_baseline": cpu_baseline,
        "serving": serving,
    }
    print(json.dumps(out), flush=True)
    plan.close()


if __name__ == "__main__":
    main()
