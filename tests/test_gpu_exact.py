"""GPU parity of the exact-mode hot path against the FP64 oracle.

Bars: raw bins within 1e-12 (FP64 arithmetic) / 1e-5 (FP32) of the oracle's,
relative to the bins' RMS (stream-mode and refinement bins: 1e-12 / 2e-5 of
the largest bin); recovered supports bit-exact; values within
1e-10 (FP64) relative to the coefficient magnitude.  Every case prints its
name, shape and seed before touching the GPU.
"""
import numpy as np
import pytest

import siggen
from oracle.exact import noiseless_sparse_fft
from oracle.hashing import hash_to_bins_raw
from oracle.params import SfftParams
from oracle.window import default_w, window_time

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    from paper_1201_2501_amd import sfft
    sfft.load()
    return torch, torch.device("cuda:0")


def plan_for(n, k, B, w, seed, **kw):
    from paper_1201_2501_amd.sfft import Plan
    return Plan(n, k, B, w, seed, **kw)


def oracle_params(plan, seed=None):
    d = plan.desc
    return SfftParams(n=d.n, k=d.k, B=d.B, w=d.w, seed=d.seed if seed is None else seed, alpha=d.alpha,
                      delta=d.delta, theta=d.theta, g_min=d.g_min, rounds=d.rounds, b_min=d.b_min,
                      patience=d.patience, stop_count=d.stop_count, stop_patience=d.stop_patience,
                      ratio_tol=d.ratio_tol, alpha_decay=d.alpha_decay, cap=d.cap, refine_shift=d.refine_shift,
                      refine_window=d.refine_window or 16, window=d.window)


RAW_CASES = [
    # (name, n, B, dtype, prec, beta, B_r)
    ("c1-pair", 1 << 14, 64, np.complex128, 1, 1, 64),
    ("c1-pair-B16", 1 << 14, 64, np.complex128, 1, 1, 16),
    ("c3-pair-f64", 1 << 22, 1024, np.complex64, 1, 1, 1024),
    ("c3-pair-f32", 1 << 22, 1024, np.complex64, 0, 1, 1024),
    ("c3-small-round", 1 << 22, 1024, np.complex64, 1, 1, 64),
    ("beta-inside", 1 << 18, 512, np.complex64, 1, 777, 512),
    ("beta-beyond-w", 1 << 18, 512, np.complex64, 1, 100003, 512),
]


@pytest.mark.parametrize("name,n,B,dtype,prec,beta,B_r", RAW_CASES)
def test_raw_bins_match_oracle(torch_dev, name, n, B, dtype, prec, beta, B_r):
    torch, dev = torch_dev
    delta = 1e-12 if dtype == np.complex128 else 1e-9
    w = default_w(n, B, 0.5, delta)
    x, sup, val = siggen.planted_signal(n, 40, 11, dtype, noise_ratio=0.01)
    in_dtype = 1 if dtype == np.complex128 else 0
    say(name, "n", n, "B", B, "B_r", B_r, "w", w, "prec", prec, "beta", beta)
    plan = plan_for(n, 40, B, w, 5, delta=delta, in_dtype=in_dtype, loc_prec=prec, b_min=16)
    xd = torch.from_numpy(x).to(dev)
    rng = np.random.default_rng(hash(name) % 1000)
    sigma = int(rng.integers(0, n // 2)) * 2 + 1
    a = int(rng.integers(0, n))
    b = int(rng.integers(0, n))
    u0, u1 = plan.hash_pair_raw(xd, sigma, a, beta, b, B_r, prec)
    torch.cuda.synchronize()
    u0 = u0.cpu().numpy()
    u1 = u1.cpu().numpy()
    G = window_time(n, B_r, w * B_r // B, 0.5, delta)
    e0 = hash_to_bins_raw(x, sigma, a, b, B_r, G)
    e1 = hash_to_bins_raw(x, sigma, (a + beta) % n, b, B_r, G)
    # relative to the bins' RMS: 1e-12 for FP64 folds, 1e-5 for FP32 (measured
    # at n = 2^22: 4e-15 and 9.4e-7)
    tol = 1e-12 if prec == 1 else 1e-5
    rms = np.sqrt(np.mean(np.abs(np.concatenate([e0, e1])) ** 2))
    err = max(np.max(np.abs(u0 - e0)), np.max(np.abs(u1 - e1)))
    print("raw-bin error", name, "of rms", err / rms, flush=True)
    assert err <= tol * rms
    plan.close()


def c1_case(seed):
    n, k, B = 1 << 14, 16, 64
    return n, k, B, default_w(n, B, 0.5, 1e-12)


def compare(res_idx, res_val, ref, rel=1e-10):
    assert np.array_equal(res_idx, ref.indices), (res_idx, ref.indices, ref.margins)
    mag = np.maximum(np.abs(ref.values), 1e-300)
    assert np.all(np.abs(res_val - ref.values) <= rel * mag + 1e-14)


@pytest.mark.parametrize("seed", range(4))
def test_plain_exact_c1_matches_oracle(torch_dev, seed):
    torch, dev = torch_dev
    n, k, B, w = c1_case(seed)
    say("plain-c1", "n", n, "k", k, "seed", seed)
    plan = plan_for(n, k, B, w, seed, delta=1e-12, in_dtype=1, loc_prec=1)
    x, sup, val = siggen.planted_signal(n, k, 100 + seed, np.complex128)
    idx, v, info, st = plan.execute(torch.from_numpy(x).to(dev))
    ref = noiseless_sparse_fft(x, oracle_params(plan))
    assert int(info[0]) == ref.rounds_used
    compare(idx, v, ref)
    assert np.array_equal(idx, sup)
    plan.close()


def run_batch(torch, dev, plan, xs, seeds):
    X = torch.from_numpy(np.stack(xs)).to(dev)
    S = torch.tensor(seeds, dtype=torch.int64, device=dev)
    bufs = plan.execute_batch(X, S)
    torch.cuda.synchronize()
    out = []
    for r in range(len(xs)):
        c = int(bufs["counts"][r])
        out.append((bufs["idx"][r, :c].cpu().numpy(), bufs["val"][r, :c].cpu().numpy(),
                    bufs["info"][r].cpu().numpy()))
    return out


def test_batched_exact_c1_matches_oracle_per_seed(torch_dev):
    torch, dev = torch_dev
    n, k, B, w = c1_case(0)
    count = 8
    say("batched-c1", "n", n, "count", count)
    plan = plan_for(n, k, B, w, 0, delta=1e-12, in_dtype=1, loc_prec=1, max_batch=count)
    xs, seeds = [], []
    for s in range(count):
        x, _, _ = siggen.planted_signal(n, k, 200 + s, np.complex128)
        xs.append(x)
        seeds.append(1000 + 17 * s)
    out = run_batch(torch, dev, plan, xs, seeds)
    for s in range(count):
        ref = noiseless_sparse_fft(xs[s], oracle_params(plan, seeds[s]))
        assert int(out[s][2][0]) == ref.rounds_used
        compare(out[s][0], out[s][1], ref)
    plan.close()


def test_graph_replays_are_identical_and_batch_independent(torch_dev):
    torch, dev = torch_dev
    n, k, B, w = c1_case(0)
    count = 6
    say("graph-replay", "n", n, "count", count)
    plan = plan_for(n, k, B, w, 0, delta=1e-12, in_dtype=1, loc_prec=1, max_batch=count)
    xs = [siggen.planted_signal(n, k, 300 + s, np.complex128)[0] for s in range(count)]
    seeds = [5 + s for s in range(count)]
    X = torch.from_numpy(np.stack(xs)).to(dev)
    S = torch.tensor(seeds, dtype=torch.int64, device=dev)
    first = None
    for rep in range(3):
        bufs = plan.execute_batch(X, S)
        torch.cuda.synchronize()
        snap = {key: t.clone() for key, t in bufs.items()}
        _ = (X.abs() * 2).sum().item()          # eager work between replays
        if first is None:
            first = snap
        else:
            for key in snap:
                assert torch.equal(snap[key], first[key]), key
    # the same signal alone (different batch) gives the same answer
    alone = plan_for(n, k, B, w, 0, delta=1e-12, in_dtype=1, loc_prec=1, max_batch=1)
    for s in (0, 3):
        o = run_batch(torch, dev, alone, [xs[s]], [seeds[s]])[0]
        c = int(first["counts"][s])
        assert np.array_equal(o[0], first["idx"][s, :c].cpu().numpy())
        assert np.allclose(o[1], first["val"][s, :c].cpu().numpy(), rtol=1e-12, atol=0)
    plan.close()
    alone.close()


@pytest.mark.parametrize("shape", ["c1", "c3"])
def test_graph_replays_match_eager_launches(torch_dev, shape, monkeypatch):
    """Every replay of the captured step (one graph without phase events,
    the hash and decode graphs with them) equals the same step launched
    kernel by kernel (SFFT_NO_GRAPH=1), with eager work and synchronisations
    between the replays."""
    from paper_1201_2501_amd import sfft

    torch, dev = torch_dev
    if shape == "c1":
        n, k, B, w = c1_case(0)
        count, kw = 6, dict(delta=1e-12, in_dtype=1, loc_prec=1)
        xs = [siggen.planted_signal(n, k, 400 + s, np.complex128)[0] for s in range(count)]
        X = torch.from_numpy(np.stack(xs)).to(dev)
    else:
        n, k, B, count = 1 << 22, 256, 1024, 4
        kw = dict(delta=1e-7, alpha=0.7, window=1, theta=0.02, b_min=64, patience=4, ratio_tol=0.002,
                  g_min=0.25, stop_count=256, stop_patience=3, group_step=3)
        w = 0
        X, _, _ = siggen.torch_planted_batch(n, k, [600 + s for s in range(count)], dev, magnitude="loguniform")
    say("graph-vs-eager", shape, "n", n, "count", count)
    S = torch.tensor([11 + s for s in range(count)], dtype=torch.int64, device=dev)
    monkeypatch.setenv("SFFT_NO_GRAPH", "1")
    eager_plan = plan_for(n, k, B, w, 0, max_batch=count, **kw)
    b = eager_plan.execute_batch(X, S)
    torch.cuda.synchronize()
    want = {key: t.clone() for key, t in b.items()}
    monkeypatch.delenv("SFFT_NO_GRAPH")
    for flags in (0, sfft.SFFT_FLAG_TIMING):
        plan = plan_for(n, k, B, w, 0, max_batch=count, flags=flags, **kw)
        for rep in range(4):
            b = plan.execute_batch(X, S)
            torch.cuda.synchronize()
            for key in want:
                assert torch.equal(b[key], want[key]), (flags, rep, key)
            _ = (X.abs() * 2).sum().item()       # eager work between replays
            b["idx"].zero_()                     # the next replay rewrites every output
        plan.close()
    eager_plan.close()


def test_plans_on_several_streams_match_one_plan(torch_dev):
    """Several batches in flight (one plan instance and stream each, calls
    queued without waiting, the way the throughput measurement runs them)
    give, call by call, the results of one plan running the batches in turn."""
    torch, dev = torch_dev
    n, k, B, w = c1_case(0)
    count, m, calls = 6, 3, 9
    say("streams-in-flight", "n", n, "count", count, "plans", m)
    kw = dict(delta=1e-12, in_dtype=1, loc_prec=1, max_batch=count)
    batches = []
    for c in range(calls):
        xs = [siggen.planted_signal(n, k, 1300 + 10 * c + s, np.complex128)[0] for s in range(count)]
        batches.append((torch.from_numpy(np.stack(xs)).to(dev),
                        torch.tensor([71 * c + s for s in range(count)], dtype=torch.int64, device=dev)))
    ref_plan = plan_for(n, k, B, w, 0, **kw)
    want = []
    for X, S in batches:
        b = ref_plan.execute_batch(X, S)
        torch.cuda.synchronize()
        want.append({key: t.clone() for key, t in b.items()})
    plans = [plan_for(n, k, B, w, 0, **kw) for _ in range(m)]
    streams = [torch.cuda.Stream() for _ in range(m)]
    # one output set per call (batch_buffers keeps one set per plan), so that
    # no call waits for another's results
    def out_set(plan):
        return dict(idx=torch.zeros((count, plan.cap), dtype=torch.int64, device=dev),
                    val=torch.zeros((count, plan.cap), dtype=torch.complex128, device=dev),
                    counts=torch.zeros(count, dtype=torch.int32, device=dev),
                    info=torch.zeros((count, 4), dtype=torch.int32, device=dev))
    outs = [out_set(plans[c % m]) for c in range(calls)]
    cur = torch.cuda.current_stream()
    for st in streams:
        st.wait_stream(cur)
    for c, (X, S) in enumerate(batches):
        plans[c % m].execute_batch(X, S, stream=streams[c % m], bufs=outs[c])
    torch.cuda.synchronize()
    for c in range(calls):
        for key in ("idx", "val", "counts", "info"):
            assert torch.equal(outs[c][key], want[c][key]), (c, key)
    for p in plans + [ref_plan]:
        p.close()


def test_plain_and_batched_agree(torch_dev):
    torch, dev = torch_dev
    n, k, B, w = c1_case(0)
    say("plain-vs-batched", "n", n)
    plan = plan_for(n, k, B, w, 42, delta=1e-12, in_dtype=1, loc_prec=1, max_batch=2)
    x, _, _ = siggen.planted_signal(n, k, 77, np.complex128)
    idx, v, info, st = plan.execute(torch.from_numpy(x).to(dev))
    o = run_batch(torch, dev, plan, [x, x], [42, 42])
    for r in range(2):
        assert np.array_equal(o[r][0], idx)
        assert np.allclose(o[r][1], v, rtol=1e-11, atol=1e-14)


def test_zero_signal_and_truncation(torch_dev):
    torch, dev = torch_dev
    n, k, B, w = c1_case(0)
    say("edge-zero-trunc", "n", n)
    plan = plan_for(n, 4, B, w, 3, delta=1e-12, in_dtype=1, loc_prec=1)
    idx, v, info, st = plan.execute(torch.zeros(n, dtype=torch.complex128, device=dev))
    assert len(idx) == 0 and int(info[0]) == plan.desc.patience
    # 12 planted coefficients with cap 4: the 4 largest are returned, flagged
    sup, val = siggen.planted_spectrum(n, 12, 9, magnitude="loguniform")
    x = siggen.time_signal(n, sup, val)
    idx, v, info, st = plan.execute(torch.from_numpy(x).to(dev))
    ref = noiseless_sparse_fft(x, oracle_params(plan))
    assert ref.truncated and (int(info[1]) & 1) == 1
    assert st == 6    # SFFT_ETRUNC
    compare(idx, v, ref)


@pytest.mark.parametrize("seed,sched", [(0, "default"), (1, "default"), (2, "tuned"), (3, "tuned"), (4, "alpha0.6"),
                                        (5, "alpha0.6"), (6, "stopk"), (7, "stopk"), (8, "lowtheta"),
                                        (9, "lowtheta"), (10, "alpha0.7"), (11, "alpha0.7"), (12, "ratio"),
                                        (13, "ratio")])
def test_c3_shape_matches_oracle(torch_dev, seed, sched):
    """n = 2^22, k = 256, log-uniform magnitudes, complex64, FP64 location
    decoding; the default schedule (b_min = B/16, 16 rounds), b_min = 32 with
    24 rounds, a shorter window (alpha = 0.6, delta = 1e-8, b_min = 64,
    patience 4), the same with the stop at k found entries, and with a lower
    bin threshold and window floor (theta = 0.01, g_min = 0.25), on a few
    signals."""
    torch, dev = torch_dev
    n, k, B = 1 << 22, 256, 1024
    alpha, delta = {"alpha0.6": (0.6, 1e-8), "stopk": (0.6, 1e-8), "lowtheta": (0.6, 1e-8),
                    "alpha0.7": (0.7, 1e-7), "ratio": (0.6, 1e-7)}.get(sched, (0.5, 1e-9))
    w = default_w(n, B, alpha, delta)
    kw = {"default": {}, "tuned": dict(b_min=32, rounds=24),
          "alpha0.6": dict(alpha=0.6, b_min=64, patience=4, rounds=24),
          "stopk": dict(alpha=0.6, b_min=64, patience=5, rounds=24, stop_count=k, stop_patience=2 + seed % 2),
          "lowtheta": dict(alpha=0.6, b_min=64, patience=4, rounds=24, theta=0.01, g_min=0.25),
          "alpha0.7": dict(alpha=0.7, b_min=64, patience=4, rounds=24, theta=0.01, g_min=0.25, stop_count=k,
                           stop_patience=3),
          "ratio": dict(alpha=0.6, b_min=64, patience=4, rounds=24, g_min=0.25, ratio_tol=0.01, stop_count=k,
                        stop_patience=3)}[sched]
    theta = kw.pop("theta", 0.02)
    say("c3-shape", sched, "n", n, "k", k, "B", B, "w", w, "seed", seed)
    plan = plan_for(n, k, B, w, 0, delta=delta, theta=theta, loc_prec=1, max_batch=2, **kw)
    if sched == "tuned":
        assert plan.round_groups() == [9, 11, 13, 17, 24]
    xs, sups, seeds = [], [], []
    for s in range(2):
        x, sup, val = siggen.planted_signal(n, k, 300 + 2 * seed + s, np.complex64, magnitude="loguniform")
        xs.append(x)
        sups.append(sup)
        seeds.append(10 * seed + s)
    out = run_batch(torch, dev, plan, xs, seeds)
    for s in range(2):
        ref = noiseless_sparse_fft(xs[s], oracle_params(plan, seeds[s]))
        assert int(out[s][2][0]) == ref.rounds_used
        compare(out[s][0], out[s][1], ref)
        assert np.array_equal(out[s][0], sups[s])
    plan.close()


@pytest.mark.parametrize("threads,chunks,group0,step,order", [(512, 1, 0, 0, 0), (1024, 1, 0, 0, 0), (256, 2, 0, 0, 0),
                                                             (1024, 2, 0, 0, 0), (256, 1, 6, 0, 0), (512, 1, 12, 0, 0),
                                                             (256, 1, 0, 4, 0), (256, 1, 0, 0, 1), (256, 1, 12, 3, 2),
                                                             (512, 2, 0, 0, 2)])
def test_c3_launch_shapes_match_oracle(torch_dev, threads, chunks, group0, step, order):
    """The launch shape the autotuner picks from (HashToBins workgroup size,
    batch chunks, size of the first round group, workgroup order) leaves
    supports and rounds unchanged and values within the FP64 bar: with
    B_r < threads a bin's partial sums are only added in another order."""
    torch, dev = torch_dev
    n, k, B = 1 << 22, 256, 1024
    w = default_w(n, B, 0.5, 1e-9)
    count = 8 if order == 2 else 4       # a multiple of 8: the per-XCD order applies
    say("c3-launch-shape", "threads", threads, "chunks", chunks, "group0", group0, "order", order, "count", count)
    plan = plan_for(n, k, B, w, 0, delta=1e-9, theta=0.02, loc_prec=1, max_batch=count, b_min=32, rounds=24,
                    hash_threads=threads, chunks=chunks, group0=group0, group_step=step, hash_order=order,
                    flags=2)     # SFFT_FLAG_TIMING: chunk count
    assert plan.desc.hash_threads == threads and plan.desc.chunks == chunks and plan.desc.hash_order == order
    g0 = group0 or 9
    assert plan.round_groups() == ([g0, 13, 21, 24] if step == 4 else [g0, 15, 21, 24] if step == 3 else
                                   plan.round_groups())
    assert plan.round_groups()[0] == g0
    xs, sups, seeds = [], [], []
    for s in range(count):
        x, sup, _ = siggen.planted_signal(n, k, 4000 + s, np.complex64, magnitude="loguniform")
        xs.append(x)
        sups.append(sup)
        seeds.append(31 * s + 7)
    out = run_batch(torch, dev, plan, xs, seeds)
    assert plan.timings()[4] == chunks
    for s in range(count):
        ref = noiseless_sparse_fft(xs[s], oracle_params(plan, seeds[s]))
        assert int(out[s][2][0]) == ref.rounds_used
        compare(out[s][0], out[s][1], ref)
        assert np.array_equal(out[s][0], sups[s])
    plan.close()


@pytest.mark.parametrize("b_min", [1024, 4096])
def test_large_k_finish_matches_oracle(torch_dev, b_min):
    """k = 2048 gives 8192 zhat entries, more than the per-round
    re-estimation blocks hold in LDS: the re-estimation runs as one
    workgroup per signal over its rounds, with the same results."""
    torch, dev = torch_dev
    n, k, B = 1 << 20, 2048, 4096
    w = default_w(n, B, 0.5, 1e-9)
    say("large-k-finish", "n", n, "k", k, "B", B, "b_min", b_min)
    plan = plan_for(n, k, B, w, 0, delta=1e-9, theta=0.25, loc_prec=1, max_batch=2, b_min=b_min, rounds=24)
    xs, sups = [], []
    for s in range(2):
        x, sup, _ = siggen.planted_signal(n, k, 5 + s, np.complex64, magnitude="unit")
        xs.append(x)
        sups.append(sup)
    seeds = [3, 4]
    out = run_batch(torch, dev, plan, xs, seeds)
    for s in range(2):
        ref = noiseless_sparse_fft(xs[s], oracle_params(plan, seeds[s]))
        assert int(out[s][2][0]) == ref.rounds_used
        compare(out[s][0], out[s][1], ref)
    plan.close()


def test_c3_round_groups_skip_only_undecoded_rounds(torch_dev):
    """The batched exact path hashes round group 0 for every signal and each
    later group only for signals still decoding: a batch whose signals stop
    in different groups still matches the oracle signal by signal."""
    torch, dev = torch_dev
    n, k, B = 1 << 22, 256, 1024
    w = default_w(n, B, 0.5, 1e-9)
    count = 6
    say("c3-round-groups", "n", n, "k", k, "count", count)
    plan = plan_for(n, k, B, w, 0, delta=1e-9, theta=0.02, loc_prec=1, max_batch=count)
    # the schedule 1024, 512, 256, 128, 64, 64, ... reaches b_min at round 4;
    # patience 3 => group 0 ends at round 8, then groups of 2, 2, 4 rounds
    assert plan.round_groups() == [8, 10, 12, 16]
    xs = [siggen.planted_signal(n, k, 1_000_003 + s, np.complex64, magnitude="loguniform")[0]
          for s in range(count)]
    seeds = [s * 7919 + 12345 for s in range(count)]
    out = run_batch(torch, dev, plan, xs, seeds)
    used = []
    for s in range(count):
        ref = noiseless_sparse_fft(xs[s], oracle_params(plan, seeds[s]))
        assert int(out[s][2][0]) == ref.rounds_used
        compare(out[s][0], out[s][1], ref)
        used.append(ref.rounds_used)
    assert len({next(e for e in [8, 10, 12, 16] if e >= r) for r in used}) >= 2, used
    plan.close()


@pytest.mark.parametrize("n,k,B", [(1 << 18, 64, 256), (1 << 20, 256, 1024)])
def test_section5_reduction_k_point_dft(torch_dev, n, k, B):
    """Section 5: the k-point DFT of x_k through the n-point exact sFFT of its
    periodic extension y_t = x_{t mod k}, whose spectrum is sqrt(n/k) x_k-hat
    on the multiples of n/k.  The lattice support puts every coefficient at
    the same offset within its bin in a round (all decoded or none), a
    structured case of the method: batched GPU = oracle, and = a direct
    k-point DFT."""
    torch, dev = torch_dev
    count = 3
    say("section5", "n", n, "k", k, "B", B, "count", count)
    ys, xks = zip(*[siggen.periodic_signal(n, k, 40 + s) for s in range(count)])
    expect_idx = np.arange(k) * (n // k)
    w = default_w(n, B, 0.5, 1e-12)
    theta = 0.05 * min(np.min(np.abs(np.fft.fft(xk) / np.sqrt(k) * np.sqrt(n / k))) for xk in xks)
    # all coefficients vanish together when the shared offset falls where G'
    # is near 0 (about 22% of offsets at alpha = 1/2): patience 6 makes an
    # empty stop at the start (0.22^6) negligible
    plan = plan_for(n, k, B, w, 0, delta=1e-12, theta=theta, in_dtype=1, loc_prec=1, max_batch=count, patience=6)
    seeds = [3 + s for s in range(count)]
    out = run_batch(torch, dev, plan, list(ys), seeds)
    for s in range(count):
        ref = noiseless_sparse_fft(ys[s], oracle_params(plan, seeds[s]))
        compare(out[s][0], out[s][1], ref)
        expect_val = np.sqrt(n / k) * np.fft.fft(xks[s]) / np.sqrt(k)
        assert np.array_equal(out[s][0], expect_idx)
        assert np.max(np.abs(out[s][1] - expect_val)) <= 1e-9 * np.max(np.abs(expect_val))
    plan.close()


@pytest.mark.parametrize("B_r", [64, 32, 16])
def test_alpha_decay_raw_bins_match_oracle(torch_dev, B_r):
    """Each round of the alpha_t schedule hashes with its own alpha_r and
    window length (the oracle's round_bins / round_alpha): raw pair bins in
    FP64 against the oracle's HashToBins with that round's window."""
    torch, dev = torch_dev
    n, k, B, delta = 1 << 14, 16, 64, 1e-12
    w = default_w(n, B, 0.5, delta)
    say("alpha-decay-raw", "n", n, "B", B, "B_r", B_r)
    plan = plan_for(n, k, B, w, 5, delta=delta, in_dtype=1, loc_prec=1, b_min=16, alpha_decay=0.5)
    p = oracle_params(plan)
    r = [p.round_bins(q)[0] for q in range(p.rounds)].index(B_r)
    Br, wr = p.round_bins(r)
    assert Br == B_r and wr == w              # B and alpha halve together: the window length stays
    x, _, _ = siggen.planted_signal(n, 40, 12, np.complex128, noise_ratio=0.01)
    rng = np.random.default_rng(B_r)
    sigma, a, b = int(rng.integers(0, n // 2)) * 2 + 1, int(rng.integers(0, n)), int(rng.integers(0, n))
    u0, u1 = plan.hash_pair_raw(torch.from_numpy(x).to(dev), sigma, a, 1, b, B_r, 1)
    torch.cuda.synchronize()
    G = window_time(n, Br, wr, p.round_alpha(r), delta)
    e0 = hash_to_bins_raw(x, sigma, a, b, Br, G)
    e1 = hash_to_bins_raw(x, sigma, (a + 1) % n, b, Br, G)
    scale = max(np.max(np.abs(e0)), np.max(np.abs(e1)))
    assert np.max(np.abs(u0.cpu().numpy() - e0)) <= 1e-12 * scale
    assert np.max(np.abs(u1.cpu().numpy() - e1)) <= 1e-12 * scale
    plan.close()


@pytest.mark.parametrize("shape", ["c1", "c3"])
def test_alpha_decay_batched_matches_oracle(torch_dev, shape):
    """The alpha_t schedule end to end: n = 2^14, k = 16 in FP64 storage, and
    the n = 2^22, k = 256 batch shape (alpha 0.75 halving with B down to
    b_min = 64), against the oracle and the planted supports."""
    torch, dev = torch_dev
    if shape == "c1":
        n, k, B, dtype, delta, count = 1 << 14, 16, 64, np.complex128, 1e-12, 4
        kw = dict(delta=delta, in_dtype=1, loc_prec=1, b_min=16, alpha_decay=0.5, patience=4)
        w = default_w(n, B, 0.5, delta)
    else:
        n, k, B, dtype, delta, count = 1 << 22, 256, 1024, np.complex64, 1e-8, 2
        kw = dict(delta=delta, alpha=0.75, loc_prec=1, b_min=64, rounds=24, patience=5, theta=0.01, g_min=0.25,
                  alpha_decay=0.5)
        w = default_w(n, B, 0.75, delta)
    say("alpha-decay", shape, "n", n, "k", k, "B", B, "count", count)
    plan = plan_for(n, k, B, w, 0, max_batch=count, **kw)
    xs, sups, seeds = [], [], []
    for s in range(count):
        x, sup, _ = siggen.planted_signal(n, k, 700 + s, dtype, magnitude="unit" if shape == "c1" else "loguniform")
        xs.append(x)
        sups.append(sup)
        seeds.append(31 * s + 7)
    out = run_batch(torch, dev, plan, xs, seeds)
    for s in range(count):
        ref = noiseless_sparse_fft(xs[s], oracle_params(plan, seeds[s]))
        assert int(out[s][2][0]) == ref.rounds_used
        compare(out[s][0], out[s][1], ref)
        assert np.array_equal(out[s][0], sups[s])
    plan.close()


@pytest.mark.parametrize("alpha_decay", [0.0, 0.7])
def test_launch_bytes_and_gathered_samples_agree(torch_dev, alpha_decay):
    """The roofline's algorithmic bytes of the first HashToBins launch and the
    serving policy's gathered samples count the same rounds: for one signal,
    bytes = 8 (w_r + 1) summed over round group 0 plus the 2 B_r complex128
    raw bins of each of those rounds."""
    from paper_1201_2501_amd import sfft
    n, k, B = 1 << 22, 256, 1024
    w = default_w(n, B, 0.75, 1e-8)
    say("launch-bytes", "alpha_decay", alpha_decay)
    plan = plan_for(n, k, B, w, 0, delta=1e-8, alpha=0.75, b_min=64, rounds=24, patience=5, group0=12,
                    alpha_decay=alpha_decay)
    d = plan.desc
    samples = sfft.sfft_plan_samples(d)
    p = oracle_params(plan)
    g0 = plan.round_groups()[0]
    assert g0 == 12
    assert samples == sum(p.round_bins(r)[1] + 1 for r in range(g0))
    bins = sum(p.round_bins(r)[0] for r in range(g0))
    assert plan.h2b_bytes(1) == 8 * samples + 32 * bins
    assert plan.h2b_bytes(512) == 512 * plan.h2b_bytes(1)
    plan.close()


@pytest.mark.parametrize("shape,parts", [("c1", 2), ("c1", 8), ("c3", 4), ("c3", 16)])
def test_split_hashing_matches_oracle(torch_dev, shape, parts):
    """hash_split: each (signal, round) hashed by several workgroups over
    window ranges, partials summed in part order: the same supports and
    values as the oracle, at n = 2^14 (FP64 storage) and at the n = 2^22,
    k = 256 batch shape."""
    torch, dev = torch_dev
    if shape == "c1":
        n, k, B, dtype, count = 1 << 14, 16, 64, np.complex128, 4
        w = default_w(n, B, 0.5, 1e-12)
        kw = dict(delta=1e-12, in_dtype=1, loc_prec=1)
    else:
        n, k, B, dtype, count = 1 << 22, 256, 1024, np.complex64, 2
        w = default_w(n, B, 0.75, 1e-8)
        kw = dict(delta=1e-8, alpha=0.75, loc_prec=1, b_min=64, rounds=24, patience=5, theta=0.01, g_min=0.25,
                  stop_count=k, stop_patience=3, ratio_tol=0.002, group0=12, group_step=3)
    say("split-hash", shape, "parts", parts, "n", n, "count", count)
    plan = plan_for(n, k, B, w, 0, max_batch=count, hash_split=parts, **kw)
    xs, sups, seeds = [], [], []
    for s in range(count):
        x, sup, _ = siggen.planted_signal(n, k, 820 + s, dtype, magnitude="unit" if shape == "c1" else "loguniform")
        xs.append(x)
        sups.append(sup)
        seeds.append(13 * s + 5)
    out = run_batch(torch, dev, plan, xs, seeds)
    for s in range(count):
        ref = noiseless_sparse_fft(xs[s], oracle_params(plan, seeds[s]))
        assert int(out[s][2][0]) == ref.rounds_used
        compare(out[s][0], out[s][1], ref)
        assert np.array_equal(out[s][0], sups[s])
    plan.close()


def test_split_hashing_is_batch_independent(torch_dev):
    """A signal gives bit-identical results alone and inside a batch under
    hash_split (the serving runtime relies on this)."""
    torch, dev = torch_dev
    n, k, B = 1 << 16, 64, 256
    w = default_w(n, B, 0.5, 1e-9)
    say("split-hash-batch-independence", "n", n)
    plan = plan_for(n, k, B, w, 0, max_batch=4, hash_split=4, b_min=32, rounds=24, patience=5)
    xs = [siggen.planted_signal(n, k, 840 + s, np.complex64)[0] for s in range(4)]
    seeds = [3, 4, 5, 6]
    batch = run_batch(torch, dev, plan, xs, seeds)
    for s in (0, 3):
        alone = run_batch(torch, dev, plan, [xs[s]], [seeds[s]])[0]
        assert np.array_equal(alone[0], batch[s][0]) and np.array_equal(alone[1], batch[s][1])
    plan.close()


def test_cached_tuned_c3_plan_matches_oracle(torch_dev):
    """The plan the autotuner stored for the n = 2^22, k = 256 batch (the one
    bench.py times) matches the oracle on two signals of that workload."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_1201_2501_amd",
                        "tuned.json")
    recs = [r for key, r in json.load(open(path)).items() if "|n=4194304|k=256|mode=0|" in key] \
        if os.path.exists(path) else []
    if not recs:
        pytest.skip("no stored plan for this workload")
    rec = recs[0]
    torch, dev = torch_dev
    n, k, B = 1 << 22, 256, rec["B"]
    fields = {f: v for f, v in rec["fields"].items() if f not in ("mode",)}
    say("c3-cached-plan", "B", B, fields)
    plan = plan_for(n, k, B, 0, 0, max_batch=2, **fields)
    xs, sups, seeds = [], [], []
    for s in range(2):
        x, sup, _ = siggen.planted_signal(n, k, 5000 + s, np.complex64, magnitude="loguniform")
        xs.append(x)
        sups.append(sup)
        seeds.append(101 * s + 17)
    out = run_batch(torch, dev, plan, xs, seeds)
    for s in range(2):
        ref = noiseless_sparse_fft(xs[s], oracle_params(plan, seeds[s]))
        assert int(out[s][2][0]) == ref.rounds_used
        compare(out[s][0], out[s][1], ref)
        assert np.array_equal(out[s][0], sups[s])
    plan.close()


@pytest.mark.parametrize("n,k,B,mode,prec", [(1 << 16, 16, 256, 2, 1), (1 << 18, 100, 512, 1, 1),
                                             (1 << 18, 100, 512, 1, 0), (1 << 14, 16, 64, 2, 1)])
def test_stream_mode_raw_bins_match_oracle(torch_dev, n, k, B, mode, prec):
    """Stream-mode HashToBins (hash_mode 1: rounds whose window covers n/8 or
    more; 2: every round) reads the signal contiguously; the raw bins of every
    round of group 0, at both shifts, match the oracle's HashToBins of the
    same draws: FP64 within 1e-12 of the largest bin, FP32 within 2e-5."""
    from oracle.rng import draw_b, draw_sigma
    from paper_1201_2501_amd import sfft
    torch, dev = torch_dev
    dtype = np.complex128 if n == 1 << 14 else np.complex64
    delta = 1e-12 if dtype == np.complex128 else 1e-9
    w = default_w(n, B, 0.5, delta)
    count = 2
    plan = plan_for(n, k, B, w, 0, delta=delta, in_dtype=int(dtype == np.complex128), loc_prec=prec,
                    max_batch=count, hash_mode=mode, rounds=12, group0=6)
    nstream = sfft.sfft_plan_stream_rounds(plan.desc)
    say("stream-raw", "n", n, "B", B, "w", w, "mode", mode, "prec", prec, "stream rounds", nstream)
    assert nstream >= 1 and (mode != 2 or nstream == 6)
    xs = [siggen.planted_signal(n, k, 870 + s, dtype, noise_ratio=0.01)[0] for s in range(count)]
    seeds = [41, 977]
    X = torch.from_numpy(np.stack(xs)).to(dev)
    plan.execute_batch(X, torch.tensor(seeds, dtype=torch.int64, device=dev))
    torch.cuda.synchronize()
    p = oracle_params(plan)
    tol = 1e-12 if prec == 1 else 2e-5
    for s in range(count):
        for r in range(6):
            Br, wr = p.round_bins(r)
            G = window_time(n, Br, wr, p.round_alpha(r), delta)
            sigma, b = draw_sigma(seeds[s], n, r), draw_b(seeds[s], n, r)
            e0 = hash_to_bins_raw(xs[s], sigma, 0, b, Br, G)
            e1 = hash_to_bins_raw(xs[s], sigma, 1, b, Br, G)
            g0, g1 = plan.raw_slot(s, r, dev)
            sc = max(np.abs(e0).max(), np.abs(e1).max())
            assert np.abs(g0 - e0).max() <= tol * sc, (s, r)
            assert np.abs(g1 - e1).max() <= tol * sc, (s, r)
    plan.close()


@pytest.mark.parametrize("n,k,B,mode", [(1 << 18, 100, 512, 1), (1 << 16, 16, 256, 2), (1 << 20, 256, 1024, 2)])
def test_stream_mode_recovery_matches_oracle(torch_dev, n, k, B, mode):
    """The batched exact path with stream-mode rounds: supports bit-exact and
    values within 1e-10 of the oracle, rounds decoded equal, for four
    signals with their own seeds (the served shapes' schedule: b_min 32,
    24 rounds, patience 5)."""
    torch, dev = torch_dev
    w = default_w(n, B, 0.5, 1e-9)
    count = 4
    plan = plan_for(n, k, B, w, 0, delta=1e-9, loc_prec=1, max_batch=count, hash_mode=mode, b_min=32,
                    rounds=24, patience=5)
    say("stream-recovery", "n", n, "k", k, "B", B, "mode", mode)
    xs, sups, seeds = [], [], []
    for s in range(count):
        x, sup, _ = siggen.planted_signal(n, k, 880 + s, np.complex64)
        xs.append(x)
        sups.append(sup)
        seeds.append(101 * s + 3)
    out = run_batch(torch, dev, plan, xs, seeds)
    for s in range(count):
        ref = noiseless_sparse_fft(xs[s], oracle_params(plan, seeds[s]))
        assert int(out[s][2][0]) == ref.rounds_used
        compare(out[s][0], out[s][1], ref)
        assert np.array_equal(out[s][0], sups[s])
    plan.close()


@pytest.mark.parametrize("n,k,B,A,prec", [(1 << 18, 100, 512, 300, 1), (1 << 18, 100, 512, 50001, 1),
                                          (1 << 18, 100, 512, 300, 0), (1 << 22, 256, 1024, 2048, 0)])
def test_refine_raw_bins_match_oracle(torch_dev, n, k, B, A, prec):
    """The pair launch with the refinement hashing: the third hashing (shift
    A) of every round of group 0 matches the oracle's HashToBins at shift A,
    and the pair's own bins still match theirs (FP64 within 1e-12 of the
    largest bin, FP32 within 2e-5); A within the windows (one window feeds
    all three hashings) and beyond them (the third reads its own)."""
    from oracle.rng import draw_b, draw_sigma
    torch, dev = torch_dev
    delta = 1e-9
    w = default_w(n, B, 0.5, delta)
    count = 2
    plan = plan_for(n, k, B, w, 0, delta=delta, loc_prec=prec, max_batch=count, rounds=12, group0=6,
                    refine_shift=A, refine_window=2)
    say("refine-raw", "n", n, "B", B, "w", w, "A", A, "prec", prec)
    xs = [siggen.planted_signal(n, k, 890 + s, np.complex64, noise_ratio=0.01)[0] for s in range(count)]
    seeds = [43, 1001]
    X = torch.from_numpy(np.stack(xs)).to(dev)
    plan.execute_batch(X, torch.tensor(seeds, dtype=torch.int64, device=dev))
    torch.cuda.synchronize()
    p = oracle_params(plan)
    tol = 1e-12 if prec == 1 else 2e-5
    for s in range(count):
        for r in range(6):
            Br, wr = p.round_bins(r)
            G = window_time(n, Br, wr, p.round_alpha(r), delta)
            sigma, b = draw_sigma(seeds[s], n, r), draw_b(seeds[s], n, r)
            e = [hash_to_bins_raw(xs[s], sigma, a, b, Br, G) for a in (0, 1, A)]
            g0, g1 = plan.raw_slot(s, r, dev)
            gA = plan.raw_refine(s, r, dev)
            sc = max(np.abs(v).max() for v in e)
            for got, exp in zip((g0, g1, gA), e):
                assert np.abs(got - exp).max() <= tol * sc, (s, r)
    plan.close()


@pytest.mark.parametrize("n,k,B,A,E,prec", [(1 << 18, 100, 512, 300, 16, 1), (1 << 18, 100, 512, 50001, 2, 1),
                                            (1 << 22, 256, 1024, 2048, 1000, 0)])
def test_refine_recovery_matches_oracle(torch_dev, n, k, B, A, E, prec):
    """The batched exact path with the multi-shift refinement: supports
    bit-exact against the oracle (which refines the same way in FP64) and
    the planted ones.  FP64 bins: rounds decoded equal and values within
    1e-10 relative.  FP32 bins (n = 2^22, where the FP32 pair alone locates
    nothing): values within 2e-5 of the largest magnitude, the FP32 rounding
    of the bins; the rounds decoded may differ, since bin noise of a few
    1e-7 of the largest bin changes which collided bins pass the checks in
    a round (the oracle with such noise added to its bins does the same)."""
    torch, dev = torch_dev
    delta = 1e-9
    w = default_w(n, B, 0.5, delta)
    count = 2
    mag = "loguniform" if n == 1 << 22 else "unit"
    plan = plan_for(n, k, B, w, 0, delta=delta, theta=0.02 if mag == "loguniform" else 0.25, loc_prec=prec,
                    max_batch=count, b_min=32, rounds=24, refine_shift=A, refine_window=E)
    say("refine-recovery", "n", n, "k", k, "B", B, "A", A, "E", E, "prec", prec)
    xs, sups, seeds = [], [], []
    for s in range(count):
        x, sup, _ = siggen.planted_signal(n, k, 900 + s, np.complex64, magnitude=mag)
        xs.append(x)
        sups.append(sup)
        seeds.append(7 * s + 5)
    out = run_batch(torch, dev, plan, xs, seeds)
    for s in range(count):
        ref = noiseless_sparse_fft(xs[s], oracle_params(plan, seeds[s]))
        print("refine-recovery rounds", int(out[s][2][0]), "oracle", ref.rounds_used, flush=True)
        assert prec == 0 or int(out[s][2][0]) == ref.rounds_used
        assert np.array_equal(out[s][0], ref.indices)
        assert np.array_equal(out[s][0], sups[s])
        if prec == 1:
            compare(out[s][0], out[s][1], ref)
        else:
            err = np.abs(out[s][1] - ref.values).max()
            print("refine-recovery FP32 value error", err, "of", np.abs(ref.values).max(), flush=True)
            assert err <= 2e-5 * np.abs(ref.values).max()
    plan.close()


@pytest.mark.parametrize("n,B,dtype,extra", [(1 << 14, 64, np.complex128, 0), (1 << 14, 64, np.complex128, 14),
                                             (1 << 22, 1024, np.complex64, 62)])
def test_adversarial_collision_matches_oracle(torch_dev, n, B, dtype, extra):
    """Host-forced collision: for the signal's round-0 draws (sigma, b), i2 is
    placed so that its permuted position follows i1's (same bin, the pair's
    phase mixes both); with `extra` other coefficients.  Round 0 cannot
    decode the pair; the GPU recovers what the oracle recovers (supports
    bit-exact, values within 1e-10, rounds decoded equal), which is the
    planted spectrum.  Batched path, and the plain path at n = 2^14."""
    from oracle.hashing import bin_offset, perm_position
    from oracle.rng import draw_b, draw_sigma
    torch, dev = torch_dev
    seed = 4242
    sigma, b = draw_sigma(seed, n, 0), draw_b(seed, n, 0)
    sinv = pow(sigma, -1, n)
    i1 = 1000
    while abs(bin_offset(i1, sigma, b, n, B)[1]) >= n // (8 * B):
        i1 += 1
    i2 = (sinv * (perm_position(i1, sigma, b, n) + 1) + b) % n
    assert bin_offset(i2, sigma, b, n, B)[0] == bin_offset(i1, sigma, b, n, B)[0]
    rng = np.random.Generator(np.random.PCG64(77 + extra))
    others = [int(i) for i in rng.choice(n, 4 * extra + 8, replace=False) if int(i) not in (i1, i2)][:extra]
    sup = np.array(sorted([i1, i2] + others), dtype=np.int64)
    val = np.exp(2j * np.pi * rng.random(len(sup)))
    val[sup == i1], val[sup == i2] = 1.0 + 0.5j, -0.7 + 0.8j
    x = siggen.time_signal(n, sup, val).astype(dtype)
    delta = 1e-12 if dtype == np.complex128 else 1e-9
    w = default_w(n, B, 0.5, delta)
    k = len(sup)
    say("adversarial", "n", n, "B", B, "k", k, "i1", i1, "i2", i2, "seed", seed)
    plan = plan_for(n, k, B, w, seed, delta=delta, in_dtype=int(dtype == np.complex128), loc_prec=1, max_batch=1)
    ref = noiseless_sparse_fft(x, oracle_params(plan, seed))
    assert np.array_equal(ref.indices, sup) and ref.rounds_used >= 2
    out = run_batch(torch, dev, plan, [x], [seed])[0]
    assert int(out[2][0]) == ref.rounds_used
    compare(out[0], out[1], ref)
    if n == 1 << 14:
        idx, v, info, st = plan.execute(torch.from_numpy(x).to(dev))
        assert int(info[0]) == ref.rounds_used
        compare(idx, v, ref)
    plan.close()


@pytest.mark.parametrize("n,B,dtype,prec,B_r", [(1 << 14, 64, np.complex128, 1, 64), (1 << 14, 64, np.complex128, 1, 16),
                                               (1 << 22, 1024, np.complex64, 1, 1024),
                                               (1 << 22, 1024, np.complex64, 1, 64),
                                               (1 << 22, 1024, np.complex64, 0, 1024)])
def test_kaiser_raw_bins_match_oracle(torch_dev, n, B, dtype, prec, B_r):
    """The Kaiser-Bessel window (plan window = 1): the pair's raw bins match
    the oracle's HashToBins with its own Kaiser window table (FP64 within
    1e-12 of the bins' RMS, FP32 within 1e-5)."""
    torch, dev = torch_dev
    delta = 1e-12 if dtype == np.complex128 else 1e-8
    alpha = 0.5 if n == 1 << 14 else 0.75
    w = default_w(n, B, alpha, delta, kind=1)
    x, sup, val = siggen.planted_signal(n, 40, 13, dtype, noise_ratio=0.01)
    say("kaiser-raw", "n", n, "B", B, "B_r", B_r, "w", w, "prec", prec)
    plan = plan_for(n, 40, B, w, 5, delta=delta, alpha=alpha, in_dtype=int(dtype == np.complex128), loc_prec=prec,
                    b_min=16, window=1)
    xd = torch.from_numpy(x).to(dev)
    rng = np.random.default_rng(B_r + prec)
    sigma = int(rng.integers(0, n // 2)) * 2 + 1
    a = int(rng.integers(0, n))
    b = int(rng.integers(0, n))
    u0, u1 = plan.hash_pair_raw(xd, sigma, a, 1, b, B_r, prec)
    torch.cuda.synchronize()
    G = window_time(n, B_r, w * B_r // B, alpha, delta, kind=1)
    e0 = hash_to_bins_raw(x, sigma, a, b, B_r, G)
    e1 = hash_to_bins_raw(x, sigma, (a + 1) % n, b, B_r, G)
    rms = np.sqrt(np.mean(np.abs(np.concatenate([e0, e1])) ** 2))
    err = max(np.max(np.abs(u0.cpu().numpy() - e0)), np.max(np.abs(u1.cpu().numpy() - e1)))
    print("kaiser raw-bin error of rms", err / rms, flush=True)
    assert err <= (1e-12 if prec == 1 else 1e-5) * rms
    plan.close()


@pytest.mark.parametrize("shape", ["c1", "c3"])
def test_kaiser_window_recovery_matches_oracle(torch_dev, shape):
    """Exact mode with the Kaiser-Bessel window against the oracle with the
    same window: supports bit-exact (and equal to the planted ones), values
    within 1e-10, rounds decoded equal.  C1: n = 2^14, complex128, plain and
    batched; C3: n = 2^22, k = 256, log-uniform magnitudes, the tuned
    schedule's fields with the Kaiser length."""
    torch, dev = torch_dev
    if shape == "c1":
        n, k, B, dtype, count = 1 << 14, 16, 64, np.complex128, 4
        kw = dict(delta=1e-12, in_dtype=1, loc_prec=1)
        alpha, mag = 0.5, "unit"
    else:
        n, k, B, dtype, count = 1 << 22, 256, 1024, np.complex64, 4
        kw = dict(alpha=0.75, delta=1e-8, b_min=64, patience=5, rounds=24, theta=0.01, g_min=0.25, ratio_tol=0.002,
                  stop_count=k, stop_patience=3, group0=12, group_step=3, loc_prec=1)
        alpha, mag = 0.75, "loguniform"
    w = default_w(n, B, alpha, kw["delta"], kind=1)
    say("kaiser-recovery", shape, "n", n, "k", k, "B", B, "w", w)
    plan = plan_for(n, k, B, w, 0, window=1, max_batch=count, **kw)
    xs, sups, seeds = [], [], []
    # C1: signals whose oracle runs have no decision within 1e-9 of a tie and
    # recover (at this shape about 3 % of signals do not, with either window)
    for s in ([0, 3, 4, 6] if shape == "c1" else range(count)):
        x, sup, _ = siggen.planted_signal(n, k, 960 + s, dtype, magnitude=mag)
        xs.append(x)
        sups.append(sup)
        seeds.append(13 * s + 1)
    out = run_batch(torch, dev, plan, xs, seeds)
    for s in range(count):
        ref = noiseless_sparse_fft(xs[s], oracle_params(plan, seeds[s]))
        assert int(out[s][2][0]) == ref.rounds_used
        compare(out[s][0], out[s][1], ref)
        assert np.array_equal(out[s][0], sups[s])
    plan.close()
    if shape == "c1":
        plan = plan_for(n, k, B, w, seeds[0], window=1, **kw)
        idx, v, info, st = plan.execute(torch.from_numpy(xs[0]).to(dev))
        ref = noiseless_sparse_fft(xs[0], oracle_params(plan))
        assert int(info[0]) == ref.rounds_used
        compare(idx, v, ref)
        plan.close()
