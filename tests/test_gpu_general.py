"""GPU parity of the general-mode path (Algorithms 2 and 3) against the FP64
oracle.

FP64 location and estimation arithmetic: supports bit-exact, values within
1e-10 relative.  FP32 arithmetic: values within 1e-4 relative; a support
difference is accepted only when the oracle run has a near-tie decision
(a vote within 1e-4 rad of s*pi, or a top-k' boundary gap below 1e-4 of the
compared magnitudes), reported by the oracle's margins.
"""
import numpy as np
import pytest

import siggen
from oracle.general import sparse_fft
from oracle.metrics import l2l2_ratio
from oracle.params import SfftParams

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    from paper_1201_2501_amd import sfft
    sfft.load()
    return torch, torch.device("cuda:0")


def make_plan(n, k, B, seed, prec, max_batch=1, delta=1e-6, est_prec=None, window=0):
    """General-mode plan: LocateInner pairs in `prec` arithmetic (0 FP32, 1
    FP64), EstimateValues hashings in `est_prec` (default: the same)."""
    from paper_1201_2501_amd.sfft import Plan, SFFT_MODE_GENERAL
    return Plan(n, k, B, 0, seed, mode=SFFT_MODE_GENERAL, delta=delta, loc_prec=prec,
                est_prec=prec if est_prec is None else est_prec, max_batch=max_batch, window=window)


def oracle_params(plan, seed=None):
    d = plan.desc
    return SfftParams(n=d.n, k=d.k, B=d.B, w=d.w, seed=d.seed if seed is None else seed, alpha=d.alpha,
                      delta=d.delta, g_min=d.g_min, rounds=d.rounds, t=d.t, s=d.s, R_loc=d.R_loc,
                      R_est=d.R_est, cap=d.cap, b_min=d.b_min, window=d.window)


def check(idx, val, ref, rel, allow_near_tie=False):
    if not np.array_equal(idx, ref.indices):
        assert allow_near_tie and (ref.vote_margin < 1e-4 or ref.select_margin < 1e-4), \
            (idx, ref.indices, ref.vote_margin, ref.select_margin)
        return False
    mag = np.maximum(np.abs(ref.values), 1e-300)
    assert np.all(np.abs(val - ref.values) <= rel * mag + 1e-12), np.max(np.abs(val - ref.values) / mag)
    return True


CASES = [
    # name, n, k, B, noise, prec
    ("small-noiseless-f64", 1 << 16, 12, 256, 0.0, 1),
    ("small-noisy-f64", 1 << 16, 12, 256, 0.05, 1),
    ("small-noisy-f32", 1 << 16, 12, 256, 0.05, 0),
    ("c2-f64", 1 << 20, 64, 1024, 0.05, 1),
    ("c2-f32", 1 << 20, 64, 1024, 0.05, 0),
]


@pytest.mark.parametrize("name,n,k,B,noise,prec", CASES)
def test_plain_general_matches_oracle(torch_dev, name, n, k, B, noise, prec):
    torch, dev = torch_dev
    seed = 3
    say("plain-general", name, "n", n, "k", k, "B", B)
    plan = make_plan(n, k, B, seed, prec)
    x, sup, val = siggen.planted_signal(n, k, 500 + k, np.complex64, noise_ratio=noise)
    idx, v, info, st = plan.execute(torch.from_numpy(x).to(dev))
    ref = sparse_fft(x, oracle_params(plan))
    same = check(idx, v, ref, 1e-10 if prec == 1 else 1e-4, allow_near_tie=(prec == 0))
    ratio, err = l2l2_ratio(x, k, idx, v)
    if noise > 0:
        assert ratio <= 2.0
    elif same:
        assert np.array_equal(idx, sup)
    plan.close()


def test_batched_general_matches_oracle_per_seed(torch_dev):
    torch, dev = torch_dev
    n, k, B = 1 << 16, 12, 256
    count = 4
    say("batched-general", "n", n, "count", count)
    plan = make_plan(n, k, B, 0, 1, max_batch=count)
    xs, seeds = [], []
    for s in range(count):
        xs.append(siggen.planted_signal(n, k, 700 + s, np.complex64, noise_ratio=0.05)[0])
        seeds.append(11 + 5 * s)
    X = torch.from_numpy(np.stack(xs)).to(dev)
    S = torch.tensor(seeds, dtype=torch.int64, device=dev)
    bufs = plan.execute_batch(X, S)
    torch.cuda.synchronize()
    for s in range(count):
        c = int(bufs["counts"][s])
        ref = sparse_fft(xs[s], oracle_params(plan, seeds[s]))
        check(bufs["idx"][s, :c].cpu().numpy(), bufs["val"][s, :c].cpu().numpy(), ref, 1e-10)
    # plain path with the same seed gives the same answer as the batch
    plain = make_plan(n, k, B, seeds[1], 1)
    idx, v, info, st = plain.execute(X[1])
    c = int(bufs["counts"][1])
    assert np.array_equal(idx, bufs["idx"][1, :c].cpu().numpy())
    assert np.allclose(v, bufs["val"][1, :c].cpu().numpy(), rtol=1e-11, atol=1e-14)
    plan.close()
    plain.close()


def test_batched_general_raw_slots_match_oracle(torch_dev):
    """Every batched HashToBins job of round 0 (LocateInner pairs and
    EstimateValues hashings) against the oracle's bins for the same draws."""
    from oracle.general import beta_range, level_widths
    from oracle.hashing import hash_to_bins_raw
    from oracle.rng import LEVEL_EST, draw_a, draw_b, draw_beta, draw_sigma
    from oracle.window import window_time
    torch, dev = torch_dev
    n, k, B = 1 << 16, 12, 256
    say("general-raw-slots", "n", n)
    plan = make_plan(n, k, B, 9, 1, max_batch=1)
    x = siggen.planted_signal(n, k, 800, np.complex64, noise_ratio=0.05)[0]
    X = torch.from_numpy(x[None, :]).to(dev)
    S = torch.tensor([9], dtype=torch.int64, device=dev)
    plan.execute_batch(X, S)
    torch.cuda.synchronize()
    d = plan.desc
    G = window_time(n, B, d.w, d.alpha, d.delta)
    sigma, b = draw_sigma(9, n, 0, 0, 0), draw_b(9, n, 0, 0, 0)
    slot = 0
    for D, W in enumerate(level_widths(n, B, d.t), start=1):
        lo, hi = beta_range(n, W, d.t, d.s)
        for q in range(d.R_loc):
            a, beta = draw_a(9, n, 0, D, q), draw_beta(9, lo, hi, 0, D, q)
            g0, g1 = plan.raw_slot(0, slot, dev)
            e0 = hash_to_bins_raw(x, sigma, a, b, B, G)
            e1 = hash_to_bins_raw(x, sigma, (a + beta) % n, b, B, G)
            sc = max(np.abs(e0).max(), np.abs(e1).max())
            assert np.abs(g0 - e0).max() <= 1e-12 * sc, ("loc", D, q, 0)
            assert np.abs(g1 - e1).max() <= 1e-12 * sc, ("loc", D, q, 1)
            slot += 1
    for e in range(d.R_est):
        se, ae, be = draw_sigma(9, n, 0, LEVEL_EST, e), draw_a(9, n, 0, LEVEL_EST, e), draw_b(9, n, 0, LEVEL_EST, e)
        g0, _ = plan.raw_slot(0, slot, dev)
        e0 = hash_to_bins_raw(x, se, ae, be, B, G)
        assert np.abs(g0 - e0).max() <= 1e-12 * np.abs(e0).max(), ("est", e)
        slot += 1
    plan.close()


def test_c4_shape_raw_hashings_and_recovery(torch_dev):
    """n = 2^26, k = 1024, unit magnitudes with 1% noise, B = 4096 (default
    rounds, FP64 location pairs): round 0's first LocateInner pair and first
    EstimateValues hashing of signal 0 against the oracle at full size, then
    supports equal to the planted ones for each signal, l2/l2 <= 2 for the
    first."""
    from oracle.general import beta_range, level_widths
    from oracle.hashing import hash_to_bins_raw
    from oracle.rng import LEVEL_EST, draw_a, draw_b, draw_beta, draw_sigma
    from oracle.window import window_time
    torch, dev = torch_dev
    n, k, B, count = 1 << 26, 1024, 4096, 2
    say("c4-shape", "n", n, "k", k, "B", B, "count", count)
    X, sups, vals = siggen.torch_planted_batch(n, k, [91_000 + s for s in range(count)], dev, magnitude="unit",
                                               noise_ratio=0.01, chunk=1)
    seeds = [17, 29]
    plan = make_plan(n, k, B, 0, 1, max_batch=count, delta=1e-7)
    d = plan.desc
    assert d.rounds == 7
    bufs = plan.execute_batch(X, torch.tensor(seeds, dtype=torch.int64, device=dev))
    torch.cuda.synchronize()
    x0 = X[0].cpu().numpy()
    G = window_time(n, B, d.w, d.alpha, d.delta)
    sigma, b = draw_sigma(seeds[0], n, 0, 0, 0), draw_b(seeds[0], n, 0, 0, 0)
    W = level_widths(n, B, d.t)[0]
    lo, hi = beta_range(n, W, d.t, d.s)
    a, beta = draw_a(seeds[0], n, 0, 1, 0), draw_beta(seeds[0], lo, hi, 0, 1, 0)
    g0, g1 = plan.raw_slot(0, 0, dev)
    e0 = hash_to_bins_raw(x0, sigma, a, b, B, G)
    e1 = hash_to_bins_raw(x0, sigma, (a + beta) % n, b, B, G)
    sc = max(np.abs(e0).max(), np.abs(e1).max())
    assert np.abs(g0 - e0).max() <= 1e-12 * sc and np.abs(g1 - e1).max() <= 1e-12 * sc
    nloc = len(level_widths(n, B, d.t)) * d.R_loc
    se, ae, be = (draw_sigma(seeds[0], n, 0, LEVEL_EST, 0), draw_a(seeds[0], n, 0, LEVEL_EST, 0),
                  draw_b(seeds[0], n, 0, LEVEL_EST, 0))
    g2, _ = plan.raw_slot(0, nloc, dev)
    e2 = hash_to_bins_raw(x0, se, ae, be, B, G)
    rel = 1e-12 if d.est_prec == 1 else 2e-5
    assert np.abs(g2 - e2).max() <= rel * np.abs(e2).max()
    for s in range(count):
        c = int(bufs["counts"][s])
        idx = bufs["idx"][s, :c].cpu().numpy()
        v = bufs["val"][s, :c].cpu().numpy()
        assert np.array_equal(idx, np.sort(sups[s]))
        if s == 0:   # the oracle's own FFT at 2^26 points takes most of a minute
            ratio, _ = l2l2_ratio(X[s].cpu().numpy(), k, idx, v)
            assert ratio <= 2.0, ratio
    plan.close()


@pytest.mark.parametrize("prec", [1, 0])
def test_batched_general_c2_shape_matches_oracle(torch_dev, prec):
    """Batched general mode at n = 2^20, k = 64, B = 1024, tail/head 0.05:
    each of four signals (own seeds) against the oracle run with its seed."""
    torch, dev = torch_dev
    n, k, B, count = 1 << 20, 64, 1024, 4
    say("batched-general-c2", "prec", prec, "count", count)
    plan = make_plan(n, k, B, 0, prec, max_batch=count)
    xs = [siggen.planted_signal(n, k, 900 + s, np.complex64, noise_ratio=0.05)[0] for s in range(count)]
    seeds = [101 + 13 * s for s in range(count)]
    X = torch.from_numpy(np.stack(xs)).to(dev)
    bufs = plan.execute_batch(X, torch.tensor(seeds, dtype=torch.int64, device=dev))
    torch.cuda.synchronize()
    for s in range(count):
        c = int(bufs["counts"][s])
        idx, v = bufs["idx"][s, :c].cpu().numpy(), bufs["val"][s, :c].cpu().numpy()
        ref = sparse_fft(xs[s], oracle_params(plan, seeds[s]))
        check(idx, v, ref, 1e-10 if prec == 1 else 1e-4, allow_near_tie=(prec == 0))
        ratio, _ = l2l2_ratio(xs[s], k, idx, v)
        assert ratio <= 2.0, (s, ratio)
    plan.close()


@pytest.fixture(scope="module")
def c4_case(torch_dev):
    """One n = 2^26, k = 1024 signal (unit magnitudes, tail/head 0.01) on the
    device and its oracle run (B = 4096, delta = 1e-7, default rounds)."""
    torch, dev = torch_dev
    n, k, B, seed = 1 << 26, 1024, 4096, 17
    X, sups, _ = siggen.torch_planted_batch(n, k, [91_000], dev, magnitude="unit", noise_ratio=0.01, chunk=1)
    plan = make_plan(n, k, B, seed, 1, delta=1e-7)
    params = oracle_params(plan)
    plan.close()
    x0 = X[0].cpu().numpy()
    ref = sparse_fft(x0, params)
    return X, x0, np.sort(sups[0]), ref, params


@pytest.mark.parametrize("loc,est", [(0, 0), (1, 0), (1, 1)], ids=["f32", "f64loc", "f64"])
def test_c4_precision_variants_match_oracle(torch_dev, c4_case, loc, est):
    """The precision split at n = 2^26, k = 1024 against the FP64 oracle:
    FP32 location and estimation hashings, FP64 location with FP32
    estimation, FP64 throughout (the final re-estimation is FP64 in all
    three).  Supports bit-exact (FP32 location: or differing only where the
    oracle has a near-tie decision); values within 1e-10 relative when the
    estimation hashings are FP64, else 1e-4."""
    torch, dev = torch_dev
    X, x0, sup, ref, params = c4_case
    say("c4-precision", "loc", loc, "est", est)
    plan = make_plan(params.n, params.k, params.B, params.seed, loc, delta=params.delta, est_prec=est)
    d = plan.desc
    assert (d.loc_prec, d.est_prec, d.w, d.rounds) == (loc, est, params.w, params.rounds)
    idx, v, info, st = plan.execute(X[0])
    same = check(idx, v, ref, 1e-10 if est == 1 else 1e-4, allow_near_tie=(loc == 0))
    if same:
        assert np.array_equal(idx, sup)
    plan.close()


@pytest.fixture(scope="module")
def c4_kaiser_case(torch_dev):
    """The c4_case signal with the Kaiser-Bessel window (the C4 bench's
    window) and its oracle run."""
    torch, dev = torch_dev
    n, k, B, seed = 1 << 26, 1024, 4096, 17
    X, sups, _ = siggen.torch_planted_batch(n, k, [91_000], dev, magnitude="unit", noise_ratio=0.01, chunk=1)
    plan = make_plan(n, k, B, seed, 1, delta=1e-7, window=1)
    params = oracle_params(plan)
    plan.close()
    x0 = X[0].cpu().numpy()
    ref = sparse_fft(x0, params)
    return X, x0, np.sort(sups[0]), ref, params


def test_c4_kaiser_window_matches_oracle(torch_dev, c4_kaiser_case):
    """n = 2^26, k = 1024 with the Kaiser-Bessel window, FP64 location and
    FP32 estimation (the C4 default) against the FP64 oracle: supports
    bit-exact, values within 1e-4 relative (FP32 estimation hashings)."""
    torch, dev = torch_dev
    X, x0, sup, ref, params = c4_kaiser_case
    say("c4-kaiser", "w", params.w)
    assert params.window == 1
    plan = make_plan(params.n, params.k, params.B, params.seed, 1, delta=params.delta, est_prec=0, window=1)
    d = plan.desc
    assert (d.window, d.w, d.rounds) == (1, params.w, params.rounds)
    idx, v, info, st = plan.execute(X[0])
    assert check(idx, v, ref, 1e-4, allow_near_tie=False)
    assert np.array_equal(idx, sup)
    plan.close()


@pytest.mark.parametrize("b_min", [256, 1024])
def test_general_b_min_schedule_matches_oracle(torch_dev, b_min):
    """General mode with a floor on the round bins (b_min = B: B and w fixed in
    every round) at n = 2^20, k = 64, B = 1024, tail/head 0.05, FP64: the
    batched path against the oracle, signal by signal."""
    from paper_1201_2501_amd.sfft import Plan, SFFT_MODE_GENERAL
    torch, dev = torch_dev
    n, k, B, count = 1 << 20, 64, 1024, 2
    say("general-b_min", b_min)
    plan = Plan(n, k, B, 0, 0, mode=SFFT_MODE_GENERAL, delta=1e-6, loc_prec=1, est_prec=1, b_min=b_min,
                max_batch=count)
    assert plan.desc.b_min == b_min
    xs = [siggen.planted_signal(n, k, 960 + s, np.complex64, noise_ratio=0.05)[0] for s in range(count)]
    seeds = [7 + 3 * s for s in range(count)]
    bufs = plan.execute_batch(torch.from_numpy(np.stack(xs)).to(dev), torch.tensor(seeds, dtype=torch.int64,
                                                                                     device=dev))
    torch.cuda.synchronize()
    for s in range(count):
        c = int(bufs["counts"][s])
        ref = sparse_fft(xs[s], oracle_params(plan, seeds[s]))
        check(bufs["idx"][s, :c].cpu().numpy(), bufs["val"][s, :c].cpu().numpy(), ref, 1e-10)
    plan.close()


@pytest.mark.parametrize("noise", [0.0, 0.05])
def test_general_kaiser_window_matches_oracle(torch_dev, noise):
    """General mode with the Kaiser-Bessel window (window = 1), FP64, batched
    over three signals with their own seeds: supports bit-exact and values
    within 1e-10 of the oracle with the same window."""
    torch, dev = torch_dev
    n, k, B, count = 1 << 16, 12, 256, 3
    say("general-kaiser", "n", n, "k", k, "B", B, "noise", noise)
    plan = make_plan(n, k, B, 0, 1, max_batch=count, window=1)
    xs = [siggen.planted_signal(n, k, 640 + s, np.complex64, noise_ratio=noise)[0] for s in range(count)]
    seeds = [5, 6, 7]
    X = torch.from_numpy(np.stack(xs)).to(dev)
    bufs = plan.execute_batch(X, torch.tensor(seeds, dtype=torch.int64, device=dev))
    torch.cuda.synchronize()
    for s in range(count):
        c = int(bufs["counts"][s])
        ref = sparse_fft(xs[s], oracle_params(plan, seeds[s]))
        check(bufs["idx"][s, :c].cpu().numpy(), bufs["val"][s, :c].cpu().numpy(), ref, 1e-10)
    plan.close()
