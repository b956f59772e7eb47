"""GPU check of the autotuner on a small exactly-sparse batch: the choice
recovers every planted support, is no slower than the reference candidate
measured in the same run, comes back from the cache, and a plan built from
it reproduces the planted supports.  Every case prints its name first."""
import numpy as np
import pytest

import siggen

pytestmark = pytest.mark.gpu


def say(*a):
    print("[gpu-case]", *a, flush=True)


def test_autotune_small_exact_batch(tmp_path):
    import torch
    from paper_1201_2501_amd import autotune, sfft

    sfft.load()
    dev = torch.device("cuda:0")
    n, k, count = 1 << 18, 32, 32
    say("autotune", "n", n, "k", k, "count", count)
    X, sups, _ = siggen.torch_planted_batch(n, k, [7000 + s for s in range(count)], dev, magnitude="loguniform")
    seeds = torch.arange(count, dtype=torch.int64, device=dev) * 13 + 5
    space = {"bins": {"B": [128, 256]}, "window": {"delta": [1e-9]},
             "schedule": {"b_min": [16, 32], "patience": [3]},
             "launch": {"hash_threads": [256, 512], "chunks": [1]}}
    base = dict(theta=0.02, rounds=24, loc_prec=sfft.SFFT_F64)
    cache = str(tmp_path / "tuned.json")

    kept = {}

    def confirm(i):
        if i not in kept:
            xb, sb, _ = siggen.torch_planted_batch(n, k, [8000 + 100 * i + s for s in range(count)], dev,
                                                   magnitude="loguniform")
            kept[i] = (xb, torch.arange(count, dtype=torch.int64, device=dev) * 29 + 3 + i, sb)
        return kept[i]

    res = autotune.tune(X, k, sfft.SFFT_MODE_EXACT, seeds=seeds, truth=sups, base=base, space=space, reps=2,
                        cache=cache, confirm=confirm, confirm_batches=2)
    assert res.quality == 1.0 and res.B in (128, 256) and res.confirm_batches == 2
    assert res.fields["b_min"] in (16, 32) and res.fields["hash_threads"] in (256, 512)
    ok = [r for r in res.table if "ms" in r]
    assert len(ok) >= 4 and all(r["quality"] == 1.0 for r in ok)
    ref_ms = ok[0]["ms"]                                  # the reference candidate runs first
    assert res.ms <= ref_ms
    hit = autotune.tune(X, k, sfft.SFFT_MODE_EXACT, seeds=seeds, truth=sups, base=base, space=space,
                        cache=cache)
    assert hit.from_cache and hit.B == res.B and hit.fields == res.fields and hit.confirm_batches == 2
    plan = sfft.Plan(n, k, res.B, 0, 0, max_batch=count, **{f: v for f, v in res.fields.items()})
    bufs = plan.execute_batch(X, seeds)
    torch.cuda.synchronize()
    counts = bufs["counts"].cpu().numpy()
    idx = bufs["idx"].cpu().numpy()
    for s in range(count):
        assert np.array_equal(idx[s, :counts[s]], np.sort(sups[s]))
    plan.close()


def test_autotune_incumbent_joins_the_search():
    """A known-good candidate outside the search space (an incumbent, e.g. a
    stored choice of another build) is timed right after the reference,
    takes part in the confirmations, and the choice is no slower than it."""
    import torch
    from paper_1201_2501_amd import autotune, sfft

    sfft.load()
    dev = torch.device("cuda:0")
    n, k, count = 1 << 18, 32, 32
    say("autotune-incumbent", "n", n, "k", k, "count", count)
    X, sups, _ = siggen.torch_planted_batch(n, k, [9000 + s for s in range(count)], dev, magnitude="loguniform")
    seeds = torch.arange(count, dtype=torch.int64, device=dev) * 17 + 1
    space = {"bins": {"B": [256]}, "window": {"delta": [1e-9]}, "schedule": {"b_min": [32], "patience": [4]}}
    base = dict(theta=0.02, rounds=24, loc_prec=sfft.SFFT_F64)
    kept = {}

    def confirm(i):
        if i not in kept:
            xb, sb, _ = siggen.torch_planted_batch(n, k, [9500 + 100 * i + s for s in range(count)], dev,
                                                   magnitude="loguniform")
            kept[i] = (xb, torch.arange(count, dtype=torch.int64, device=dev) * 23 + 7 + i, sb)
        return kept[i]

    inc = dict(B=128, b_min=16, patience=4, delta=1e-9)
    res = autotune.tune(X, k, sfft.SFFT_MODE_EXACT, seeds=seeds, truth=sups, base=base, space=space, reps=2,
                        confirm=confirm, confirm_batches=2, incumbents=[inc])
    rec = res.table[1]
    assert rec["cand"]["B"] == 128 and rec["cand"]["b_min"] == 16 and "ms" in rec
    assert res.quality == 1.0
    assert res.ms <= res.table[0]["ms"]                  # no slower than the reference
    if res.B == 128:                                     # the incumbent (or a launch variant of it) won
        assert res.ms <= rec["ms"] * 1.02
    # with a wide margin a confirmed incumbent is kept whatever else is faster
    keep = autotune.tune(X, k, sfft.SFFT_MODE_EXACT, seeds=seeds, truth=sups, base=base, space=space, reps=2,
                         confirm=confirm, confirm_batches=2, incumbents=[inc], incumbent_margin=100.0)
    inc_rec = keep.table[1]
    if inc_rec["quality"] == 1.0 and keep.B != 128:
        # only a failed confirmation may drop it
        assert keep.quality == 1.0
    elif inc_rec["quality"] == 1.0:
        assert keep.fields["b_min"] == 16


def test_autotune_small_general_batch(tmp_path):
    """General mode: candidates are accepted on their recall of the planted
    heads (within the slack of the reference candidate's), the choice keeps
    that recall on a fresh batch, and it is no slower than the reference."""
    import torch
    from paper_1201_2501_amd import autotune, sfft

    sfft.load()
    dev = torch.device("cuda:0")
    n, k, count = 1 << 18, 16, 16
    say("autotune-general", "n", n, "k", k, "count", count)

    def batch(base):
        X, sups, _ = siggen.torch_planted_batch(n, k, [base + s for s in range(count)], dev, magnitude="unit",
                                                noise_ratio=0.05)
        return X, torch.arange(count, dtype=torch.int64, device=dev) * 7 + base, sups

    X, seeds, sups = batch(12_000)
    kept = {}

    def confirm(i):
        if i not in kept:
            kept[i] = batch(13_000 + 100 * i)
        return kept[i]

    space = {"bins": {"B": [256, 512]}, "window": {"delta": [1e-6]},
             "schedule": {"R_est": [5, 7], "R_loc": [3]}, "launch": {"hash_threads": [256, 512]}}
    res = autotune.tune(X, k, sfft.SFFT_MODE_GENERAL, seeds=seeds, truth=sups, space=space, reps=2,
                        cache=str(tmp_path / "t.json"), confirm=confirm, confirm_batches=1)
    ok = [r for r in res.table if "ms" in r]
    ref = ok[0]
    assert res.B in (256, 512) and res.fields["R_est"] in (5, 7)
    assert res.quality >= ref["quality"] - 0.005 and res.ms <= ref["ms"]
    plan = sfft.Plan(n, k, res.B, 0, 0, max_batch=count, **res.fields)
    Xc, sc, supc = confirm(0)
    bufs = plan.execute_batch(Xc, sc)
    torch.cuda.synchronize()
    counts = bufs["counts"].cpu().numpy()
    idx = bufs["idx"].cpu().numpy()
    recall = np.mean([len(np.intersect1d(idx[s, :counts[s]], supc[s])) / k for s in range(count)])
    assert recall >= 0.95
    plan.close()
