"""Autotuner of the batched sparse FFT: chooses the bin count B, the flat
window (Gaussian or Kaiser-Bessel) and its length w (through its accuracy
delta), the round schedule and the launch
shape of a batch of one shape by measuring candidate plans on calibration
signals on the device.

The method fixes its parameters only up to constants (B = O(k), a window of
O(B log(n/delta)) samples, the number of rounds), so their best values depend
on the signals and the device.  A candidate is accepted only if its results
are as good as those of a conservative reference candidate on the same
calibration batch:

  * exact mode: every signal's recovered support equals the planted support
    (when `truth` is given) or the reference candidate's support;
  * general mode: the mean fraction of planted (or reference) coefficients
    found is within `recall_slack` of the reference candidate's.

Among accepted candidates the fastest (median time of `reps` replayed batch
steps, HIP events) wins.  The search is coordinate-wise with a small beam,
stage by stage in the order of the space (by default: the bin count, the
window, the round schedule, the decode thresholds, the count stop), each
stage varying its fields around each of the `beam` fastest accepted
candidates so far; the launch-shape stages (HashToBins workgroup size, batch
chunks, first round group), which cannot change results, run last, around
the configuration that survives confirmation.

One calibration batch cannot show a per-signal failure rate of 1e-3, and a
shorter window or an earlier stop can have one.  With `confirm` (a function
returning fresh batches; it is called again for the same index, so it should
keep them), after every result-affecting stage the `confirm_top` fastest
accepted configurations not yet confirmed run on `confirm_batches` new
batches beside the reference candidate (one plan per configuration; launch
variants of a configuration give the same results).  A configuration
survives when it recovers every signal the reference recovers (exact mode)
or stays within recall_slack of the reference's recall (general mode);
rejected configurations no longer count as accepted, so later stages start
from confirmed ones.  The fastest confirmed configuration wins.

Results are cached in a JSON file keyed by device, shape, batch size and the
library's kernel sources, so a shape is tuned once per device and build.

    from paper_1201_2501_amd import autotune
    res = autotune.tune(x, k, truth=supports, cache="tuned.json")
    plan = Plan(n, k, res.B, 0, 0, max_batch=len(x), **res.fields)
"""
import hashlib
import json
import os
import statistics
import time
from dataclasses import dataclass, field

import numpy as np

from . import sfft

PKG = os.path.dirname(os.path.abspath(__file__))
_SOURCES = ("sfft_kernels.hip", "sfft_pair.hpp", "sfft_decode.hip", "sfft_host.cpp", "sfft_common.hpp", "sfft_internal.hpp",
            "sfft_device.hpp")


def library_hash():
    """Hash of the library sources the tuned timings depend on."""
    h = hashlib.sha256()
    for f in _SOURCES:
        path = os.path.join(PKG, "csrc", f)
        if os.path.exists(path):
            h.update(open(path, "rb").read())
    return h.hexdigest()[:16]


def pow2_range(lo, hi):
    out, v = [], 1
    while v <= hi:
        if v >= lo:
            out.append(v)
        v <<= 1
    return out


def default_space(n, k, mode, theta=0.25):
    """Candidate values per stage, searched in this order.  B stays within
    the kernels' limit (4096) and at most n/16; exact mode starts at 2k
    bins, general mode at 4k.  theta: the caller's bin threshold (exact
    mode also tries half of it: a coefficient is hidden in a round only when
    G' |c| < theta, so a lower threshold needs fewer empty rounds)."""
    if mode == sfft.SFFT_MODE_EXACT:
        lo = max(64, 2 * k)
        Bs = pow2_range(lo, min(4096, n // 16)) or [min(4096, max(2, n // 16))]
        Bs = [b for b in Bs if b >= 512] or Bs[-2:]
        return {
            "bins": {"B": Bs},
            "window": {"window": [0, 1], "delta": [1e-10, 1e-9, 1e-8, 1e-7, 1e-6], "alpha": [0.5, 0.6, 0.7, 0.75, 0.8]},
            "schedule": {"b_min": [16, 32, 64], "patience": [3, 4, 5]},
            "decode": {"theta": [theta, theta / 2], "g_min": [0.25, 0.4], "ratio_tol": [0.0, 0.002, 0.01]},
            "stop": {"stop_count": [0, k], "stop_patience": [2, 3], "patience": [3, 4, 5]},
            "launch": {"hash_threads": [256, 512, 1024], "chunks": [1, 2]},
            "groups": {"group0_offset": [0, -1, 1, 2], "group_step": [0, 3, 4]},
        }
    lo = max(256, 4 * k)
    Bs = pow2_range(lo, min(4096, n // 16)) or [min(4096, max(2, n // 16))]
    return {
        "bins": {"B": Bs[:3]},
        "window": {"window": [0, 1], "delta": [1e-7, 1e-6]},
        "schedule": {"R_est": [5, 7, 9], "R_loc": [3, 4]},
        "launch": {"hash_threads": [256, 512, 1024], "chunks": [1, 2]},
    }


def first_floor_round(B, b_min):
    """Exact mode: the first round whose bin count B >> r has reached b_min."""
    r = 0
    while (B >> r) > max(b_min, 1) and (B >> (r + 1)) >= max(b_min, 1):
        r += 1
    return r


# stages and fields that choose only the launch shape: results do not depend on them
LAUNCH_STAGES = ("launch", "groups")
LAUNCH_FIELDS = ("hash_threads", "chunks", "group0", "group0_offset", "group_step")


def signature(cand):
    """The fields of a candidate that can change its results."""
    return tuple(sorted((f, v) for f, v in cand.items() if f not in LAUNCH_FIELDS))


def launch_changes(cand):
    """Number of launch fields set away from the library defaults."""
    return (int(cand.get("hash_threads", 256) != 256) + int(cand.get("chunks", 1) not in (0, 1)) +
            int(bool(cand.get("group0"))) + int(bool(cand.get("group_step"))))


def normalize(cand):
    """Drop fields that do not change the plan (stop_patience without
    stop_count) and turn group0_offset (rounds relative to the library's
    default first round group: first b_min round + patience + 1) into
    group0, so equal plans compare equal."""
    c = dict(cand)
    if not c.get("stop_count"):
        c.pop("stop_patience", None)
    if not c.get("group_step"):
        c.pop("group_step", None)
    off = c.pop("group0_offset", None)
    if off is not None:
        c.pop("group0", None)
        if off:
            auto = first_floor_round(c["B"], c.get("b_min") or max(2, c["B"] >> 4)) + c.get("patience", 3) + 1
            c["group0"] = max(1, min(auto + off, c.get("rounds") or 16))
    return c


def reference_candidate(space, mode, base):
    """The conservative candidate every other one is compared with: the
    largest B, the smallest delta and the slowest-stopping schedule."""
    c = dict(base)
    c["B"] = max(space["bins"]["B"])
    c["delta"] = min(space["window"]["delta"])
    c["window"] = 0
    if "alpha" in space["window"]:
        c["alpha"] = min(space["window"]["alpha"])
    if mode == sfft.SFFT_MODE_EXACT:
        c["b_min"] = max(space["schedule"]["b_min"])
        c["patience"] = max(space["schedule"]["patience"])
        c["stop_count"] = 0
    else:
        c["R_est"] = max(space["schedule"]["R_est"])
        c["R_loc"] = max(space["schedule"]["R_loc"])
    c["hash_threads"] = 256
    c["chunks"] = 1
    return normalize(c)


@dataclass
class TuneResult:
    B: int
    fields: dict
    ms: float
    rate: float
    quality: float
    key: str
    from_cache: bool = False
    table: list = field(default_factory=list)
    confirm_batches: int = 0

    def as_dict(self):
        return {"B": self.B, "fields": self.fields, "ms": self.ms, "rate": self.rate, "quality": self.quality,
                "key": self.key, "from_cache": self.from_cache, "candidates": len(self.table),
                "confirm_batches": self.confirm_batches}


def device_tag(device):
    """Architecture and compute-unit count of a torch device (stable across
    runtimes, unlike the marketing name)."""
    import torch

    pr = torch.cuda.get_device_properties(device)
    arch = getattr(pr, "gcnArchName", "") or pr.name
    return "%s-%dcu" % (arch.split(":")[0], pr.multi_processor_count)


def cache_key(n, k, mode, count, in_dtype, device_name):
    return "%s|n=%d|k=%d|mode=%d|count=%d|dtype=%d|lib=%s" % (device_name, n, k, mode, count, in_dtype,
                                                              library_hash())


def lookup(cache, n, k, mode, count, in_dtype, device_name, any_build=False):
    """The cached TuneResult of a shape, or None.  any_build: without an entry
    for the current library build, take one stored by another build for the
    same device and shape (its plan is valid; its timings may not be
    current); from_cache is then "other build"."""
    key = cache_key(n, k, mode, count, in_dtype, device_name)
    data = _load_cache(cache)
    rec, how = data.get(key), True
    if not rec and any_build:
        prefix = key[:key.rindex("|lib=")]
        others = [(kk, r) for kk, r in data.items() if kk.startswith(prefix + "|lib=")]
        if others:
            key, rec = others[-1]
            how = "other build"
    if not rec:
        return None
    return TuneResult(B=rec["B"], fields=rec["fields"], ms=rec["ms"], rate=rec["rate"], quality=rec["quality"],
                      key=key, from_cache=how, confirm_batches=rec.get("confirm_batches", 0))


def _load_cache(path):
    if not path or not os.path.exists(path):
        return {}
    try:
        return json.load(open(path))
    except ValueError:
        return {}


def _store_cache(path, key, rec):
    if not path:
        return
    data = _load_cache(path)
    data[key] = rec
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


class _Runner:
    """Builds, times and scores candidate plans on one calibration batch."""

    def __init__(self, x, k, mode, seeds, truth, reps, log):
        import torch

        self.torch = torch
        self.x, self.k, self.mode, self.seeds = x, k, mode, seeds
        self.n, self.count = int(x.shape[1]), int(x.shape[0])
        self.in_dtype = sfft.SFFT_C128 if x.dtype == torch.complex128 else sfft.SFFT_C64
        self.truth = None if truth is None else [np.sort(np.asarray(t, dtype=np.int64)) for t in truth]
        self.reps, self.log = reps, log
        self.ref_supports = None
        self.table = []

    def run(self, cand, x=None, seeds=None, reps=None):
        """(median ms per batch step, per-signal supports) of one candidate
        on the calibration batch (or on x, seeds), or None when its plan is
        not valid for this shape."""
        torch = self.torch
        if x is None:
            x, seeds = self.x, self.seeds
        count = int(x.shape[0])
        fields = {f: v for f, v in cand.items() if f not in ("B", "in_dtype", "max_batch")}
        try:
            plan = sfft.Plan(self.n, self.k, cand["B"], 0, 0, in_dtype=self.in_dtype, max_batch=count, **fields)
        except sfft.SfftError as e:
            self.table.append({"cand": cand, "error": str(e)})
            return None
        try:
            bufs = plan.batch_buffers(count, x.device)
            plan.execute_batch(x, seeds, bufs=bufs)                  # capture + warm-up
            torch.cuda.synchronize()
            times = []
            for _ in range(self.reps if reps is None else reps):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                plan.execute_batch(x, seeds, bufs=bufs)
                e1.record()
                torch.cuda.synchronize()
                times.append(e0.elapsed_time(e1))
            counts = bufs["counts"].cpu().numpy()
            idx = bufs["idx"].cpu().numpy()
            sups = [idx[s, :counts[s]].copy() for s in range(count)]
        finally:
            plan.close()
        return (statistics.median(times) if times else float("nan")), sups

    def run_batches(self, cand, batches):
        """Supports of one candidate on each (x, seeds) of `batches`, from one
        plan; None when its plan is not valid."""
        torch = self.torch
        fields = {f: v for f, v in cand.items() if f not in ("B", "in_dtype", "max_batch")}
        count = max(int(x.shape[0]) for x, _ in batches)
        try:
            plan = sfft.Plan(self.n, self.k, cand["B"], 0, 0, in_dtype=self.in_dtype, max_batch=count, **fields)
        except sfft.SfftError:
            return None
        out = []
        try:
            for x, seeds in batches:
                bufs = plan.execute_batch(x, seeds)
                torch.cuda.synchronize()
                counts = bufs["counts"].cpu().numpy()
                idx = bufs["idx"].cpu().numpy()
                out.append([idx[s, :counts[s]].copy() for s in range(int(x.shape[0]))])
        finally:
            plan.close()
        return out

    def quality(self, sups, target=None):
        """Exact mode: fraction of signals whose support equals the target;
        general mode: mean fraction of target coefficients found."""
        if target is None:
            target = self.truth if self.truth is not None else self.ref_supports
        if self.mode == sfft.SFFT_MODE_EXACT:
            return float(np.mean([np.array_equal(s, t) for s, t in zip(sups, target)]))
        return float(np.mean([len(np.intersect1d(s, t)) / max(1, len(t)) for s, t in zip(sups, target)]))

    def survives(self, sups, ref_sups, truth, slack):
        """Whether a candidate's supports on a confirmation batch are as good
        as the reference candidate's on the same batch."""
        if truth is None:
            if self.mode == sfft.SFFT_MODE_EXACT:
                return all(np.array_equal(s, r) for s, r in zip(sups, ref_sups))
            return self.quality(sups, ref_sups) >= 1.0 - slack - 1e-12
        if self.mode == sfft.SFFT_MODE_EXACT:
            return all(np.array_equal(s, t) or not np.array_equal(r, t) for s, r, t in zip(sups, ref_sups, truth))
        return self.quality(sups, truth) >= self.quality(ref_sups, truth) - slack - 1e-12

    def evaluate(self, cand):
        out = self.run(cand)
        if out is None:
            return None
        ms, sups = out
        q = self.quality(sups) if (self.truth is not None or self.ref_supports is not None) else 1.0
        rec = {"cand": dict(cand), "ms": round(ms, 4), "quality": q}
        self.table.append(rec)
        if self.log:
            self.log("autotune: %s -> %.3f ms, quality %.4f" % (
                ", ".join("%s=%s" % kv for kv in sorted(cand.items())), ms, q))
        return rec, sups


def tune(x, k, mode=sfft.SFFT_MODE_EXACT, seeds=None, truth=None, base=None, space=None, reps=3,
         budget_s=120.0, cache=None, recall_slack=0.005, log=None, force=False, confirm=None,
         confirm_batches=4, confirm_top=16, beam=3, launch_margin=0.01, passes=2, incumbents=None,
         incumbent_margin=0.02):
    """Tune the plan of a batch x ([count, n] complex device tensor) with
    sparsity k.  base: plan fields kept fixed (e.g. theta, rounds, loc_prec,
    flags); space: {"bins": {...}, "window": {...}, "schedule": {...}, ...}
    lists of candidate values (default_space when None); truth: per-signal
    planted supports, else the reference candidate's supports are the
    target; confirm: i -> (x_i, seeds_i, truth_i or None), fresh batches of
    the same shape for the confirmations (called again for the same i);
    incumbents: complete candidates (plan fields with "B") known to be good,
    e.g. a stored choice of another library build: they are timed after the
    reference and take part in the beam and the confirmations like any
    other candidate, so that a search whose beam wanders (its order follows
    measured times) still compares against them; a confirmed incumbent is
    kept unless the choice is faster than it by more than incumbent_margin
    (timings of close variants differ by about 1 % from run to run, so
    without it a re-tune can swap one equivalent plan for another).
    Returns a TuneResult; with
    `cache`, a stored result for the same key is returned without measuring
    (unless force)."""
    import torch

    n, count = int(x.shape[1]), int(x.shape[0])
    base = dict(base or {})
    base.setdefault("mode", mode)
    space = space or default_space(n, k, mode, base.get("theta", 0.25))
    in_dtype = sfft.SFFT_C128 if x.dtype == torch.complex128 else sfft.SFFT_C64
    tag = device_tag(x.device)
    key = cache_key(n, k, mode, count, in_dtype, tag)
    if cache and not force:
        hit = lookup(cache, n, k, mode, count, in_dtype, tag)
        if hit:
            return hit

    runner = _Runner(x, k, mode, seeds, truth, reps, log)
    t_start = time.time()
    ref = reference_candidate(space, mode, base)
    out = runner.evaluate(ref)
    if out is None:
        raise RuntimeError("autotune: the reference candidate %r is not a valid plan" % ref)
    ref_rec, ref_sups = out
    runner.ref_supports = ref_sups
    inc_cands = []
    for inc in incumbents or []:
        cand = normalize(dict(base, **inc))
        inc_cands.append(cand)
        if not any(r.get("cand") == cand for r in runner.table):
            runner.evaluate(cand)
    if truth is None:
        ref_rec["quality"] = 1.0
    floor = ref_rec["quality"] - (recall_slack if mode == sfft.SFFT_MODE_GENERAL else 0.0)
    rejected = set()

    def accepted(rec):
        return rec["quality"] >= floor - 1e-12 and signature(rec["cand"]) not in rejected

    def ranked_accepted():
        return sorted((r for r in runner.table if "ms" in r and accepted(r)), key=lambda r: r["ms"])

    def stage(name, starts):
        grid = space.get(name, {})
        names = sorted(grid)
        combos = [{}]
        for f in names:
            combos = [dict(c, **{f: v}) for c in combos for v in grid[f]]
        for current in starts:
            for combo in combos:
                if time.time() - t_start > budget_s:
                    return
                cand = normalize(dict(current, **combo))
                if any(r.get("cand") == cand for r in runner.table):
                    continue
                runner.evaluate(cand)

    result_stages = [name for name in space if name not in LAUNCH_STAGES]
    launch_stages = [name for name in space if name in LAUNCH_STAGES]
    passed = {signature(ref_rec["cand"])}
    ref_on_batch = {}
    confirmed = 0

    def confirm_top_new():
        """Confirm the fastest accepted configurations not yet confirmed; a
        configuration that misses a signal the reference recovers on any
        confirmation batch is rejected (its candidates stop counting as
        accepted)."""
        nonlocal confirmed
        todo, seen = [], set()
        for r in ranked_accepted():
            sig = signature(r["cand"])
            if sig in passed or sig in seen:
                continue
            seen.add(sig)
            todo.append(r)
            if len(todo) == confirm_top:
                break
        if not todo:
            return
        batches, truths = [], []
        for i in range(confirm_batches):
            xb, sb, tb = confirm(i)
            batches.append((xb, sb))
            truths.append(None if tb is None else [np.sort(np.asarray(t, dtype=np.int64)) for t in tb])
        for i, b in enumerate(batches):
            if i not in ref_on_batch:
                got = runner.run_batches(ref_rec["cand"], [b])
                ref_on_batch[i] = got[0] if got else None
        for rec in todo:
            outs = runner.run_batches(rec["cand"], batches)
            ok = outs is not None and all(
                ref_on_batch[i] is not None and runner.survives(o, ref_on_batch[i], truths[i], recall_slack)
                for i, o in enumerate(outs))
            sig = signature(rec["cand"])
            if ok:
                passed.add(sig)
            else:
                rejected.add(sig)
                if log:
                    log("autotune: confirmation rejects %s" % ", ".join(
                        "%s=%s" % kv for kv in sorted(rec["cand"].items())))
        confirmed = confirm_batches

    use_confirm = confirm is not None and confirm_batches > 0
    # the stages interact (a shorter window can pass only with the decode
    # settings found later), so the result stages are searched `passes` times
    for _ in range(passes):
        for name in result_stages:
            stage(name, [dict(r["cand"]) for r in ranked_accepted()[:beam]])
            if use_confirm:
                confirm_top_new()
    survivors = passed if use_confirm else None

    def eligible():
        return [r for r in ranked_accepted() if survivors is None or signature(r["cand"]) in survivors]

    # launch shape around the fastest surviving configuration; a shape away
    # from the library defaults must be faster by more than launch_margin
    winner = eligible()[0]
    wsig = signature(winner["cand"])

    def variants():
        return [r for r in eligible() if signature(r["cand"]) == wsig]

    for name in launch_stages:
        stage(name, [dict(r["cand"]) for r in variants()[:beam]])
    fastest = variants()[0]["ms"]
    best = min((r for r in variants() if r["ms"] <= fastest * (1.0 + launch_margin)),
               key=lambda r: (launch_changes(r["cand"]), r["ms"]))
    for r in eligible():
        if r["cand"] in inc_cands and r["ms"] <= best["ms"] * (1.0 + incumbent_margin):
            best = r
            break

    cand = dict(best["cand"])
    B = int(cand.pop("B"))
    res = TuneResult(B=B, fields=cand, ms=best["ms"], rate=count / (best["ms"] * 1e-3), quality=best["quality"],
                     key=key, table=runner.table)
    if cache:
        _store_cache(cache, key, {"B": B, "fields": cand, "ms": res.ms, "rate": round(res.rate, 1),
                                  "quality": res.quality, "candidates": len(runner.table),
                                  "reference_ms": ref_rec["ms"], "confirm_batches": confirmed})
    res.confirm_batches = confirmed
    return res
