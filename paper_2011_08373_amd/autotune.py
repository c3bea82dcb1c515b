"""Autotuner of the radix sort: digit widths and scatter tile shapes.

For a set of kernels (one size class) it times each (digits, tile shape)
pair with the library's own hipEvent timings of record generation and the
sort passes and keeps the fastest; then it tries every tile for each pass on
its own, the other passes fixed, and keeps a pass's tile where it is faster.  Digits are either of one width (8..11
bits) or automatic with a narrow lowest digit (6..9 bits; the rest of the
key in digits of at most 10 bits).  Results are cached in tuning.json next to
this file, keyed by the GPU architecture and a size class: log2 of the access
count and the radix key's width in bits (which sets how many passes each
digit width needs).  They are applied through rp_set_tuning before a run.

    python -m paper_2011_08373_amd.autotune [--out FILE] [--passes] [workload ...]

tunes the named workloads (default: the stress kernel in both modes, the
plain-large kernel in both modes and the batched kernels) and rewrites their
entries (in FILE instead of tuning.json when given; it starts from a copy of
tuning.json).  With --passes, a size class already in the cache keeps its
digits and common tile and only the per-pass tiles are tuned again.
"""
from __future__ import annotations

import json
import math
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning.json")
_out = [None]                 # where tune() writes (None: CACHE)
# (digit bits, lowest digit bits): one width (rb, 0), or automatic widths
# with a narrow lowest digit (0, low)
DIGITS = [(0, 6), (0, 7), (0, 8), (0, 9), (8, 0), (9, 0), (10, 0), (11, 0)]
SHAPES = 10                   # radix-scatter tile shapes 0..9
CANDIDATES = [(dg, shape) for dg in DIGITS for shape in range(SHAPES)]


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def bucket(n_accesses: int, key_bits: int) -> str:
    return "2^%d/k%d" % (max(0, int(math.log2(max(1, n_accesses)))), int(key_bits))


def _load() -> dict:
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def lookup(n_accesses: int, key_bits: int):
    return _load().get(_arch(), {}).get(bucket(n_accesses, key_bits))


def apply(n_accesses: int, key_bits: int) -> bool:
    """Set the knobs from the cache; False if this size class is not tuned."""
    from . import librepair as L
    best = lookup(n_accesses, key_bits)
    if not best:
        return False
    L.set_tuning(L.TUNE_SORT_DIGIT_BITS, best["digit_bits"])
    L.set_tuning(L.TUNE_LOW_DIGIT_BITS, best.get("low_digit_bits", 0))
    L.set_tuning(L.TUNE_SCATTER_SHAPE, best["shape"])
    L.set_tuning(L.TUNE_PASS_SHAPES, L.pass_shapes_value(best.get("pass_shapes", [])))
    return True


def _time(L, kms, batch, ws, reps):
    """Best of reps runs' generation + sort time (ms), None if a run fails
    (e.g. the workspace cannot hold this digit width)."""
    times = []
    for _ in range(reps):
        if batch:
            ok = L.repair_batch(kms, ws=ws)[0] == 0
        else:
            ok = L.repair(kms, ws=ws)["ret"] in (L.OK, L.UNSAT)
        if not ok:
            return None
        s = L.last_stats()
        times.append(s["ms_sort"] + s["ms_gen"])
    return min(times)


def tune(kms, reps: int = 3, ws=None, candidates=None, passes_only: bool = False) -> dict:
    """Time every candidate on a batch (or one kernel) and cache the best."""
    from . import librepair as L
    batch = isinstance(kms, (list, tuple)) or isinstance(kms, L.BatchArg)
    if batch and not isinstance(kms, L.BatchArg):
        kms = L.BatchArg(kms)
    elif not batch:
        kms = L.KernelArg(kms)
    key_bits = L.sort_key_bits(kms)
    results = []
    L.set_tuning(L.TUNE_PASS_SHAPES, L.PASS_SHAPES_DEFAULT)
    cached = None
    if passes_only:
        if batch:
            L.repair_batch(kms, ws=ws)
        else:
            L.repair(kms, ws=ws)
        cached = lookup(L.last_stats()["accesses"], key_bits)
    if cached:
        candidates = [((cached["digit_bits"], cached.get("low_digit_bits", 0)), cached["shape"])]
    for (rb, low), shape in candidates or CANDIDATES:
        L.set_tuning(L.TUNE_SORT_DIGIT_BITS, rb)
        L.set_tuning(L.TUNE_LOW_DIGIT_BITS, low)
        L.set_tuning(L.TUNE_SCATTER_SHAPE, shape)
        t = _time(L, kms, batch, ws, reps)
        if t is not None:
            results.append((t, rb, low, shape, L.last_stats()["accesses"]))
    if not results:
        raise RuntimeError("no sort configuration ran")
    results.sort()
    t, rb, low, shape, acc = results[0]
    # then each pass's tile on its own, the other passes fixed
    L.set_tuning(L.TUNE_SORT_DIGIT_BITS, rb)
    L.set_tuning(L.TUNE_LOW_DIGIT_BITS, low)
    L.set_tuning(L.TUNE_SCATTER_SHAPE, shape)
    passes = L.last_stats()["sort_passes"]
    per_pass = [shape] * min(passes, 7)
    for p in range(len(per_pass)):
        for sh in range(SHAPES):
            if sh == per_pass[p]:
                continue
            trial = per_pass[:p] + [sh] + per_pass[p + 1:]
            L.set_tuning(L.TUNE_PASS_SHAPES, L.pass_shapes_value(trial))
            tt = _time(L, kms, batch, ws, reps)
            if tt is not None and tt < 0.995 * t:    # a clear gain, not noise
                t, per_pass = tt, trial
    pass_shapes = [None if sh == shape else sh for sh in per_pass]
    if all(sh is None for sh in pass_shapes):
        pass_shapes = []
    L.set_tuning(L.TUNE_PASS_SHAPES, L.pass_shapes_value(pass_shapes))
    dest = _out[0] or CACHE
    data = _load() if dest == CACHE or not os.path.exists(dest) else json.load(open(dest))
    data.setdefault(_arch(), {})[bucket(acc, key_bits)] = dict(
        digit_bits=rb, low_digit_bits=low, shape=shape, pass_shapes=pass_shapes, ms=t)
    with open(dest, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    L.set_tuning(L.TUNE_SORT_DIGIT_BITS, rb)
    L.set_tuning(L.TUNE_LOW_DIGIT_BITS, low)
    L.set_tuning(L.TUNE_SCATTER_SHAPE, shape)
    return dict(digit_bits=rb, low_digit_bits=low, shape=shape, pass_shapes=pass_shapes, ms=t,
                key_bits=key_bits, table=[(r[1], r[2], r[3], r[0]) for r in results])


# (plain-large's two modes share a size class: the literal one, tuned last,
# keeps it)
WORKLOADS = ("stress-literal", "stress-planted", "plain-large-planted", "plain-large-literal",
             "batched")


def main(argv):
    import torch
    from . import librepair as L, synth
    if argv[:1] == ["--out"]:
        _out[0] = argv[1]
        argv = argv[2:]
    passes_only = argv[:1] == ["--passes"]
    if passes_only:
        argv = argv[1:]
    torch.cuda.set_device(0)
    ws = L.Workspace()
    for name in argv or WORKLOADS:
        if name == "batched":
            kms = synth.generate_batch(mode="planted")
            reps = 3
        else:
            cfg, mode = name.rsplit("-", 1)
            kms = synth.generate(cfg, mode=mode)
            reps = 2 if cfg == "stress" else 3
        r = tune(kms, reps=reps, ws=ws, passes_only=passes_only)
        best = sorted(r["table"], key=lambda e: e[3])[:5]
        print(json.dumps({"workload": name, "key_bits": r["key_bits"],
                          "digit_bits": r["digit_bits"], "low_digit_bits": r["low_digit_bits"],
                          "shape": r["shape"], "pass_shapes": r["pass_shapes"], "ms": r["ms"],
                          "best5": best}), flush=True)
        ws.t = None
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main(sys.argv[1:])
