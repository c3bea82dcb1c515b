"""Autotuner of the radix sort: digit widths and scatter tile shape.

For a set of kernels (one size class) it times each (digits, tile shape)
pair with the library's own hipEvent timings of record generation and the
sort passes and keeps the fastest.  Digits are either of one width (8..11
bits) or automatic with a narrow lowest digit (6..9 bits; the rest of the
key in digits of at most 10 bits).  Results are cached in tuning.json next to
this file, keyed by the GPU architecture and a size class: log2 of the access
count and the radix key's width in bits (which sets how many passes each
digit width needs).  They are applied through rp_set_tuning before a run.

    python -m paper_2011_08373_amd.autotune [--out FILE] [workload ...]

tunes the named workloads (default: the stress kernel in both modes, the
plain-large kernel in both modes and the batched kernels) and rewrites their
entries (in FILE instead of tuning.json when given; it starts from a copy of
tuning.json).
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
CANDIDATES = [(dg, shape) for dg in DIGITS for shape in range(10)]


def has_narrow_pass(key_bits: int, digit_bits: int, low_digit_bits: int) -> bool:
    """Whether the library's digit plan for this key has a pass of at most 7
    bits (the passes RP_TUNE_NARROW_SHAPE applies to): only automatic widths
    above a narrow lowest digit give one (digits of one width are 8..11)."""
    rest = key_bits - low_digit_bits if key_bits > low_digit_bits else 0
    n = (rest + 9) // 10
    if digit_bits == 0 and low_digit_bits and rest > 0 and rest >= 6 * n:
        widths = [low_digit_bits] + [rest // n + (1 if i < rest % n else 0) for i in range(n)]
        return min(widths) <= 7
    return False


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
    L.set_tuning(L.TUNE_NARROW_SHAPE, best.get("narrow_shape", 10))
    return True


def tune(kms, reps: int = 3, ws=None, candidates=None) -> dict:
    """Time every candidate on a batch (or one kernel) and cache the best."""
    from . import librepair as L
    batch = isinstance(kms, (list, tuple)) or isinstance(kms, L.BatchArg)
    if batch and not isinstance(kms, L.BatchArg):
        kms = L.BatchArg(kms)
    elif not batch:
        kms = L.KernelArg(kms)
    key_bits = L.sort_key_bits(kms)
    results = []
    L.set_tuning(L.TUNE_NARROW_SHAPE, 10)
    for (rb, low), shape in candidates or CANDIDATES:
        L.set_tuning(L.TUNE_SORT_DIGIT_BITS, rb)
        L.set_tuning(L.TUNE_LOW_DIGIT_BITS, low)
        L.set_tuning(L.TUNE_SCATTER_SHAPE, shape)
        times = []
        for _ in range(reps):
            if batch:
                ok = L.repair_batch(kms, ws=ws)[0] == 0
            else:
                ok = L.repair(kms, ws=ws)["ret"] in (L.OK, L.UNSAT)
            if not ok:            # e.g. the workspace cannot hold this digit width
                break
            s = L.last_stats()
            times.append(s["ms_sort"] + s["ms_gen"])
        if len(times) == reps:
            results.append((min(times), rb, low, shape, L.last_stats()["accesses"]))
    if not results:
        raise RuntimeError("no sort configuration ran")
    results.sort()
    t, rb, low, shape, acc = results[0]
    # then the tile of the narrow-digit passes (at most 7 bits) on their own
    L.set_tuning(L.TUNE_SORT_DIGIT_BITS, rb)
    L.set_tuning(L.TUNE_LOW_DIGIT_BITS, low)
    L.set_tuning(L.TUNE_SCATTER_SHAPE, shape)
    narrow = 10
    for ns in range(10 if has_narrow_pass(key_bits, rb, low) else 0):
        if ns == shape:
            continue
        L.set_tuning(L.TUNE_NARROW_SHAPE, ns)
        times = []
        for _ in range(reps):
            if batch:
                ok = L.repair_batch(kms, ws=ws)[0] == 0
            else:
                ok = L.repair(kms, ws=ws)["ret"] in (L.OK, L.UNSAT)
            if not ok:
                break
            s = L.last_stats()
            times.append(s["ms_sort"] + s["ms_gen"])
        if len(times) == reps and min(times) < t:
            t, narrow = min(times), ns
    L.set_tuning(L.TUNE_NARROW_SHAPE, narrow)
    dest = _out[0] or CACHE
    data = _load() if dest == CACHE or not os.path.exists(dest) else json.load(open(dest))
    data.setdefault(_arch(), {})[bucket(acc, key_bits)] = dict(
        digit_bits=rb, low_digit_bits=low, shape=shape, narrow_shape=narrow, ms=t)
    with open(dest, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    L.set_tuning(L.TUNE_SORT_DIGIT_BITS, rb)
    L.set_tuning(L.TUNE_LOW_DIGIT_BITS, low)
    L.set_tuning(L.TUNE_SCATTER_SHAPE, shape)
    return dict(digit_bits=rb, low_digit_bits=low, shape=shape, narrow_shape=narrow, ms=t,
                key_bits=key_bits, table=[(r[1], r[2], r[3], r[0]) for r in results])


WORKLOADS = ("stress-literal", "stress-planted", "plain-large-literal", "plain-large-planted",
             "batched")


def main(argv):
    import torch
    from . import librepair as L, synth
    if argv[:1] == ["--out"]:
        _out[0] = argv[1]
        argv = argv[2:]
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
        r = tune(kms, reps=reps, ws=ws)
        best = sorted(r["table"], key=lambda e: e[3])[:5]
        print(json.dumps({"workload": name, "key_bits": r["key_bits"],
                          "digit_bits": r["digit_bits"], "low_digit_bits": r["low_digit_bits"],
                          "shape": r["shape"], "narrow_shape": r["narrow_shape"], "ms": r["ms"],
                          "best5": best}), flush=True)
        ws.t = None
        torch.cuda.empty_cache()


if __name__ == "__main__":
    main(sys.argv[1:])
