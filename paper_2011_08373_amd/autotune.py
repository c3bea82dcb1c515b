"""Autotuner of the radix sort: digit width and scatter tile shape.

For a set of kernels (one size class) it times each (digit bits, tile shape)
pair with the library's own hipEvent timings of the sort passes and keeps the
fastest.  Results are cached in tuning.json next to this file, keyed by the
GPU architecture and a size bucket (log2 of the access count), and applied
through rp_set_tuning before a run.
"""
from __future__ import annotations

import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuning.json")
CANDIDATES = [(rb, shape) for rb in (8, 9, 10, 11) for shape in range(10)]


def _arch() -> str:
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def bucket(n_accesses: int) -> str:
    return "2^%d" % max(0, int(math.log2(max(1, n_accesses))))


def _load() -> dict:
    if os.path.exists(CACHE):
        with open(CACHE) as f:
            return json.load(f)
    return {}


def lookup(n_accesses: int):
    return _load().get(_arch(), {}).get(bucket(n_accesses))


def apply(n_accesses: int) -> bool:
    """Set the knobs from the cache; False if this size class is not tuned."""
    from . import librepair as L
    best = lookup(n_accesses)
    if not best:
        return False
    L.set_tuning(L.TUNE_SORT_DIGIT_BITS, best["digit_bits"])
    L.set_tuning(L.TUNE_SCATTER_SHAPE, best["shape"])
    return True


def tune(kms, reps: int = 3, ws=None) -> dict:
    """Time every candidate on a batch (or one kernel) and cache the best."""
    from . import librepair as L
    batch = isinstance(kms, (list, tuple)) or isinstance(kms, L.BatchArg)
    results = []
    for rb, shape in CANDIDATES:
        L.set_tuning(L.TUNE_SORT_DIGIT_BITS, rb)
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
            results.append((min(times), rb, shape, L.last_stats()["accesses"]))
    if not results:
        raise RuntimeError("no sort configuration ran")
    results.sort()
    t, rb, shape, acc = results[0]
    data = _load()
    data.setdefault(_arch(), {})[bucket(acc)] = dict(digit_bits=rb, shape=shape, ms=t)
    with open(CACHE, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    L.set_tuning(L.TUNE_SORT_DIGIT_BITS, rb)
    L.set_tuning(L.TUNE_SCATTER_SHAPE, shape)
    return dict(digit_bits=rb, shape=shape, ms=t, table=[(r[1], r[2], r[0]) for r in results])
