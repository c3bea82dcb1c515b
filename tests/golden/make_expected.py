"""Write the oracle's results for the full-size synthetic workloads.

Calls only the CPU oracle (oracle/) on seeded inputs from the generator.
Output: tests/golden/expected_<name>.json.  Run from the repository root:

    python tests/golden/make_expected.py [name ...]

Names: plain_large, max_points, batched, stress_literal, stress_planted
(default: all).  The stress kernel (about 1.9G accesses) is checked with
the oracle's one-instance-at-a-time route on every host core (a few minutes
per Verify call and 7 GB of memory); the batched kernels are repaired on a
pool of host threads, one kernel per thread.
"""
import json
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

from oracle import oracle as O  # noqa: E402
from paper_2011_08373_amd import synth  # noqa: E402
from golden_util import encode_pairs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
REPAIR_KEYS = ("status", "assign", "weight", "added", "removed", "rounds", "n_clauses",
               "trajectory")


def _write(name, out, t):
    path = os.path.join(HERE, "expected_%s.json" % name)
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(name, "%.1fs" % (time.time() - t), path, flush=True)


def record(name, km, xs, compact=False):
    """Verify (pairs, divergent slots, access count) and GenerateClause under
    each x, and the repair loop with every trace learned per call."""
    t = time.time()
    out = dict(config=km.meta.get("config"), seed=km.meta.get("seed"),
               mode=km.meta.get("mode"), checks={}, clauses={})
    for x in xs:
        st, pairs, div, nrec = O.check(km, x)
        c = dict(status=st, divergent=div, n_records=nrec, n_pairs=len(pairs))
        if compact:
            c["pairs_z"] = encode_pairs(pairs, km.n_points)
        else:
            c["pairs"] = [list(p) for p in pairs]
        out["checks"][str(x)] = c
        st, cl = O.clauses(km, x)
        out["clauses"][str(x)] = [list(q) for q in cl]
        print("  %s x=%#x: %d pairs, %d clauses, %.0fs" % (name, x, len(pairs), len(cl),
                                                          time.time() - t), flush=True)
    # learn-all policy only: the one-trace policy needs one full-size
    # Verify per learned clause, hours of oracle time at this size
    out["repair_policy0"] = O.repair(km, policy=0)
    if "x_star" in km.meta:
        out["x_star"] = km.meta["x_star"]
    _write(name, out, t)
    return out


def plain_large():
    km = synth.generate("plain-large", mode="literal")
    record("plain_large_literal", km, [0])
    kp = synth.generate("plain-large", mode="planted")
    r = O.repair(kp)
    record("plain_large_planted", kp, [0, kp.meta["x_star"], r["assign"]])


def max_points():
    km = synth.max_points_kernel()
    r = O.repair(km)
    record("max_points", km, [0, km.meta["x_star"], r["assign"]], compact=True)


def stress(mode):
    O.set_route(1, 0)
    try:
        km = synth.generate("stress", mode=mode)
        if mode == "literal":
            # no barrier and every barrier enabled
            xs = [0, (1 << km.n_slots) - 1]
            record("stress_literal", km, xs, compact=True)
        else:
            # the route to the result is known only after the repair: the
            # repair runs first (a few minutes), then the three checks
            r = O.repair(km, policy=0)
            record("stress_planted", km, [0, km.meta["x_star"], r["assign"]], compact=True)
    finally:
        O.set_route(0)


def batched(threads=None):
    """Every kernel of the 1,024-kernel batched workload, planted and
    literal: the repair result of each, and Verify / GenerateClause at x = 0
    for 16 planted kernels spread over the size range (the largest
    included)."""
    t = time.time()
    threads = threads or os.cpu_count() or 4
    O.set_route(0)
    out = dict(config="batched", seed=3, n=1024)
    for mode in ("planted", "literal"):
        kms = synth.generate_batch(mode=mode)

        def one(k):
            r = O.repair(k, policy=0)
            return {key: r[key] for key in REPAIR_KEYS}
        with ThreadPoolExecutor(threads) as ex:
            out["repair_" + mode] = list(ex.map(one, kms))
        print("  batched %s: %.0fs" % (mode, time.time() - t), flush=True)
        if mode == "planted":
            size = [(int(k.blocks) * int(k.threads) * int((k.points["kind"] == 0).sum()), q)
                    for q, k in enumerate(kms)]
            size.sort()
            pick = sorted({size[int(round(f * (len(size) - 1)))][1]
                           for f in [q / 15 for q in range(16)]})
            out["checked"] = {}
            for q in pick:
                km = kms[q]
                st, pairs, div, nrec = O.check(km, 0)
                st2, cl = O.clauses(km, 0)
                out["checked"][str(q)] = dict(status=st, pairs=[list(p) for p in pairs],
                                              divergent=div, n_records=nrec,
                                              clauses=[list(c) for c in cl])
    _write("batched", out, t)


def main():
    names = sys.argv[1:] or ["plain_large", "max_points", "batched", "stress_literal",
                             "stress_planted"]
    for n in names:
        if n == "plain_large":
            plain_large()
        elif n == "max_points":
            max_points()
        elif n == "batched":
            batched()
        elif n == "stress_literal":
            stress("literal")
        elif n == "stress_planted":
            stress("planted")
        else:
            raise SystemExit("unknown name %s" % n)


if __name__ == "__main__":
    main()
