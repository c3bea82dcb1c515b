"""Write the oracle's results for the full-size synthetic workloads.

Calls only the CPU oracle (oracle/) on seeded inputs from the generator.
Output: tests/golden/expected_<name>.json.  Run from the repository root:

    python tests/golden/make_expected.py
"""
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import oracle as O  # noqa: E402
from paper_2011_08373_amd import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def record(name, km, xs):
    t = time.time()
    out = dict(config=km.meta.get("config"), seed=km.meta.get("seed"),
               mode=km.meta.get("mode"), checks={}, clauses={})
    for x in xs:
        st, pairs, div, nrec = O.check(km, x)
        out["checks"][str(x)] = dict(status=st, pairs=[list(p) for p in pairs], divergent=div,
                                     n_records=nrec)
        st, cl = O.clauses(km, x)
        out["clauses"][str(x)] = [list(c) for c in cl]
    # learn-all policy only: the one-trace policy needs one full-size
    # Verify per learned clause, hours of oracle time at this size
    out["repair_policy0"] = O.repair(km, policy=0)
    if "x_star" in km.meta:
        out["x_star"] = km.meta["x_star"]
    path = os.path.join(HERE, "expected_%s.json" % name)
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
    print(name, "%.1fs" % (time.time() - t), path)


def main():
    km = synth.generate("plain-large", mode="literal")
    record("plain_large_literal", km, [0])
    kp = synth.generate("plain-large", mode="planted")
    r = O.repair(kp)
    record("plain_large_planted", kp, [0, kp.meta["x_star"], r["assign"]])


if __name__ == "__main__":
    main()
