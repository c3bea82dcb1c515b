"""Loading of the paper's worked examples stored under tests/golden/."""
import glob
import json
import os

from paper_2011_08373_amd import synth

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def kernel_from_json(d):
    k = d["kernel"]
    return synth.make_kernel(k["blocks"], k["threads"], k["arrays"], k["guards"],
                             k["points"], k["slots"])


def listing_fixtures():
    out = []
    for path in sorted(glob.glob(os.path.join(GOLDEN, "*.json"))):
        name = os.path.splitext(os.path.basename(path))[0]
        if name in ("solver_examples", "weights") or name.startswith("expected_"):
            continue
        with open(path) as f:
            out.append((name, json.load(f)))
    return out


def load(name):
    with open(os.path.join(GOLDEN, name + ".json")) as f:
        return json.load(f)
