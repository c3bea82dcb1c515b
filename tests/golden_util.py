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


def encode_pairs(pairs, P):
    """Racing pairs [(level, i, j)] in ascending order as a compact string:
    the deltas of the codes level*P*P + i*P + j, zlib-compressed, base64."""
    import base64
    import zlib
    codes = [lv * P * P + i * P + j for lv, i, j in pairs]
    deltas = [codes[0]] + [b - a for a, b in zip(codes, codes[1:])] if codes else []
    return base64.b64encode(zlib.compress(",".join(map(str, deltas)).encode(), 9)).decode()


def decode_pairs(text, P):
    import base64
    import zlib
    raw = zlib.decompress(base64.b64decode(text)).decode()
    out, code = [], 0
    for d in (raw.split(",") if raw else []):
        code += int(d)
        out.append((code // (P * P), (code // P) % P, code % P))
    return out
