"""Summaries of rocprofv3 CSV output for the committed profiles.

  python -m paper_2011_08373_amd.profsum stats RUN_kernel_stats.csv
      Markdown table of the kernel statistics (calls, average, total, share).

  python -m paper_2011_08373_amd.profsum counters RUN_counter_collection.csv RECORDS
      Markdown table of every counter of a counter-collection run, per
      kernel: the average per dispatch and per 64 records (RECORDS: the
      access records one dispatch of the streaming kernels processes).

  python -m paper_2011_08373_amd.profsum traffic FETCH.csv WRITE.csv KEY MATCH SOURCE COPY_BYTES
      HBM bytes per launch of the kernel named MATCH, or else of the kernels
      whose names contain it (e.g. "rp::j0_kernel"; several instantiations
      are averaged over all their dispatches) from two counter-collection runs (one
      with FETCH_SIZE, one with WRITE_SIZE; the counters read KiB per
      dispatch).  Each counter is scaled by what it reads for the largest
      plain device copy of COPY_BYTES bytes in the same run (bench.py
      --calib), so the figure is in true bytes.  Prints the entry and merges
      it into profiles/traffic.json under KEY, with the sha256 of
      SOURCE: bench.py reports the figure only while SOURCE is unchanged.
"""
import csv
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _short(name):
    name = name.split("(")[0].replace("void ", "")
    return name.strip()


def stats_table(path):
    rows = list(csv.DictReader(open(path)))
    tot = sum(float(r["TotalDurationNs"]) for r in rows) or 1.0
    out = ["| kernel | calls | avg us | total us | min us | max us | share |",
           "|---|---:|---:|---:|---:|---:|---:|"]
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    for r in rows:
        out.append("| %s | %s | %.1f | %.1f | %.1f | %.1f | %.1f%% |" % (
            _short(r["Name"]), r["Calls"], float(r["AverageNs"]) / 1e3,
            float(r["TotalDurationNs"]) / 1e3, float(r["MinNs"]) / 1e3,
            float(r["MaxNs"]) / 1e3, 100.0 * float(r["TotalDurationNs"]) / tot))
    return "\n".join(out)


def _per_dispatch(path, counter):
    """{kernel short name: [value per dispatch]} for one counter."""
    vals = defaultdict(list)
    for r in csv.DictReader(open(path)):
        if r.get("Counter_Name") != counter:
            continue
        vals[_short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return vals


def counters_table(path, records):
    vals = defaultdict(lambda: defaultdict(list))
    for r in csv.DictReader(open(path)):
        vals[_short(r["Kernel_Name"])][r["Counter_Name"]].append(float(r["Counter_Value"]))
    names = sorted({c for d in vals.values() for c in d})
    out = ["| kernel | dispatches | " + " | ".join(names) + " |",
           "|---|---:|" + "---:|" * len(names)]
    groups = float(records) / 64.0
    for k in sorted(vals):
        d = vals[k]
        n = max(len(v) for v in d.values())
        cells = []
        for c in names:
            v = d.get(c)
            if not v:
                cells.append("")
                continue
            avg = sum(v) / len(v)
            cells.append("%.4g (%.1f / 64 rec)" % (avg, avg / groups))
        out.append("| %s | %d | %s |" % (k, n, " | ".join(cells)))
    return "\n".join(out)


def traffic(fetch_csv, write_csv, key, match, source, copy_bytes):
    out = {}
    for counter, path in (("FETCH_SIZE", fetch_csv), ("WRITE_SIZE", write_csv)):
        v = _per_dispatch(path, counter)
        copies = [x for k, xs in v.items() if "copy" in k.lower() for x in xs]
        if not copies:
            raise SystemExit("no copy kernel in %s: run bench.py with --calib" % path)
        ref = max(copies) * 1024.0            # bytes the counter reads for the copy
        factor = copy_bytes / ref
        names = [k for k in v if k == match] or [k for k in v if match in k]
        if not names:
            raise SystemExit("kernel %s not in %s" % (match, path))
        # several kernels (the instantiations of one kernel for different
        # digit widths): the average over all their dispatches, as bench.py
        # averages its launch times over all of them
        xs = [x for k in sorted(names) for x in v[k]]
        out[counter] = {"kib_per_dispatch": sum(xs) / len(xs), "dispatches": len(xs),
                        "copy_factor": factor,
                        "bytes_per_launch": sum(xs) / len(xs) * 1024.0 * factor}
    with open(os.path.join(ROOT, source), "rb") as fh:
        sha = hashlib.sha256(fh.read()).hexdigest()
    entry = {"source": source, "sha256": sha, "match": match, "kernels": sorted(names),
             "fetch_bytes_per_launch": out["FETCH_SIZE"]["bytes_per_launch"],
             "write_bytes_per_launch": out["WRITE_SIZE"]["bytes_per_launch"],
             "bytes_per_launch": out["FETCH_SIZE"]["bytes_per_launch"] +
                                 out["WRITE_SIZE"]["bytes_per_launch"],
             "counters": out}
    f = os.path.join(ROOT, "profiles", "traffic.json")
    data = json.load(open(f)) if os.path.exists(f) else {}
    data[key] = entry
    with open(f, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    return entry


def main(argv):
    if len(argv) >= 2 and argv[0] == "stats":
        print(stats_table(argv[1]))
    elif len(argv) >= 3 and argv[0] == "counters":
        print(counters_table(argv[1], float(argv[2])))
    elif len(argv) >= 7 and argv[0] == "traffic":
        print(json.dumps(traffic(argv[1], argv[2], argv[3], argv[4], argv[5], float(argv[6])),
                         indent=1))
    else:
        print(__doc__)
        return 2
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
