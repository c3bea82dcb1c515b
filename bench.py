"""Benchmark of the repair hot path on one MI355X.

One step = one full rp_repair call (Alg. 1: record generation, the one-time
radix sort, then Verify / GenerateClause / Solve rounds until a verdict) on
the plain-large synthetic kernel: 256 blocks x 256 threads, 512 program
points, 32 barrier slots (8 grid-level), two shared and two global arrays of
1M int32 words.  The metric is race-checked accesses per second: every
(point, block, thread) access is race-checked once per Verify call.

Prints one JSON line.  Inputs are synthetic and seeded; device buffers are
resident before the timed region starts.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def _ensure_built():
    lib = os.path.join(ROOT, "paper_2011_08373_amd", "lib", "librepair.so")
    if not os.path.exists(lib):
        from paper_2011_08373_amd import build as hipbuild
        hipbuild.build()


def cpu_baseline(km, rounds_gpu):
    """The CPU oracle (single thread) on one full repair of the same kernel."""
    from oracle import oracle as O
    t = time.perf_counter()
    r = O.repair(km)
    dt = time.perf_counter() - t
    acc = int(km.meta.get("accesses", 0))
    return dict(value=acc * r["rounds"] / dt, unit="race-checked accesses/s", cores=1,
                kind="oracle", sample="one full repair of the plain-large kernel "
                "(%d Verify calls, %.1f s)" % (r["rounds"], dt),
                matches_gpu_rounds=r["rounds"] == rounds_gpu)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--mode", default="literal", choices=("literal", "planted"))
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calib", action="store_true",
                    help="run a 512 MiB device copy first (reference for byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    _ensure_built()
    import torch
    from paper_2011_08373_amd import librepair as L, synth
    torch.cuda.set_device(0)
    if args.calib:
        a = torch.empty(64 << 20, dtype=torch.int64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    km = synth.generate("plain-large", mode=args.mode)
    ws = L.Workspace()
    ws.get(L.workspace_bytes(km, L.OP_REPAIR))
    for _ in range(args.warmup):
        L.repair(km, ws=ws)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r = L.repair(km, ws=ws)
        stats.append(L.last_stats())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms = (t1 - t0) * 1e3 / args.steps
    acc = stats[-1]["accesses"]
    km.meta["accesses"] = acc
    checked = acc * r["rounds"]
    value = checked / (ms / 1e3)
    # dominant kernel: the radix-sort pass (reads and writes 8 B per record)
    launches = sum(s["sort_launches"] for s in stats)
    kms = sum(s["ms_sort_kernels"] for s in stats)
    rec = stats[-1]["records"]
    pass_ms = kms / max(1, launches)
    achieved = 16.0 * rec / (pass_ms / 1e3) / 1e9 if pass_ms > 0 else 0.0
    out = {
        "metric": "race-checked accesses/sec",
        "value": value,
        "unit": "accesses/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "plain-large %s: 256 blocks x 256 threads, 512 points, "
                               "32 slots (8 grid), 2 shared + 2 global arrays of 1M words, "
                               "seed 2" % args.mode,
                   "accesses": acc, "records": rec, "verify_calls": r["rounds"],
                   "repair_status": r["status"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "scatter_kernel (one radix pass: reads and writes 8 B per record)",
                     "avg_launch_ms": pass_ms},
        "phases_ms": {k: sum(s[k] for s in stats) / len(stats)
                      for k in ("ms_gen", "ms_sort", "ms_check", "ms_clause", "ms_solve",
                                "ms_total")},
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(km, r["rounds"])
    print(json.dumps(out))


if __name__ == "__main__":
    main()
