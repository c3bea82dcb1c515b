"""Benchmark of the repair hot path on one MI355X.

One step = one full rp_repair call (Alg. 1: record generation, the one-time
radix sort, then Verify / GenerateClause / Solve rounds until a verdict) on
the plain-large synthetic kernel: 256 blocks x 256 threads, 512 program
points, 32 barrier slots (8 grid-level), two shared and two global arrays of
1M int32 words.  The metric is race-checked accesses per second: every
(point, block, thread) access is race-checked once per Verify call.

More legs are reported beside the headline (same JSON line; --legs picks):
  planted  the same kernel with a planted safe barrier set (several Verify
           calls, ends SAFE);
  stress   4,096 blocks x 1,024 threads, 1,024 points, eight 16M-word arrays
           (2.0G records after the reduction, a 16 GB log; 2.4G planted):
           throughput and kernel rooflines far outside the last-level cache;
  batched  the 1,024-kernel batched workload (planted mode): repaired kernels
           per second of one rp_repair_batch call against the plain
           one-kernel-at-a-time rp_repair loop on the same kernels;
  rounds   Verify calls per kernel over the batched kernels under each
           learning policy (all traces / one trace per call) and Solve
           strategy (exact / mhs), and with the option switches;
  served   Poisson arrivals (2,000 jobs/s by default) drawn from the same
           1,024 kernels into a continuous-batching server with a 64 GB
           arena: p50/p99 latency from submission to verdict, throughput;
  instrumented  1,024 small structured programs (branches, loops, calls,
           pre-existing barriers) through the library's instrumentation pass
           and one rp_repair_batch call: host microseconds per program,
           kernels per second, Verify calls per kernel.

Prints one JSON line.  Inputs are synthetic and seeded; device buffers are
resident before the timed region starts.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "plain-large": "plain-large %s: 256 blocks x 256 threads, 512 points, 32 slots (8 grid), "
                   "2 shared + 2 global arrays of 1M words, seed 2",
    "stress": "stress %s: 4096 blocks x 1024 threads, 1024 points (half accesses), 64 slots "
              "(16 grid), 4 shared + 4 global arrays of 16M words, seed 5",
}


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


def model_accesses(km):
    """(point, block, thread) accesses of a kernel model: the size class the
    autotuner's cache is keyed by."""
    total = 0
    for p in km.points:
        if int(p["kind"]) != 0:
            continue
        m, r = (int(v) for v in km.guards[int(p["guard"])])
        if r < km.threads:
            total += (km.threads - r + m - 1) // m
    return total * km.blocks


def apply_tuning(L, n_accesses):
    """The autotuner's sort configuration for this size class, else the
    library's defaults (automatic digit width, 512 x 8 scatter tiles)."""
    from paper_2011_08373_amd import autotune
    best = autotune.lookup(n_accesses) if n_accesses else None
    if best:
        autotune.apply(n_accesses)
        return dict(digit_bits=best["digit_bits"], shape=best["shape"], autotuned=True)
    L.set_tuning(L.TUNE_SORT_DIGIT_BITS, 0)
    L.set_tuning(L.TUNE_SCATTER_SHAPE, 4)
    return dict(digit_bits="auto", shape=4, autotuned=False)


def run_main(L, torch, km, steps, warmup):
    """Times `steps` full rp_repair calls on one kernel (inputs resident),
    with the autotuner's sort configuration for its size class.  The timed
    calls record hipEvents around the streaming kernels only (timing level
    1); one more call after the timed region records every phase (level 2)
    for the phase breakdown."""
    ws = L.Workspace()
    ka = L.KernelArg(km)          # the C view of the descriptors, built once
    sort_cfg = apply_tuning(L, model_accesses(km))
    ws.get(L.workspace_bytes(ka, L.OP_REPAIR))
    level = L.set_tuning(L.TUNE_TIMING, 1)
    for _ in range(warmup):
        L.repair(ka, ws=ws)
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(steps):
        r = L.repair(ka, ws=ws)
        stats.append(L.last_stats())
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    L.set_tuning(L.TUNE_TIMING, 2)
    L.repair(ka, ws=ws)
    phases = L.last_stats()
    L.set_tuning(L.TUNE_TIMING, level)
    del ws
    stats[-1]["sort_config"] = sort_cfg
    stats[-1]["phases"] = {k: phases[k] for k in ("ms_upload", "ms_gen", "ms_sort", "ms_j0",
                                                  "ms_check", "ms_clause", "ms_solve", "ms_total")}
    return r, (t1 - t0) * 1e3 / steps, stats


def _traffic(kernel):
    """HBM bytes per launch from committed counter data, if the kernel's
    source is unchanged since the counters were taken; else None."""
    import hashlib
    f = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(f):
        return None
    with open(f) as fh:
        data = json.load(fh)
    e = data.get(kernel)
    if not e:
        return None
    src = os.path.join(ROOT, e["source"])
    if not os.path.exists(src):
        return None
    with open(src, "rb") as fh:
        if hashlib.sha256(fh.read()).hexdigest() != e["sha256"]:
            return None
    return e["bytes_per_launch"]


def kernel_rooflines(stats, traffic_prefix=""):
    """Algorithmic bytes per launch / average hipEvent launch time, for the
    kernels timed one by one on the library's stream.  Counter traffic is
    looked up under traffic_prefix + kernel name (it depends on the workload)."""
    n = len(stats)
    last = stats[-1]
    rec = last["records"]
    out = {}

    def entry(name, bytes_per_launch, total_ms, launches):
        if launches <= 0 or total_ms <= 0:
            return
        avg = total_ms / launches
        gbs = bytes_per_launch / (avg / 1e3) / 1e9
        out[name] = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": _traffic(traffic_prefix + name),
                     "avg_launch_ms": avg, "bytes_per_launch": bytes_per_launch,
                     "ms_per_step": total_ms / n}
    # radix scatter pass: reads and writes 8 B per record
    entry("scatter_kernel", 16 * rec, sum(s["ms_sort_kernels"] for s in stats),
          sum(s["sort_launches"] for s in stats))
    # first-partner scan (once per repair): reads 8 B per record
    entry("j0_kernel", 8 * rec, sum(s["ms_conf_kernels"] for s in stats),
          sum(s["conf_launches"] for s in stats))
    # record generation: writes 8 B per record
    entry("gen_kernel", 8 * rec, sum(s["ms_gen"] for s in stats), n)
    return out


def stress_leg(L, torch, steps):
    """The stress kernel (4,096 blocks x 1,024 threads, 1,024 points, eight
    16M-word arrays): a log of 16-20 GB, far beyond the 256 MB last-level
    cache, so the kernel rooflines here are HBM figures."""
    from paper_2011_08373_amd import synth
    out = {}
    for mode in ("literal", "planted"):
        km = synth.generate("stress", mode=mode)
        r, ms, stats = run_main(L, torch, km, steps, 1)
        acc = stats[-1]["accesses"]
        out[mode] = {"value": acc * r["rounds"] / (ms / 1e3), "unit": "accesses/s",
                     "ms_per_step": ms, "accesses": acc, "records": stats[-1]["records"],
                     "sort": stats[-1]["sort_config"],
                     "verify_calls": r["rounds"], "repair_status": r["status"],
                     "kernels": kernel_rooflines(stats, "stress/"),
                     "phases_ms": stats[-1]["phases"]}
        torch.cuda.empty_cache()
    out["workload"] = WORKLOADS["stress"] % "literal and planted"
    return out


def batched_leg(L, torch, kms):
    """One batched call over all kernels vs the plain per-kernel loop."""
    b = L.BatchArg(kms)
    ws = L.Workspace()
    ws.get(L.batch_workspace_bytes(b))
    L.repair_batch(b, ws=ws)                       # warm-up
    torch.cuda.synchronize()
    # sort knobs of this size class from the autotuner's cache, if tuned
    tuned = apply_tuning(L, L.last_stats()["accesses"])["autotuned"]
    if tuned:
        L.repair_batch(b, ws=ws)
        torch.cuda.synchronize()
    t = time.perf_counter()
    st, res = L.repair_batch(b, ws=ws)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    bstats = L.last_stats()
    # plain loop: one rp_repair per kernel, in order
    ws1 = L.Workspace()
    ws1.get(max(L.workspace_bytes(k, L.OP_REPAIR) for k in kms))
    L.repair(kms[0], ws=ws1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    plain = [L.repair(k, ws=ws1) for k in kms]
    torch.cuda.synchronize()
    tp = time.perf_counter() - t
    same = all(plain[q]["status"] == res[q]["status"] and plain[q]["assign"] == res[q]["assign"]
               for q in range(len(kms)))
    rep = sum(1 for r in res if r["status"] == 0)
    uns = sum(1 for r in res if r["status"] == 1)
    return {"workload": "batched planted: %d kernels, threads log-uniform in [64, 65536], "
                        "points uniform in [16, 1024], slots uniform in [2, 40], seed 3" % len(kms),
            "kernels_per_s_batched": len(kms) / tb, "kernels_per_s_plain": len(kms) / tp,
            "speedup": tp / tb, "ms_batched": tb * 1e3, "ms_plain": tp * 1e3,
            "repaired": rep, "unsat": uns, "other": len(kms) - rep - uns,
            "batched_equals_plain": same, "records": bstats["records"],
            "accesses": bstats["accesses"], "rounds": bstats["rounds"],
            "phases_ms": {k: bstats[k] for k in ("ms_gen", "ms_sort", "ms_j0", "ms_check",
                                                 "ms_clause", "ms_solve", "ms_total")},
            "autotuned": tuned}


def rounds_leg(L, torch, kms):
    """Verify calls per kernel of the repair loop under each learning policy
    and Solve strategy (and the paper's option switches), over the batched
    kernels in one rp_repair_batch call each.  Policy and strategy change
    only the route: the repaired barrier sets must equal the exact,
    all-traces ones."""
    b = L.BatchArg(kms)
    ws = L.Workspace()
    configs = [
        ("exact solve, all traces", dict(policy=0, solver=0)),
        ("mhs, all traces", dict(policy=0, solver=1)),
        ("exact solve, one trace", dict(policy=1, solver=0)),
        ("mhs, one trace", dict(policy=1, solver=1)),
        ("mhs, one trace, no grid barriers", dict(policy=1, solver=1, grid=0)),
        ("mhs, one trace, pre-existing barriers kept", dict(policy=1, solver=1, inspect=0)),
        ("mhs, one trace, both", dict(policy=1, solver=1, grid=0, inspect=0)),
    ]
    out, base = {}, None
    for name, kw in configs:
        L.repair_batch(b, ws=ws, **kw)                 # warm-up
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, res = L.repair_batch(b, ws=ws, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        calls = sorted(r["rounds"] for r in res)
        got = [(r["status"], r["assign"]) for r in res]
        if base is None:
            base = got
        e = {"verify_calls": sum(calls), "per_kernel_mean": sum(calls) / len(calls),
             "per_kernel_median": calls[len(calls) // 2], "per_kernel_max": calls[-1],
             "repaired": sum(1 for r in res if r["status"] == 0), "ms": dt * 1e3,
             "status": st}
        if "grid" not in kw and "inspect" not in kw:
            e["same_result_as_exact_all"] = got == base
        out[name] = e
    return out


def instrumented_leg(L, torch, n, seed=11):
    """Structured programs through rp_instrument, then one batched repair
    under the default strategy and under the paper's (mhs, one trace)."""
    from paper_2011_08373_amd import synth
    progs = synth.generate_programs(n, seed=seed)
    out = {"workload": "instrumented: %d random structured programs (1-4 blocks x 32-128 "
                       "threads, nested branches, loops of 2-4 trips, calls, pre-existing "
                       "barriers), grid-level instrumentation on, seed %d" % (n, seed)}
    L.instrument(progs[0])
    t = time.perf_counter()
    inst = [L.instrument(p) for p in progs]
    ti = time.perf_counter() - t
    kms = [k for st, k in inst if st == 0]
    out["instrument_us_per_program"] = ti / n * 1e6
    out["instrumented"] = len(kms)
    out["slots_mean"] = sum(k.n_slots for k in kms) / max(1, len(kms))
    out["points_mean"] = sum(k.n_points for k in kms) / max(1, len(kms))
    b = L.BatchArg(kms)
    ws = L.Workspace()
    for name, kw in (("exact solve, all traces", {}), ("mhs, one trace", dict(policy=1, solver=1))):
        L.repair_batch(b, ws=ws, **kw)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, res = L.repair_batch(b, ws=ws, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t
        calls = sorted(r["rounds"] for r in res)
        out[name] = {"kernels_per_s": len(kms) / dt, "ms": dt * 1e3, "status": st,
                     "repaired": sum(1 for r in res if r["status"] == 0),
                     "unsat": sum(1 for r in res if r["status"] == 1),
                     "verify_calls_per_kernel": sum(calls) / max(1, len(calls)),
                     "verify_calls_max": calls[-1] if calls else 0}
    return out


def served_leg(L, torch, kms, rate, seconds, arena_gb):
    """Poisson arrivals into the continuous-batching server."""
    from paper_2011_08373_amd import synth
    warm = 1.0
    arr = synth.poisson_arrivals(rate, warm + seconds, seed=4)
    srv = L.Server(arena_bytes=int(arena_gb * (1 << 30)), max_resident=1024)
    lat = {}
    n_sub = 0
    t0 = time.perf_counter()
    max_res = 0
    limit = warm + seconds + 60.0          # drain the backlog, but not forever
    while len(lat) < len(arr) and time.perf_counter() - t0 < limit:
        now = time.perf_counter() - t0
        while n_sub < len(arr) and arr[n_sub] <= now:
            st = srv.submit(kms[n_sub % len(kms)], n_sub)
            if st != 0:
                raise RuntimeError("submit failed: %d" % st)
            n_sub += 1
        nres, npend = srv.step()
        max_res = max(max_res, nres)
        for jid, r, l in srv.poll():
            lat[jid] = l
        if nres == 0 and npend == 0 and n_sub < len(arr):
            time.sleep(max(0.0, min(0.001, arr[n_sub] - (time.perf_counter() - t0))))
    t_end = time.perf_counter() - t0
    srv.close()
    ids = [i for i in range(len(arr)) if arr[i] >= warm]
    ls = sorted(lat[i] for i in ids if i in lat)

    def pct(p):
        return ls[min(len(ls) - 1, max(0, int(math.ceil(p * len(ls))) - 1))] if ls else None
    return {"workload": "served: Poisson arrivals at %.0f jobs/s drawn from the batched "
                        "kernels, %.0f GB arena, 1 s warm-up + %.1f s measured" % (rate, arena_gb, seconds),
            "jobs_measured": len(ids), "jobs_finished": len(ls),
            "p50_s": pct(0.50), "p99_s": pct(0.99),
            "throughput_jobs_per_s": len(arr) / t_end, "offered_jobs_per_s": rate,
            "max_resident": max_res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--mode", default="literal", choices=("literal", "planted"))
    ap.add_argument("--config", default="plain-large", choices=("plain-large", "stress"),
                    help="kernel of the headline leg (the stress kernel for profiling runs)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--legs", default="main,planted,stress,batched,rounds,served,instrumented")
    ap.add_argument("--stress-steps", type=int, default=3)
    ap.add_argument("--batched-n", type=int, default=1024)
    ap.add_argument("--serve-rate", type=float, default=2000.0)
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--serve-arena-gb", type=float, default=64.0)
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
    km = synth.generate(args.config, mode=args.mode)
    r, ms, stats = run_main(L, torch, km, args.steps, args.warmup)
    acc = stats[-1]["accesses"]
    km.meta["accesses"] = acc
    checked = acc * r["rounds"]
    value = checked / (ms / 1e3)
    kern = kernel_rooflines(stats, "" if args.config == "plain-large" else args.config + "/")
    dom = max(kern, key=lambda k: kern[k]["ms_per_step"])
    roof = dict(kern[dom])
    roof["kernel"] = dom
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
        "config": {"workload": WORKLOADS[args.config] % args.mode,
                   "accesses": acc, "records": stats[-1]["records"],
                   "verify_calls": r["rounds"], "repair_status": r["status"],
                   "sort": stats[-1]["sort_config"]},
        "roofline": {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic",
                                          "kernel", "avg_launch_ms", "bytes_per_launch")},
        "kernels": kern,
        # warm: Verify on the resident run log (the conflict-scan kernel of
        # each round); cold: the whole repair, generation and sort included
        "warm_check_accesses_per_s": (acc * sum(s["conf_launches"] for s in stats) /
                                      (sum(s["ms_conf_kernels"] for s in stats) / 1e3)
                                      if sum(s["ms_conf_kernels"] for s in stats) > 0 else None),
        # one call with every phase timed, after the timed region
        "phases_ms": stats[-1]["phases"],
    }
    if args.config == "plain-large" and args.mode == "literal" and "planted" in set(args.legs.split(",")):
        # context: the same kernel with a planted safe barrier set (repair
        # runs several Verify calls and ends SAFE)
        kp = synth.generate("plain-large", mode="planted")
        rp, msp, stp = run_main(L, torch, kp, max(1, args.steps // 2), 1)
        kp_acc = stp[-1]["accesses"]
        kk = kernel_rooflines(stp)
        out["planted"] = {"value": kp_acc * rp["rounds"] / (msp / 1e3), "ms_per_step": msp,
                          "verify_calls": rp["rounds"], "repair_status": rp["status"],
                          "weight": rp["weight"],
                          "j0_kernel_frac": kk["j0_kernel"]["frac"],
                          "phases_ms": stp[-1]["phases"]}
    if not args.no_cpu and args.config == "plain-large":
        out["cpu_baseline"] = cpu_baseline(km, r["rounds"])
    legs = set(args.legs.split(","))
    torch.cuda.empty_cache()
    if "stress" in legs:
        out["stress"] = stress_leg(L, torch, args.stress_steps)
    if "batched" in legs or "served" in legs or "rounds" in legs:
        kms = synth.generate_batch(n=args.batched_n, mode="planted")
        if "batched" in legs:
            out["batched"] = batched_leg(L, torch, kms)
        if "rounds" in legs:
            out["rounds"] = rounds_leg(L, torch, kms)
        if "served" in legs:
            out["served"] = served_leg(L, torch, kms, args.serve_rate, args.serve_seconds,
                                       args.serve_arena_gb)
    if "instrumented" in legs:
        out["instrumented"] = instrumented_leg(L, torch, args.batched_n)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
