"""Benchmark of the repair hot path on one MI355X.

One step = one full rp_repair call (Alg. 1: record generation, the one-time
radix sort and first-partner table, then Verify / GenerateClause / Solve
rounds until a verdict) on the stress kernel: 4,096 blocks x 1,024 threads,
1,024 program points (half of them accesses), 64 barrier slots (16
grid-level), four shared and four global arrays of 16M int32 words, about
2.0G access records (a 16 GB log, far beyond the 256 MB last-level cache).
The metric is race-checked accesses per second: every (point, block,
thread) access is race-checked once per Verify call.

More legs are reported beside the headline (same JSON line; --legs picks):
  planted  the same kernel with a planted safe barrier set (several Verify
           calls, ends SAFE); its per-Verify rate is reported apart from the
           Verify-call multiplier;
  plain    the plain-large kernel (256 blocks x 256 threads, 512 points, four
           1M-word arrays), literal and planted: a 213 MB log that the
           last-level cache partly holds;
  batched  the 1,024-kernel batched workload (planted mode): repaired kernels
           per second of one rp_repair_batch call against the plain
           one-kernel-at-a-time rp_repair loop on the same kernels (both with
           their descriptors marshalled before the timer starts);
  rounds   Verify calls per kernel over the batched kernels under each
           learning policy (all traces / one trace per call) and Solve
           strategy (exact / mhs), and with the option switches;
  served   Poisson arrivals drawn from the same 1,024 kernels into a
           continuous-batching server with a 64 GB arena, at the offered
           rate and at rates above the plain loop's capacity: p50/p99 latency
           from submission to verdict and the rate of jobs finished inside
           the measured window;
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


def host_info():
    """CPU model, logical cores and RAM of the host the oracle runs on."""
    model, mem = None, None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as f:
            for line in f:
                if line.startswith("MemTotal"):
                    mem = round(int(line.split()[1]) / (1 << 20), 1)
                    break
    except OSError:
        pass
    return dict(cpu_model=model, nproc=os.cpu_count(), ram_gib=mem)


# host threads the oracle may use: the machine's CPU share for one GPU
ORACLE_THREADS = 16
# blocks of the stress kernel the oracle repairs: all 4,096 (about 15 s on
# 16 threads; a quarter of them took under 4 s, below the 10 s a baseline
# needs to be timed reliably)
STRESS_SAMPLE_BLOCKS = 4096


def cpu_baseline(name, mode, km_full):
    """The CPU oracle timed on the host cores on a bounded sample of the
    headline workload: one full repair (Alg. 1 in the paper's order) of the
    same kernel model restricted to its first STRESS_SAMPLE_BLOCKS blocks
    (stress), or of the whole kernel (plain-large, one thread)."""
    from oracle import oracle as O
    from paper_2011_08373_amd import synth
    if name == "stress":
        threads = max(1, min(ORACLE_THREADS, os.cpu_count() or 1))
        if STRESS_SAMPLE_BLOCKS >= km_full.blocks:
            km = km_full
            sample = ("one full repair (per-instance location-grouped checker on %d threads) "
                      "of the whole stress kernel's %s model" % (threads, mode))
        else:
            km = synth.generate(name, mode=mode, blocks=STRESS_SAMPLE_BLOCKS)
            sample = ("one full repair (per-instance location-grouped checker on %d threads) "
                      "of the stress kernel's %s model restricted to its first %d of %d "
                      "blocks (same points, threads and arrays)"
                      % (threads, mode, STRESS_SAMPLE_BLOCKS, km_full.blocks))
        O.set_route(1, threads)
    else:
        threads = 1
        km = km_full
        sample = "one full repair of the plain-large %s kernel on one thread" % mode
        O.set_route(0)
    try:
        acc = model_accesses(km)
        t = time.perf_counter()
        r = O.repair(km)
        dt = time.perf_counter() - t
    finally:
        O.set_route(0)
    out = dict(value=acc * r["rounds"] / dt, unit="race-checked accesses/s", cores=threads,
               kind="oracle", sample=sample + " (%d accesses, %d Verify call(s), %.1f s)"
               % (acc, r["rounds"], dt), seconds=dt)
    out.update(host_info())
    return out


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


def apply_tuning(L, n_accesses, key_bits):
    """The autotuner's sort configuration for this size class (access count
    and key width), else the library's defaults (automatic digit width,
    512 x 8 scatter tiles)."""
    from paper_2011_08373_amd import autotune
    best = autotune.lookup(n_accesses, key_bits) if n_accesses else None
    if best:
        autotune.apply(n_accesses, key_bits)
        return dict(digit_bits=best["digit_bits"] or "auto",
                    low_digit_bits=best.get("low_digit_bits", 0), shape=best["shape"],
                    pass_shapes=best.get("pass_shapes", []), key_bits=key_bits,
                    autotuned=True)
    L.set_tuning(L.TUNE_SORT_DIGIT_BITS, 0)
    L.set_tuning(L.TUNE_LOW_DIGIT_BITS, 6)
    L.set_tuning(L.TUNE_SCATTER_SHAPE, 4)
    L.set_tuning(L.TUNE_PASS_SHAPES, L.PASS_SHAPES_DEFAULT)
    return dict(digit_bits="auto", low_digit_bits=6, shape=4, pass_shapes=[],
                key_bits=key_bits, autotuned=False)


def run_main(L, torch, km, steps, warmup):
    """Times `steps` full rp_repair calls on one kernel (inputs resident),
    with the autotuner's sort configuration for its size class.  The timed
    calls record hipEvents around the streaming kernels only (timing level
    1); one more call after the timed region records every phase (level 2)
    for the phase breakdown."""
    ws = L.Workspace()
    ka = L.KernelArg(km)          # the C view of the descriptors, built once
    sort_cfg = apply_tuning(L, model_accesses(km), L.sort_key_bits(ka))
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


def phase_roofline(stats):
    """The race-check phase of one repair (record generation, every radix
    pass with its counts and column scans, the first-partner scan), timed
    with the streaming kernels' hipEvents, against its algorithmic bytes:
    8 B per record written by generation, 16 B per record and radix pass,
    8 B per record read by the scan."""
    n = len(stats)
    last = stats[-1]
    rec = last["records"]
    passes = last.get("sort_passes", 0)
    ms = sum(s["ms_gen"] + s["ms_sort"] + s["ms_j0"] for s in stats) / n
    if ms <= 0:
        return None
    byts = rec * (8 + 16 * passes + 8)
    gbs = byts / (ms / 1e3) / 1e9
    return {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": gbs / HBM_PEAK_GBS, "ms_per_step": ms, "bytes_per_step": byts,
            "sort_passes": passes}


def kernel_leg(L, torch, name, mode, steps, warmup=1):
    """Full repairs of one named kernel (the stress kernel's 16-20 GB log is
    far beyond the 256 MB last-level cache; plain-large's 213 MB log is
    partly held by it).  `accesses_per_s_per_verify` divides the accesses by
    the repair time once; `value` multiplies them by the Verify calls, whose
    rounds after the first cost O(points) on the resident first-partner
    table."""
    from paper_2011_08373_amd import synth
    km = synth.generate(name, mode=mode)
    r, ms, stats = run_main(L, torch, km, steps, warmup)
    acc = stats[-1]["accesses"]
    out = {"workload": WORKLOADS[name] % mode,
           "value": acc * r["rounds"] / (ms / 1e3), "unit": "race-checked accesses/s",
           "accesses_per_s_per_verify": acc / (ms / 1e3),
           "verify_calls": r["rounds"], "ms_per_step": ms, "steps": steps,
           "accesses": acc, "records": stats[-1]["records"],
           "sort": stats[-1]["sort_config"], "repair_status": r["status"],
           "weight": r.get("weight"),
           "kernels": kernel_rooflines(stats, "" if name == "plain-large" else name + "/"),
           "phases_ms": stats[-1]["phases"]}
    torch.cuda.empty_cache()
    return out


def batched_leg(L, torch, kms):
    """One batched call over all kernels vs the plain per-kernel loop."""
    b = L.BatchArg(kms)
    ws = L.Workspace()
    ws.get(L.batch_workspace_bytes(b))
    L.repair_batch(b, ws=ws)                       # warm-up
    torch.cuda.synchronize()
    # sort knobs of this size class from the autotuner's cache, if tuned
    tuned = apply_tuning(L, L.last_stats()["accesses"], L.sort_key_bits(b))["autotuned"]
    if tuned:
        L.repair_batch(b, ws=ws)
        torch.cuda.synchronize()
    t = time.perf_counter()
    st, res = L.repair_batch(b, ws=ws)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t
    bstats = L.last_stats()
    # plain loop: one rp_repair per kernel, in order, with each kernel's C
    # view and workspace size prepared before the timer (as the batched
    # call's BatchArg is)
    kas = b.args
    # each plain call takes the automatic digit width of its own key
    L.set_tuning(L.TUNE_SORT_DIGIT_BITS, 0)
    ws1 = L.Workspace()
    ws1.get(max(ka.need(L.OP_REPAIR) for ka in kas))
    L.repair(kas[0], ws=ws1)
    torch.cuda.synchronize()
    t = time.perf_counter()
    plain = [L.repair(ka, ws=ws1) for ka in kas]
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
            # the race-check phase of the batched call, as for the main leg
            "race_check_phase": phase_roofline([bstats]),
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


def served_leg(L, torch, kms, rate, seconds, arena_gb, seed=4):
    """Poisson arrivals into the continuous-batching server: 1 s of warm-up,
    then `seconds` measured.  Latency is submission to verdict for the jobs
    that arrive inside the measured window; throughput counts the verdicts
    delivered inside it (so it can exceed neither the offered rate by much
    nor the server's capacity)."""
    from paper_2011_08373_amd import synth
    warm = 1.0
    arr = synth.poisson_arrivals(rate, warm + seconds, seed=seed)
    srv = L.Server(arena_bytes=int(arena_gb * (1 << 30)), max_resident=1024)
    lat, done_at = {}, {}
    n_sub = 0
    t0 = time.perf_counter()
    max_res = 0
    limit = warm + seconds + 30.0          # drain the backlog, but not forever
    while len(lat) < len(arr) and time.perf_counter() - t0 < limit:
        now = time.perf_counter() - t0
        while n_sub < len(arr) and arr[n_sub] <= now:
            st = srv.submit(kms[n_sub % len(kms)], n_sub)
            if st != 0:
                raise RuntimeError("submit failed: %d" % st)
            n_sub += 1
        nres, npend = srv.step()
        max_res = max(max_res, nres)
        t_poll = time.perf_counter() - t0
        for jid, r, l in srv.poll():
            lat[jid] = l
            done_at[jid] = t_poll
        if nres == 0 and npend == 0 and n_sub < len(arr):
            time.sleep(max(0.0, min(0.001, arr[n_sub] - (time.perf_counter() - t0))))
    srv.close()
    ids = [i for i in range(len(arr)) if arr[i] >= warm]
    ls = sorted(lat[i] for i in ids if i in lat)
    in_window = sum(1 for t in done_at.values() if warm <= t < warm + seconds)

    def pct(p):
        return ls[min(len(ls) - 1, max(0, int(math.ceil(p * len(ls))) - 1))] if ls else None
    return {"offered_jobs_per_s": rate, "seconds": seconds,
            "jobs_arrived": len(ids), "jobs_finished": len(ls),
            "p50_s": pct(0.50), "p99_s": pct(0.99),
            "throughput_jobs_per_s": in_window / seconds,
            "max_resident": max_res}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--mode", default="literal", choices=("literal", "planted"))
    ap.add_argument("--config", default="stress", choices=("stress", "plain-large"),
                    help="kernel of the headline leg")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--legs", default="main,planted,plain,batched,rounds,served,instrumented")
    ap.add_argument("--leg-steps", type=int, default=20,
                    help="timed repairs of the planted and plain legs")
    ap.add_argument("--batched-n", type=int, default=1024)
    ap.add_argument("--serve-rates", default="2000,4000,8000",
                    help="offered Poisson rates (jobs/s) of the served leg")
    ap.add_argument("--serve-seconds", type=float, default=10.0)
    ap.add_argument("--serve-arena-gb", type=float, default=64.0)
    ap.add_argument("--calib", action="store_true",
                    help="run a 512 MiB device copy first (reference for byte counters)")
    ap.add_argument("--digit-order", type=int, default=None, choices=(0, 1),
                    help="radix digit order: 0 lowest first, 1 highest first "
                         "(default: the library's)")
    ap.add_argument("--scan-pipeline", type=int, default=None, choices=(0, 1),
                    help="first-partner scan: 1 issues the next range's loads before "
                         "the current range is scanned (default: the library's)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    _ensure_built()
    import torch
    from paper_2011_08373_amd import librepair as L, synth
    torch.cuda.set_device(0)
    if args.digit_order is not None:
        L.set_tuning(L.TUNE_DIGIT_ORDER, args.digit_order)
    if args.scan_pipeline is not None:
        L.set_tuning(L.TUNE_SCAN_PIPELINE, args.scan_pipeline)
    legs = set(args.legs.split(","))
    if args.calib:
        a = torch.empty(64 << 20, dtype=torch.int64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    km = synth.generate(args.config, mode=args.mode)
    r, ms, stats = run_main(L, torch, km, args.steps, args.warmup)
    acc = stats[-1]["accesses"]
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
        # the race-check phase (generation, sort, first-partner table) against
        # its algorithmic bytes: 8 B written per record by generation, 16 B
        # per radix pass, 8 B read by the first-partner scan
        "race_check_phase": phase_roofline(stats),
        # the once-per-kernel first-partner scan alone: accesses per second of
        # that scan (later Verify calls reuse its table)
        "first_partner_scan_accesses_per_s": (
            acc * sum(s["conf_launches"] for s in stats) /
            (sum(s["ms_conf_kernels"] for s in stats) / 1e3)
            if sum(s["ms_conf_kernels"] for s in stats) > 0 else None),
        # one call with every phase timed, after the timed region
        "phases_ms": stats[-1]["phases"],
    }
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(args.config, args.mode, km)
    del km
    torch.cuda.empty_cache()
    if "planted" in legs:
        other = "planted" if args.mode == "literal" else "literal"
        out["planted" if other == "planted" else "literal"] = kernel_leg(
            L, torch, args.config, other, args.leg_steps)
    if "plain" in legs and args.config != "plain-large":
        out["plain_large"] = {m: kernel_leg(L, torch, "plain-large", m, args.leg_steps)
                              for m in ("literal", "planted")}
    if "batched" in legs or "served" in legs or "rounds" in legs:
        kms = synth.generate_batch(n=args.batched_n, mode="planted")
        if "batched" in legs:
            out["batched"] = batched_leg(L, torch, kms)
        if "rounds" in legs:
            out["rounds"] = rounds_leg(L, torch, kms)
        if "served" in legs:
            runs = [served_leg(L, torch, kms, float(rate), args.serve_seconds,
                               args.serve_arena_gb)
                    for rate in args.serve_rates.split(",") if rate]
            out["served"] = {
                "workload": "served: Poisson arrivals drawn from the batched kernels, "
                            "%.0f GB arena, 1 s warm-up + %.1f s measured per rate"
                            % (args.serve_arena_gb, args.serve_seconds),
                "runs": runs,
                "plain_loop_kernels_per_s": out.get("batched", {}).get("kernels_per_s_plain")}
    if "instrumented" in legs:
        out["instrumented"] = instrumented_leg(L, torch, args.batched_n)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
