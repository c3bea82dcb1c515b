"""HIP path (through the C ABI) against the CPU oracle, element by element.

The whole path is integer: every comparison is exact.
"""
import json
import os

import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_08373_amd import synth
import bruteforce as BF
from golden_util import GOLDEN, kernel_from_json, listing_fixtures

pytestmark = pytest.mark.gpu

FIXTURES = listing_fixtures()
REPAIR_KEYS = ("status", "assign", "weight", "added", "removed", "rounds", "n_clauses",
               "trajectory")


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2011_08373_amd import librepair
    return librepair


def same_repair(g, o):
    return {k: g[k] for k in REPAIR_KEYS} == {k: o[k] for k in REPAIR_KEYS}


@pytest.mark.parametrize("name,fx", FIXTURES, ids=[n for n, _ in FIXTURES])
def test_listing(L, name, fx):
    km = kernel_from_json(fx)
    for x, exp in fx["expect"].get("check", {}).items():
        g = L.check(km, int(x))
        o = O.check(km, int(x))
        assert g[:4] == o, (name, x)
        assert [list(p) for p in g[1]] == exp["pairs"]
        assert g[2] == exp["divergent"]
    for x, exp in fx["expect"].get("clauses", {}).items():
        g = L.clauses(km, int(x))
        assert g == O.clauses(km, int(x)), (name, x)
        assert [list(c) for c in g[1]] == exp
    for policy in (0, 1):
        g = L.repair(km, policy=policy)
        o = O.repair(km, policy=policy)
        assert same_repair(g, o), (name, policy, g, o)


def test_plain_small_1000_seeds(L):
    # the small plain configuration: 1 block x 64 threads, 16 points
    mism = []
    for seed in range(1000):
        km = synth.generate("plain-small", seed=seed)
        g = L.repair(km)
        o = O.repair(km)
        if not same_repair(g, o):
            mism.append((seed, g, o))
        if seed % 25 == 0:
            rng = np.random.default_rng(seed)
            for x in [0] + rng.integers(0, 16, size=2).tolist():
                assert L.check(km, x)[:4] == O.check(km, x), (seed, x)
                assert L.clauses(km, x) == O.clauses(km, x), (seed, x)
    assert not mism, mism[:3]


def test_plain_small_planted(L):
    for seed in range(200):
        km = synth.generate("plain-small", mode="planted", seed=seed)
        for policy in (0, 1):
            g = L.repair(km, policy=policy)
            o = O.repair(km, policy=policy)
            assert same_repair(g, o), (seed, policy)


def test_tiny_random_kernels(L):
    for seed in range(400):
        rng = np.random.default_rng(40_000 + seed)
        km = BF.tiny_kernel(rng)
        for policy in (0, 1):
            g = L.repair(km, policy=policy)
            o = O.repair(km, policy=policy)
            assert same_repair(g, o), (seed, policy, g, o)
        for x in rng.integers(0, 1 << max(1, km.n_slots), size=3).tolist():
            assert L.check(km, x)[:4] == O.check(km, x), (seed, x)
            assert L.clauses(km, x) == O.clauses(km, x), (seed, x)


def test_block_conditions(L):
    # guards with a condition on the block id (padding records in the
    # same-block log, executing blocks only in the cross-block log)
    for seed in range(300):
        rng = np.random.default_rng(80_000 + seed)
        km = BF.tiny_kernel(rng, max_blocks=4, block_conds=True)
        for policy in (0, 1):
            g = L.repair(km, policy=policy)
            o = O.repair(km, policy=policy)
            assert same_repair(g, o), (seed, policy, g, o)
        for x in rng.integers(0, 1 << max(1, km.n_slots), size=2).tolist():
            assert L.check(km, x)[:4] == O.check(km, x), (seed, x)
            assert L.clauses(km, x) == O.clauses(km, x), (seed, x)
    # kernels of the batched distribution with several generation items and
    # sort tiles; four arrays, so the padding array id takes one more bit
    cfg = synth.config("batched")
    kms = []
    for seed in range(10):
        rng = np.random.default_rng(81_000 + seed)
        c = dict(cfg)
        c.update(blocks=int(rng.integers(2, 9)), threads=64 * int(rng.integers(1, 5)),
                 P=int(rng.integers(64, 400)), S=int(rng.integers(4, 24)), S_grid=3)
        km = synth.with_block_conditions(synth.planted_kernel(c, rng), rng, frac=0.7)
        kms.append(km)
        g = L.repair(km)
        o = O.repair(km)
        assert same_repair(g, o), (seed, g, o)
        for x in (0, g["assign"], o["trajectory"][0]):
            assert L.check(km, x)[:4] == O.check(km, x), (seed, x)
    st, res = L.repair_batch(kms)
    assert st == 0
    for q, km in enumerate(kms):
        o = O.repair(km)
        assert {k: res[q][k] for k in REPAIR_KEYS if k != "trajectory"} == \
            {k: o[k] for k in REPAIR_KEYS if k != "trajectory"}, q


def test_tiny_options(L):
    for seed in range(150):
        rng = np.random.default_rng(50_000 + seed)
        km = BF.tiny_kernel(rng)
        for grid, inspect in ((0, 1), (1, 0), (0, 0)):
            g = L.repair(km, grid=grid, inspect=inspect)
            o = O.repair(km, grid=grid, inspect=inspect)
            assert same_repair(g, o), (seed, grid, inspect)
        g = L.repair(km, max_rounds=1)
        o = O.repair(km, max_rounds=1)
        assert same_repair(g, o), seed


def _clause_sets(rng, S, n):
    out = []
    for _ in range(n):
        u = rng.random()
        p = int(rng.integers(0, 1 << S))
        q = int(rng.integers(0, 1 << S))
        if u < 0.6:
            out.append((p | (1 << int(rng.integers(0, S))), 0))
        elif u < 0.85:
            out.append((0, 1 << int(rng.integers(0, S))))
        else:
            out.append((p & ~q, q & ~p))
    return out


def test_solver_random(L):
    rng = np.random.default_rng(5)
    for _ in range(300):
        S = int(rng.integers(1, 16))
        cl = _clause_sets(rng, S, int(rng.integers(0, 20)))
        w = rng.integers(1, 9, size=S).tolist()
        g = L.min_barriers(cl, w, S)
        o = O.min_barriers(cl, w, S)
        if o[0] == 1:
            assert g[0] == 1
        else:
            assert g == o, (cl, w)


def test_solver_wide_components(L):
    # components wider than the enumeration limit take the branch and bound
    rng = np.random.default_rng(6)
    for trial in range(20):
        S = int(rng.integers(21, 65))
        cl = []
        for _ in range(int(rng.integers(20, 80))):
            lo = int(rng.integers(0, S - 1))
            hi = int(rng.integers(lo, min(S, lo + 6)))
            cl.append((((1 << (hi + 1)) - 1) & ~((1 << lo) - 1), 0))
        cl += [(0, 1 << int(rng.integers(0, S))) for _ in range(3)]
        cl.append((((1 << S) - 1) if S < 64 else (1 << 64) - 1, 0))
        w = rng.integers(1, 5, size=S).tolist()
        g = L.min_barriers(cl, w, S)
        o = O.min_barriers(cl, w, S)
        assert g == o, trial


def test_solver_examples(L):
    with open(os.path.join(GOLDEN, "solver_examples.json")) as f:
        fx = json.load(f)
    for case in fx["cases"]:
        g = L.min_barriers(case["clauses"], case["weights"], case["n_slots"])
        exp = case["expect"]
        assert g[0] == exp["status"], case["name"]
        if g[0] == 0:
            assert (g[1], g[2]) == (exp["assign"], exp["weight"]), case["name"]


def _expected(name):
    path = os.path.join(GOLDEN, "expected_%s.json" % name)
    with open(path) as f:
        return json.load(f)


@pytest.mark.parametrize("name,mode", [("plain_large_literal", "literal"),
                                       ("plain_large_planted", "planted")])
def test_plain_large_full_size(L, name, mode):
    # 256 blocks x 256 threads, 512 points, 32 slots, four 1M-word arrays
    exp = _expected(name)
    km = synth.generate("plain-large", mode=mode)
    for x, c in exp["checks"].items():
        g = L.check(km, int(x))
        assert g[0] == 0
        assert g[3] == c["n_records"]
        assert g[2] == c["divergent"]
        assert [list(p) for p in g[1]] == c["pairs"], x
        assert [list(q) for q in L.clauses(km, int(x))[1]] == exp["clauses"][x], x
    g = L.repair(km, policy=0)
    o = exp["repair_policy0"]
    assert same_repair(g, o), (g, o)


@pytest.mark.parametrize("name,mode", [("plain_large_literal", "literal"),
                                       ("plain_large_planted", "planted")])
def test_scan_variants_full_size(L, name, mode):
    # the first-partner scan with the next range's loads in flight or not,
    # and with the record fields taken from the low word or from the whole
    # record: the same repair as the oracle's stored result
    exp = _expected(name)["repair_policy0"]
    km = synth.generate("plain-large", mode=mode)
    old = (L.set_tuning(L.TUNE_SCAN_PIPELINE, 0), L.set_tuning(L.TUNE_SCAN_FIELDS, 0))
    try:
        for pipe in (0, 1):
            for fields in (0, 1):
                L.set_tuning(L.TUNE_SCAN_PIPELINE, pipe)
                L.set_tuning(L.TUNE_SCAN_FIELDS, fields)
                g = L.repair(km, policy=0)
                assert same_repair(g, exp), (pipe, fields, g, exp)
    finally:
        L.set_tuning(L.TUNE_SCAN_PIPELINE, old[0])
        L.set_tuning(L.TUNE_SCAN_FIELDS, old[1])


def test_pass_shapes_full_size(L):
    # every tile shape on each pass of plain-large's 6, 7 and 6-bit plan in
    # turn, the other passes on a 1024 x 8 tile, and two per-pass mixes of
    # its 10 and 9-bit plan: the same races as the oracle's stored result
    exp = _expected("plain_large_literal")
    km = synth.generate("plain-large", mode="literal")
    x, c = next(iter(exp["checks"].items()))
    old = (L.set_tuning(L.TUNE_SCATTER_SHAPE, 3),
           L.set_tuning(L.TUNE_PASS_SHAPES, L.PASS_SHAPES_DEFAULT),
           L.set_tuning(L.TUNE_SORT_DIGIT_BITS, 0), L.set_tuning(L.TUNE_LOW_DIGIT_BITS, 6))
    try:
        cases = [(6, [None] * p + [sh]) for p in range(3) for sh in range(10)]
        cases += [(9, [6, 8]), (9, [7, 0])]
        for low, shapes in cases:
            L.set_tuning(L.TUNE_LOW_DIGIT_BITS, low)
            L.set_tuning(L.TUNE_PASS_SHAPES, L.pass_shapes_value(shapes))
            g = L.check(km, int(x))
            assert L.last_stats()["sort_passes"] == (3 if low == 6 else 2), (low, shapes)
            assert g[0] == 0 and g[3] == c["n_records"], (low, shapes)
            assert [list(p) for p in g[1]] == c["pairs"], (low, shapes)
    finally:
        L.set_tuning(L.TUNE_SCATTER_SHAPE, old[0])
        L.set_tuning(L.TUNE_PASS_SHAPES, old[1])
        L.set_tuning(L.TUNE_SORT_DIGIT_BITS, old[2])
        L.set_tuning(L.TUNE_LOW_DIGIT_BITS, old[3])


def test_sort_knobs_full_size(L):
    # every digit plan (one width of 8..11 bits, or a 6..9-bit lowest digit
    # with the rest of the 19 key bits in digits of at most 10 bits, one
    # width where the rest is too short) and scatter tile
    # shape, with the scatter's grid at its resident size and at one
    # workgroup per compute unit (so the ~1,600 sort chunks of this log are
    # handed out by ticket), with the highest and with the lowest key digit
    # sorted first: the same races as the oracle's stored result
    exp = _expected("plain_large_literal")
    km = synth.generate("plain-large", mode="literal")
    x, c = next(iter(exp["checks"].items()))
    old = (L.set_tuning(L.TUNE_SORT_DIGIT_BITS, 0), L.set_tuning(L.TUNE_SCATTER_SHAPE, 4),
           L.set_tuning(L.TUNE_SCATTER_WGS, 0), L.set_tuning(L.TUNE_DIGIT_ORDER, 1),
           L.set_tuning(L.TUNE_LOW_DIGIT_BITS, 6))
    try:
        for order in (1, 0):
            for bits, low in ((0, 6), (0, 7), (0, 8), (0, 9), (8, 0), (9, 0), (10, 0), (11, 0)):
                for shape in range(10):
                    for wgs in (0, 1):
                        case = (order, bits, low, shape, wgs)
                        L.set_tuning(L.TUNE_DIGIT_ORDER, order)
                        L.set_tuning(L.TUNE_SORT_DIGIT_BITS, bits)
                        L.set_tuning(L.TUNE_LOW_DIGIT_BITS, low)
                        L.set_tuning(L.TUNE_SCATTER_SHAPE, shape)
                        L.set_tuning(L.TUNE_SCATTER_WGS, wgs)
                        g = L.check(km, int(x))
                        assert g[0] == 0 and g[3] == c["n_records"], case
                        assert g[2] == c["divergent"], case
                        assert [list(p) for p in g[1]] == c["pairs"], case
    finally:
        L.set_tuning(L.TUNE_SORT_DIGIT_BITS, old[0])
        L.set_tuning(L.TUNE_SCATTER_SHAPE, old[1])
        L.set_tuning(L.TUNE_SCATTER_WGS, old[2])
        L.set_tuning(L.TUNE_DIGIT_ORDER, old[3])
        L.set_tuning(L.TUNE_LOW_DIGIT_BITS, old[4])


def _many_clause_kernel(seed, n_slots=64):
    # one block of 64 threads, one shared array; groups of accesses (one
    # write, or up to eight reads) separated by barrier slots, so every race
    # has a slot between its points and no clause is empty: a few hundred
    # learned clauses with many distinct slot sets, and the clause sort of
    # the Verify round spans several waves of its workgroup
    rng = np.random.default_rng(seed)
    pts = []
    for s in range(n_slots + 1):
        if rng.random() < 0.4:
            pts.append(dict(kind=0, is_write=1, a=1, c=int(rng.integers(-2, 3))))
        else:
            for _ in range(int(rng.integers(1, 9))):
                pts.append(dict(kind=0, is_write=0, a=int(rng.integers(0, 2)),
                                c=int(rng.integers(-2, 3))))
        if s < n_slots:
            pts.append(dict(kind=1, slot=s))
    slots = [(0, 0, int(rng.integers(1, 4))) for _ in range(n_slots)]
    return synth.make_kernel(1, 64, [(128, 0)], [(1, 0)], pts, slots)


def test_clause_sort_many_clauses(L):
    for seed in range(4):
        km = _many_clause_kernel(seed)
        rng = np.random.default_rng(100 + seed)
        for x in [0] + [int(v) for v in rng.integers(0, 1 << 62, size=3)]:
            assert L.clauses(km, x) == O.clauses(km, x), (seed, x)


def test_edge_empty_and_degenerate(L):
    km = synth.make_kernel(1, 1, [], [(1, 0)], [], [])
    assert L.check(km, 0)[:4] == O.check(km, 0)
    assert same_repair(L.repair(km), O.repair(km))
    # no slots, one racing write: UNSAT
    km = synth.make_kernel(1, 8, [(16, 0)], [(1, 0)], [dict(kind=0, is_write=1, a=0)], [])
    assert L.check(km, 0)[:4] == O.check(km, 0)
    assert same_repair(L.repair(km), O.repair(km))
    # one thread, one block: nothing can race
    km = synth.make_kernel(1, 1, [(4, 1)], [(1, 0)],
                           [dict(kind=0, is_write=1), dict(kind=1, slot=0),
                            dict(kind=0, is_write=1)], [(0, 1, 1)])
    assert same_repair(L.repair(km), O.repair(km))
    # array sizes that are not powers of two, negative strides
    pts = [dict(kind=0, is_write=1, a=-1, b=3, c=-2), dict(kind=1, slot=0),
           dict(kind=0, is_write=0, a=2, b=5, c=1), dict(kind=1, slot=1, guard=1),
           dict(kind=0, is_write=1, a=1, b=7, c=0)]
    km = synth.make_kernel(3, 7, [(13, 1)], [(1, 0), (3, 1)], pts,
                           [(0, 0, 2), (1, 1, 5)])
    for x in range(4):
        assert L.check(km, x)[:4] == O.check(km, x, literal=True), x
    assert same_repair(L.repair(km), O.repair(km))


def test_ragged_tiles(L):
    # record counts that leave partial sort and scan tiles, several blocks
    for T, B in ((63, 3), (65, 5), (200, 41), (257, 2)):
        cfg = synth.config("plain-small")
        cfg.update(blocks=B, threads=T, arrays=[(4096, 0), (8192, 1)], P=40, S=8, S_grid=2,
                   a_set=(-1, 0, 1, 2), b_set=(0, T), guard_frac=0.3, loop_frac=0.3, unroll=3)
        for seed in range(3):
            rng = np.random.default_rng(seed)
            km = synth.planted_kernel(cfg, rng)
            assert same_repair(L.repair(km), O.repair(km)), (T, B, seed)
            assert L.check(km, 0)[:4] == O.check(km, 0), (T, B, seed)


def test_errors(L):
    good = synth.generate("plain-small", seed=1)
    bad = good.copy()
    bad.points["array"][0] = 7
    assert L.validate(bad) == L.ERR_INVALID
    assert L.check(bad, 0)[0] == L.ERR_INVALID
    assert L.repair(bad)["status"] == L.ERR_INVALID
    # output capacity: the needed count comes back
    st, pairs, div, nrec, n = L.check(good, 0, cap=0)
    o = O.check(good, 0)
    if o[1]:
        assert st == L.ERR_CAPACITY and n == len(o[1])
    # workspace too small
    ws = L.Workspace()
    ws.get(16)
    import ctypes as C
    ka = L.KernelArg(good)
    out = L.RpOut()
    o = L.RpOpts(0, 1, 1, 0, 0)
    st = L.lib().rp_repair(ka.ref, C.byref(o), C.byref(out), None, 0,
                           C.c_void_p(ws.t.data_ptr()), 16, None)
    assert st == L.ERR_WORKSPACE


def _mixed_kernels():
    kms = []
    for seed in range(12):
        kms.append(synth.generate("plain-small", mode="planted", seed=seed))
        kms.append(synth.generate("plain-small", seed=100 + seed))
    for seed in range(16):
        kms.append(BF.tiny_kernel(np.random.default_rng(60_000 + seed)))
    # a few medium kernels from the batched distribution (small sizes)
    cfg = synth.config("batched")
    for seed in range(6):
        rng = np.random.default_rng(70_000 + seed)
        c = dict(cfg)
        c.update(blocks=int(rng.integers(1, 5)), threads=64 * int(rng.integers(1, 5)),
                 P=int(rng.integers(16, 200)), S=int(rng.integers(2, 20)), S_grid=2)
        kms.append(synth.planted_kernel(c, rng))
    return kms


def test_batch_equals_plain(L):
    kms = _mixed_kernels()
    st, res = L.repair_batch(kms)
    assert st == 0
    for q, km in enumerate(kms):
        o = O.repair(km)
        g = {k: res[q][k] for k in REPAIR_KEYS if k != "trajectory"}
        assert g == {k: o[k] for k in REPAIR_KEYS if k != "trajectory"}, q
    # order does not matter
    perm = np.random.default_rng(1).permutation(len(kms)).tolist()
    st, res2 = L.repair_batch([kms[q] for q in perm])
    assert st == 0
    for a, q in enumerate(perm):
        assert res2[a] == res[q], (a, q)


def test_batch_many_kernels(L):
    # more than 64 kernels: each round reads back only the count of running
    # jobs, the verdicts once at the end; several rounds replay the graph
    kms = [BF.tiny_kernel(np.random.default_rng(90_000 + q), bias=True) for q in range(80)]
    for kw in (dict(), dict(policy=1)):
        st, res = L.repair_batch(kms, **kw)
        assert st == 0
        assert max(r["rounds"] for r in res) >= 3
        for q, km in enumerate(kms):
            o = O.repair(km, **kw)
            g = {k: res[q][k] for k in REPAIR_KEYS if k != "trajectory"}
            assert g == {k: o[k] for k in REPAIR_KEYS if k != "trajectory"}, (kw, q)


def test_timing_levels(L):
    km = synth.generate("plain-small", seed=3)
    old = L.set_tuning(L.TUNE_TIMING, 0)
    try:
        r0 = L.repair(km)
        s = L.last_stats()
        assert s["ms_total"] == 0 and s["ms_gen"] == 0 and s["ms_sort"] == 0
        L.set_tuning(L.TUNE_TIMING, 1)
        r1 = L.repair(km)
        s = L.last_stats()
        assert s["ms_total"] > 0 and s["ms_gen"] > 0 and s["ms_sort"] > 0
        assert s["ms_clause"] == 0                 # rounds are not split at level 1
        L.set_tuning(L.TUNE_TIMING, 2)
        r2 = L.repair(km)
        s = L.last_stats()
        assert s["ms_total"] > 0 and s["ms_clause"] > 0
        # timing never changes a result
        assert same_repair(r0, r1) and same_repair(r1, r2)
    finally:
        L.set_tuning(L.TUNE_TIMING, old)


def test_batch_policy_and_options(L):
    kms = _mixed_kernels()[:24]
    for kw in (dict(policy=1), dict(grid=0), dict(inspect=0), dict(max_rounds=1)):
        st, res = L.repair_batch(kms, **kw)
        assert st == 0
        for q, km in enumerate(kms):
            o = O.repair(km, **kw)
            g = {k: res[q][k] for k in REPAIR_KEYS if k != "trajectory"}
            assert g == {k: o[k] for k in REPAIR_KEYS if k != "trajectory"}, (kw, q)


def test_batch_invalid_member(L):
    kms = _mixed_kernels()[:8]
    bad = kms[3].copy()
    bad.points["array"][0] = 9
    bad.points["kind"][0] = 0
    kms[3] = bad
    st, res = L.repair_batch(kms)
    assert st == 0
    assert res[3]["status"] == L.ERR_INVALID
    for q in (0, 1, 2, 4, 5, 6, 7):
        o = O.repair(kms[q])
        assert res[q]["status"] == o["status"] and res[q]["assign"] == o["assign"], q


def test_server_continuous_batching(L):
    # jobs arrive over several steps; each result equals the job's result
    # alone, and newly admitted jobs share rounds with resident ones
    kms = _mixed_kernels()
    srv = L.Server(arena_bytes=3 << 20, max_resident=8)
    try:
        big = synth.generate("plain-large")
        assert srv.submit(big, 999) == L.ERR_BUDGET
        results, overlap, nxt, steps = {}, False, 0, 0
        while len(results) < len(kms):
            for _ in range(3):   # three arrivals per step
                if nxt < len(kms):
                    assert srv.submit(kms[nxt], nxt) == 0
                    nxt += 1
            before = {i for i in results}
            nres, npend = srv.step()
            steps += 1
            if nres >= 2:
                overlap = True
            for jid, r, lat in srv.poll():
                assert jid not in before and lat >= 0
                results[jid] = r
            assert steps < 2000
        assert overlap
        for q, km in enumerate(kms):
            o = O.repair(km)
            g = {k: results[q][k] for k in REPAIR_KEYS if k != "trajectory"}
            assert g == {k: o[k] for k in REPAIR_KEYS if k != "trajectory"}, q
    finally:
        srv.close()


def test_server_recreate_same_results(L):
    kms = _mixed_kernels()[:10]
    outs = []
    for _ in range(2):
        srv = L.Server(arena_bytes=64 << 20, max_resident=64)
        for q, km in enumerate(kms):
            assert srv.submit(km, q) == 0
        res = {}
        while len(res) < len(kms):
            srv.step()
            for jid, r, lat in srv.poll():
                res[jid] = r
        srv.close()
        outs.append(res)
    assert outs[0] == outs[1]


NONE = 0xFFFFFFFF


def _first_from_pairs(pairs, P):
    first = np.full((2, P), NONE, np.uint64)
    for lv, i, j in pairs:
        if j < first[lv][i]:
            first[lv][i] = j
    return first


@pytest.mark.parametrize("pipe,fields", [(0, 0), (1, 0), (0, 1), (1, 1)])
def test_first_partners(L, pipe, fields):
    old = (L.set_tuning(L.TUNE_SCAN_PIPELINE, pipe), L.set_tuning(L.TUNE_SCAN_FIELDS, fields))
    try:
        _first_partners_cases(L)
    finally:
        L.set_tuning(L.TUNE_SCAN_PIPELINE, old[0])
        L.set_tuning(L.TUNE_SCAN_FIELDS, old[1])


def _first_partners_cases(L):
    for seed in range(200):
        rng = np.random.default_rng(80_000 + seed)
        km = BF.tiny_kernel(rng)
        for x in [0] + rng.integers(0, 1 << max(1, km.n_slots), size=2).tolist():
            st, first, div = L.first_partners(km, x)
            o = O.check(km, x)
            assert st == 0 and div == o[2]
            assert (first.astype(np.uint64) == _first_from_pairs(o[1], km.n_points)).all(), (seed, x)
    for seed in range(0, 1000, 50):
        km = synth.generate("plain-small", seed=seed)
        st, first, div = L.first_partners(km, 0)
        assert (first.astype(np.uint64) == _first_from_pairs(O.check(km, 0)[1], km.n_points)).all()


def chain_kernel(n_slots=24):
    """One block of 64 threads, two shared arrays X and Y; accesses alternate
    between them with a barrier slot after each: on each array the accesses
    alternate write A[tid] / read A[tid + 1], so every access races with the
    next one on its array, two accesses later.  The races give the clauses
    {s_k, s_k+1}: one constraint component of n_slots slots (a path), wider
    than the enumeration limit, so Solve takes the branch and bound."""
    pts = []
    for k in range(n_slots + 1):
        arr = k % 2
        write = (k // 2) % 2 == 0
        pts.append(dict(kind=0, is_write=int(write), array=arr, a=1, c=0 if write else 1))
        if k < n_slots:
            pts.append(dict(kind=1, slot=k))
    return synth.make_kernel(1, 64, [(128, 0), (128, 0)], [(1, 0)], pts,
                             [(0, 0, 1 + (s % 3)) for s in range(n_slots)])


def test_solver_node_budget(L):
    # the exact search's node budget is a tuning knob; a component that
    # needs more nodes ends its job with RP_ERR_SEARCH (a status of its own)
    km = chain_kernel(24)
    o = O.repair(km)
    assert o["status"] == 0
    g = L.repair(km)
    assert same_repair(g, o), (g, o)
    old = L.set_tuning(L.TUNE_SOLVER_NODES, 4)
    try:
        g = L.repair(km)
        assert g["status"] == L.ERR_SEARCH and g["ret"] == L.ERR_SEARCH, g
        st, full = O.full_clauses(km)
        s = L.min_barriers(full, km.weights.tolist(), km.n_slots)
        assert s[0] == L.ERR_SEARCH
    finally:
        L.set_tuning(L.TUNE_SOLVER_NODES, old)
    assert L.min_barriers(full, km.weights.tolist(), km.n_slots) == \
        O.min_barriers(full, km.weights.tolist(), km.n_slots)


def test_batch_job_error_leaves_the_others(L):
    # one job of a batch fails on the device (its exact search spends the
    # node budget): it alone reads RP_ERR_SEARCH, every other job finishes
    # with the oracle's result
    kms = [synth.generate("plain-small", mode="planted", seed=s) for s in range(6)]
    kms.insert(3, chain_kernel(24))
    old = L.set_tuning(L.TUNE_SOLVER_NODES, 4)
    try:
        st, res = L.repair_batch(kms)
    finally:
        L.set_tuning(L.TUNE_SOLVER_NODES, old)
    assert st == 0
    for q, km in enumerate(kms):
        if q == 3:
            assert res[q]["status"] == L.ERR_SEARCH
            continue
        o = O.repair(km)
        assert {k: res[q][k] for k in REPAIR_KEYS if k != "trajectory"} == \
            {k: o[k] for k in REPAIR_KEYS if k != "trajectory"}, q


def test_solver_hard_components(L):
    # random clause sets over 40-64 slots forming one component, with mixed
    # and negative clauses: the branch and bound against the oracle's
    rng = np.random.default_rng(16)
    for trial in range(12):
        S = int(rng.integers(40, 65))
        cl = []
        for s in range(S - 1):                       # a spine keeps it connected
            cl.append(((1 << s) | (1 << (s + 1)), 0))
        for _ in range(int(rng.integers(S, 3 * S))):
            p = 0
            for _ in range(int(rng.integers(1, 4))):
                p |= 1 << int(rng.integers(0, S))
            cl.append((p, 0))
        for _ in range(int(rng.integers(0, 6))):
            cl.append((0, 1 << int(rng.integers(0, S))))
        w = rng.integers(1, 12, size=S).tolist()
        g = L.min_barriers(cl, w, S)
        o = O.min_barriers(cl, w, S)
        assert g == o, trial
