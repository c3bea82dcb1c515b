"""HIP path against the oracle's stored results at full workload sizes.

The expected values under tests/golden/expected_*.json are written by
tests/golden/make_expected.py, which calls only the CPU oracle.  Every
comparison is exact (the whole path is integer):

  * the kernel at the 4,096-point limit: Verify (every racing pair),
    GenerateClause and the repair loop;
  * the 1,024-kernel batched workload (threads log-uniform in [64, 65536]):
    every kernel's repair result (verdict, barrier set, weight, changes,
    Verify calls, constraint count) from one batched call in planted and in
    literal mode; Verify and GenerateClause on 16 kernels
    spread over the size range, the largest included; the same kernels
    through the continuous-batching server;
  * the stress kernel (4,096 blocks x 1,024 threads, 1,024 points, eight
    16M-word arrays, about 2G access records): Verify and GenerateClause at
    every stored assignment and the repair loop, literal and planted.
"""
import json
import os

import pytest

from paper_2011_08373_amd import synth
from golden_util import GOLDEN, decode_pairs

pytestmark = pytest.mark.gpu

REPAIR_KEYS = ("status", "assign", "weight", "added", "removed", "rounds", "n_clauses",
               "trajectory")


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2011_08373_amd import librepair
    return librepair


def _expected(name):
    path = os.path.join(GOLDEN, "expected_%s.json" % name)
    if not os.path.exists(path):
        pytest.fail("stored oracle result %s is missing (tests/golden/make_expected.py)" % path)
    with open(path) as f:
        return json.load(f)


def _pairs(c, P):
    if "pairs_z" in c:
        return decode_pairs(c["pairs_z"], P)
    return [tuple(p) for p in c["pairs"]]


def _same_repair(g, o, keys=REPAIR_KEYS):
    return {k: g[k] for k in keys} == {k: o[k] for k in keys}


# batched and served results carry no per-round trajectory
BATCH_KEYS = tuple(k for k in REPAIR_KEYS if k != "trajectory")


def _check_and_clauses(L, km, exp):
    P = km.n_points
    for x, c in exp["checks"].items():
        print("  check x=%#x" % int(x), flush=True)
        st, pairs, div, nrec, n = L.check(km, int(x))
        assert st == 0, (x, st)
        assert nrec == c["n_records"], x
        assert div == c["divergent"], x
        assert n == c["n_pairs"], x
        assert [tuple(p) for p in pairs] == _pairs(c, P), x
        st, cl = L.clauses(km, int(x))
        assert st == 0, (x, st)
        assert [list(q) for q in cl] == exp["clauses"][x], x


def test_max_points(L):
    # 4,096 points, 64 slots, 16 arrays: the largest program the model admits
    exp = _expected("max_points")
    km = synth.max_points_kernel()
    assert km.n_points == 4096
    _check_and_clauses(L, km, exp)
    assert _same_repair(L.repair(km, policy=0), exp["repair_policy0"])


@pytest.fixture(scope="module")
def batched_expected():
    return _expected("batched")


@pytest.mark.parametrize("mode", ["planted", "literal"])
def test_batched_full_size(L, batched_expected, mode):
    # one rp_repair_batch call over all 1,024 kernels of the workload
    exp = batched_expected["repair_" + mode]
    kms = synth.generate_batch(mode=mode)
    assert len(kms) == len(exp) == 1024
    st, res = L.repair_batch(kms)
    assert st == 0
    bad = [q for q in range(len(kms)) if not _same_repair(res[q], exp[q], BATCH_KEYS)]
    assert not bad, (len(bad), bad[:5], res[bad[0]], exp[bad[0]]) if bad else None


def test_batched_checked_kernels(L, batched_expected):
    # Verify and GenerateClause at x = 0 on 16 kernels spread over the size
    # range of (point, block, thread) accesses, the largest included
    kms = synth.generate_batch(mode="planted")
    checked = batched_expected["checked"]
    assert len(checked) >= 12

    def accesses(k):
        return k.blocks * k.threads * int((k.points["kind"] == 0).sum())
    sizes = []
    for q, c in checked.items():
        km = kms[int(q)]
        sizes.append(accesses(km))
        st, pairs, div, nrec, n = L.check(km, 0)
        assert st == 0 and nrec == c["n_records"] and div == c["divergent"], q
        assert [list(p) for p in pairs] == c["pairs"], q
        st, cl = L.clauses(km, 0)
        assert st == 0 and [list(v) for v in cl] == c["clauses"], q
    assert max(sizes) == max(accesses(k) for k in kms)


def test_served_full_size(L, batched_expected):
    # the same kernels through the continuous-batching server: jobs arrive
    # 48 per step while earlier ones are resident; every verdict equals the
    # oracle's result for that kernel alone
    exp = batched_expected["repair_planted"]
    kms = synth.generate_batch(mode="planted")
    srv = L.Server(arena_bytes=64 << 30, max_resident=256)
    try:
        results, nxt, steps, overlap = {}, 0, 0, 0
        while len(results) < len(kms):
            for _ in range(48):
                if nxt < len(kms):
                    assert srv.submit(kms[nxt], nxt) == 0
                    nxt += 1
            nres, npend = srv.step()
            overlap = max(overlap, nres)
            steps += 1
            for jid, r, lat in srv.poll():
                assert jid not in results
                results[jid] = r
            assert steps < 20000
        assert overlap >= 2
    finally:
        srv.close()
    bad = [q for q in range(len(kms)) if not _same_repair(results[q], exp[q], BATCH_KEYS)]
    assert not bad, (len(bad), bad[:5])


@pytest.mark.parametrize("mode", ["literal", "planted"])
def test_stress_full_size(L, mode):
    # about 2G access records: every racing pair and clause at each stored
    # assignment, and the repair loop
    import torch
    exp = _expected("stress_" + mode)
    km = synth.generate("stress", mode=mode)
    try:
        _check_and_clauses(L, km, exp)
        g = L.repair(km, policy=0)
        assert _same_repair(g, exp["repair_policy0"]), (g, exp["repair_policy0"])
    finally:
        L._ws.t = None
        torch.cuda.empty_cache()
