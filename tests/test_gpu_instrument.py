"""Instrumented programs (Section 2.2) repaired on the GPU: the library's
pass followed by its repair loop, against the oracle's pass followed by the
oracle's repair loop."""
import pytest

from oracle import instrument as OI
from oracle import oracle as O
from paper_2011_08373_amd import synth
from paper_2011_08373_amd.synth import st_access, st_call, st_end, st_if

pytestmark = pytest.mark.gpu

KEYS = ("status", "assign", "weight", "added", "removed", "rounds", "n_clauses")


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2011_08373_amd import librepair
    return librepair


def test_listing3_repaired_before_the_branch(L):
    p = synth.Program(1, 64, [(128, 0)], [(1, 0), (2, 0)],
                      [[st_access(0, 0, a=1, c=1), st_if(1), st_call(1), st_end()],
                       [st_access(0, 1, a=1, c=0)]])
    st, k = L.instrument(p, grid=1)
    assert st == 0
    r = L.repair(k)
    assert (r["status"], r["assign"], r["weight"], r["rounds"]) == (0, 1 << 2, 1, 2)


@pytest.mark.parametrize("grid", [0, 1])
def test_instrumented_programs_batch(L, grid):
    progs = synth.generate_programs(96, seed=5 + grid)
    kms = []
    for p in progs:
        st, k = L.instrument(p, grid=grid)
        so, ko = OI.instrument(p, grid=grid)
        assert st == so == 0, p.meta
        kms.append((k, ko))
    for kw in (dict(), dict(policy=1), dict(policy=1, solver=1)):
        st, res = L.repair_batch([k for k, _ in kms], **kw)
        assert st == 0
        for q, (k, ko) in enumerate(kms):
            o = O.repair(ko, **kw)
            assert {x: res[q][x] for x in KEYS} == {x: o[x] for x in KEYS}, (grid, kw, q)
