"""The instrumentation pass (Section 2.2): the oracle pinned against the
paper's listings and closed forms, and the library's pass (host-only C ABI
call, no GPU) equal to the oracle on random programs."""
import math

import numpy as np
import pytest

from oracle import instrument as OI
from oracle import oracle as O
from paper_2011_08373_amd import synth
from paper_2011_08373_amd.synth import (BLOCK, GRID, GLOBAL, SHARED, st_access, st_barrier,
                                        st_call, st_end, st_if, st_loop)
from golden_util import kernel_from_json, load


@pytest.fixture(scope="module")
def L():
    from paper_2011_08373_amd import librepair
    return librepair


def prog(functions, guards=((1, 0),), arrays=((128, SHARED),), blocks=1, threads=64):
    return synth.Program(blocks, threads, [tuple(a) for a in arrays], [tuple(g) for g in guards],
                         functions)


def same_kernel(k1, k2):
    bg1 = None if k1.block_guards is None else k1.block_guards.tobytes()
    bg2 = None if k2.block_guards is None else k2.block_guards.tobytes()
    return (k1.blocks, k1.threads) == (k2.blocks, k2.threads) and bg1 == bg2 and all(
        np.asarray(getattr(k1, f)).tobytes() == np.asarray(getattr(k2, f)).tobytes()
        for f in ("arrays", "guards", "points", "slots"))


# The listings as programs.  Their instrumented models were written by hand
# from the listings (tests/golden/), before this pass existed.
READ_NEXT = dict(a=1, c=1)          # A[tid + 1]
WRITE_OWN = dict(a=1, c=0)          # A[tid]
LISTINGS = {
    # Listing 1: temp = A[tid+1]; A[tid] = temp
    "listing1_race": (prog([[st_access(0, 0, **READ_NEXT), st_access(0, 1, **WRITE_OWN)]]), 0),
    # Listing 3: read; if (temp < 50) write(A, tid) -- the data-dependent
    # branch modelled by tid % 2 == 0; grid-level instrumentation enabled
    "listing3_scope": (prog([[st_access(0, 0, **READ_NEXT), st_if(1), st_call(1), st_end()],
                             [st_access(0, 1, **WRITE_OWN)]], guards=((1, 0), (2, 0))), 1),
    # Listing 5: if (tid % 2 == 0) { temp = A[tid+1]; A[tid] = temp; }
    "listing5_as_written": (prog([[st_if(1), st_access(0, 0, **READ_NEXT),
                                   st_access(0, 1, **WRITE_OWN), st_end()]],
                                 guards=((1, 0), (2, 0))), 0),
    # Listing 6: A[tid] = A[tid+1]
    "listing6_single_line": (prog([[st_access(0, 0, **READ_NEXT), st_access(0, 1, **WRITE_OWN)]]), 0),
    # Listing 7: A[0] = tid
    "listing7_write_write": (prog([[st_access(0, 1, a=0, c=0)]]), 0),
    # Listing 8: temp = read(A, tid); write(A, tid, temp) -- both accesses
    # inside called functions
    "listing8_interfunction": (prog([[st_call(1), st_call(2)], [st_access(0, 0, **READ_NEXT)],
                                     [st_access(0, 1, **WRITE_OWN)]]), 0),
}


@pytest.mark.parametrize("name", sorted(LISTINGS))
def test_listings_instrument_to_their_models(L, name):
    p, grid = LISTINGS[name]
    want = kernel_from_json(load(name))
    st, k = OI.instrument(p, grid=grid)
    assert st == 0 and same_kernel(k, want), name
    st, k = L.instrument(p, grid=grid)
    assert st == 0 and same_kernel(k, want), name


def test_listing3_repair_is_the_barrier_before_the_branch():
    # the paper's point: the barrier beside the call inside the branch (b3)
    # would diverge; the repair enables b2, before the branch
    p, _ = LISTINGS["listing3_scope"]
    st, k = OI.instrument(p, grid=1)
    b3 = 4                         # slots: b1 b4 b2 b5 b3 b6
    assert O.check(k, 1 << b3)[:3] == (0, [], 1 << b3)
    r = O.repair(k)
    assert r["status"] == 0 and r["assign"] == 1 << 2 and r["weight"] == 1
    st, k0 = OI.instrument(p, grid=0)   # block-level only: b1 b2 b3
    assert k0.n_slots == 3 and O.repair(k0)["assign"] == 1 << 1


def test_listing2_preexisting_barrier_in_branch():
    # Listing 2: if (tid % 2 == 0) { temp = A[tid+1]; __syncthreads(); A[tid] = temp; }
    p = prog([[st_if(1), st_access(0, 0, **READ_NEXT), st_barrier(BLOCK),
               st_access(0, 1, **WRITE_OWN), st_end()]], guards=((1, 0), (2, 0)))
    st, k = OI.instrument(p, grid=0)
    assert st == 0
    # site before the branch (all threads), site before the read, the
    # programmer's barrier, site before the write (even threads)
    assert k.points["kind"].tolist() == [1, 1, 0, 1, 1, 0]
    assert k.points["slot"][[0, 1, 3, 4]].tolist() == [0, 1, 2, 3]
    assert k.points["guard"].tolist() == [0, 1, 1, 1, 1, 1]
    assert k.slots["preexisting"].tolist() == [0, 0, 1, 0]
    assert [tuple(g) for g in k.guards.tolist()] == [(1, 0), (2, 0)]
    # no two threads meet, the divergent programmer's barrier goes
    r = O.repair(k)
    assert (r["status"], r["assign"], r["removed"]) == (0, 0, 1 << 2)   # removed: a slot mask


def test_loops_unroll_with_loop_variable_terms_and_weights(L):
    # for (i = 0; i < 3; i++) A[tid + 4*i + 1] = ...
    p = prog([[st_loop(3), st_access(0, 1, a=1, c=1, d=4), st_end()]])
    for inst in (OI.instrument, L.instrument):
        st, k = inst(p, grid=0)
        assert st == 0
        assert k.points["kind"].tolist() == [1, 1, 0] * 3
        assert k.points["slot"].tolist() == [0, 1, 0] * 3
        assert k.points["c"][2::3].tolist() == [1, 5, 9]
        assert k.slots["weight"].tolist() == [10, 10]          # lw^1
    # two nested loops, grid twins: head of the outer loop at depth 1, head
    # of the inner loop and the access at depth 2
    p = prog([[st_loop(2), st_loop(2), st_access(0, 0), st_end(), st_end()]])
    st, k = OI.instrument(p, grid=1)
    assert k.slots["weight"].tolist() == [10, 22, 100, 112, 100, 112]
    assert k.slots["level"].tolist() == [BLOCK, GRID] * 3
    assert k.n_points == 2 * (2 + 2 * (2 + 2 + 1))
    st, k = OI.instrument(p, grid=1, gw=5, lw=3)
    assert k.slots["weight"].tolist() == [3, 8, 9, 14, 9, 14]


def test_preexisting_barrier_in_a_function_per_call_site():
    p = prog([[st_call(1), st_loop(2), st_call(1), st_end()],
              [st_access(0, 0), st_barrier(GRID)]], blocks=2)
    st, k = OI.instrument(p, grid=0)
    assert st == 0
    # call site 1: site, access, barrier (slot 1); call site 2 inside the
    # loop: head site, call site, access, barrier (slot 4) -- twice
    pre = k.slots["preexisting"].tolist()
    assert pre == [0, 1, 0, 0, 1]
    assert k.slots["weight"].tolist() == [1, 13, 10, 10, 22]
    assert k.slots["level"].tolist() == [BLOCK, GRID, BLOCK, BLOCK, GRID]


def test_block_branch_with_grid_barrier(L):
    # if (blockIdx.x % 2 == 0) { A[tid] = ...; g.sync(); } ... B[tid] read by all
    p = synth.Program(2, 8, [(16, GLOBAL)], [(1, 0), (1, 0)],
                      [[st_if(1), st_access(0, 1, a=1, b=8), st_barrier(GRID), st_end(),
                        st_access(0, 0, a=1, b=0)]],
                      block_guards=[(1, 0), (2, 0)])
    for inst in (OI.instrument, L.instrument):
        st, k = inst(p, grid=1)
        assert st == 0
        assert [tuple(g) for g in k.guards.tolist()] == [(1, 0), (1, 0)]
        assert [tuple(g) for g in k.block_guards.tolist()] == [(1, 0), (2, 0)]
        # the pre-existing grid barrier runs in block 0 only: it diverges
        pre = int(np.flatnonzero(k.slots["preexisting"])[0])
        assert O.check(k, 1 << pre)[2] == 1 << pre
    st, k = OI.instrument(p, grid=1)
    # block 0 writes words 0..7, every block reads words 0..7 afterwards: the
    # cross-block race needs a grid barrier that every block reaches -- the
    # one before the read (slot of the site before the last access)
    r = O.repair(k)
    assert r["status"] == 0
    assert r["removed"] == 1 << pre
    chosen = [s for s in range(k.n_slots) if (r["assign"] >> s) & 1]
    assert [int(k.slots["level"][s]) for s in chosen] == [GRID]
    # that slot's occurrences run in every block
    occ = [q for q in range(k.n_points) if k.points["kind"][q] == 1 and k.points["slot"][q] == chosen[0]]
    assert all(k.block_guards[k.points["guard"][q]]["m"] == 1 for q in occ)


def test_guard_meet_is_the_residue_class_of_both():
    for m1 in range(1, 9):
        for m2 in range(1, 9):
            for r1 in range(m1):
                for r2 in range(m2):
                    lcm = m1 * m2 // math.gcd(m1, m2)
                    both = {t for t in range(3 * lcm) if t % m1 == r1 and t % m2 == r2}
                    g = OI.residue_meet((m1, r1), (m2, r2))
                    if not both:
                        assert g is None
                    else:
                        m, r = g
                        assert both == {t for t in range(3 * lcm) if t % m == r}


def test_library_guard_meet_on_nested_branches(L):
    guards = [(1, 0), (2, 0), (2, 1), (3, 1), (4, 3), (6, 5), (5, 2)]
    for g1 in range(1, len(guards)):
        for g2 in range(1, len(guards)):
            p = prog([[st_if(g1), st_if(g2), st_access(0, 0), st_end(), st_end()]], guards=guards)
            s1, k1 = L.instrument(p, grid=0)
            s2, k2 = OI.instrument(p, grid=0)
            assert s1 == s2
            (m1, r1), (m2, r2) = guards[g1], guards[g2]
            both = {t for t in range(120) if t % m1 == r1 and t % m2 == r2}
            if not both:
                assert s1 == -1
                continue
            assert same_kernel(k1, k2)
            m, r = k1.guards[k1.points["guard"][-1]].tolist()
            assert both == {t for t in range(120) if t % m == r}


def _counts(p, grid):
    """Closed-form slot and point counts of the instrumented program."""
    F = p.functions
    reach = {}

    def touches(f):
        if f not in reach:
            reach[f] = any(s["kind"] == synth.S_ACCESS or
                           (s["kind"] == synth.S_CALL and touches(s["count"])) for s in F[f])
        return reach[f]

    def pre(f):
        return sum(1 for s in F[f] if s["kind"] == synth.S_BARRIER) + \
            sum(pre(s["count"]) for s in F[f] if s["kind"] == synth.S_CALL)

    per_site = 1 + grid
    sites = sum(1 for s in F[0] if s["kind"] in (synth.S_ACCESS, synth.S_IF, synth.S_LOOP)) + \
        sum(1 for s in F[0] if s["kind"] == synth.S_CALL and touches(s["count"]))

    def points(f, lo, hi):
        n, i = 0, lo
        site = per_site if f == 0 else 0
        while i < hi:
            s = F[f][i]
            k = s["kind"]
            if k in (synth.S_IF, synth.S_LOOP):
                depth, j = 1, i + 1
                while depth:
                    depth += {synth.S_IF: 1, synth.S_LOOP: 1, synth.S_END: -1}.get(F[f][j]["kind"], 0)
                    j += 1
                inner = points(f, i + 1, j - 1)
                n += site + inner if k == synth.S_IF else s["count"] * (site + inner)
                i = j
                continue
            if k == synth.S_ACCESS:
                n += 1 + site
            elif k == synth.S_BARRIER:
                n += 1
            elif k == synth.S_CALL:
                n += (site if touches(s["count"]) else 0) + points(s["count"], 0, len(F[s["count"]]))
            i += 1
        return n

    return per_site * sites + pre(0), points(0, 0, len(F[0]))


def test_counts_closed_form():
    for grid in (0, 1):
        for p in synth.generate_programs(150, seed=21):
            st, k = OI.instrument(p, grid=grid)
            assert st == 0
            assert (k.n_slots, k.n_points) == _counts(p, grid), p.meta
            # every slot's weight is lw^d or gw + lw^d by its level
            for lv, w in zip(k.slots["level"].tolist(), k.slots["weight"].tolist()):
                base = w - 12 if lv == GRID else w
                assert base >= 1 and 10 ** round(math.log10(base)) == base


@pytest.mark.parametrize("grid,gw,lw", [(1, 12, 10), (0, 12, 10), (1, 5, 3)])
def test_library_equals_oracle(L, grid, gw, lw):
    n_ok = 0
    for p in synth.generate_programs(250, seed=7 + grid + lw):
        s1, k1 = L.instrument(p, grid=grid, gw=gw, lw=lw)
        s2, k2 = OI.instrument(p, grid=grid, gw=gw, lw=lw)
        assert s1 == s2, p.meta
        if s1 == 0:
            n_ok += 1
            assert same_kernel(k1, k2), p.meta
            assert L.validate(k1) == 0
    assert n_ok > 200


def test_malformed_programs(L):
    acc = st_access(0, 0)
    cases = [
        prog([[acc, st_end()]]),                                   # END without region
        prog([[st_if(0), acc]]),                                   # unclosed
        prog([[st_call(1)], [st_call(2)], [st_call(1)]]),          # recursion
        prog([[st_call(0)]]),                                      # the kernel is not callable
        prog([[st_call(3)], [acc]]),                               # no such function
        prog([[st_loop(0), acc, st_end()]]),                       # zero trips
        prog([[st_if(5), acc, st_end()]]),                         # no such guard
        prog([[st_if(1), st_if(2), acc, st_end(), st_end()]],
             guards=((1, 0), (2, 0), (2, 1))),                      # no thread takes both
        prog([[st_access(4, 0)]]),                                 # no such array
        prog([[acc] * 40]),                                        # 80 slots with grid twins
        prog([[st_loop(4000), acc, st_end()]]),                    # 12000 points
        prog([[st_loop(2), st_access(0, 1, c=2 ** 31 - 1, d=1), st_end()]]),   # word offset overflow
        prog([[st_loop(2), st_loop(2), st_loop(2), st_loop(2), st_loop(2), st_loop(2),
               st_loop(2), st_loop(2), st_loop(2), st_loop(2), acc] + [st_end()] * 10]),  # 10^10
    ]
    for q, p in enumerate(cases):
        assert OI.instrument(p)[0] == -1, q
        assert L.instrument(p)[0] == -1, q
    # a program the limits admit
    assert L.instrument(prog([[acc] * 32]))[0] == 0
    assert L.instrument(prog([[acc] * 32]), grid=1)[0] == 0
