"""The CPU oracle pinned to the paper's worked examples and to closed forms.

Each fixture under tests/golden/ cites the listing or section it encodes.
"""
import pytest

from oracle import oracle as O
from paper_2011_08373_amd import synth
from golden_util import kernel_from_json, listing_fixtures, load

FIXTURES = listing_fixtures()


@pytest.mark.parametrize("name,fx", FIXTURES, ids=[n for n, _ in FIXTURES])
def test_listing_check(name, fx):
    km = kernel_from_json(fx)
    assert O.validate(km) == 0
    for x, exp in fx["expect"].get("check", {}).items():
        for literal in (True, False):
            st, pairs, div, _ = O.check(km, int(x), literal=literal)
            assert st == 0
            assert [list(p) for p in pairs] == exp["pairs"], (name, x, literal)
            assert div == exp["divergent"], (name, x, literal)


@pytest.mark.parametrize("name,fx", FIXTURES, ids=[n for n, _ in FIXTURES])
def test_listing_clauses(name, fx):
    km = kernel_from_json(fx)
    for x, exp in fx["expect"].get("clauses", {}).items():
        st, cl = O.clauses(km, int(x))
        assert st == 0
        assert [list(c) for c in cl] == exp, (name, x)


@pytest.mark.parametrize("name,fx", FIXTURES, ids=[n for n, _ in FIXTURES])
@pytest.mark.parametrize("policy", [0, 1])
def test_listing_repair(name, fx, policy):
    km = kernel_from_json(fx)
    exp = fx["expect"]["repair"]
    r = O.repair(km, policy=policy)
    assert r["status"] == exp["status"], name
    if exp["status"] == 0:
        for key in ("assign", "weight", "added", "removed"):
            assert r[key] == exp[key], (name, key)
        assert O.check(km, r["assign"])[1] == []
    if policy == 0:
        assert r["rounds"] == exp["rounds"], name


def test_listing1_fixed_by_exactly_one_barrier():
    # Section 1: the race of Listing 1 is avoided by one __syncthreads()
    km = kernel_from_json(load("listing1_race"))
    r = O.repair(km)
    assert bin(r["assign"]).count("1") == 1


def test_solver_examples():
    fx = load("solver_examples")
    for case in fx["cases"]:
        for method in (0, 1, 2):
            st, a, w = O.min_barriers(case["clauses"], case["weights"], case["n_slots"], method)
            exp = case["expect"]
            assert st == exp["status"], (case["name"], method)
            if st == 0:
                assert (a, w) == (exp["assign"], exp["weight"]), (case["name"], method)


def test_mixed_clauses_greedy_fails():
    # Section 2.4: the positive clauses' minimal hitting set {b1, b2}
    # violates the negative clause, so the exact answer needs 3 barriers.
    case = load("solver_examples")["cases"][0]
    pos = [p for p, n in case["clauses"] if n == 0]
    greedy = 0b11
    assert all(greedy & p for p in pos)
    assert not all((greedy & p) or (~greedy & n) for p, n in case["clauses"])


def test_weight_formula():
    fx = load("weights")
    for c in fx["cases"]:
        assert synth.paper_weight(c["level"], c["depth"]) == c["weight"]


# ---------------------------------------------------------------- closed forms

def _two_access(T, N, c1, c2, w1, w2, a1=1, a2=1, blocks=1, space=0, b=0):
    pts = [dict(kind=0, is_write=w1, a=a1, b=b, c=c1), dict(kind=1, slot=0),
           dict(kind=0, is_write=w2, a=a2, b=b, c=c2)]
    return synth.make_kernel(blocks, T, [(N, space)], [(1, 0)], pts, [(0, 0, 1)])


@pytest.mark.parametrize("T", [5, 8, 31, 64])
def test_closed_form_shift(T):
    # a = 1, b = 0, same shared array, N >= T + 4: thread t' = t + c1 - c2
    # exists (|c1 - c2| <= 4 < T) and no wrap collides, so the two accesses
    # meet on distinct threads exactly when c1 != c2.
    N = T + 4
    for c1 in range(-2, 3):
        for c2 in range(-2, 3):
            for w1, w2 in ((1, 0), (0, 1), (1, 1)):
                km = _two_access(T, N, c1, c2, w1, w2)
                st, pairs, div, _ = O.check(km, 0)
                conflict = (0, 0, 2) in pairs
                assert conflict == (c1 != c2), (T, c1, c2, w1, w2)
                assert O.pair_conflict(km, 0, 2, 0) == int(c1 != c2)
                # the barrier between them always separates
                assert (0, 0, 2) not in O.check(km, 1)[1]


@pytest.mark.parametrize("a", [1, -1, 2])
def test_closed_form_injective_write(a):
    # a write whose map tid -> address is injective (|a| <= 2, 2T <= N)
    # never conflicts with itself
    T, N = 32, 64
    km = _two_access(T, N, 0, 1, 1, 1, a1=a, a2=a)
    pairs = O.check(km, 0)[1]
    assert (0, 0, 0) not in pairs and (0, 2, 2) not in pairs


@pytest.mark.parametrize("m", [1, 2, 4])
def test_closed_form_constant_write(m):
    # a = 0 write with >= 2 active threads always conflicts with itself
    T, N = 16, 64
    pts = [dict(kind=0, is_write=1, a=0, c=3, guard=1)]
    km = synth.make_kernel(1, T, [(N, 0)], [(1, 0), (m, 0)], pts, [])
    pairs = O.check(km, 0)[1]
    assert pairs == [(0, 0, 0)]
    r = O.repair(km)
    assert r["status"] == 1 and r["rounds"] == 1


def test_global_array_cross_block_closed_form():
    # GLOBAL array, a = 1, b = T: blocks own disjoint words; the only
    # cross-block meeting of read A[t+1+bT] and write A[t+bT] is thread T-1
    # of block k with thread 0 of block k+1.
    T, B = 8, 4
    km = _two_access(T, T * B + 4, 1, 0, 0, 1, blocks=B, space=1, b=T)
    pairs = O.check(km, 0)[1]
    assert (0, 0, 2) in pairs and (1, 0, 2) in pairs
    assert (1, 2, 2) not in pairs and (0, 2, 2) not in pairs
    # a block barrier between them does not order different blocks
    assert O.check(km, 1)[1] == [(1, 0, 2)]


def test_negative_mod_is_euclidean():
    # a = -1, c = -2: thread t touches (-t - 2) mod N; thread 0 -> N - 2.
    T, N = 4, 16
    pts = [dict(kind=0, is_write=1, a=-1, c=-2), dict(kind=0, is_write=0, a=0, c=N - 2)]
    km = synth.make_kernel(1, T, [(N, 0)], [(1, 0)], pts, [])
    pairs = O.check(km, 0)[1]
    # thread 0 writes N-2, threads 1..3 read N-2
    assert pairs == [(0, 0, 1)]
    pts[1]["c"] = N - 1  # nobody writes N-1 (addresses N-2..N-5)
    km = synth.make_kernel(1, T, [(N, 0)], [(1, 0)], pts, [])
    assert O.check(km, 0)[1] == []


def test_validation_rules():
    base = dict(blocks=1, threads=4, arrays=[(8, 0)], guards=[(1, 0)],
                points=[dict(kind=1, slot=0), dict(kind=0, is_write=1, a=1)],
                slots=[(0, 0, 1)])
    assert O.validate(synth.make_kernel(**base)) == 0
    bad = []
    b = dict(base); b["threads"] = 0; bad.append(b)
    b = dict(base); b["guards"] = [(2, 2)]; bad.append(b)
    b = dict(base); b["slots"] = [(0, 0, 0)]; bad.append(b)
    b = dict(base); b["points"] = [dict(kind=1, slot=1), dict(kind=0)]; bad.append(b)
    b = dict(base); b["points"] = [dict(kind=0, array=3)]; b["slots"] = []; bad.append(b)
    b = dict(base); b["slots"] = [(0, 0, 1), (0, 0, 1)]; bad.append(b)  # slot 1 never occurs
    b = dict(base); b["guards"] = [(1, 0), (2, 0)]
    b["points"] = [dict(kind=1, slot=0), dict(kind=1, slot=0, guard=1)]; bad.append(b)
    b = dict(base); b["points"] = [dict(kind=3)]; b["slots"] = []; bad.append(b)
    for b in bad:
        assert O.validate(synth.make_kernel(**b)) == -1, b


def test_empty_kernel():
    km = synth.make_kernel(1, 1, [], [(1, 0)], [], [])
    st, pairs, div, n = O.check(km, 0)
    assert (st, pairs, div, n) == (0, [], 0, 0)
    r = O.repair(km)
    assert r["status"] == 0 and r["assign"] == 0 and r["rounds"] == 1


def test_options_grid_and_inspect():
    km = kernel_from_json(load("grid_barrier_repair"))
    # grid-level barriers disabled: only a grid barrier can fix it -> UNSAT
    assert O.repair(km, grid=0)["status"] == 1
    # pre-existing barrier kept when not inspected
    fx = load("listing2_divergence")
    km = kernel_from_json(fx)
    r = O.repair(km, inspect=0)
    # the kept barrier diverges: no repair exists that keeps it
    assert r["status"] == 1
    km1 = kernel_from_json(load("listing1_race"))
    km1.slots["preexisting"][0] = 1
    r = O.repair(km1, inspect=0)
    assert r["status"] == 0 and r["assign"] == 3 and r["removed"] == 0


def test_options_preexisting_grid_barrier():
    # the grid switch turns off every grid slot, the programmer's included;
    # the inspection switch keeps every pre-existing slot on.  Both at once on
    # a pre-existing grid barrier: UNSAT at the first Solve, no Verify call
    km = kernel_from_json(load("grid_barrier_repair"))
    km.slots["preexisting"][2] = 1
    for grid, inspect, want in ((1, 1, (0, 4, 2)), (1, 0, (0, 4, 1)),
                                (0, 1, (1, None, 1)), (0, 0, (1, None, 0))):
        r = O.repair(km, grid=grid, inspect=inspect)
        st, assign, rounds = want
        assert (r["status"], r["rounds"]) == (st, rounds), (grid, inspect, r)
        if st == 0:
            assert r["assign"] == assign and r["added"] == 0 and r["removed"] == 0


def test_max_rounds():
    km = kernel_from_json(load("listing1_race"))
    r = O.repair(km, max_rounds=1)
    assert r["status"] == -5 and r["rounds"] == 1
    assert O.repair(km, max_rounds=2)["status"] == 0
