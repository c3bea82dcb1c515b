"""The CPU oracle against brute force and against itself on tiny/small inputs."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_08373_amd import synth
import bruteforce as BF


@pytest.mark.parametrize("chunk", range(8))
def test_repair_equals_bruteforce(chunk):
    # Lemma: the repair loop with an exact Solve stops at the canonical
    # minimum-weight safe assignment (or proves there is none).
    for seed in range(chunk * 150, (chunk + 1) * 150):
        rng = np.random.default_rng(10_000 + seed)
        km = BF.tiny_kernel(rng)
        assert O.validate(km) == 0, seed
        best = BF.best_safe(km)
        for policy in (0, 1):
            r = O.repair(km, policy=policy)
            if best is None:
                assert r["status"] == 1, (seed, policy)
            else:
                assert r["status"] == 0, (seed, policy)
                assert r["assign"] == best, (seed, policy)
        # Safe(x) <=> x satisfies the assignment-independent constraint set
        st, full = O.full_clauses(km)
        conf = BF.conflicting_pairs(km)
        for x in range(1 << km.n_slots):
            sat = all((x & p) or (~x & n) for p, n in full)
            assert sat == BF.safe(km, x, conf), (seed, x)


@pytest.mark.parametrize("chunk", range(4))
def test_check_literal_grouped_bruteforce(chunk):
    for seed in range(chunk * 100, (chunk + 1) * 100):
        rng = np.random.default_rng(20_000 + seed)
        km = BF.tiny_kernel(rng)
        conf = BF.conflicting_pairs(km)
        st, pairs0, _, _ = O.check(km, 0, literal=True)
        assert set(pairs0) == conf, seed
        for x in rng.integers(0, 1 << max(1, km.n_slots), size=4).tolist():
            a = O.check(km, x, literal=True)
            b = O.check(km, x, literal=False)
            assert a == b, (seed, x)
        for (lv, i, j) in conf:
            assert O.pair_conflict(km, i, j, lv) == 1
        for _ in range(6):
            i, j = sorted(rng.integers(0, km.n_points, size=2).tolist())
            for lv in (0, 1):
                assert O.pair_conflict(km, i, j, lv) == int((lv, i, j) in conf), (seed, i, j, lv)


@pytest.mark.parametrize("chunk", range(4))
def test_block_conditions_bruteforce(chunk):
    # guards with a condition on the block id: records of the executing
    # blocks only; a grid barrier diverges when part of the grid reaches it
    for seed in range(chunk * 120, (chunk + 1) * 120):
        rng = np.random.default_rng(40_000 + seed)
        km = BF.tiny_kernel(rng, max_blocks=4, block_conds=True)
        assert O.validate(km) == 0, seed
        conf = BF.conflicting_pairs(km)
        assert set(O.check(km, 0, literal=True)[1]) == conf, seed
        for x in [0] + rng.integers(0, 1 << max(1, km.n_slots), size=3).tolist():
            a = O.check(km, x, literal=True)
            assert a == O.check(km, x, literal=False), (seed, x)
            assert (not a[1] and not a[2]) == BF.safe(km, x, conf), (seed, x)
        best = BF.best_safe(km)
        for policy in (0, 1):
            r = O.repair(km, policy=policy)
            if best is None:
                assert r["status"] == 1, (seed, policy)
            else:
                assert (r["status"], r["assign"]) == (0, best), (seed, policy)


def test_grid_divergence_and_block_conditions_pins():
    # two blocks of 4 threads, one global array of 8 words
    def kern(block_guards, level, is_write_b=1, b=0):
        return synth.make_kernel(
            2, 4, [(8, 1)], [(1, 0), (1, 0)],
            [dict(kind=0, is_write=1, array=0, guard=1, a=1, b=b, c=0),
             dict(kind=1, slot=0, guard=1),
             dict(kind=0, is_write=is_write_b, array=0, guard=0, a=1, b=b, c=0)],
            [(level, 0, 1)], block_guards=block_guards)
    # a grid barrier only block 0 reaches diverges; a block barrier does not
    assert O.check(kern([(1, 0), (2, 0)], 1), 1)[2] == 1
    assert O.check(kern([(1, 0), (2, 0)], 0), 1)[2] == 0
    assert O.check(kern([(1, 0), (1, 0)], 1), 1)[2] == 0
    assert O.check(kern(None, 1), 1)[2] == 0
    # every block writes words 0..3 at point 0: the two blocks race there
    # (0 with 0, cross-block) unless only one block executes it
    st, pairs, div, n = O.check(kern(None, 0), 0)
    assert (1, 0, 0) in pairs and n == 16
    st, pairs, div, n = O.check(kern([(1, 0), (2, 1)], 0), 0)
    assert (1, 0, 0) not in pairs and (1, 0, 2) in pairs and n == 12
    # the repair: only a grid barrier orders the blocks, and with the write
    # restricted to block 0 that barrier diverges -> no repair
    r = O.repair(kern([(1, 0), (2, 0)], 1))
    assert r["status"] == 1
    r = O.repair(kern(None, 1))
    assert r["status"] == 1          # point 0 races with itself across blocks
    r = O.repair(kern([(1, 0), (2, 0)], 0, b=4))
    assert r["status"] == 0 and r["assign"] == 0   # block-owned words: no race


def test_check_literal_grouped_plain_small():
    for seed in range(0, 1000, 37):
        km = synth.generate("plain-small", seed=seed)
        rng = np.random.default_rng(seed)
        for x in [0] + rng.integers(0, 16, size=3).tolist():
            assert O.check(km, x, literal=True) == O.check(km, x, literal=False), (seed, x)


def _random_clauses(rng, S, n):
    out = []
    for _ in range(n):
        kind = rng.random()
        p = int(rng.integers(0, 1 << S))
        q = int(rng.integers(0, 1 << S))
        if kind < 0.6:
            out.append((p | (1 << int(rng.integers(0, S))), 0))
        elif kind < 0.85:
            out.append((0, 1 << int(rng.integers(0, S))))
        else:
            out.append((p & ~q, q & ~p))
    return out


def test_solver_methods_agree_with_bruteforce():
    rng = np.random.default_rng(7)
    for _ in range(400):
        S = int(rng.integers(1, 11))
        cl = _random_clauses(rng, S, int(rng.integers(0, 14)))
        w = rng.integers(1, 6, size=S).tolist()
        best = BF.best_clause_solution(cl, w, S)
        for method in (0, 1, 2):
            st, a, wt = O.min_barriers(cl, w, S, method)
            if best is None:
                assert st == 1
            else:
                assert (st, a) == (0, best), (cl, w, method)
                assert wt == BF.key(best, w)[0]


def test_bnb_matches_exhaustive_large_components():
    # components wider than 20 slots take the branch-and-bound route
    rng = np.random.default_rng(11)
    for _ in range(12):
        S = 24
        cl = []
        for _ in range(30):
            lo = int(rng.integers(0, S - 1))
            hi = int(rng.integers(lo, min(S, lo + 5)))
            cl.append((((1 << (hi + 1)) - 1) & ~((1 << lo) - 1), 0))
        cl += [(0, 1 << int(rng.integers(0, S))) for _ in range(3)]
        cl.append(((1 << S) - 1, 0))  # ties everything into one component
        w = rng.integers(1, 4, size=S).tolist()
        a = O.min_barriers(cl, w, S, 1)
        b = O.min_barriers(cl, w, S, 2)
        assert a == b


def test_reduce_definition():
    rng = np.random.default_rng(3)
    for _ in range(200):
        cl = _random_clauses(rng, 6, int(rng.integers(0, 12)))
        red = O.reduce(cl)
        uniq = sorted(set(cl))
        exp = [c for c in uniq if not any(d != c and (d[0] & ~c[0]) == 0 and (d[1] & ~c[1]) == 0
                                          for d in uniq)]
        assert red == exp


def tiny_planted_config(rng):
    T = int(rng.integers(2, 9))
    B = int(rng.integers(1, 3))
    return dict(blocks=B, threads=T, arrays=[(4 * T, 0), (4 * T * B, 1)],
                P=int(rng.integers(4, 13)), S=int(rng.integers(1, 7)),
                S_grid=int(rng.integers(0, 3)), write_frac=0.5, a_set=(-1, 0, 1, 2),
                b_set=(0, T), c_rng=(-2, 2), guard_frac=0.2, loop_frac=0.2, unroll=2,
                access_frac=1.0, pre_frac=0.3, weight_mode="paper")


@pytest.mark.parametrize("chunk", range(4))
def test_planted_tiny_bruteforce(chunk):
    # planted kernels are repairable; the result is the brute-force optimum
    # and never heavier than the hidden assignment
    n_nonzero = 0
    for seed in range(chunk * 100, (chunk + 1) * 100):
        rng = np.random.default_rng(30_000 + seed)
        km = synth.planted_kernel(tiny_planted_config(rng), rng)
        assert O.validate(km) == 0
        xs = km.meta["x_star"]
        assert BF.safe(km, xs), seed
        best = BF.best_safe(km)
        r = O.repair(km)
        assert r["status"] == 0 and r["assign"] == best, seed
        w = [int(v) for v in km.slots["weight"]]
        assert BF.key(best, w) <= BF.key(xs, w)
        n_nonzero += best != 0
    assert n_nonzero >= 8
