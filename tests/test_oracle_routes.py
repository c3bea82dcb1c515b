"""The oracle's one-instance-at-a-time route against brute force and against
the whole-kernel route.

Route 1 evaluates the conflict relation per (array, block) for the
same-block relation and per (global array, address stripe) for the
cross-block one, spread over host threads; it is what makes the full-size
stress and batched workloads fit the host.  Every location lies in exactly
one part, so both routes must give the same relation: checked here against
the pure-Python brute force (every record pair) on tiny kernels, with the
stripe size forced down to one record so that every cross-block part is a
single address class, and against route 0 on larger random kernels.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_08373_amd import synth
import bruteforce as BF


@pytest.fixture(autouse=True)
def _restore_route():
    yield
    O.set_route(0)


@pytest.mark.parametrize("chunk", range(3))
def test_per_instance_route_bruteforce(chunk):
    for seed in range(chunk * 150, (chunk + 1) * 150):
        rng = np.random.default_rng(70_000 + seed)
        km = BF.tiny_kernel(rng, max_blocks=4, block_conds=bool(seed % 2))
        conf = BF.conflicting_pairs(km)
        O.set_route(1, 1 + seed % 4, 1 + seed % 3)
        st, pairs, div, nrec = O.check(km, 0)
        assert st == 0 and set(pairs) == conf, seed
        for x in rng.integers(0, 1 << max(1, km.n_slots), size=3).tolist():
            b = O.check(km, x)
            O.set_route(0)
            a = O.check(km, x, literal=True)
            O.set_route(1, 1 + seed % 4, 1 + seed % 3)
            assert a == b, (seed, x)


@pytest.mark.parametrize("chunk", range(2))
def test_per_instance_route_repair_bruteforce(chunk):
    for seed in range(chunk * 120, (chunk + 1) * 120):
        rng = np.random.default_rng(80_000 + seed)
        km = BF.tiny_kernel(rng, max_blocks=3, bias=True)
        best = BF.best_safe(km)
        O.set_route(1, 2, 2)
        for policy in (0, 1):
            r = O.repair(km, policy=policy)
            if best is None:
                assert r["status"] == 1, (seed, policy)
            else:
                assert r["status"] == 0 and r["assign"] == best, (seed, policy)


def _medium_kernel(rng):
    """A few hundred to a few thousand records per array: blocks 2-6, threads
    8-40, small word counts so that addresses wrap and locations collide."""
    B = int(rng.integers(2, 7))
    T = int(rng.integers(8, 41))
    arrays = [(int(rng.integers(16, 200)), int(rng.integers(0, 2))) for _ in range(3)]
    guards = [(1, 0), (2, int(rng.integers(0, 2))), (3, int(rng.integers(0, 3)))]
    points = []
    for _ in range(int(rng.integers(10, 40))):
        points.append(dict(kind=0, is_write=int(rng.random() < 0.4),
                           array=int(rng.integers(0, 3)), guard=int(rng.integers(0, 3)),
                           a=int(rng.integers(-3, 4)), b=int(rng.choice([0, 1, T, -T, 7])),
                           c=int(rng.integers(-5, 6))))
    return synth.make_kernel(B, T, arrays, guards, points, [])


def test_per_instance_route_equals_whole_kernel_route():
    for seed in range(60):
        rng = np.random.default_rng(90_000 + seed)
        km = _medium_kernel(rng)
        O.set_route(0)
        a = O.check(km, 0)
        fa = O.full_clauses(km)
        O.set_route(1, 1 + seed % 5, [0, 1, 50, 400][seed % 4])
        b = O.check(km, 0)
        fb = O.full_clauses(km)
        assert a == b, seed
        assert fa == fb, seed


def test_per_instance_route_plain_small_repairs():
    for seed in range(40):
        km = synth.generate("plain-small", mode="literal", seed=seed)
        O.set_route(0)
        a = O.repair(km)
        O.set_route(1, 3)
        assert O.repair(km) == a, seed
