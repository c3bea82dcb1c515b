"""The mhs strategy (Section 2.4) on the HIP path against the oracle: the
greedy minimal hitting set per round, the exact fallback, the final exact
query.  Every field is compared exactly, trajectory included."""
import numpy as np
import pytest

import bruteforce as BF
from golden_util import kernel_from_json, listing_fixtures, load
from oracle import oracle as O
from paper_2011_08373_amd import synth

pytestmark = pytest.mark.gpu

FIXTURES = listing_fixtures()
KEYS = ("status", "assign", "weight", "added", "removed", "rounds", "n_clauses", "trajectory")


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2011_08373_amd import librepair
    return librepair


def same(g, o):
    return {k: g[k] for k in KEYS} == {k: o[k] for k in KEYS}


def test_final_exact_query_fixture(L):
    fx = load("mhs_final_query")
    km = kernel_from_json(fx)
    g = L.repair(km, solver=1)
    exp = fx["expect"]["repair_mhs"]
    for k in ("status", "assign", "weight", "rounds", "added", "removed", "trajectory"):
        assert g[k] == exp[k], k
    assert L.repair(km, solver=0)["trajectory"] == fx["expect"]["repair"]["trajectory"]


@pytest.mark.parametrize("name,fx", FIXTURES, ids=[n for n, _ in FIXTURES])
def test_listings(L, name, fx):
    km = kernel_from_json(fx)
    for policy in (0, 1):
        g = L.repair(km, policy=policy, solver=1)
        o = O.repair(km, policy=policy, solver=1)
        assert same(g, o), (name, policy, g, o)


@pytest.mark.parametrize("mode", ["literal", "planted"])
def test_plain_small(L, mode):
    mism = []
    for seed in range(300):
        km = synth.generate("plain-small", mode=mode, seed=seed)
        if mode == "planted":
            km.slots["weight"][:] = np.random.default_rng(seed).integers(1, 6, km.n_slots)
        for policy in (0, 1):
            g = L.repair(km, policy=policy, solver=1)
            o = O.repair(km, policy=policy, solver=1)
            if not same(g, o):
                mism.append((seed, policy, g, o))
    assert not mism, mism[:2]


def test_tiny_weighted(L):
    rng = np.random.default_rng(31)
    for t in range(300):
        km = BF.tiny_kernel(rng, bias=True)
        if km.n_slots:
            km.slots["weight"][:] = rng.integers(1, 6, km.n_slots)
        for policy in (0, 1):
            g = L.repair(km, policy=policy, solver=1)
            o = O.repair(km, policy=policy, solver=1)
            assert same(g, o), (t, policy, g, o)


def test_options_and_round_limit(L):
    km = kernel_from_json(load("mhs_final_query"))
    for mr in (1, 2, 3):
        g = L.repair(km, solver=1, max_rounds=mr)
        o = O.repair(km, solver=1, max_rounds=mr)
        assert same(g, o), mr
    km = synth.generate("plain-small", mode="planted", seed=3)
    for grid, inspect in ((0, 1), (1, 0), (0, 0)):
        g = L.repair(km, solver=1, grid=grid, inspect=inspect)
        o = O.repair(km, solver=1, grid=grid, inspect=inspect)
        assert same(g, o), (grid, inspect)


def test_plain_large_planted(L):
    km = synth.generate("plain-large", mode="planted")
    g = L.repair(km, solver=1)
    o = O.repair(km, solver=1)
    assert same(g, o)
    assert g["assign"] == L.repair(km)["assign"]


def test_batch_equals_plain(L):
    kms = [synth.generate("plain-small", mode="planted", seed=s) for s in range(40)]
    kms.append(kernel_from_json(load("mhs_final_query")))
    st, res = L.repair_batch(kms, solver=1)
    assert st == 0
    for q, km in enumerate(kms):
        o = O.repair(km, solver=1)
        for k in ("status", "assign", "weight", "rounds", "n_clauses"):
            assert res[q][k] == o[k], (q, k)


def test_invalid_solver(L):
    km = kernel_from_json(load("mhs_final_query"))
    assert L.repair(km, solver=2)["ret"] == L.ERR_INVALID
