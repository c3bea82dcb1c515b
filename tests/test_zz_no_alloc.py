"""rp_repair_noalloc (the repair loop in the library's fixed per-device
array) against rp_repair (caller-allocated workspace), through the C ABI.

Results must be identical, trajectory included: two calls in a row with the
second on a smaller kernel, kernels near the array's size limit, the
learning policies and Solve strategies, and the option switches.  A kernel
whose workspace exceeds the array is rejected before any device work.
"""
import numpy as np
import pytest

from oracle import oracle as O
from paper_2011_08373_amd import synth

pytestmark = pytest.mark.gpu

KEYS = ("status", "assign", "weight", "added", "removed", "rounds", "n_clauses", "trajectory")


@pytest.fixture(scope="module")
def L():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    from paper_2011_08373_amd import librepair
    return librepair


def _same(a, b):
    return {k: a[k] for k in KEYS} == {k: b[k] for k in KEYS}


def _near_limit(L, kms, lo_frac):
    """The largest kernel whose repair workspace lies in [lo_frac, 1] x the
    fixed array."""
    cap = L.noalloc_scratch_bytes()
    best = None
    for k in kms:
        w = L.workspace_bytes(k, L.OP_REPAIR)
        if lo_frac * cap <= w <= cap and (best is None or w > best[0]):
            best = (w, k)
    assert best is not None
    return best[1]


def test_two_calls_second_smaller(L):
    kms = synth.generate_batch(mode="planted")
    big = _near_limit(L, kms, 0.5)
    small = synth.generate("plain-small", mode="planted", seed=7)
    assert L.workspace_bytes(small, L.OP_REPAIR) < L.workspace_bytes(big, L.OP_REPAIR)
    for km in (big, small):
        g = L.repair_noalloc(km)
        r = L.repair(km)
        assert g["ret"] == r["ret"]
        assert _same(g, r), (g, r)
    o = O.repair(small)
    assert _same(L.repair_noalloc(small), o)


def test_policies_and_options(L):
    for seed in range(12):
        km = synth.generate("plain-small", mode="planted" if seed % 2 else "literal", seed=seed)
        for kw in (dict(), dict(policy=1), dict(solver=1), dict(grid=0, inspect=0),
                   dict(policy=1, solver=1, max_rounds=2)):
            g = L.repair_noalloc(km, **kw)
            r = L.repair(km, **kw)
            assert g["ret"] == r["ret"] and _same(g, r), (seed, kw)


def test_batched_kernels_in_a_row(L):
    # kernels of the batched workload that fit the array, largest first,
    # each checked against the workspace entry point
    kms = synth.generate_batch(mode="planted")
    cap = L.noalloc_scratch_bytes()
    fit = [k for k in kms if L.workspace_bytes(k, L.OP_REPAIR) <= cap]
    fit.sort(key=lambda k: -L.workspace_bytes(k, L.OP_REPAIR))
    rng = np.random.default_rng(5)
    pick = fit[:4] + [fit[int(q)] for q in rng.integers(4, len(fit), size=12)]
    for km in pick:
        g = L.repair_noalloc(km)
        r = L.repair(km)
        assert g["ret"] == r["ret"] and _same(g, r)


def test_too_large_is_rejected(L):
    km = synth.generate("plain-large", mode="planted")
    assert L.workspace_bytes(km, L.OP_REPAIR) > L.noalloc_scratch_bytes()
    g = L.repair_noalloc(km)
    assert g["ret"] == L.ERR_WORKSPACE
    # the array is still usable afterwards
    small = synth.generate("plain-small", mode="planted", seed=3)
    assert _same(L.repair_noalloc(small), L.repair(small))
