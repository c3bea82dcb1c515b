"""Pins of the oracle's mhs strategy (Section 2.4): the greedy minimal hitting
set of the positive clauses, the exact fallback when it breaks a negative
clause, and the final exact query that makes the repaired set minimum."""
import itertools

import numpy as np
import pytest

import bruteforce as BF
from golden_util import kernel_from_json, load
from oracle import oracle as O
from paper_2011_08373_amd import synth


def test_greedy_paper_example_breaks_negative_clause():
    # Section 2.4: mhs of the positive clauses is {b1, b2}, which the clause
    # (not b1 or not b2) forbids; the exact answer needs three barriers.
    case = load("solver_examples")["cases"][0]
    st, x = O.greedy_mhs(case["clauses"], case["weights"], case["n_slots"])
    assert st == 0 and x == 0b11
    assert not all((x & p) or (~x & n) for p, n in case["clauses"])
    st, a, w = O.min_barriers(case["clauses"], case["weights"], case["n_slots"])
    assert (a, w) == (0b001110, 3)


def test_greedy_two_literal_clause_takes_lower_slot():
    # Appendix A.1's clause (a or b): both answers hit it; ties go to the lower slot
    assert O.greedy_mhs([(0b11, 0)], [1, 1], 2) == (0, 0b01)


def test_greedy_weighted_ratio():
    # one clause per unit weight: b (1/1) beats a (1/3)
    assert O.greedy_mhs([(0b11, 0)], [3, 1], 2) == (0, 0b10)
    # s0 hits two clauses at weight 3 (2/3), s1 and s2 one each at weight 1
    assert O.greedy_mhs([(0b011, 0), (0b101, 0)], [3, 1, 1], 3) == (0, 0b110)


def test_greedy_minimality_pass_drops_first_pick():
    # s0 hits four clauses and is taken first; s1 and s2 are then needed for
    # the clauses only they hit, after which s0 is redundant and dropped
    cl = [(0b011, 0), (0b011, 0), (0b101, 0), (0b101, 0), (0b010, 0), (0b100, 0)]
    assert O.greedy_mhs(cl, [1, 1, 1], 3) == (0, 0b110)


def test_greedy_empty_clause_is_unsat():
    assert O.greedy_mhs([(0b1, 0), (0, 0)], [1], 1)[0] == 1


def test_greedy_ignores_negative_clauses():
    assert O.greedy_mhs([(0, 0b1), (0, 0b10)], [1, 1], 2) == (0, 0)


def _brute_min_weight(cl, w, S):
    best = None
    for x in range(1 << S):
        if all(x & p for p, n in cl if n == 0):
            W = sum(w[s] for s in range(S) if (x >> s) & 1)
            best = W if best is None else min(best, W)
    return best


def test_greedy_is_a_minimal_hitting_set_random():
    rng = np.random.default_rng(21)
    for _ in range(400):
        S = int(rng.integers(1, 9))
        w = [int(v) for v in rng.integers(1, 5, S)]
        cl = [(int(rng.integers(1, 1 << S)), 0) for _ in range(int(rng.integers(1, 8)))]
        st, x = O.greedy_mhs(cl, w, S)
        assert st == 0
        assert all(x & p for p, _ in cl)                     # hits every clause
        for s in range(S):                                    # and is minimal
            if (x >> s) & 1:
                assert not all((x & ~(1 << s)) & p for p, _ in cl)
        W = sum(w[s] for s in range(S) if (x >> s) & 1)
        assert W >= _brute_min_weight(cl, w, S)               # never beats the optimum


def test_final_exact_query_changes_the_greedy_answer():
    fx = load("mhs_final_query")
    km = kernel_from_json(fx)
    for key, solver in (("repair", 0), ("repair_mhs", 1)):
        exp = fx["expect"][key]
        r = O.repair(km, solver=solver)
        for k in ("status", "assign", "weight", "rounds", "added", "removed", "trajectory"):
            assert r[k] == exp[k], (key, k)
    # the greedy's safe answer is verified, then replaced by the optimum
    assert O.safe_literal(km, 0b101) == 1 and O.safe_literal(km, 0b010) == 1


@pytest.mark.parametrize("mode", ["literal", "planted"])
def test_mhs_result_equals_exact_plain_small(mode):
    # Lemma: the loop stops at a safe x that is the optimum of every clause
    # learned so far, so the learning route cannot change the result
    for seed in range(200):
        km = synth.generate("plain-small", mode=mode, seed=seed)
        a, b = O.repair(km), O.repair(km, solver=1)
        assert (a["status"], a["assign"], a["weight"]) == (b["status"], b["assign"], b["weight"])


def test_mhs_result_equals_brute_force_tiny():
    rng = np.random.default_rng(23)
    for t in range(300):
        km = BF.tiny_kernel(rng, bias=bool(t % 2))
        for policy in (0, 1):
            r = O.repair(km, policy=policy, solver=1)
            best = BF.best_safe(km)
            if best is None:
                assert r["status"] == 1
            else:
                assert r["status"] == 0 and r["assign"] == best


def test_mhs_options_and_round_limit():
    fx = load("mhs_final_query")
    km = kernel_from_json(fx)
    r = O.repair(km, solver=1, max_rounds=2)
    assert r["status"] == -5 and r["rounds"] == 2
    r = O.repair(km, solver=1, max_rounds=3)
    assert r["status"] == 0 and r["rounds"] == 3
