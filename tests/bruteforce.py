"""Pure-Python brute force for tiny kernels (test helper, independent of the oracle).

Straight from the definitions: every pair of (point, block, thread) access
records, every assignment of the barrier variables.  Only usable for a few
hundred records and <= 8 slots.
"""
import numpy as np


def tiny_kernel(rng, max_points=10, max_slots=6, max_threads=8, max_blocks=2, bias=None,
                block_conds=False):
    """Random tiny kernel; ``bias`` favours repairable shapes (injective
    addresses, denser barriers) so the repair loop has work to do;
    ``block_conds`` gives guards a condition on the block id as well."""
    bias = bool(rng.random() < 0.5) if bias is None else bias
    from paper_2011_08373_amd import synth
    B = int(rng.integers(1, max_blocks + 1))
    T = int(rng.integers(1, max_threads + 1))
    lo_words = 2 * T * B if bias else 4
    arrays = [(int(rng.integers(lo_words, lo_words + 13)), int(rng.integers(0, 2)))
              for _ in range(int(rng.integers(1, 3)))]
    guards = [(1, 0)]
    for _ in range(int(rng.integers(0, 3))):
        m = int(rng.integers(2, 4))
        guards.append((m, int(rng.integers(0, m))))
    P = int(rng.integers(1, max_points + 1))
    S_max = int(rng.integers(0, max_slots + 1))
    points, slots, slot_guard = [], [], []
    for _ in range(P):
        u = rng.random()
        if u < (0.5 if bias else 0.35) and (len(slots) < S_max or slots):
            if len(slots) < S_max and (not slots or rng.random() < 0.7):
                g = int(rng.integers(0, len(guards)))
                slot_guard.append(g)
                slots.append((int(rng.integers(0, 2)), int(rng.integers(0, 2)),
                              int(rng.integers(1, 6))))
                points.append(dict(kind=1, slot=len(slots) - 1, guard=g))
            else:
                s = int(rng.integers(0, len(slots)))
                points.append(dict(kind=1, slot=s, guard=slot_guard[s]))
        elif u < 0.92:
            b_choices = [T] if bias else [-2, -1, 0, 1, 2, T]
            a_choices = [-1, 1, 2] if bias else [-2, -1, 0, 1, 2]
            points.append(dict(kind=0, is_write=int(rng.random() < 0.5),
                               array=int(rng.integers(0, len(arrays))),
                               guard=int(rng.integers(0, len(guards))),
                               a=int(a_choices[int(rng.integers(0, len(a_choices)))]),
                               b=int(b_choices[int(rng.integers(0, len(b_choices)))]),
                               c=int(rng.integers(-3, 4))))
        else:
            points.append(dict(kind=2))
    bg = None
    if block_conds:
        bg = []
        for _ in guards:
            if rng.random() < 0.5:
                m = int(rng.integers(2, 4))
                bg.append((m, int(rng.integers(0, m))))
            else:
                bg.append((1, 0))
    return synth.make_kernel(B, T, arrays, guards, points, slots, block_guards=bg)


def _runs(km, g, k, t):
    """Thread t of block k executes a point with guard g."""
    m, r = (int(v) for v in km.guards[g])
    if t % m != r:
        return False
    if km.block_guards is None:
        return True
    bm, br = (int(v) for v in km.block_guards[g])
    return k % bm == br


def _records(km):
    pts = km.points
    out = []
    for i in range(len(pts)):
        if int(pts["kind"][i]) != 0:
            continue
        m, r = (int(v) for v in km.guards[int(pts["guard"][i])])
        arr = int(pts["array"][i])
        n = int(km.arrays["words"][arr])
        a, b, c = int(pts["a"][i]), int(pts["b"][i]), int(pts["c"][i])
        for k in range(km.blocks):
            for t in range(km.threads):
                if _runs(km, int(pts["guard"][i]), k, t):
                    out.append((i, k, t, arr, (a * t + b * k + c) % n))
    return out


def conflicting_pairs(km):
    """{(level, i, j)} of point pairs with a conflicting record pair."""
    recs = _records(km)
    pts = km.points
    space = km.arrays["space"]
    out = set()
    for x in range(len(recs)):
        for y in range(x + 1, len(recs)):
            i, k, t, arr, ad = recs[x]
            j, k2, t2, arr2, ad2 = recs[y]
            if arr != arr2 or ad != ad2 or (k, t) == (k2, t2):
                continue
            if not (pts["is_write"][i] or pts["is_write"][j]):
                continue
            if k != k2 and int(space[arr]) != 1:
                continue
            out.add((0 if k == k2 else 1, min(i, j), max(i, j)))
    return out


def safe(km, x, conflicts=None):
    conflicts = conflicting_pairs(km) if conflicts is None else conflicts
    pts = km.points
    for lv, i, j in conflicts:
        sep = False
        for u in range(i + 1, j):
            if int(pts["kind"][u]) != 1:
                continue
            s = int(pts["slot"][u])
            if (x >> s) & 1 and (lv == 0 or int(km.slots["level"][s]) == 1):
                sep = True
                break
        if not sep:
            return False
    for u in range(len(pts)):
        if int(pts["kind"][u]) != 1 or not (x >> int(pts["slot"][u])) & 1:
            continue
        g = int(pts["guard"][u])
        per_block = [sum(1 for t in range(km.threads) if _runs(km, g, k, t))
                     for k in range(km.blocks)]
        if int(km.slots["level"][int(pts["slot"][u])]) == 1:
            # a grid barrier is reached by the whole grid or by nobody
            if 0 < sum(per_block) < km.blocks * km.threads:
                return False
        elif any(0 < n < km.threads for n in per_block):
            return False
    return True


def key(x, w):
    W = sum(int(w[s]) for s in range(len(w)) if (x >> s) & 1)
    return (W, bin(x).count("1"), x)


def best_safe(km):
    """Canonical minimum-key safe assignment by enumeration, or None."""
    conf = conflicting_pairs(km)
    w = [int(v) for v in km.slots["weight"]]
    best = None
    for x in range(1 << km.n_slots):
        if safe(km, x, conf) and (best is None or key(x, w) < key(best, w)):
            best = x
    return best


def best_clause_solution(clauses, w, S):
    best = None
    for x in range(1 << S):
        if all((x & p) or (~x & n) for p, n in clauses):
            if best is None or key(x, w) < key(best, w):
                best = x
    return best
