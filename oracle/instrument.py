"""Instrumentation pass of Section 2.2, written plainly (TEST INFRASTRUCTURE ONLY).

Only tests/, the smoke entry point and the benchmark's CPU-baseline leg may
import this module.  It shares no code with the HIP library's pass.

The paper's rules, as this model takes them:
  * the instrumentation adds a barrier guarded by a fresh Boolean barrier
    variable before every read or write of a shared variable, and before a
    call of a function that touches one;
  * it also adds them at scope boundaries -- the entry point of a branch
    statement and the head of a loop -- so that a barrier can be enabled
    where it causes no barrier divergence (the example kernel's solution is
    the barrier before the branch, not the ones beside the accesses);
  * with grid-level instrumentation enabled every such place also gets a
    grid-level barrier variable (the example kernel's b4..b6 after b1..b3);
  * pre-existing barriers are guarded by barrier variables too, so that the
    repair may remove them;
  * weights (Section 2.4): gw*gb + lw^ld.
A branch condition has a thread part and a block part (each tid or bid
mod m == r); nested branches meet part by part.
Sites go into the kernel body only (the example kernel has none inside the
called function).  Loops are unrolled and calls inlined; a site's copies
share its variable.

The program format is the generator's ``Program`` (statement dicts, regions
closed by END); call chains longer than 64 functions are rejected.
``instrument`` returns (status, Kernel or None) with status 0 or -1
(malformed program, or a model beyond 64 slots / 4096 points).
"""
from __future__ import annotations

ACCESS_S, BARRIER_S, IF_S, LOOP_S, CALL_S, END_S = 0, 1, 2, 3, 4, 5
OK, ERR_INVALID = 0, -1
MAX_SLOTS, MAX_POINTS = 64, 4096


class Invalid(Exception):
    pass


def parse(stmts):
    """Statement list -> tree of nodes (kind, statement index, dict, children)."""
    root = []
    stack = [root]
    opened = []
    for idx, st in enumerate(stmts):
        k = st["kind"]
        if k in (ACCESS_S, BARRIER_S, CALL_S):
            stack[-1].append((k, idx, st, None))
        elif k in (IF_S, LOOP_S):
            node = (k, idx, st, [])
            stack[-1].append(node)
            stack.append(node[3])
            opened.append(idx)
        elif k == END_S:
            if not opened:
                raise Invalid("END without IF/LOOP")
            stack.pop()
            opened.pop()
        else:
            raise Invalid("unknown statement kind")
    if opened:
        raise Invalid("unclosed region")
    return root


def residue_meet(g1, g2):
    """The threads with tid % m1 == r1 and tid % m2 == r2, as (m, r), found by
    trying every residue below lcm(m1, m2); None when no thread qualifies."""
    (m1, r1), (m2, r2) = g1, g2
    a, b = m1, m2
    while b:
        a, b = b, a % b
    lcm = m1 // a * m2
    if lcm >= 1 << 32:
        return None
    for t in range(lcm):
        if t % m1 == r1 and t % m2 == r2:
            return (lcm, t)
    return None


def instrument(prog, grid: int = 1, gw: int = 12, lw: int = 10):
    try:
        return OK, _instrument(prog, grid, gw, lw)
    except Invalid:
        return ERR_INVALID, None


def _instrument(prog, grid, gw, lw):
    from paper_2011_08373_amd import synth   # the input format only
    if prog.blocks < 1 or prog.threads < 1 or not prog.functions:
        raise Invalid("empty program")
    if grid not in (0, 1) or lw < 1:
        raise Invalid("options")
    for w, sp in prog.arrays:
        if w < 1 or sp not in (0, 1):
            raise Invalid("array")
    bguards = prog.block_guards if getattr(prog, "block_guards", None) is not None \
        else [(1, 0)] * len(prog.guards)
    if len(bguards) != len(prog.guards):
        raise Invalid("block conditions")
    for m, r in list(prog.guards) + list(bguards):
        if m < 1 or not 0 <= r < m:
            raise Invalid("guard")
    F = len(prog.functions)
    trees = [parse(f) for f in prog.functions]
    for f in range(F):
        for st in prog.functions[f]:
            if st["kind"] == ACCESS_S and (st["array"] >= len(prog.arrays) or st["is_write"] not in (0, 1)):
                raise Invalid("access")
            if st["kind"] == BARRIER_S and st["level"] not in (0, 1):
                raise Invalid("barrier level")
            if st["kind"] == IF_S and st["guard"] >= len(prog.guards):
                raise Invalid("branch guard")
            if st["kind"] == LOOP_S and st["count"] < 1:
                raise Invalid("trip count")
            if st["kind"] == CALL_S and not 1 <= st["count"] < F:
                raise Invalid("callee")

    # which functions touch an array, directly or through calls; recursion is
    # rejected (every function is checked, called or not)
    memo = {}

    def touches(f, active):
        if f in active:
            raise Invalid("recursion")
        if f in memo:
            return memo[f]
        if len(active) >= 64:
            raise Invalid("call chain longer than 64")
        active = active | {f}
        hit = False
        for st in prog.functions[f]:
            if st["kind"] == ACCESS_S:
                hit = True
            elif st["kind"] == CALL_S and touches(st["count"], active):
                hit = True
        memo[f] = hit
        return hit

    for f in range(F):
        touches(f, frozenset())

    # a condition is a pair: (thread residue class, block residue class)
    guards = [((1, 0), (1, 0))]
    points = []
    slots = []
    slot_ids = {}

    def guard_index(g):
        if g not in guards:
            guards.append(g)
        return guards.index(g)

    def weight(level, depth):
        w = (gw if level == 1 else 0) + lw ** depth
        if w < 1 or w >= 1 << 32:
            raise Invalid("weight")
        return w

    def emit_barrier(key, level, pre, g, depth):
        if key not in slot_ids:
            slot_ids[key] = len(slots)
            slots.append((level, pre, weight(level, depth)))
        points.append(dict(kind=synth.BARRIER, guard=guard_index(g), slot=slot_ids[key]))

    def emit_site(path, f, idx, g, depth):
        emit_barrier((path, f, idx, "block"), 0, 0, g, depth)
        if grid:
            emit_barrier((path, f, idx, "grid"), 1, 0, g, depth)

    def check_size():
        if len(points) > MAX_POINTS or len(slots) > MAX_SLOTS:
            raise Invalid("model too large")

    def run(nodes, f, path, g, depth, it):
        for kind, idx, st, body in nodes:
            check_size()
            if kind == ACCESS_S:
                if f == 0:
                    emit_site(path, f, idx, g, depth)
                c = st["c"] + st["d"] * it
                if not -(1 << 31) <= c < (1 << 31):
                    raise Invalid("word offset")
                points.append(dict(kind=synth.ACCESS, is_write=st["is_write"], array=st["array"],
                                   guard=guard_index(g), a=st["a"], b=st["b"], c=c))
            elif kind == BARRIER_S:
                emit_barrier((path, f, idx, "pre"), st["level"], 1, g, depth)
            elif kind == IF_S:
                if f == 0:
                    emit_site(path, f, idx, g, depth)
                inner_t = residue_meet(g[0], tuple(prog.guards[st["guard"]]))
                inner_b = residue_meet(g[1], tuple(bguards[st["guard"]]))
                if inner_t is None or inner_b is None:
                    raise Invalid("no thread takes the branch")
                run(body, f, path, (inner_t, inner_b), depth, it)
            elif kind == LOOP_S:
                for i in range(st["count"]):
                    if f == 0:
                        emit_site(path, f, idx, g, depth + 1)
                    run(body, f, path, g, depth + 1, i)
                    check_size()
            elif kind == CALL_S:
                callee = st["count"]
                if f == 0 and memo[callee]:
                    emit_site(path, f, idx, g, depth)
                run(trees[callee], callee, path + ((f, idx),), g, depth, it)
        check_size()

    run(trees[0], 0, (), ((1, 0), (1, 0)), 0, 0)
    block_part = [b for _, b in guards]
    return synth.make_kernel(prog.blocks, prog.threads, prog.arrays, [t for t, _ in guards],
                             points, slots, dict(prog.meta, instrumented=True, grid=grid),
                             block_part if any(m > 1 for m, _ in block_part) else None)
