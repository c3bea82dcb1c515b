"""Seeded synthetic kernel models for the barrier-repair path.

This module only *builds inputs*: it draws kernel models (arrays, guards,
program points, barrier slots, weights) from seeded distributions.  It holds
none of the repair method's arithmetic (no addresses, intervals, races,
clauses or solving), so the CPU oracle and the HIP library can both consume
its output without sharing any method code.

Model (the instrumented program P of the repair algorithm, Section 2.3):
  * ``blocks`` x ``threads`` threads; arrays are SHARED (one instance per
    block) or GLOBAL (one instance);
  * points 0..P-1 in post-unroll program order; a point is an ACCESS
    (read/write of ``array`` at (a*tid + b*bid + c) mod words), a BARRIER
    occurrence of a slot (a barrier variable b_s of Section 2.2/2.3), or NOP;
  * every ACCESS/BARRIER carries a guard (m, r): executed by threads with
    tid mod m == r (thread-parity style branches, Listing 2);
  * slots are numbered by first occurrence; slot weights follow either the
    paper's formula gw*gb + lw^ld (Section 2.4; defaults gw=12, lw=10 from
    Section 4.1) or the multiplicative rule of the large synthetic configs.

Two modes:
  * ``literal``: the configs' distributions verbatim;
  * ``planted``: a hidden safe assignment x* is drawn first and accesses are
    built so that x* separates every conflict; every planted kernel is
    repairable with weight <= W(x*).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

ACCESS, BARRIER, NOP = 0, 1, 2
SHARED, GLOBAL = 0, 1
BLOCK, GRID = 0, 1

ARRAY_DT = np.dtype([("words", "<u4"), ("space", "u1")], align=True)
GUARD_DT = np.dtype([("m", "<u4"), ("r", "<u4")], align=True)
POINT_DT = np.dtype([("kind", "u1"), ("is_write", "u1"), ("array", "<u2"),
                     ("guard", "<u2"), ("slot", "<u2"), ("a", "<i4"),
                     ("b", "<i4"), ("c", "<i4")], align=True)
SLOT_DT = np.dtype([("level", "u1"), ("preexisting", "u1"), ("weight", "<u4")],
                   align=True)
assert ARRAY_DT.itemsize == 8 and GUARD_DT.itemsize == 8
assert POINT_DT.itemsize == 20 and SLOT_DT.itemsize == 8


@dataclass
class Kernel:
    """A kernel model; arrays are C-layout structured numpy arrays."""
    blocks: int
    threads: int
    arrays: np.ndarray
    guards: np.ndarray
    points: np.ndarray
    slots: np.ndarray
    meta: dict = field(default_factory=dict)
    block_guards: np.ndarray | None = None   # [n_guards] (m, r) on bid, or None

    @property
    def n_points(self) -> int:
        return int(self.points.shape[0])

    @property
    def n_slots(self) -> int:
        return int(self.slots.shape[0])

    @property
    def weights(self) -> np.ndarray:
        return np.ascontiguousarray(self.slots["weight"], dtype=np.uint32)

    def copy(self) -> "Kernel":
        return Kernel(self.blocks, self.threads, self.arrays.copy(),
                      self.guards.copy(), self.points.copy(), self.slots.copy(),
                      dict(self.meta),
                      None if self.block_guards is None else self.block_guards.copy())


def make_kernel(blocks, threads, arrays, guards, points, slots, meta=None,
                block_guards=None) -> Kernel:
    """Build a Kernel from plain Python lists.

    arrays: [(words, space)], guards: [(m, r)] on the thread id,
    block_guards: None or [(m, r)] on the block id, one per guard,
    points: [dict(kind=..., is_write=..., array=..., guard=..., slot=..., a=, b=, c=)],
    slots:  [(level, preexisting, weight)].
    """
    arr = np.zeros(len(arrays), ARRAY_DT)
    for n, (w, s) in enumerate(arrays):
        arr[n] = (w, s)
    gd = np.zeros(len(guards), GUARD_DT)
    for n, (m, r) in enumerate(guards):
        gd[n] = (m, r)
    pt = np.zeros(len(points), POINT_DT)
    for n, p in enumerate(points):
        pt[n] = (p.get("kind", ACCESS), p.get("is_write", 0), p.get("array", 0),
                 p.get("guard", 0), p.get("slot", 0), p.get("a", 0),
                 p.get("b", 0), p.get("c", 0))
    sl = np.zeros(len(slots), SLOT_DT)
    for n, (lv, pre, w) in enumerate(slots):
        sl[n] = (lv, pre, w)
    bg = None
    if block_guards is not None:
        bg = np.zeros(len(block_guards), GUARD_DT)
        for n, (m, r) in enumerate(block_guards):
            bg[n] = (m, r)
    return Kernel(int(blocks), int(threads), arr, gd, pt, sl, dict(meta or {}), bg)


# ---------------------------------------------------------------------------
# Weights (Section 2.4 formula; Section 4.1 defaults)
# ---------------------------------------------------------------------------

def paper_weight(level: int, loop_depth: int, gw: int = 12, lw: int = 10) -> int:
    """weight = gw*gb + lw^ld, gb = 1 for a grid-level barrier, ld = loop depth."""
    gb = 1 if level == GRID else 0
    return gw * gb + lw ** loop_depth


def baseline_weight(level: int, trip_count: int) -> int:
    """1 per block barrier, times the trip count inside a loop, times 10 for grid."""
    return (10 if level == GRID else 1) * max(1, trip_count)


# ---------------------------------------------------------------------------
# Configurations
# ---------------------------------------------------------------------------

def config(name: str) -> dict:
    """Generator parameters of the five synthetic workloads."""
    base2 = dict(write_frac=0.3, a_set=(-1, 0, 1, 2), b_set=(0, 256), c_rng=(-2, 2),
                 guard_frac=0.10, loop_frac=0.10, unroll=8, access_frac=1.0,
                 pre_frac=0.25, weight_mode="baseline")
    if name == "plain-small":
        return dict(blocks=1, threads=64, arrays=[(128, SHARED)], P=16, S=4, S_grid=0,
                    write_frac=0.4, a_set=(1, 2), b_set=(0,), c_rng=(-2, 2),
                    guard_frac=0.0, loop_frac=0.0, unroll=1, access_frac=1.0,
                    pre_frac=0.25, weight_mode="baseline", seed=0)
    if name == "plain-large":
        d = dict(base2)
        d.update(blocks=256, threads=256,
                 arrays=[(1 << 20, SHARED)] * 2 + [(1 << 20, GLOBAL)] * 2,
                 P=512, S=32, S_grid=8, seed=2)
        return d
    if name == "batched":
        d = dict(base2)
        d.update(arrays=[(1 << 20, SHARED)] * 2 + [(1 << 20, GLOBAL)] * 2,
                 n_kernels=1024, seed=3)
        return d
    if name == "stress":
        return dict(blocks=4096, threads=1024,
                    arrays=[(1 << 24, SHARED)] * 4 + [(1 << 24, GLOBAL)] * 4,
                    P=1024, S=64, S_grid=16, write_frac=0.25, a_set=(-1, 0, 1, 2),
                    b_set=(0, 256), c_rng=(-2, 2), guard_frac=0.15, loop_frac=0.10,
                    unroll=16, access_frac=0.5, pre_frac=0.25,
                    weight_mode="baseline", seed=5)
    raise KeyError(name)


# ---------------------------------------------------------------------------
# Program skeleton: regions, loops, guards, slot placement
# ---------------------------------------------------------------------------

def _skeleton(rng, P, S, S_grid, guard_frac, loop_frac, unroll, access_frac, pre_frac):
    """Draw regions and slot placement.

    Returns (stmts, seq, slot_static) where ``stmts`` are static statements
    (dict with region info) and ``seq`` the post-unroll list of
    (static statement index, iteration).
    """
    regions = []
    length = 0
    while length < P:
        rem = P - length
        guard = None
        if rng.random() < guard_frac:
            m = int(rng.choice((2, 4)))
            guard = (m, int(rng.integers(0, m)))
        if unroll > 1 and rng.random() < loop_frac:
            body = int(rng.integers(2, 9))
            if body * unroll <= rem:
                regions.append(dict(n=body, trip=unroll, guard=guard))
                length += body * unroll
                continue
        n = min(int(rng.integers(4, 17)), rem)
        regions.append(dict(n=n, trip=1, guard=guard))
        length += n
    stmts = []
    for rid, rg in enumerate(regions):
        for j in range(rg["n"]):
            stmts.append(dict(region=rid, trip=rg["trip"], guard=rg["guard"]))
    S = min(S, len(stmts) // 2 if len(stmts) >= 2 else len(stmts))
    slot_pos = sorted(rng.choice(len(stmts), size=S, replace=False).tolist()) if S else []
    for k in slot_pos:
        stmts[k]["slot"] = True
    S_grid = min(S_grid, S)
    grid_of = set(rng.choice(S, size=S_grid, replace=False).tolist()) if S_grid else set()
    for n, k in enumerate(slot_pos):
        stmts[k]["level"] = GRID if n in grid_of else BLOCK
        stmts[k]["pre"] = bool(rng.random() < pre_frac)
    seq = []
    start = 0
    for rg in regions:
        ids = list(range(start, start + rg["n"]))
        for it in range(rg["trip"]):
            seq.extend((k, it) for k in ids)
        start += rg["n"]
    n_barrier_post = sum(1 for k, _ in seq if stmts[k].get("slot"))
    n_other_post = len(seq) - n_barrier_post
    q = 1.0 if access_frac >= 1.0 else min(1.0, access_frac * P / max(1, n_other_post))
    for st in stmts:
        if not st.get("slot"):
            st["access"] = bool(rng.random() < q)
    return stmts, seq


def _weight(mode, level, trip):
    if mode == "paper":
        return paper_weight(level, 1 if trip > 1 else 0)
    return baseline_weight(level, trip)


def _assemble(blocks, threads, arrays, stmts, seq, weight_mode, fields, meta):
    """Unroll static statements into points, renumber slots by first occurrence."""
    guards = [(1, 0)]
    gidx = {(1, 0): 0}

    def guard_id(g):
        if g is None:
            return 0
        if g not in gidx:
            gidx[g] = len(guards)
            guards.append(g)
        return gidx[g]

    slot_id = {}
    slots = []
    points = []
    for k, _it in seq:
        st = stmts[k]
        g = guard_id(st["guard"])
        if st.get("slot"):
            if k not in slot_id:
                slot_id[k] = len(slots)
                slots.append((st["level"], 1 if st["pre"] else 0,
                              _weight(weight_mode, st["level"], st["trip"])))
            points.append(dict(kind=BARRIER, guard=g, slot=slot_id[k]))
        elif k in fields:
            f = fields[k]
            points.append(dict(kind=ACCESS, guard=g, **f))
        else:
            points.append(dict(kind=NOP, guard=g))
    meta = dict(meta)
    meta["static_slot_of"] = slot_id
    return make_kernel(blocks, threads, arrays, guards, points, slots, meta)


def literal_kernel(cfg: dict, rng) -> Kernel:
    """Kernel with the configuration's distributions taken verbatim."""
    stmts, seq = _skeleton(rng, cfg["P"], cfg["S"], cfg["S_grid"], cfg["guard_frac"],
                           cfg["loop_frac"], cfg["unroll"], cfg["access_frac"],
                           cfg["pre_frac"])
    fields = {}
    lo, hi = cfg["c_rng"]
    for k, st in enumerate(stmts):
        if st.get("slot") or not st.get("access"):
            continue
        fields[k] = dict(array=int(rng.integers(0, len(cfg["arrays"]))),
                         is_write=int(rng.random() < cfg["write_frac"]),
                         a=int(rng.choice(cfg["a_set"])), b=int(rng.choice(cfg["b_set"])),
                         c=int(rng.integers(lo, hi + 1)))
    return _assemble(cfg["blocks"], cfg["threads"], cfg["arrays"], stmts, seq,
                     cfg["weight_mode"], fields, dict(mode="literal"))


def _owned_patterns(cfg, space, words, rng):
    """(a, b) choices whose map (bid, tid) -> address is injective where it matters."""
    T, B = cfg["threads"], cfg["blocks"]
    out = []
    for a in cfg["a_set"]:
        if a in (1, -1) and T <= words:
            out.append(a)
        elif a == 2 and 2 * T <= words:
            out.append(a)
    if space == GLOBAL:
        out = [a for a in out if a in (1, -1)]
        bs = [b for b in cfg["b_set"] if (B == 1 or (b >= T and b * (B - 1) + T <= words))]
        if not bs and T * B <= words:
            bs = [T]
        if not bs:
            return []
        return [(a, b) for a in out for b in bs]
    return [(a, b) for a in out for b in cfg["b_set"]]


def planted_kernel(cfg: dict, rng) -> Kernel:
    """Kernel built around a hidden safe assignment x* (stored in meta['x_star']).

    x* enables each unguarded slot with probability 1/2.  Within each x*
    interval (block-level for SHARED arrays, grid-level for GLOBAL ones) an
    array is either read-only or owned by one address pattern that is
    injective over the threads that can meet at one instance.
    """
    stmts, seq = _skeleton(rng, cfg["P"], cfg["S"], cfg["S_grid"], cfg["guard_frac"],
                           cfg["loop_frac"], cfg["unroll"], cfg["access_frac"],
                           cfg["pre_frac"])
    on = {}
    for k, st in enumerate(stmts):
        if st.get("slot"):
            on[k] = (st["guard"] is None) and bool(rng.random() < 0.5)
    # interval ids of every post-unroll position (block level, grid level)
    ib = ig = 0
    pos_iv = []
    for k, _it in seq:
        st = stmts[k]
        if st.get("slot") and on[k]:
            ib += 1
            if st["level"] == GRID:
                ig += 1
        pos_iv.append((ib, ig))
    copies = {}
    for pos, (k, _it) in enumerate(seq):
        copies.setdefault(k, []).append(pos)
    arrays = cfg["arrays"]
    pats = [_owned_patterns(cfg, sp, w, rng) for (w, sp) in arrays]
    lo, hi = cfg["c_rng"]
    mode = {}          # (array, interval) -> ("ro",) | ("own", a, b, c)
    fields = {}
    for k, st in enumerate(stmts):
        if st.get("slot") or not st.get("access"):
            continue
        for arr in rng.permutation(len(arrays)).tolist():
            lvl = 1 if arrays[arr][1] == GLOBAL else 0
            ivs = sorted({pos_iv[p][lvl] for p in copies[k]})
            seen = [mode.get((arr, iv)) for iv in ivs]
            owns = {m[1:] for m in seen if m is not None and m[0] == "own"}
            if len(owns) > 1:
                continue
            if owns:
                a, b, c = next(iter(owns))
                has_ro = any(m is not None and m[0] == "ro" for m in seen)
                w = 0 if has_ro else int(rng.random() < cfg["write_frac"])
                for iv in ivs:
                    mode.setdefault((arr, iv), ("own", a, b, c))
                fields[k] = dict(array=arr, is_write=w, a=a, b=b, c=c)
                break
            if any(m is not None for m in seen) or not pats[arr] or rng.random() < 0.5:
                # read-only in every interval this statement touches
                for iv in ivs:
                    mode.setdefault((arr, iv), ("ro",))
                fields[k] = dict(array=arr, is_write=0, a=int(rng.choice(cfg["a_set"])),
                                 b=int(rng.choice(cfg["b_set"])),
                                 c=int(rng.integers(lo, hi + 1)))
                break
            a, b = pats[arr][int(rng.integers(0, len(pats[arr])))]
            c = int(rng.integers(lo, hi + 1))
            for iv in ivs:
                mode[(arr, iv)] = ("own", a, b, c)
            fields[k] = dict(array=arr, is_write=int(rng.random() < cfg["write_frac"]),
                             a=a, b=b, c=c)
            break
    kern = _assemble(cfg["blocks"], cfg["threads"], arrays, stmts, seq,
                     cfg["weight_mode"], fields, dict(mode="planted"))
    x_star = 0
    for k, sid in kern.meta["static_slot_of"].items():
        if on.get(k):
            x_star |= 1 << sid
    kern.meta["x_star"] = x_star
    return kern


def generate(name: str, mode: str = "literal", seed: int | None = None, **over) -> Kernel:
    """One kernel of a named configuration."""
    cfg = config(name)
    cfg.update(over)
    s = cfg["seed"] if seed is None else seed
    rng = np.random.default_rng(s)
    k = literal_kernel(cfg, rng) if mode == "literal" else planted_kernel(cfg, rng)
    k.meta.update(config=name, seed=s)
    return k


def max_points_kernel(seed: int = 15) -> Kernel:
    """A kernel at the point limit of the model (4,096 points), in planted
    mode with the large workload's distributions: 2 blocks x 64 threads,
    8 shared + 8 global arrays of 256 words, 64 slots (16 grid-level)."""
    k = generate("plain-large", mode="planted", seed=seed, P=4096, S=64, S_grid=16, blocks=2,
                 threads=64, arrays=[(256, SHARED)] * 8 + [(256, GLOBAL)] * 8)
    k.meta.update(config="max-points")
    return k


def batch_shape(rng):
    """Threads log-uniform in [64, 65536] (multiple of 64); points, slots uniform."""
    total = int(round(2.0 ** rng.uniform(6, 16) / 64.0)) * 64
    total = max(64, min(65536, total))
    T = min(256, total)
    total = max(T, (total // T) * T)
    B = total // T
    P = int(rng.integers(16, 1025))
    S = int(rng.integers(2, 41))
    return B, T, P, S, int(round(S / 4))


def generate_batch(n: int | None = None, mode: str = "literal", seed: int | None = None,
                   name: str = "batched") -> list:
    """Kernels of the batched configuration; kernel i uses SeedSequence(seed).spawn(n)[i]."""
    cfg = config(name)
    n = cfg["n_kernels"] if n is None else n
    s = cfg["seed"] if seed is None else seed
    out = []
    for i, child in enumerate(np.random.SeedSequence(s).spawn(n)):
        rng = np.random.default_rng(child)
        B, T, P, S, Sg = batch_shape(rng)
        c = dict(cfg)
        c.update(blocks=B, threads=T, P=P, S=S, S_grid=Sg)
        k = literal_kernel(c, rng) if mode == "literal" else planted_kernel(c, rng)
        k.meta.update(config=name, seed=s, index=i)
        out.append(k)
    return out


def with_block_conditions(km: Kernel, rng, frac: float = 0.4, moduli=(2, 3, 4)) -> Kernel:
    """A copy of ``km`` whose guards (all but guard 0) get, each with
    probability ``frac``, a condition bid % m == r on the block id as well."""
    out = km.copy()
    bg = np.zeros(len(km.guards), GUARD_DT)
    bg["m"] = 1
    for g in range(1, len(km.guards)):
        if rng.random() < frac:
            m = int(rng.choice(moduli))
            bg[g] = (m, int(rng.integers(0, m)))
    out.block_guards = bg
    return out


def poisson_arrivals(rate: float, duration: float, seed: int = 4) -> np.ndarray:
    """Arrival times (seconds) of a Poisson process of the given rate."""
    rng = np.random.default_rng(seed)
    n = int(rate * duration * 1.5) + 16
    t = np.cumsum(rng.exponential(1.0 / rate, size=n))
    return t[t < duration]


# ---------------------------------------------------------------------------
# Structured programs (the input of the instrumentation pass, Section 2.2)
# ---------------------------------------------------------------------------

S_ACCESS, S_BARRIER, S_IF, S_LOOP, S_CALL, S_END = 0, 1, 2, 3, 4, 5


@dataclass
class Program:
    """A structured kernel: ``functions[0]`` is the kernel body, the others
    are device functions.  A function is a list of statement dicts in which
    S_IF (``guard``: index into ``guards``) and S_LOOP (``count`` trips) open
    a region that S_END closes; S_ACCESS has ``array``, ``is_write``, ``a``,
    ``b``, ``c``, ``d``; S_BARRIER (pre-existing) has ``level``; S_CALL has
    ``count`` = callee index.  ``block_guards`` (None, or one (m, r) per
    guard) adds a condition on the block id to each guard."""
    blocks: int
    threads: int
    arrays: list
    guards: list
    functions: list
    meta: dict = field(default_factory=dict)
    block_guards: list | None = None


def st_access(array, is_write, a=1, b=0, c=0, d=0):
    return dict(kind=S_ACCESS, array=array, is_write=int(is_write), a=a, b=b, c=c, d=d)


def st_barrier(level=BLOCK):
    return dict(kind=S_BARRIER, level=level)


def st_if(guard):
    return dict(kind=S_IF, guard=guard)


def st_loop(count):
    return dict(kind=S_LOOP, count=count)


def st_call(callee):
    return dict(kind=S_CALL, count=callee)


def st_end():
    return dict(kind=S_END)


def random_program(rng, max_sites: int = 20, max_pre: int = 6) -> Program:
    """A small random structured kernel: nested branches (thread-parity
    conditions, and block-parity ones when there are several blocks),
    uniform loops with loop-variable address terms, calls of device
    functions and pre-existing barriers.  ``max_sites`` bounds the
    statements of the kernel body that take an instrumented barrier
    (accesses, branches, loops, calls); ``max_pre`` the pre-existing ones."""
    B = int(rng.choice([1, 2, 4]))
    T = int(rng.choice([32, 64, 128]))
    n_arr = int(rng.integers(1, 4))
    arrays = []
    for _ in range(n_arr):
        space = int(rng.integers(0, 2))
        words = T * (B if space == GLOBAL else 1) * int(rng.choice([1, 2]))
        arrays.append((words, space))
    guards = [(1, 0), (2, 0), (2, 1)]
    for m in (3, 4):
        guards.append((m, int(rng.integers(0, m))))
    # branches on the block id (thread part {1, 0}) when there are blocks
    bguards = [(1, 0)] * len(guards)
    if B > 1:
        for bm, br in ((2, 0), (2, 1), (B, 0)):
            guards.append((1, 0))
            bguards.append((bm, br))
    state = dict(sites=0, pre=0)

    def fits(g, outer):
        # some thread of some block takes both: each part is the enclosing
        # one again, or has a modulus coprime with it
        for pa, pb in ((guards[g], guards[outer]), (bguards[g], bguards[outer])):
            if pa != pb and math.gcd(pa[0], pb[0]) != 1:
                return False
        return True

    def access():
        arr = int(rng.integers(0, n_arr))
        w = bool(rng.random() < 0.4)
        a = int(rng.choice([1, 1, 1, -1, 2])) if w else int(rng.choice([1, 1, -1, 0, 2]))
        b = T if arrays[arr][1] == GLOBAL and (w or rng.random() < 0.7) else 0
        c = int(rng.integers(-2, 3))
        d = int(rng.choice([0, 0, 1, 2]))
        return st_access(arr, w, a, b, c, d)

    def pre_barrier():
        state["pre"] += 1
        lv = GRID if B > 1 and rng.random() < 0.25 else BLOCK
        return st_barrier(lv)

    n_dev = int(rng.integers(0, 3))
    functions = [None]
    for _ in range(n_dev):
        body = []
        for _ in range(int(rng.integers(1, 4))):
            r = rng.random()
            if r < 0.15 and state["pre"] < max_pre:
                body.append(pre_barrier())
            elif r < 0.3:
                body += [st_loop(int(rng.integers(2, 4))), access(), st_end()]
            else:
                body.append(access())
        functions.append(body)

    def block(depth, n, outer):
        out = []
        for _ in range(n):
            if state["sites"] >= max_sites:
                break
            r = rng.random()
            if r < 0.12 and state["pre"] < max_pre:
                out.append(pre_barrier())
                continue
            state["sites"] += 1
            if r < 0.24 and depth < 2:
                # nested conditions: the enclosing one again, or one whose
                # modulus is coprime with it, so some thread takes both
                cand = [g for g in range(len(guards)) if g == outer or fits(g, outer)]
                g = int(rng.choice(cand))
                out.append(st_if(g))
                out += block(depth + 1, int(rng.integers(1, 4)), g if g else outer)
                out.append(st_end())
            elif r < 0.34 and depth < 2:
                out.append(st_loop(int(rng.integers(2, 5))))
                out += block(depth + 1, int(rng.integers(1, 4)), outer)
                out.append(st_end())
            elif r < 0.44 and n_dev:
                out.append(st_call(int(rng.integers(1, n_dev + 1))))
            else:
                out.append(access())
        return out

    functions[0] = block(0, int(rng.integers(3, 9)), 0)
    return Program(B, T, arrays, guards, functions,
                   block_guards=bguards if B > 1 else None)


def generate_programs(n: int, seed: int = 11, **kw) -> list:
    """Programs of the instrumented workload; program i uses
    SeedSequence(seed).spawn(n)[i]."""
    out = []
    for i, child in enumerate(np.random.SeedSequence(seed).spawn(n)):
        p = random_program(np.random.default_rng(child), **kw)
        p.meta.update(seed=seed, index=i)
        out.append(p)
    return out
