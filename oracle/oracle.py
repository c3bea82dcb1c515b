"""ctypes wrapper of the CPU oracle (TEST INFRASTRUCTURE ONLY).

Only tests/, the smoke entry point and the benchmark's CPU-baseline leg may
import this module.  It shares no code with the HIP library: it reads a
kernel model by field name (the generator's plain numpy arrays) and copies it
into the oracle's own C structs.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")

OK, UNSAT, ERR_INVALID, ERR_CAPACITY, ERR_ROUNDS = 0, 1, -1, -2, -5


def build(force: bool = False) -> str:
    """Compile the oracle with the host compiler (no GPU code involved)."""
    src = os.path.join(HERE, "oracle.cpp")
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < max(
            os.path.getmtime(src), os.path.getmtime(os.path.join(HERE, "oracle.h"))):
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-shared", "-fPIC",
                               "-Wall", "-pthread", "-o", tmp, src])
        os.replace(tmp, LIB)
    return LIB


class _Array(C.Structure):
    _fields_ = [("words", C.c_uint32), ("space", C.c_uint8)]


class _Guard(C.Structure):
    _fields_ = [("m", C.c_uint32), ("r", C.c_uint32)]


class _Point(C.Structure):
    _fields_ = [("kind", C.c_uint8), ("is_write", C.c_uint8), ("array", C.c_uint16),
                ("guard", C.c_uint16), ("slot", C.c_uint16), ("a", C.c_int32),
                ("b", C.c_int32), ("c", C.c_int32)]


class _Slot(C.Structure):
    _fields_ = [("level", C.c_uint8), ("preexisting", C.c_uint8), ("weight", C.c_uint32)]


class _Kernel(C.Structure):
    _fields_ = [("blocks", C.c_uint32), ("threads", C.c_uint32), ("n_arrays", C.c_uint32),
                ("n_guards", C.c_uint32), ("n_points", C.c_uint32), ("n_slots", C.c_uint32),
                ("arrays", C.POINTER(_Array)), ("guards", C.POINTER(_Guard)),
                ("points", C.POINTER(_Point)), ("slots", C.POINTER(_Slot)),
                ("block_guards", C.POINTER(_Guard))]


class Clause(C.Structure):
    _fields_ = [("pos", C.c_uint64), ("neg", C.c_uint64)]


class _Pair(C.Structure):
    _fields_ = [("i", C.c_uint16), ("j", C.c_uint16), ("level", C.c_uint8), ("pad", C.c_uint8)]


class _Opts(C.Structure):
    _fields_ = [("policy", C.c_uint8), ("grid", C.c_uint8), ("inspect", C.c_uint8),
                ("solver", C.c_uint8), ("max_rounds", C.c_uint32)]


class _Result(C.Structure):
    _fields_ = [("status", C.c_int32), ("rounds", C.c_uint32), ("n_clauses", C.c_uint32),
                ("pad", C.c_uint32), ("assign", C.c_uint64), ("weight", C.c_uint64),
                ("added", C.c_uint64), ("removed", C.c_uint64)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        build()
        L = C.CDLL(LIB)
        K = C.POINTER(_Kernel)
        u64p = C.POINTER(C.c_uint64)
        L.or_validate.argtypes = [K]
        L.or_check.argtypes = [K, C.c_uint64, C.c_int, C.POINTER(_Pair), C.c_uint64,
                               u64p, u64p, u64p]
        L.or_pair_conflict.argtypes = [K, C.c_uint32, C.c_uint32, C.c_int]
        L.or_clauses.argtypes = [K, C.c_uint64, C.POINTER(Clause), C.c_uint64, u64p]
        L.or_full_clauses.argtypes = [K, C.POINTER(Clause), C.c_uint64, u64p]
        L.or_reduce.argtypes = [C.POINTER(Clause), C.c_uint64]
        L.or_reduce.restype = C.c_uint64
        L.or_min_barriers.argtypes = [C.POINTER(Clause), C.c_uint64, C.POINTER(C.c_uint32),
                                      C.c_uint32, C.c_int, u64p, u64p]
        L.or_repair.argtypes = [K, C.POINTER(_Opts), C.POINTER(_Result), u64p, C.c_uint32]
        L.or_greedy_mhs.argtypes = [C.POINTER(Clause), C.c_uint64, C.POINTER(C.c_uint32),
                                    C.c_uint32, u64p]
        L.or_safe_literal.argtypes = [K, C.c_uint64]
        L.or_set_route.argtypes = [C.c_int, C.c_int, C.c_uint64]
        _lib = L
    return _lib


class _Held:
    """Keeps the C copies of one kernel model alive."""

    def __init__(self, km):
        arrs = km.arrays
        self.arrays = (_Array * max(1, len(arrs)))()
        for n in range(len(arrs)):
            self.arrays[n].words = int(arrs["words"][n])
            self.arrays[n].space = int(arrs["space"][n])
        g = km.guards
        self.guards = (_Guard * max(1, len(g)))()
        for n in range(len(g)):
            self.guards[n].m = int(g["m"][n])
            self.guards[n].r = int(g["r"][n])
        p = km.points
        self.points = (_Point * max(1, len(p)))()
        cols = {f: p[f].tolist() for f in ("kind", "is_write", "array", "guard", "slot",
                                            "a", "b", "c")}
        for n in range(len(p)):
            q = self.points[n]
            q.kind, q.is_write, q.array = cols["kind"][n], cols["is_write"][n], cols["array"][n]
            q.guard, q.slot = cols["guard"][n], cols["slot"][n]
            q.a, q.b, q.c = cols["a"][n], cols["b"][n], cols["c"][n]
        s = km.slots
        self.slots = (_Slot * max(1, len(s)))()
        for n in range(len(s)):
            self.slots[n].level = int(s["level"][n])
            self.slots[n].preexisting = int(s["preexisting"][n])
            self.slots[n].weight = int(s["weight"][n])
        bg = getattr(km, "block_guards", None)
        self.block_guards = None
        if bg is not None:
            self.block_guards = (_Guard * max(1, len(bg)))()
            for n in range(len(bg)):
                self.block_guards[n].m = int(bg["m"][n])
                self.block_guards[n].r = int(bg["r"][n])
        self.k = _Kernel(int(km.blocks), int(km.threads), len(arrs), len(g), len(p), len(s),
                         self.arrays, self.guards, self.points, self.slots,
                         self.block_guards)

    @property
    def ptr(self):
        return C.byref(self.k)


def set_route(route: int, threads: int = 0, part_records: int = 0) -> int:
    """Location-grouped checker route: 0 whole kernel at once, 1 one array
    instance at a time on `threads` host threads (0: every core), cross-block
    parts of about `part_records` records (0: 2^25).  Returns the previous
    route."""
    return lib().or_set_route(int(route), int(threads), int(part_records))


def validate(km) -> int:
    return lib().or_validate(_Held(km).ptr)


def check(km, x: int = 0, literal: bool = False):
    """Races and divergence under x.

    Returns (status, pairs, divergent_mask, n_records); pairs is a list of
    (level, i, j) in ascending order.
    """
    h = _Held(km)
    n = C.c_uint64(0)
    div = C.c_uint64(0)
    nrec = C.c_uint64(0)
    st = lib().or_check(h.ptr, x, int(literal), None, 0, C.byref(n), C.byref(div),
                        C.byref(nrec))
    if st not in (OK, ERR_CAPACITY):
        return st, [], 0, 0
    buf = (_Pair * max(1, n.value))()
    st = lib().or_check(h.ptr, x, int(literal), buf, n.value, C.byref(n), C.byref(div),
                        C.byref(nrec))
    pairs = [(buf[q].level, buf[q].i, buf[q].j) for q in range(n.value)]
    return st, pairs, div.value, nrec.value


def pair_conflict(km, i: int, j: int, level: int) -> int:
    return lib().or_pair_conflict(_Held(km).ptr, i, j, level)


def _clauses_call(fn, h, *args):
    n = C.c_uint64(0)
    st = fn(h.ptr, *args, None, 0, C.byref(n))
    if st not in (OK, ERR_CAPACITY):
        return st, []
    buf = (Clause * max(1, n.value))()
    st = fn(h.ptr, *args, buf, n.value, C.byref(n))
    return st, [(buf[q].pos, buf[q].neg) for q in range(n.value)]


def clauses(km, x: int = 0):
    """(status, [(pos, neg), ...]) reduced and sorted."""
    return _clauses_call(lib().or_clauses, _Held(km), C.c_uint64(x))


def full_clauses(km):
    return _clauses_call(lib().or_full_clauses, _Held(km))


def reduce(cl):
    buf = (Clause * max(1, len(cl)))()
    for q, (p, n) in enumerate(cl):
        buf[q].pos, buf[q].neg = p, n
    m = lib().or_reduce(buf, len(cl))
    return [(buf[q].pos, buf[q].neg) for q in range(m)]


def min_barriers(cl, weights, n_slots: int, method: int = 0):
    """(status, assign, weight)."""
    buf = (Clause * max(1, len(cl)))()
    for q, (p, n) in enumerate(cl):
        buf[q].pos, buf[q].neg = int(p), int(n)
    w = (C.c_uint32 * max(1, n_slots))(*[int(v) for v in weights[:n_slots]])
    a = C.c_uint64(0)
    wt = C.c_uint64(0)
    st = lib().or_min_barriers(buf, len(cl), w, n_slots, method, C.byref(a), C.byref(wt))
    return st, a.value, wt.value


def repair(km, policy: int = 0, grid: int = 1, inspect: int = 1, max_rounds: int = 0,
           solver: int = 0):
    """Alg. 1; returns a dict with status, assign, weight, added, removed,
    rounds, n_clauses and the trajectory of assignments.  solver 0: exact
    Solve every round; 1: greedy minimal hitting set (Section 2.4)."""
    h = _Held(km)
    o = _Opts(policy, grid, inspect, solver, max_rounds)
    r = _Result()
    cap = 4096
    traj = (C.c_uint64 * cap)()
    st = lib().or_repair(h.ptr, C.byref(o), C.byref(r), traj, cap)
    out = dict(status=r.status, assign=r.assign, weight=r.weight, added=r.added,
               removed=r.removed, rounds=r.rounds, n_clauses=r.n_clauses)
    out["trajectory"] = [traj[q] for q in range(min(r.rounds, cap))]
    out["ret"] = st
    return out


def greedy_mhs(cl, weights, n_slots: int):
    """(status, assign) of the greedy minimal hitting set of the positive clauses."""
    buf = (Clause * max(1, len(cl)))()
    for q, (p, n) in enumerate(cl):
        buf[q].pos, buf[q].neg = int(p), int(n)
    w = (C.c_uint32 * max(1, n_slots))(*[int(v) for v in weights[:n_slots]])
    a = C.c_uint64(0)
    st = lib().or_greedy_mhs(buf, len(cl), w, n_slots, C.byref(a))
    return st, a.value


def safe_literal(km, x: int) -> int:
    return lib().or_safe_literal(_Held(km).ptr, x)


def kernel_arrays_copy(km):
    """Plain copy of the model's numpy arrays (for mutation in tests)."""
    return {k: np.array(getattr(km, k)) for k in ("arrays", "guards", "points", "slots")}
