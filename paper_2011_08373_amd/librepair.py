"""ctypes binding of librepair.so (the C ABI declared in include/librepair.h).

Argument marshalling only: every step of the repair path runs in the HIP
library.  PyTorch provides the device workspace (``torch.empty`` on the
current CUDA/HIP device) and the stream handle.  Importing this module fails
loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "librepair.so")

OK, UNSAT = 0, 1
ERR_INVALID, ERR_CAPACITY, ERR_WORKSPACE, ERR_DEVICE, ERR_ROUNDS, ERR_BUDGET = -1, -2, -3, -4, -5, -6
ERR_SEARCH = -7
OP_CHECK, OP_CLAUSES, OP_REPAIR, OP_FIRST = 0, 1, 2, 4

if not os.path.exists(LIB_PATH):
    raise ImportError("librepair.so is not built (run paper_2011_08373_amd/build.py): %s"
                      % LIB_PATH)


class RpKernel(C.Structure):
    _fields_ = [("blocks", C.c_uint32), ("threads", C.c_uint32), ("n_arrays", C.c_uint32),
                ("n_guards", C.c_uint32), ("n_points", C.c_uint32), ("n_slots", C.c_uint32),
                ("arrays", C.c_void_p), ("guards", C.c_void_p), ("points", C.c_void_p),
                ("slots", C.c_void_p), ("block_guards", C.c_void_p)]


class RpClause(C.Structure):
    _fields_ = [("pos", C.c_uint64), ("neg", C.c_uint64)]


class RpOpts(C.Structure):
    _fields_ = [("policy", C.c_uint8), ("grid", C.c_uint8), ("inspect", C.c_uint8),
                ("solver", C.c_uint8), ("max_rounds", C.c_uint32)]


class RpOut(C.Structure):
    _fields_ = [("status", C.c_int32), ("rounds", C.c_uint32), ("n_clauses", C.c_uint32),
                ("pad", C.c_uint32), ("assign", C.c_uint64), ("weight", C.c_uint64),
                ("added", C.c_uint64), ("removed", C.c_uint64)]


class RpStats(C.Structure):
    _fields_ = [("ms_gen", C.c_double), ("ms_sort", C.c_double), ("ms_check", C.c_double),
                ("ms_clause", C.c_double), ("ms_solve", C.c_double), ("ms_total", C.c_double),
                ("ms_sort_pass_max", C.c_double), ("ms_sort_kernels", C.c_double),
                ("ms_j0", C.c_double),
                ("records", C.c_uint64),
                ("accesses", C.c_uint64), ("records_scanned", C.c_uint64),
                ("sort_passes", C.c_uint32), ("sort_launches", C.c_uint32),
                ("rounds", C.c_uint32), ("conf_launches", C.c_uint32),
                ("ms_upload", C.c_double), ("ms_conf_kernels", C.c_double)]


class RpFunction(C.Structure):
    _fields_ = [("n_stmts", C.c_uint32), ("stmts", C.c_void_p)]


class RpProgram(C.Structure):
    _fields_ = [("blocks", C.c_uint32), ("threads", C.c_uint32), ("n_arrays", C.c_uint32),
                ("n_guards", C.c_uint32), ("n_functions", C.c_uint32),
                ("arrays", C.c_void_p), ("guards", C.c_void_p), ("functions", C.c_void_p),
                ("block_guards", C.c_void_p)]


class RpInstrumentOpts(C.Structure):
    _fields_ = [("grid", C.c_uint8), ("pad", C.c_uint8 * 3), ("gw", C.c_uint32),
                ("lw", C.c_uint32)]


STMT_DT = np.dtype([("kind", "u1"), ("is_write", "u1"), ("level", "u1"), ("pad", "u1"),
                    ("array", "<u2"), ("guard", "<u2"), ("count", "<u4"), ("a", "<i4"),
                    ("b", "<i4"), ("c", "<i4"), ("d", "<i4")], align=True)
assert STMT_DT.itemsize == 28

PAIR_DT = np.dtype([("i", "<u2"), ("j", "<u2"), ("level", "u1"), ("pad", "u1")])
assert PAIR_DT.itemsize == 6

_L = C.CDLL(LIB_PATH)
_K = C.POINTER(RpKernel)
_u64p = C.POINTER(C.c_uint64)
_L.rp_status_string.restype = C.c_char_p
_L.rp_validate.argtypes = [_K]
_L.rp_workspace_bytes.argtypes = [_K, C.c_int]
_L.rp_workspace_bytes.restype = C.c_size_t
_L.rp_check.argtypes = [_K, C.c_uint64, C.c_void_p, C.c_uint64, _u64p, _u64p, _u64p,
                        C.c_void_p, C.c_size_t, C.c_void_p]
_L.rp_clauses.argtypes = [_K, C.c_uint64, C.c_void_p, C.c_uint64, _u64p, C.c_void_p,
                          C.c_size_t, C.c_void_p]
_L.rp_first_partners.argtypes = [_K, C.c_uint64, C.c_void_p, _u64p, C.c_void_p, C.c_size_t,
                                 C.c_void_p]
_L.rp_solve_workspace_bytes.argtypes = [C.c_uint64]
_L.rp_solve_workspace_bytes.restype = C.c_size_t
_L.rp_min_barriers.argtypes = [C.c_void_p, C.c_uint64, C.c_void_p, C.c_uint32, _u64p, _u64p,
                               C.c_void_p, C.c_size_t, C.c_void_p]
_L.rp_repair.argtypes = [_K, C.POINTER(RpOpts), C.POINTER(RpOut), C.c_void_p, C.c_uint32,
                         C.c_void_p, C.c_size_t, C.c_void_p]
_L.rp_noalloc_scratch_bytes.argtypes = []
_L.rp_noalloc_scratch_bytes.restype = C.c_size_t
_L.rp_repair_noalloc.argtypes = [_K, C.POINTER(RpOpts), C.POINTER(RpOut), C.c_void_p, C.c_uint32,
                                 C.c_void_p]
_L.rp_batch_workspace_bytes.argtypes = [C.POINTER(C.POINTER(RpKernel)), C.c_uint32]
_L.rp_batch_workspace_bytes.restype = C.c_size_t
_L.rp_repair_batch.argtypes = [C.POINTER(C.POINTER(RpKernel)), C.c_uint32, C.POINTER(RpOpts),
                               C.POINTER(RpOut), C.c_void_p, C.c_size_t, C.c_void_p]
_L.rp_server_tables_bytes.argtypes = [C.c_uint32]
_L.rp_server_tables_bytes.restype = C.c_size_t
_L.rp_server_job_bytes.argtypes = [_K]
_L.rp_server_job_bytes.restype = C.c_size_t
_L.rp_server_create.argtypes = [C.c_void_p, C.c_size_t, C.POINTER(RpOpts), C.c_uint32,
                                C.c_void_p, C.POINTER(C.c_void_p)]
_L.rp_server_submit.argtypes = [C.c_void_p, _K, C.c_uint64]
_L.rp_server_step.argtypes = [C.c_void_p, C.POINTER(C.c_uint32), C.POINTER(C.c_uint32)]
_L.rp_server_poll.argtypes = [C.c_void_p, C.POINTER(C.c_uint64), C.POINTER(RpOut),
                              C.POINTER(C.c_double), C.c_uint32, C.POINTER(C.c_uint32)]
_L.rp_server_destroy.argtypes = [C.c_void_p]
_L.rp_last_stats.argtypes = [C.POINTER(RpStats)]
_L.rp_last_stats.restype = None
_L.rp_set_sort_digit_bits.argtypes = [C.c_int]
_L.rp_set_tuning.argtypes = [C.c_int, C.c_int]
_L.rp_sort_key_bits.argtypes = [C.POINTER(C.POINTER(RpKernel)), C.c_uint32]
_L.rp_sort_key_bits.restype = C.c_uint32
_u32p = C.POINTER(C.c_uint32)
_L.rp_instrument.argtypes = [C.POINTER(RpProgram), C.POINTER(RpInstrumentOpts),
                             C.c_void_p, C.c_void_p, C.c_uint32, _u32p, C.c_void_p, C.c_uint32,
                             _u32p, C.c_void_p, C.c_uint32, _u32p]
TUNE_SORT_DIGIT_BITS, TUNE_SCATTER_SHAPE, TUNE_TIMING, TUNE_SCATTER_WGS = 0, 1, 2, 3
TUNE_SOLVER_NODES = 4
TUNE_SCAN_PIPELINE = 5
TUNE_DIGIT_ORDER = 6
TUNE_LOW_DIGIT_BITS = 7
TUNE_SCAN_FIELDS = 8
TUNE_PASS_SHAPES = 9
PASS_SHAPES_DEFAULT = 0x0FFFFFFF     # every radix pass on TUNE_SCATTER_SHAPE's tile


def pass_shapes_value(shapes) -> int:
    """TUNE_PASS_SHAPES value of a per-pass list of tile shapes (execution
    order; None or 15 = the TUNE_SCATTER_SHAPE tile)."""
    v = PASS_SHAPES_DEFAULT
    for p, sh in enumerate(list(shapes)[:7]):
        if sh is not None:
            v = (v & ~(15 << (4 * p))) | (int(sh) << (4 * p))
    return v


def lib():
    return _L


def status_string(st: int) -> str:
    return _L.rp_status_string(int(st)).decode()


class KernelArg:
    """C view of a kernel model; keeps the numpy buffers alive."""

    def __init__(self, km):
        from . import synth
        self.arrays = np.ascontiguousarray(km.arrays, dtype=synth.ARRAY_DT)
        self.guards = np.ascontiguousarray(km.guards, dtype=synth.GUARD_DT)
        self.points = np.ascontiguousarray(km.points, dtype=synth.POINT_DT)
        self.slots = np.ascontiguousarray(km.slots, dtype=synth.SLOT_DT)
        bg = getattr(km, "block_guards", None)
        self.block_guards = None if bg is None else np.ascontiguousarray(bg, dtype=synth.GUARD_DT)
        if self.block_guards is not None and len(self.block_guards) != len(self.guards):
            raise ValueError("block_guards needs one entry per guard")

        def ptr(a):
            return a.ctypes.data if a is not None and a.size else None

        self.k = RpKernel(int(km.blocks), int(km.threads), len(self.arrays), len(self.guards),
                          len(self.points), len(self.slots), ptr(self.arrays), ptr(self.guards),
                          ptr(self.points), ptr(self.slots), ptr(self.block_guards))

        self._need = {}

    @property
    def ref(self):
        return C.byref(self.k)

    def need(self, op: int) -> int:
        """Workspace bytes of op for this model (cached while the sort
        tuning, on which the size depends, is unchanged)."""
        key = (int(op), _tuning_epoch[0])
        if key not in self._need:
            self._need[key] = int(_L.rp_workspace_bytes(self.ref, int(op)))
        return self._need[key]


def _arg(km):
    """A kernel model or a KernelArg already built from one (callers that
    repeat calls on one model build it once)."""
    return km if isinstance(km, KernelArg) else KernelArg(km)


_tls = threading.local()


def _traj(cap: int):
    """Trajectory output buffer, one per thread and capacity."""
    cap = max(1, int(cap))
    bufs = getattr(_tls, "traj", None)
    if bufs is None:
        bufs = _tls.traj = {}
    if cap not in bufs:
        bufs[cap] = (C.c_uint64 * cap)()
    return bufs[cap]


class Workspace:
    """A reusable device workspace (a torch uint8 tensor)."""

    def __init__(self):
        self.t = None

    def get(self, nbytes: int):
        import torch
        if self.t is None or self.t.numel() < nbytes:
            self.t = None
            torch.cuda.empty_cache()
            self.t = torch.empty(max(1, int(nbytes)), dtype=torch.uint8, device="cuda")
        return self.t.data_ptr(), self.t.numel()


_ws = Workspace()


def _stream(stream=None):
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


def validate(km) -> int:
    return _L.rp_validate(_arg(km).ref)


def workspace_bytes(km, op: int) -> int:
    return _arg(km).need(op)


def check(km, x: int = 0, cap: int | None = None, ws=None, stream=None):
    """Verify under x.  Returns (status, pairs, divergent, n_records, n_pairs)
    with pairs a list of (level, i, j) in ascending order (empty unless OK)."""
    ka = _arg(km)
    need = int(_L.rp_workspace_bytes(ka.ref, OP_CHECK))
    if need == 0:
        return ERR_INVALID, [], 0, 0, 0
    ptr, size = (ws or _ws).get(need)
    P = int(km.n_points)
    cap = P * (P + 1) if cap is None else int(cap)
    buf = np.zeros(max(1, cap), PAIR_DT)
    n = C.c_uint64(0)
    div = C.c_uint64(0)
    nrec = C.c_uint64(0)
    st = _L.rp_check(ka.ref, C.c_uint64(int(x)), buf.ctypes.data if cap else None, cap,
                     C.byref(n), C.byref(div), C.byref(nrec), C.c_void_p(ptr), size,
                     _stream(stream))
    if st != OK:
        return st, [], div.value, nrec.value, n.value
    b = buf[:n.value]
    pairs = list(zip(b["level"].tolist(), b["i"].tolist(), b["j"].tolist()))
    return st, pairs, div.value, nrec.value, n.value


def first_partners(km, x: int = 0, ws=None, stream=None):
    """(status, first[2][P] as a numpy array, divergent); 0xFFFFFFFF = none."""
    ka = _arg(km)
    need = int(_L.rp_workspace_bytes(ka.ref, OP_FIRST))
    if need == 0:
        return ERR_INVALID, None, 0
    ptr, size = (ws or _ws).get(need)
    out = np.zeros((2, max(1, int(km.n_points))), np.uint32)
    div = C.c_uint64(0)
    st = _L.rp_first_partners(ka.ref, C.c_uint64(int(x)), out.ctypes.data, C.byref(div),
                              C.c_void_p(ptr), size, _stream(stream))
    return st, out[:, :int(km.n_points)], div.value


def clauses(km, x: int = 0, cap: int | None = None, ws=None, stream=None):
    """(status, [(pos, neg), ...]) reduced and sorted."""
    ka = _arg(km)
    need = int(_L.rp_workspace_bytes(ka.ref, OP_CLAUSES))
    if need == 0:
        return ERR_INVALID, []
    ptr, size = (ws or _ws).get(need)
    cap = 4 * len(ka.points) + 256 if cap is None else int(cap)
    buf = (RpClause * max(1, cap))()
    n = C.c_uint64(0)
    st = _L.rp_clauses(ka.ref, C.c_uint64(int(x)), buf if cap else None, cap, C.byref(n),
                       C.c_void_p(ptr), size, _stream(stream))
    if st != OK:
        return st, []
    return st, [(buf[q].pos, buf[q].neg) for q in range(n.value)]


def min_barriers(cl, weights, n_slots: int, ws=None, stream=None):
    """(status, assign, weight)."""
    n = len(cl)
    buf = (RpClause * max(1, n))()
    for q, (p, g) in enumerate(cl):
        buf[q].pos, buf[q].neg = int(p), int(g)
    w = (C.c_uint32 * max(1, n_slots))(*[int(v) for v in list(weights)[:n_slots]])
    need = int(_L.rp_solve_workspace_bytes(n))
    ptr, size = (ws or _ws).get(need)
    a = C.c_uint64(0)
    wt = C.c_uint64(0)
    st = _L.rp_min_barriers(buf, n, w, int(n_slots), C.byref(a), C.byref(wt), C.c_void_p(ptr),
                            size, _stream(stream))
    return st, a.value, wt.value


def repair(km, policy: int = 0, grid: int = 1, inspect: int = 1, max_rounds: int = 0,
           ws=None, stream=None, traj_cap: int = 4096, solver: int = 0):
    """Alg. 1 on the GPU; dict like the oracle's repair().  solver 0: exact
    Solve every round; 1: the mhs strategy (Section 2.4)."""
    ka = _arg(km)
    need = ka.need(OP_REPAIR)
    if need == 0:
        return dict(status=ERR_INVALID, ret=ERR_INVALID)
    ptr, size = (ws or _ws).get(need)
    o = RpOpts(policy, grid, inspect, solver, max_rounds)
    out = RpOut()
    traj = _traj(traj_cap)
    st = _L.rp_repair(ka.ref, C.byref(o), C.byref(out), traj, traj_cap, C.c_void_p(ptr), size,
                      _stream(stream))
    r = dict(status=out.status, assign=out.assign, weight=out.weight, added=out.added,
             removed=out.removed, rounds=out.rounds, n_clauses=out.n_clauses, ret=st)
    r["trajectory"] = [traj[q] for q in range(min(out.rounds, traj_cap))]
    return r


def noalloc_scratch_bytes() -> int:
    """Size of the fixed per-device array rp_repair_noalloc works in."""
    return int(_L.rp_noalloc_scratch_bytes())


def repair_noalloc(km, policy: int = 0, grid: int = 1, inspect: int = 1, max_rounds: int = 0,
                   stream=None, traj_cap: int = 4096, solver: int = 0):
    """rp_repair_noalloc: the repair loop with no workspace argument (the
    library's fixed per-device array); dict like repair()."""
    ka = _arg(km)
    o = RpOpts(policy, grid, inspect, solver, max_rounds)
    out = RpOut()
    traj = _traj(traj_cap)
    st = _L.rp_repair_noalloc(ka.ref, C.byref(o), C.byref(out), traj, traj_cap, _stream(stream))
    r = dict(status=out.status, assign=out.assign, weight=out.weight, added=out.added,
             removed=out.removed, rounds=out.rounds, n_clauses=out.n_clauses, ret=st)
    r["trajectory"] = [traj[q] for q in range(min(out.rounds, traj_cap))]
    return r


class BatchArg:
    """C views of many kernel models."""

    def __init__(self, kms):
        self.args = [k if isinstance(k, KernelArg) else KernelArg(k) for k in kms]
        self.ptrs = (C.POINTER(RpKernel) * max(1, len(kms)))(
            *[C.pointer(a.k) for a in self.args])
        self.n = len(kms)
        self._need = {}

    def need(self) -> int:
        """Workspace bytes of a batched repair of these kernels (cached while
        the sort tuning, on which the size depends, is unchanged)."""
        key = _tuning_epoch[0]
        if key not in self._need:
            self._need[key] = int(_L.rp_batch_workspace_bytes(self.ptrs, self.n))
        return self._need[key]


def batch_workspace_bytes(kms) -> int:
    b = kms if isinstance(kms, BatchArg) else BatchArg(kms)
    return b.need()


def repair_batch(kms, policy: int = 0, grid: int = 1, inspect: int = 1, max_rounds: int = 0,
                 ws=None, stream=None, solver: int = 0):
    """Alg. 1 over many kernels in one batched run; (status, [result dict per kernel]).
    Runs on a dedicated non-default stream unless one is given, so that each
    round can be replayed as a captured graph."""
    import torch
    b = kms if isinstance(kms, BatchArg) else BatchArg(kms)
    ptr, size = (ws or _ws).get(b.need())
    o = RpOpts(policy, grid, inspect, solver, max_rounds)
    outs = (RpOut * max(1, b.n))()
    st_obj = stream if stream is not None else _batch_stream()
    torch.cuda.current_stream().synchronize()
    st = _L.rp_repair_batch(b.ptrs, b.n, C.byref(o), outs, C.c_void_p(ptr), size,
                            C.c_void_p(st_obj.cuda_stream))
    res = []
    for q in range(b.n):
        r = outs[q]
        res.append(dict(status=r.status, assign=r.assign, weight=r.weight, added=r.added,
                        removed=r.removed, rounds=r.rounds, n_clauses=r.n_clauses))
    return st, res


_bstream = None


def _batch_stream():
    global _bstream
    import torch
    if _bstream is None:
        _bstream = torch.cuda.Stream()
    return _bstream


class Server:
    """Continuous-batching repair server over a torch-allocated device arena."""

    def __init__(self, arena_bytes: int, max_resident: int = 1024, policy: int = 0, grid: int = 1,
                 inspect: int = 1, max_rounds: int = 0, stream=None, solver: int = 0):
        import torch
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device="cuda")
        self.stream = stream if stream is not None else torch.cuda.Stream()
        torch.cuda.current_stream().synchronize()
        o = RpOpts(policy, grid, inspect, solver, max_rounds)
        h = C.c_void_p()
        st = _L.rp_server_create(C.c_void_p(self.arena.data_ptr()), int(arena_bytes), C.byref(o),
                                 int(max_resident), C.c_void_p(self.stream.cuda_stream),
                                 C.byref(h))
        if st != OK:
            raise RuntimeError("rp_server_create: " + status_string(st))
        self.h = h
        self._held = {}

    def job_bytes(self, km) -> int:
        return int(_L.rp_server_job_bytes(_arg(km).ref))

    def submit(self, km, job_id: int) -> int:
        return _L.rp_server_submit(self.h, _arg(km).ref, C.c_uint64(int(job_id)))

    def step(self):
        nr = C.c_uint32(0)
        npd = C.c_uint32(0)
        st = _L.rp_server_step(self.h, C.byref(nr), C.byref(npd))
        if st != OK:
            raise RuntimeError("rp_server_step: " + status_string(st))
        return nr.value, npd.value

    def poll(self, cap: int = 4096):
        ids = (C.c_uint64 * cap)()
        outs = (RpOut * cap)()
        lat = (C.c_double * cap)()
        n = C.c_uint32(0)
        st = _L.rp_server_poll(self.h, ids, outs, lat, cap, C.byref(n))
        if st != OK:
            raise RuntimeError("rp_server_poll: " + status_string(st))
        res = []
        for q in range(n.value):
            r = outs[q]
            res.append((ids[q], dict(status=r.status, assign=r.assign, weight=r.weight,
                                     added=r.added, removed=r.removed, rounds=r.rounds,
                                     n_clauses=r.n_clauses), lat[q]))
        return res

    def close(self):
        if self.h:
            _L.rp_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def last_stats() -> dict:
    s = RpStats()
    _L.rp_last_stats(C.byref(s))
    return {f: getattr(s, f) for f, _ in RpStats._fields_}


def set_sort_digit_bits(bits: int) -> int:
    return _L.rp_set_sort_digit_bits(int(bits))


_tuning_epoch = [0]      # bumped by every tuning change (workspace sizes depend on it)


def sort_key_bits(kms) -> int:
    """Radix key bits of one kernel model or of a batch sorted together."""
    if isinstance(kms, BatchArg):
        b = kms
    elif isinstance(kms, (list, tuple)):
        b = BatchArg(kms)
    else:
        b = BatchArg([kms])
    return int(_L.rp_sort_key_bits(b.ptrs, b.n))


def set_tuning(knob: int, value: int) -> int:
    if knob in (TUNE_SORT_DIGIT_BITS, TUNE_SCATTER_SHAPE,
                TUNE_LOW_DIGIT_BITS):   # they change workspace sizes
        _tuning_epoch[0] += 1
    return _L.rp_set_tuning(int(knob), int(value))


def instrument(prog, grid: int = 1, gw: int = 12, lw: int = 10):
    """rp_instrument on a ``synth.Program``: (status, Kernel or None)."""
    from . import synth
    arrays = np.zeros(len(prog.arrays), synth.ARRAY_DT)
    for n, (w, sp) in enumerate(prog.arrays):
        arrays[n] = (w, sp)
    guards = np.zeros(len(prog.guards), synth.GUARD_DT)
    for n, (m, r) in enumerate(prog.guards):
        guards[n] = (m, r)
    pbg = getattr(prog, "block_guards", None)
    bguards = None
    if pbg is not None:
        bguards = np.zeros(len(pbg), synth.GUARD_DT)
        for n, (m, r) in enumerate(pbg):
            bguards[n] = (m, r)
    bodies = []
    for fn in prog.functions:
        b = np.zeros(len(fn), STMT_DT)
        for n, st in enumerate(fn):
            b[n] = (st["kind"], st.get("is_write", 0), st.get("level", 0), 0,
                    st.get("array", 0), st.get("guard", 0), st.get("count", 0),
                    st.get("a", 0), st.get("b", 0), st.get("c", 0), st.get("d", 0))
        bodies.append(b)
    fns = (RpFunction * max(1, len(bodies)))()
    for n, b in enumerate(bodies):
        fns[n].n_stmts = len(b)
        fns[n].stmts = b.ctypes.data if len(b) else None
    pr = RpProgram(prog.blocks, prog.threads, len(arrays), len(guards), len(bodies),
                   arrays.ctypes.data if len(arrays) else None,
                   guards.ctypes.data if len(guards) else None, C.addressof(fns),
                   bguards.ctypes.data if bguards is not None and len(bguards) else None)
    o = RpInstrumentOpts()
    o.grid, o.gw, o.lw = grid, gw, lw
    ng, npt, ns = C.c_uint32(0), C.c_uint32(0), C.c_uint32(0)
    st = _L.rp_instrument(C.byref(pr), C.byref(o), None, None, 0, C.byref(ng), None, 0,
                          C.byref(npt), None, 0, C.byref(ns))
    if st != ERR_CAPACITY:
        return st, None
    g = np.zeros(ng.value, synth.GUARD_DT)
    bg = np.zeros(ng.value, synth.GUARD_DT)
    pt = np.zeros(npt.value, synth.POINT_DT)
    sl = np.zeros(ns.value, synth.SLOT_DT)
    st = _L.rp_instrument(C.byref(pr), C.byref(o), g.ctypes.data, bg.ctypes.data, len(g),
                          C.byref(ng), pt.ctypes.data, len(pt), C.byref(npt), sl.ctypes.data,
                          len(sl), C.byref(ns))
    if st != OK:
        return st, None
    # no block condition anywhere: the kernel model leaves block_guards out
    return st, synth.Kernel(prog.blocks, prog.threads, arrays, g, pt, sl,
                            dict(prog.meta, instrumented=True, grid=grid),
                            bg if (bg["m"] > 1).any() else None)
