"""The C ABI without a GPU: the library loads, exports every function the
header declares, and its host-side logic (validation, workspace sizing,
status strings, tuning knobs) behaves as documented.  No call here launches
a kernel."""
import ctypes as C
import os
import re

import pytest

from paper_2011_08373_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "librepair.h")
LIB = os.path.join(ROOT, "paper_2011_08373_amd", "lib", "librepair.so")


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(LIB):
        from paper_2011_08373_amd import build
        build.build()
    from paper_2011_08373_amd import librepair
    return librepair


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"\b(rp_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("rp_check", "rp_clauses", "rp_min_barriers", "rp_repair", "rp_validate",
              "rp_workspace_bytes", "rp_repair_batch", "rp_server_create", "rp_status_string"):
        assert n in names, n


def test_every_declared_function_is_exported(L):
    lib = C.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_status_strings(L):
    seen = set()
    for st in (L.OK, L.UNSAT, L.ERR_INVALID, L.ERR_CAPACITY, L.ERR_WORKSPACE, L.ERR_DEVICE,
               L.ERR_ROUNDS, L.ERR_BUDGET, L.ERR_SEARCH):
        s = L.status_string(st)
        assert isinstance(s, str) and s and s != "unknown status"
        seen.add(s)
    assert len(seen) == 9


def test_validation_without_device(L):
    km = synth.generate("plain-small", seed=0)
    assert L.validate(km) == L.OK
    bad = synth.make_kernel(1, 8, [(16, 0)], [(1, 0)],
                            [dict(kind=0, is_write=1, array=3)], [])   # no array 3
    assert L.validate(bad) == L.ERR_INVALID
    bad = synth.make_kernel(0, 8, [(16, 0)], [(1, 0)], [], [])          # no blocks
    assert L.validate(bad) == L.ERR_INVALID
    bad = synth.make_kernel(1, 8, [(16, 0)], [(2, 2)], [], [])          # r >= m
    assert L.validate(bad) == L.ERR_INVALID
    # slots must be numbered by first occurrence
    bad = synth.make_kernel(1, 8, [(16, 0)], [(1, 0)],
                            [dict(kind=1, slot=1), dict(kind=1, slot=0)], [(0, 0, 1), (0, 0, 1)])
    assert L.validate(bad) == L.ERR_INVALID


def test_workspace_follows_the_sort_tuning(L):
    km = synth.generate("plain-large", mode="literal")
    ka = L.KernelArg(km)
    old_bits = L.set_tuning(L.TUNE_SORT_DIGIT_BITS, 8)
    old_shape = L.set_tuning(L.TUNE_SCATTER_SHAPE, 4)
    try:
        n8 = ka.need(L.OP_REPAIR)
        assert n8 > 0 and n8 == L.workspace_bytes(km, L.OP_REPAIR)
        # wider digits: larger per-chunk count tables; the cached size must follow
        L.set_tuning(L.TUNE_SORT_DIGIT_BITS, 11)
        n11 = ka.need(L.OP_REPAIR)
        assert n11 > n8
        assert n11 == L.workspace_bytes(km, L.OP_REPAIR)
    finally:
        L.set_tuning(L.TUNE_SORT_DIGIT_BITS, old_bits)
        L.set_tuning(L.TUNE_SCATTER_SHAPE, old_shape)


def test_tuning_knobs(L):
    old = L.set_tuning(L.TUNE_SORT_DIGIT_BITS, 9)
    try:
        assert L.set_tuning(L.TUNE_SORT_DIGIT_BITS, 10) == 9
        assert L.set_tuning(L.TUNE_SORT_DIGIT_BITS, 7) == -1      # out of range
        assert L.set_tuning(L.TUNE_SCATTER_SHAPE, 10) == -1
        assert L.set_tuning(L.TUNE_SCATTER_SHAPE, -1) == -1
        assert L.set_tuning(99, 0) == -1
    finally:
        L.set_tuning(L.TUNE_SORT_DIGIT_BITS, old)
    old = L.set_tuning(L.TUNE_TIMING, 2)
    try:
        assert old == 1                                          # the default
        assert L.set_tuning(L.TUNE_TIMING, 0) == 2
        assert L.set_tuning(L.TUNE_TIMING, 3) == -1
        assert L.set_tuning(L.TUNE_TIMING, -1) == -1
    finally:
        L.set_tuning(L.TUNE_TIMING, old)
    old = L.set_tuning(L.TUNE_SCATTER_WGS, 4)
    try:
        assert old == 0                                          # the occupancy query
        assert L.set_tuning(L.TUNE_SCATTER_WGS, 9) == -1
        assert L.set_tuning(L.TUNE_SCATTER_WGS, 0) == 4
    finally:
        L.set_tuning(L.TUNE_SCATTER_WGS, old)
    old = L.set_tuning(L.TUNE_SOLVER_NODES, 10)
    try:
        assert old == 28                                         # 2^28 nodes by default
        assert L.set_tuning(L.TUNE_SOLVER_NODES, 3) == -1
        assert L.set_tuning(L.TUNE_SOLVER_NODES, 41) == -1
        assert L.set_tuning(L.TUNE_SOLVER_NODES, 28) == 10
    finally:
        L.set_tuning(L.TUNE_SOLVER_NODES, old)
    old = L.set_tuning(L.TUNE_SCAN_PIPELINE, 0)
    try:
        assert old == 1                                          # next range's loads in flight
        assert L.set_tuning(L.TUNE_SCAN_PIPELINE, 2) == -1
        assert L.set_tuning(L.TUNE_SCAN_PIPELINE, 1) == 0
    finally:
        L.set_tuning(L.TUNE_SCAN_PIPELINE, old)
    old = L.set_tuning(L.TUNE_DIGIT_ORDER, 0)
    try:
        assert old == 1                                          # highest digit first
        assert L.set_tuning(L.TUNE_DIGIT_ORDER, 2) == -1
        assert L.set_tuning(L.TUNE_DIGIT_ORDER, 1) == 0
    finally:
        L.set_tuning(L.TUNE_DIGIT_ORDER, old)
    old = L.set_tuning(L.TUNE_LOW_DIGIT_BITS, 0)
    try:
        assert old == 6                                          # a 6-bit lowest digit
        for bad in (5, 10, -1):
            assert L.set_tuning(L.TUNE_LOW_DIGIT_BITS, bad) == -1
        assert L.set_tuning(L.TUNE_LOW_DIGIT_BITS, 9) == 0
    finally:
        L.set_tuning(L.TUNE_LOW_DIGIT_BITS, old)
    old = L.set_tuning(L.TUNE_PASS_SHAPES, L.pass_shapes_value([None, 9, 4]))
    try:
        assert old == L.PASS_SHAPES_DEFAULT                      # every pass on the main tile
        # a nibble of 10..14, a negative value or bits above pass 6 are rejected
        for bad in (-1, 0x0FFFFFFA, 0x0FFFFEFF, 0x1FFFFFFF):
            assert L.set_tuning(L.TUNE_PASS_SHAPES, bad) == -1
        assert L.set_tuning(L.TUNE_PASS_SHAPES, 0) == 0x0FFFF49F   # passes 0..6 on shape 0
        assert L.set_tuning(L.TUNE_PASS_SHAPES, L.PASS_SHAPES_DEFAULT) == 0
    finally:
        L.set_tuning(L.TUNE_PASS_SHAPES, old)
    old = L.set_tuning(L.TUNE_SCAN_FIELDS, 1)
    try:
        assert old == 0                                          # 32-bit fields where they fit
        assert L.set_tuning(L.TUNE_SCAN_FIELDS, 2) == -1
        assert L.set_tuning(L.TUNE_SCAN_FIELDS, -1) == -1
        assert L.set_tuning(L.TUNE_SCAN_FIELDS, 0) == 1
    finally:
        L.set_tuning(L.TUNE_SCAN_FIELDS, old)


def test_invalid_kernel_does_no_device_work(L):
    bad = synth.make_kernel(0, 8, [(16, 0)], [(1, 0)], [], [])
    assert L.workspace_bytes(bad, L.OP_REPAIR) == 0


def test_pass_shapes_value(L):
    # per-pass tiles pack 4 bits per pass in execution order; unset passes
    # (None) keep 15, the common tile, and passes past 6 are not encoded
    assert L.pass_shapes_value([]) == L.PASS_SHAPES_DEFAULT == 0x0FFFFFFF
    assert L.pass_shapes_value([6, 9]) == 0x0FFFFF96
    assert L.pass_shapes_value([None, None, 4]) == 0x0FFFF4FF
    assert L.pass_shapes_value([0] * 9) == 0                  # 7 passes of 4 bits
