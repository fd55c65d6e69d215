"""C-ABI checks that need no GPU: exports, struct layout, validation, planning."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import rsm_workloads as W
from paper_1105_4424_amd import _abi, rsm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rsm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(rsm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_function():
    lib = _abi.load()
    names = declared_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(_abi.EXPORTS) == names
    out = subprocess.run(["nm", "-D", "--defined-only", _abi.LIB_PATH], capture_output=True,
                         text=True).stdout
    for n in names:
        assert re.search(r" T %s$" % n, out, re.M), n


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(r"""
#include <stdio.h>
#include <stddef.h>
#include "rsm.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu %zu\n", sizeof(rsm_space), sizeof(rsm_tiler), sizeof(rsm_task),
         sizeof(rsm_stage), sizeof(rsm_problem), sizeof(rsm_batch_info), sizeof(rsm_port_placement));
  printf("%zu %zu %zu %zu %zu %zu\n", offsetof(rsm_tiler, pattern_rank), offsetof(rsm_tiler, origin),
         offsetof(rsm_tiler, paving), offsetof(rsm_tiler, fitting), offsetof(rsm_problem, d_in),
         offsetof(rsm_task, coeffs));
  return 0;
}
""")
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I" + os.path.join(ROOT, "include"), str(src), "-o", str(exe)])
    sizes, offs = [list(map(int, l.split())) for l in
                   subprocess.check_output([str(exe)]).decode().strip().splitlines()]
    assert sizes == [ctypes.sizeof(c) for c in (_abi.Space, _abi.Tiler, _abi.Task, _abi.Stage,
                                                _abi.Problem, _abi.BatchInfo, _abi.PortPlacement)]
    assert offs == [_abi.Tiler.pattern_rank.offset, _abi.Tiler.origin.offset,
                    _abi.Tiler.paving.offset, _abi.Tiler.fitting.offset, _abi.Problem.d_in.offset,
                    _abi.Task.coeffs.offset]


def test_status_strings():
    lib = _abi.load()
    for s in range(9):
        assert lib.rsm_status_string(s).decode().startswith("RSM_")
    assert lib.rsm_abi_version() == 1


def _expect(status_name, fn):
    with pytest.raises(rsm.RsmError) as e:
        fn()
    assert e.value.name == status_name, str(e.value)


def test_validation_errors():
    ok_t = W.Tiler((8,), [0], [[1]], [[1]], (2,))
    out = W.identity_output((4,))
    # non-positive array extent
    _expect("RSM_E_SHAPE", lambda: rsm.validate(
        W.Problem((4,), [W.Tiler((0,), [0], [[1]], [[1]], (2,))], out, W.SUM)))
    # non-positive pattern extent
    _expect("RSM_E_SHAPE", lambda: rsm.validate(
        W.Problem((4,), [W.Tiler((8,), [0], [[1]], [[1]], (0,))], out, W.SUM)))
    # rank too large
    big = W.Tiler((2,) * 9, [0] * 9, np.zeros((9, 1)), np.zeros((9, 0)), ())
    _expect("RSM_E_RANK", lambda: rsm.validate(W.Problem((4,), [big], out, W.SUM)))
    # SUM with a multi-element output pattern
    out2 = W.Tiler((4, 2), [0, 0], [[1], [0]], [[0], [1]], (2,))
    _expect("RSM_E_SHAPE", lambda: rsm.validate(W.Problem((4,), [ok_t], out2, W.SUM)))
    # COPY with mismatched pattern sizes
    _expect("RSM_E_SHAPE", lambda: rsm.validate(W.Problem((4,), [ok_t], out, W.COPY)))
    # DOT with one input
    _expect("RSM_E_INVALID", lambda: rsm.validate(W.Problem((4,), [ok_t], out, W.DOT)))
    # 62-bit overflow of the index arithmetic
    huge = W.Tiler((1 << 40,), [0], [[1]], [[1]], (1 << 23,))
    _expect("RSM_E_OVERFLOW", lambda: rsm.validate(W.Problem((1 << 21,), [huge], W.identity_output((1 << 21,)), W.SUM)))
    # the valid one passes
    rsm.validate(W.Problem((4,), [ok_t], out, W.SUM))


def test_single_assignment_check():
    t = W.Tiler((6,), [0], [[1]], np.zeros((1, 0)), ())
    collide = W.Tiler((3,), [0], [[1]], np.zeros((1, 0)), ())
    p = W.Problem((6,), [t], collide, W.COPY)
    rsm.validate(p)                       # not checked by default
    _expect("RSM_E_OVERLAP", lambda: rsm.validate(p, check_single_assign=True))
    rsm.validate(W.Problem((6,), [t], W.identity_output((6,)), W.COPY), check_single_assign=True)


def test_planner_routes_workloads_to_their_kernels():
    x, p0 = W.small_sum()
    assert rsm.plan(p0) == "pattern_reduce"
    ts = W.two_stage_filter(frames=2, rows=16, cols=32)
    assert rsm.plan(ts.h) == "fir_cols_vec4"
    assert rsm.plan(ts.v) == "fir_rows"
    assert rsm.plan(ts.h, flags=_abi.FORCE_GENERIC) == "generic"
    # overlapping windows on a common 16-byte phase: 16-byte vectors into
    # registers; on request, or off that phase, row segments staged in LDS
    tw = W.two_stage_filter(frames=1, rows=8, cols=40, taps=13, pave=8, h_origin=-6)
    assert rsm.plan(tw.h) == "fir_cols_window_vec"
    assert rsm.plan_placed(tw.h, ["local", "any", "any"])[0] == "fir_cols_lds"
    tg = W.two_stage_filter(frames=1, rows=8, cols=40, taps=6, pave=8, h_origin=2)
    assert rsm.plan(tg.h) == "fir_cols_window_vec"   # gaps between windows
    t3 = W.two_stage_filter(frames=1, rows=8, cols=39, taps=13, pave=8, h_origin=-6)
    assert rsm.plan(t3.h) == "fir_cols_lds"          # rows of 39 floats: no common phase
    t7 = W.two_stage_filter(frames=1, rows=8, cols=40, taps=15, pave=8, h_origin=-6)
    assert rsm.plan(t7.h) == "fir_cols_lds"          # phase 2 + 15 taps: more than four vectors
    te = W.two_stage_filter(frames=1, rows=8, cols=40, taps=8, pave=8, h_origin=-3)
    assert rsm.plan(te.h) == "fir_cols"          # exact cover off the 16-byte grid: registers
    assert rsm.plan_placed(tw.h, ["private", "any", "constant"])[0] == "fir_cols"
    assert rsm.plan_placed(tw.h, ["private", "any", "private"])[0] == "fir_cols_window_vec"
    import torch
    mm = W.matmul_tilers(256, 256, 256)
    mm.compute = "bf16"
    assert rsm.plan(mm, dtypes=(torch.bfloat16,)).startswith("gemm_mfma_bf16")
    mm.compute = "f32"
    assert rsm.plan(mm).startswith("gemm_mfma_f32")
    # random tilers fall back to the generic kernel (or the small-pattern one)
    rng = W.rng_for(5)
    t = W.random_tiler(rng, 2, pattern_rank=2, max_pattern_side=9)
    name = rsm.plan(W.Problem((3, 3), [t], W.identity_output((3, 3)), W.SUM))
    assert name in ("generic", "pattern_reduce")


def test_planner_routes_adjoints_to_their_kernels():
    A = _abi.PLAN_ADJOINT
    ts = W.two_stage_filter(frames=2, rows=16, cols=32)
    assert rsm.plan(ts.h, flags=A) == "fir_adjoint_vec4"        # exact paving, injective
    assert rsm.plan(ts.v, flags=A) == "fir_adjoint"
    assert rsm.plan(ts.h, flags=A | _abi.FORCE_GENERIC) == "generic_adjoint"
    # 13 taps every 8 columns / rows: windows overlap (and wrap at the origin)
    tw = W.two_stage_filter(frames=1, rows=24, cols=40, taps=13, pave=8, h_origin=-6, v_origin=-6)
    assert rsm.plan(tw.h, flags=A) == "fir_adjoint_overlap_cols"   # taps along columns
    assert rsm.plan(tw.v, flags=A) == "fir_adjoint_gather"         # taps along rows
    # windows that wrap onto each other without overlapping: 8 taps every 8
    # columns, 6 windows on 40 columns
    t6 = W.Tiler((2, 4, 40), [0, 0, 0], np.diag([1, 1, 8]), [[0], [0], [1]], (8,))
    assert rsm.plan(W.Problem((2, 4, 6), [t6], W.identity_output((2, 4, 6)), W.WSUM),
                    flags=A) == "fir_adjoint_overlap_cols"
    # column steps above 16: the per-element gather
    t20 = W.Tiler((2, 4, 40), [0, 0, 0], np.diag([1, 1, 20]), [[0], [0], [1]], (8,))
    assert rsm.plan(W.Problem((2, 4, 3), [t20], W.identity_output((2, 4, 3)), W.WSUM),
                    flags=A) == "fir_adjoint_gather"
    # two repetitions reading the same rows (zero row step): no gather form
    t0 = W.Tiler((2, 4, 40), [0, 0, 0], np.diag([1, 0, 8]), [[0], [0], [1]], (8,))
    assert rsm.plan(W.Problem((2, 3, 5), [t0], W.identity_output((2, 3, 5)), W.WSUM),
                    flags=A) == "generic_adjoint"
    # 2-D windows: generic
    p2 = W.filter2d_problem(20, 24, 3, 1)
    assert rsm.plan(p2, flags=A) == "generic_adjoint"


def test_port_placement_follows_the_planned_kernel():
    # the memory space of every port (the paper's MemoryMapping, realised on
    # gfx950) for each kernel family, with the staged bytes per workgroup
    import torch
    x, p0 = W.small_sum()
    assert rsm.plan_ports(p0) == [("private", 1024), ("global", 0)]
    ts = W.two_stage_filter(frames=2, rows=16, cols=32)
    # 8 column taps: each thread's window in registers, weights uniform
    assert rsm.plan_ports(ts.h) == [("private", 256 * 8 * 4), ("global", 0), ("constant", 32)]
    # forced onto the generic kernel: every port read and written in place
    assert rsm.plan_ports(ts.h, flags=_abi.FORCE_GENERIC) == [("global", 0)] * 3
    # k x k windows: input region staged in LDS, weights read as constants
    f = W.filter2d_problem(200, 300, 9, 1)
    ports = rsm.plan_ports(f)
    assert [sp for sp, _ in ports] == ["local", "global", "constant"]
    assert ports[2][1] == 9 * 9 * 4
    # region rows x padded pitch of the tile class a single run uses:
    # (32 - 1) + 9 rows, pitch 60 + 4 * 3 + 4 floats
    assert ports[0][1] == (31 + 9) * 76 * 4
    # matrix products: both operands double-buffered in LDS, the output tile
    # in accumulators (256 x 256 tiles from 200 tiles of output upward)
    mm = W.matmul_tilers(4096, 4096, 4096)
    mm.compute = "bf16"
    assert rsm.plan_ports(mm, dtypes=(torch.bfloat16,)) == [("local", 2 * 256 * 144)] * 2 + [
        ("private", 256 * 256 * 4)]
    small = W.matmul_tilers(256, 256, 256)
    small.compute = "bf16"
    assert rsm.plan_ports(small, dtypes=(torch.bfloat16,)) == [("local", 2 * 128 * 144)] * 2 + [
        ("private", 128 * 128 * 4)]
    # a too-short port array is an error
    lib = _abi.load()
    n = ctypes.c_int32(0)
    ports1 = (_abi.PortPlacement * 1)()
    import paper_1105_4424_amd.rsm as R
    task = _abi.Task(W.SUM, _abi.F32, None)
    tin = (_abi.Tiler * 1)(R._tiler(p0.inputs[0], _abi.F32))
    st = lib.rsm_plan_ports(ctypes.byref(R._space(p0.rep_shape)), tin, 1,
                            ctypes.byref(R._tiler(p0.output, _abi.F32)), ctypes.byref(task), 0, ports1, 1,
                            ctypes.byref(n))
    assert st != 0 and n.value == 2


def test_empty_repetition_space_is_a_no_op_plan():
    t = W.Tiler((8,), [0], [[1]], [[1]], (2,))
    assert rsm.plan(W.Problem((0,), [t], W.identity_output((0,)) if False else
                              W.Tiler((1,), [0], [[1]], np.zeros((1, 0)), ()), W.SUM)) == "empty"


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError, match="not built"):
        _abi.load(str(tmp_path / "nope.so"))


def test_cg_solve_host_checks():
    # argument errors are reported before any device work
    lib = _abi.load()
    info = _abi.CgInfo()

    def call(n=4, nnz=4, tol=1e-10, max_iter=4, check_every=1, info_p=ctypes.byref(info)):
        return lib.rsm_cg_solve(n, nnz, None, None, None, None, None, tol, max_iter, check_every, 0,
                                None, None, None, info_p, None)

    name = lambda s: lib.rsm_status_string(s).decode()
    assert name(call(info_p=None)) == "RSM_E_INVALID"
    assert name(call(n=-1)) == "RSM_E_SHAPE"
    assert name(call(nnz=1 << 31)) == "RSM_E_UNSUPPORTED"
    assert name(call(tol=-1.0)) == "RSM_E_INVALID"
    assert name(call(tol=float("nan"))) == "RSM_E_INVALID"
    assert name(call(max_iter=-1)) == "RSM_E_INVALID"
    assert name(call(check_every=0)) == "RSM_E_INVALID"
    assert name(call()) == "RSM_E_INVALID"          # NULL device pointers
    # an empty system is solved with no work
    assert name(call(n=0, nnz=0)) == "RSM_OK"
    assert info.iterations == 0 and info.converged == 1 and info.breakdown == 0


def test_placement_request_routes_the_kernel_family():
    # a request names the memory space of each port (inputs, output,
    # coefficients); the planner takes the first family that meets it
    import torch
    ts = W.two_stage_filter(frames=2, rows=16, cols=32)
    P = rsm.plan_placed
    assert P(ts.h, None) == ("fir_cols_vec4", rsm.plan_ports(ts.h))
    # the window staged in LDS (input, output and weights local)
    name, ports = P(ts.h, ["local", "any", "any"])
    assert name == "fir_cols_lds" and [s for s, _ in ports] == ["local", "local", "local"]
    assert ports[0][1] == (8 * 255 + 8) * 4 and ports[2][1] == 8 * 4
    assert P(ts.h, ["any", "any", "local"])[0] == "fir_cols_lds"
    assert P(ts.h, ["any", "local", "any"])[0] == "fir_cols_lds"
    # taps in registers, weights uniform (the default family)
    assert P(ts.h, ["private", "global", "constant"])[0] == "fir_cols_vec4"
    # weights per lane: one pattern element per lane
    assert P(ts.h, ["any", "any", "private"])[0] == "pattern_reduce"
    # everything in place
    assert P(ts.h, ["global", "any", "any"]) == ("generic", [("global", 0)] * 3)
    # rows: weights in LDS, taps in registers; no family stages row taps in LDS
    assert P(ts.v, ["any", "any", "local"])[0] == "fir_rows_lds_weights"
    with pytest.raises(rsm.RsmError) as e:
        P(ts.v, ["local", "any", "any"])
    assert e.value.name == "RSM_E_UNSUPPORTED"
    # an input array is not uniform across a workgroup: never constant
    with pytest.raises(rsm.RsmError) as e:
        P(ts.h, ["constant", "any", "any"])
    assert e.value.name == "RSM_E_UNSUPPORTED"
    # the output port is written: constant memory contradicts its direction
    with pytest.raises(rsm.RsmError) as e:
        P(ts.h, ["any", "constant", "any"])
    assert e.value.name == "RSM_E_INVALID"
    # one space per port
    with pytest.raises(rsm.RsmError) as e:
        P(ts.h, ["any", "any"])
    assert e.value.name == "RSM_E_INVALID"
    # k x k windows: LDS tile by default (weights read as constants), one
    # element per lane up to 64 elements, in place on the generic kernel;
    # never weights in LDS
    f5 = W.filter2d_problem(70, 90, 5, 1)
    assert P(f5, None)[0] == "filter2d_k5_s1"
    assert P(f5, ["local", "global", "constant"])[0] == "filter2d_k5_s1"
    assert P(f5, ["private", "any", "any"])[0] == "pattern_reduce"
    assert P(f5, ["global", "any", "any"])[0] == "generic"
    with pytest.raises(rsm.RsmError) as e:
        P(f5, ["any", "any", "local"])
    assert e.value.name == "RSM_E_UNSUPPORTED"
    f9 = W.filter2d_problem(70, 90, 9, 1)
    with pytest.raises(rsm.RsmError) as e:
        P(f9, ["private", "any", "any"])    # 81 elements: more than a lane group holds
    assert e.value.name == "RSM_E_UNSUPPORTED"
    # matrix product: operands in LDS, accumulators in registers, or in place
    mm = W.matmul_tilers(256, 256, 256)
    assert P(mm, ["local", "local", "private"])[0] == "gemm_mfma_f32_nn"
    assert P(mm, ["global", "any", "any"])[0] == "generic"
    with pytest.raises(rsm.RsmError) as e:
        P(mm, ["any", "any", "local"])
    assert e.value.name == "RSM_E_UNSUPPORTED"
    # polyphase stage: windows and weights in registers by default; the
    # staged columns kernel keeps everything in LDS
    pp = W.polyphase_downscaler(frames=1, rows=18, cols=48)
    name, ports = P(pp.h, None)
    assert name == "polyphase_cols_vec"
    assert [s for s, _ in ports] == ["private", "global", "private"]
    assert ports[0][1] == 256 * 16 * 4 and ports[2][1] == 256 * 16 * 3 * 4
    assert P(pp.h, ["local", "local", "local"])[0] == "polyphase_cols"
    assert P(pp.h, ["any", "local", "any"])[0] == "polyphase_cols"
    assert P(pp.h, ["global", "any", "any"])[0] == "generic"
    assert P(pp.v, ["private", "global", "local"])[0] == "polyphase_rows"


def _raw(problem, dtype=_abi.F32):
    """ctypes descriptors of a problem with FP32 arrays."""
    n = len(problem.inputs)
    tin = (_abi.Tiler * n)(*[rsm._tiler(t, dtype) for t in problem.inputs])
    return rsm._space(problem.rep_shape), tin, n, rsm._tiler(problem.output, _abi.F32)


def test_prepared_task_plans_once_on_the_host():
    lib = _abi.load()
    ts = W.two_stage_filter(frames=2, rows=16, cols=32)
    for prob, fam in ((ts.h, "fir_cols_vec4"), (ts.v, "fir_rows"), (W.small_sum()[1], "pattern_reduce")):
        assert rsm.Prepared(prob).name == fam == rsm.plan(prob)
    assert rsm.Prepared(ts.h, flags=_abi.FORCE_GENERIC).name == "generic"
    # weights are given per call: a WSUM task prepares without them
    rep, tin, n, out = _raw(ts.h)
    h = ctypes.c_void_p()
    task = _abi.Task(_abi.TASK_WSUM, _abi.F32, None)
    assert lib.rsm_prepare(ctypes.byref(rep), tin, n, ctypes.byref(out), ctypes.byref(task), 0,
                           ctypes.byref(h)) == _abi.OK and h.value
    # ... and refuses a call without them, before any launch
    ptrs = (ctypes.c_void_p * 1)(16)
    assert lib.rsm_run_prepared(h, ptrs, ctypes.c_void_p(16), None, None) == _abi.E_INVALID
    assert b"coefficients" in lib.rsm_last_error()
    lib.rsm_prepared_destroy(h)
    lib.rsm_prepared_destroy(None)
    # flags other than the single-assignment check and the generic kernel
    for f in (_abi.ACCUMULATE, _abi.NO_FUSE, _abi.PLAN_ADJOINT, 0x1000):
        h = ctypes.c_void_p(7)
        assert lib.rsm_prepare(ctypes.byref(rep), tin, n, ctypes.byref(out), ctypes.byref(task), f,
                               ctypes.byref(h)) == _abi.E_INVALID
        assert not h.value
    # invalid descriptors fail as rsm_run does, with no handle
    bad = W.Problem((4,), [W.Tiler((0,), [0], [[1]], [[1]], (2,))], W.identity_output((4,)), W.SUM)
    _expect("RSM_E_SHAPE", lambda: rsm.Prepared(bad))
    t = W.Tiler((6,), [0], [[1]], np.zeros((1, 0)), ())
    collide = W.Problem((6,), [t], W.Tiler((3,), [0], [[1]], np.zeros((1, 0)), ()), W.COPY)
    rsm.Prepared(collide)
    _expect("RSM_E_OVERLAP", lambda: rsm.Prepared(collide, flags=_abi.CHECK_SINGLE_ASSIGN))
    assert lib.rsm_run_prepared(None, ptrs, ctypes.c_void_p(16), None, None) == _abi.E_INVALID


def test_run_keeps_plans_by_descriptor():
    # an empty repetition space runs nothing, so rsm_run returns on the host
    # and the cache can be watched without a GPU
    lib = _abi.load()
    t = W.Tiler((8,), [0], [[1]], [[1]], (2,))
    p = W.Problem((0,), [t], W.Tiler((1,), [0], [[1]], np.zeros((1, 0)), ()), W.SUM)
    rep, tin, n, out = _raw(p)
    task = _abi.Task(_abi.TASK_SUM, _abi.F32, None)
    ptrs = (ctypes.c_void_p * 1)(None)

    def call(rep=rep, tin=tin, out=out, flags=0):
        return lib.rsm_run(ctypes.byref(rep), tin, ptrs, n, ctypes.byref(out), None, ctypes.byref(task), flags,
                           None)

    h0 = lib.rsm_plan_cache_hits()
    assert call() == _abi.OK
    assert call() == _abi.OK and call() == _abi.OK
    assert lib.rsm_plan_cache_hits() == h0 + 2
    # another origin, other flags: new entries, not hits
    tin2 = (_abi.Tiler * 1)(rsm._tiler(W.Tiler((8,), [1], [[1]], [[1]], (2,)), _abi.F32))
    assert call(tin=tin2) == _abi.OK and call(flags=_abi.CHECK_SINGLE_ASSIGN) == _abi.OK
    assert lib.rsm_plan_cache_hits() == h0 + 2
    # entries beyond the pattern rank are not part of the descriptor
    tin3 = (_abi.Tiler * 1)(rsm._tiler(t, _abi.F32))
    tin3[0].fitting[0][5] = 99
    assert call(tin=tin3) == _abi.OK
    assert lib.rsm_plan_cache_hits() == h0 + 3
    # a failing descriptor is never kept: it fails every time
    tin4 = (_abi.Tiler * 1)(rsm._tiler(t, _abi.F32))
    tin4[0].array_shape[0] = 0
    assert call(tin=tin4) == _abi.E_SHAPE and call(tin=tin4) == _abi.E_SHAPE
    assert lib.rsm_plan_cache_hits() == h0 + 3
    # the cache holds 32 descriptors: after 40 others the first is planned again
    for k in range(40):
        assert call(tin=(_abi.Tiler * 1)(rsm._tiler(W.Tiler((8,), [k + 2], [[1]], [[1]], (2,)), _abi.F32))) == 0
    h1 = lib.rsm_plan_cache_hits()
    assert call() == _abi.OK and lib.rsm_plan_cache_hits() == h1
    assert call() == _abi.OK and lib.rsm_plan_cache_hits() == h1 + 1
