"""Placement requests (the paper's MemoryMapping: one address space per
port) honoured on the GPU: every placement the planner accepts runs its
kernel family through rsm_run_placed and matches the FP64 oracle at 1e-5 of
each output's |term| sum.  Requests no family meets are refused before any
launch.
"""
import numpy as np
import pytest
import torch

import oracle
import rsm_workloads as W
from paper_1105_4424_amd import _abi, rsm

from .helpers import check_close, dev, host, say

pytestmark = pytest.mark.gpu

A = "any"


def _run(p, inputs, spaces, coeffs=None, expect=None):
    name, ports = rsm.plan_placed(p, spaces)
    if expect is not None:
        assert name == expect, (spaces, name)
    for want, (got, _) in zip(spaces, ports):
        assert want == A or want == got, (spaces, ports)
    out = torch.full(p.output.array_shape, float("nan"), device="cuda")
    rsm.run_placed(p, [dev(x) for x in inputs], out, spaces, coeffs=None if coeffs is None else dev(coeffs))
    ref = oracle.run(p, inputs)
    check_close(host(out), ref.out, ref.abs_sum, what="%s %s" % (name, spaces))
    return name


# 8 taps along columns (origin -3: windows off 16-byte boundaries, wrapping
# at the left border) and along rows, 2 frames of 64 x 200
@pytest.mark.parametrize("spaces,family", [
    ((A, A, A), "fir_cols"),
    (("private", "global", "constant"), "fir_cols"),
    (("local", A, A), "fir_cols_lds"),
    ((A, "local", "local"), "fir_cols_lds"),
    ((A, A, "private"), "pattern_reduce"),
    (("global", "global", "global"), "generic"),
])
def test_column_taps_every_placement(spaces, family):
    ts = W.two_stage_filter(frames=2, rows=64, cols=200, taps=8, seed=71, h_origin=-3)
    say("placement", spaces)
    _run(ts.h, [ts.x], list(spaces), ts.c_h, family)


# 13 taps every 8 columns (origin -6: windows overlap by 5 and wrap at both
# borders), 2 frames of 64 x 200
@pytest.mark.parametrize("spaces,family", [
    ((A, A, A), "fir_cols_window_vec"),
    (("private", "global", "private"), "fir_cols_window_vec"),
    (("private", A, "constant"), "fir_cols"),
    (("local", A, A), "fir_cols_lds"),
    (("global", A, A), "generic"),
])
def test_overlapping_column_taps_every_placement(spaces, family):
    ts = W.two_stage_filter(frames=2, rows=64, cols=200, taps=13, pave=8, seed=74, h_origin=-6)
    say("placement", spaces)
    _run(ts.h, [ts.x], list(spaces), ts.c_h, family)


# polyphase stage (13 taps every 8 columns, 3 outputs per window)
@pytest.mark.parametrize("spaces,family", [
    ((A, A, A), "polyphase_cols_vec"),
    ((A, "local", A), "polyphase_cols"),
    (("global", A, A), "generic"),
])
def test_polyphase_columns_every_placement(spaces, family):
    pp = W.polyphase_downscaler(frames=1, rows=24, cols=200)
    say("placement", spaces)
    _run(pp.h, [pp.x], list(spaces), pp.c_h, family)


@pytest.mark.parametrize("spaces,family", [
    ((A, A, A), "fir_rows"),
    ((A, A, "local"), "fir_rows_lds_weights"),
    ((A, A, "private"), "pattern_reduce"),
    (("global", A, A), "generic"),
])
def test_row_taps_every_placement(spaces, family):
    ts = W.two_stage_filter(frames=2, rows=72, cols=128, taps=8, seed=72, v_origin=-5)
    mid = oracle.run(ts.h, [ts.x]).out.astype(np.float32)
    _run(ts.v, [mid], list(spaces), ts.c_v, family)


@pytest.mark.parametrize("k,spaces,family", [
    (5, (A, A, A), "filter2d_k5_s1"),
    (5, ("private", A, A), "pattern_reduce"),
    (5, ("global", A, A), "generic"),
    (9, (A, A, A), "filter2d_k9_s1"),
    (9, ("global", A, A), "generic"),
])
def test_window_every_placement(k, spaces, family):
    rng = W.rng_for(73 + k)
    p = W.filter2d_problem(70, 90, k, 1, coeffs=(rng.uniform(-1, 1, (k, k)) / (k * k)).astype(np.float32))
    x = rng.standard_normal((70, 90)).astype(np.float32)
    _run(p, [x], list(spaces), p.coeffs, family)


@pytest.mark.parametrize("spaces,family", [
    (("local", "local", "private"), "gemm_mfma_f32_nn"),
    (("global", A, A), "generic"),
])
def test_matrix_product_every_placement(spaces, family):
    a, b, _, _ = W.matmul_inputs(200, 136, 96, seed=74)
    p = W.matmul_tilers(200, 136, 96)
    _run(p, [a, b], list(spaces), None, family)


def test_placements_of_one_task_agree():
    # the same horizontal stage through every family that can run it: the
    # results agree to the FP32 bound and equal the default run where the
    # family is the default one
    ts = W.two_stage_filter(frames=2, rows=64, cols=256, taps=8, seed=75)
    x, c = dev(ts.x), dev(ts.c_h)
    outs = {}
    for spaces in ((A, A, A), ("local", A, A), (A, A, "private"), ("global", A, A)):
        name, _ = rsm.plan_placed(ts.h, list(spaces))
        o = torch.empty(ts.h.rep_shape, device="cuda")
        rsm.run_placed(ts.h, [x], o, list(spaces), coeffs=c)
        outs[name] = o
    dflt = torch.empty(ts.h.rep_shape, device="cuda")
    rsm.run(ts.h, [x], dflt, coeffs=c)
    assert torch.equal(outs["fir_cols_vec4"], dflt)
    ref = oracle.run(ts.h, [ts.x])
    for name, o in outs.items():
        check_close(host(o), ref.out, ref.abs_sum, what=name)


def test_unmet_requests_are_refused_before_any_launch():
    ts = W.two_stage_filter(frames=1, rows=16, cols=64, taps=8, seed=76)
    out = torch.full(ts.h.rep_shape, 7.0, device="cuda")
    for spaces, status in ((["constant", A, A], "RSM_E_UNSUPPORTED"), ([A, "constant", A], "RSM_E_INVALID"),
                           ([A, A], "RSM_E_INVALID")):
        with pytest.raises(rsm.RsmError) as e:
            rsm.run_placed(ts.h, [dev(ts.x)], out, spaces, coeffs=dev(ts.c_h))
        assert e.value.name == status
    torch.cuda.synchronize()
    assert bool(torch.all(out == 7.0))
