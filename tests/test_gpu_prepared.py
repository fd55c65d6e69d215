"""Tasks run without validation and planning per call: rsm_run_prepared
(validated and planned once) and rsm_run's plans kept by descriptor.  Both
launch the same kernels as a planned rsm_run, so their results equal it bit
for bit, and the oracle bounds them at 1e-5 of each value's |term| sum.
"""
import numpy as np
import pytest
import torch

import oracle
import rsm_workloads as W
from paper_1105_4424_amd import _abi, rsm

from .helpers import bf16_dev, check_close, dev, host, say

pytestmark = pytest.mark.gpu


def _cases():
    x0, p0 = W.small_sum()
    ts = W.two_stage_filter(frames=2, rows=64, cols=136, taps=8, seed=81, h_origin=-4)
    k5 = W.filter2d_problem(70, 90, 5, 2, coeffs=(W.rng_for(82).uniform(-1, 1, (5, 5)) / 25).astype(np.float32))
    x5 = W.rng_for(83).standard_normal((70, 90)).astype(np.float32)
    pp = W.polyphase_downscaler(frames=1, rows=36, cols=96)
    mid = oracle.run(ts.h, [ts.x]).out.astype(np.float32)
    return [
        ("pattern_reduce", p0, [x0], None),
        ("fir_cols_vec4", ts.h, [ts.x], ts.c_h),
        ("fir_rows", ts.v, [mid], ts.c_v),
        ("filter2d_k5_s2", k5, [x5], k5.coeffs),
        ("polyphase_cols_vec", pp.h, [pp.x], pp.c_h),
    ]


@pytest.mark.parametrize("k", range(5), ids=["pattern_reduce", "fir_cols_vec4", "fir_rows", "filter2d", "polyphase"])
def test_prepared_equals_planned_run(k):
    fam, p, xs, c = _cases()[k]
    say("prepared", fam)
    pr = rsm.Prepared(p)
    assert pr.name == fam
    ins = [dev(x) for x in xs]
    cd = None if c is None else dev(c)
    want = torch.full(p.output.array_shape, float("nan"), device="cuda")
    rsm.run(p, ins, want, coeffs=cd)
    got = torch.full(p.output.array_shape, float("nan"), device="cuda")
    for _ in range(3):   # repeated calls reuse the handle
        pr.run(ins, got, coeffs=cd)
        assert torch.equal(got, want)
    ref = oracle.run(p, xs)
    check_close(host(got), ref.out, ref.abs_sum, what=fam)
    pr.close()
    with pytest.raises(RuntimeError):
        pr.run(ins, got, coeffs=cd)


def test_prepared_matrix_product_bf16():
    M, N, K = 320, 264, 200
    a, b, ab, bb = W.matmul_inputs(M, N, K, seed=84)
    p = W.matmul_tilers(M, N, K)
    p.compute = "bf16"
    pr = rsm.Prepared(p, dtypes=(torch.bfloat16,))
    assert pr.name.startswith("gemm_mfma_bf16")
    A, B = bf16_dev(ab), bf16_dev(bb)
    got = torch.empty((M, N), device="cuda")
    want = torch.empty((M, N), device="cuda")
    pr.run([A, B], got)
    rsm.run(p, [A, B], want)
    assert torch.equal(got, want)
    # the wrong dtype is refused before the call
    with pytest.raises(TypeError):
        pr.run([A.float(), B.float()], got)


def test_prepared_input_off_16_byte_boundary_is_planned_again():
    # the handle planned the 16-byte lane-pair kernel; an input view that
    # starts 4 bytes later is run by the kernel a plain call would choose
    ts = W.two_stage_filter(frames=1, rows=32, cols=128, taps=8, seed=85)
    pr = rsm.Prepared(ts.h)
    assert pr.name == "fir_cols_vec4"
    base = torch.empty(ts.x.size + 4, device="cuda")
    xv = base[1:1 + ts.x.size].view(ts.x.shape)
    xv.copy_(dev(ts.x))
    assert xv.data_ptr() % 16 == 4
    c = dev(ts.c_h)
    got = torch.full(ts.h.rep_shape, float("nan"), device="cuda")
    pr.run([xv], got, coeffs=c)
    want = torch.full(ts.h.rep_shape, float("nan"), device="cuda")
    rsm.run(ts.h, [xv], want, coeffs=c)
    assert torch.equal(got, want)
    ref = oracle.run(ts.h, [ts.x])
    check_close(host(got), ref.out, ref.abs_sum, what="offset input")


def test_run_plan_cache_hits_and_changed_descriptors():
    # repeated calls hit the kept plan; a call that differs only in the
    # origin (a different task) must not reuse it
    # (a shape no other test of this process uses: the kept plans are per thread)
    ts = W.two_stage_filter(frames=1, rows=24, cols=152, taps=8, seed=86)
    ts2 = W.two_stage_filter(frames=1, rows=24, cols=152, taps=8, seed=86, h_origin=-3)
    x, c = dev(ts.x), dev(ts.c_h)
    h0 = rsm.plan_cache_hits()
    outs = []
    for prob in (ts.h, ts.h, ts2.h, ts2.h, ts.h):
        o = torch.full(prob.rep_shape, float("nan"), device="cuda")
        rsm.run(prob, [x], o, coeffs=c)
        outs.append(o)
    assert rsm.plan_cache_hits() - h0 >= 3
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[4])
    assert torch.equal(outs[2], outs[3])
    for prob, o in ((ts.h, outs[0]), (ts2.h, outs[2])):
        ref = oracle.run(prob, [ts.x])
        check_close(host(o), ref.out, ref.abs_sum, what="origin %s" % (prob.inputs[0].origin,))
    # the same descriptors with an input off the 16-byte boundary are another
    # entry (the lane-pair kernel's 16-byte loads cannot read it): another
    # kernel, within the same bound
    base = torch.empty(ts.x.size + 4, device="cuda")
    xv = base[1:1 + ts.x.size].view(ts.x.shape)
    xv.copy_(x)
    o = torch.full(ts.h.rep_shape, float("nan"), device="cuda")
    h1 = rsm.plan_cache_hits()
    rsm.run(ts.h, [xv], o, coeffs=c)
    assert rsm.plan_cache_hits() == h1
    ref = oracle.run(ts.h, [ts.x])
    check_close(host(o), ref.out, ref.abs_sum, what="offset input")


def test_prepared_weights_required_at_run():
    ts = W.two_stage_filter(frames=1, rows=16, cols=64, taps=8, seed=87)
    pr = rsm.Prepared(ts.h)
    out = torch.full(ts.h.rep_shape, 5.0, device="cuda")
    with pytest.raises(rsm.RsmError) as e:
        pr.run([dev(ts.x)], out)
    assert e.value.name == "RSM_E_INVALID"
    torch.cuda.synchronize()
    assert bool(torch.all(out == 5.0))


def test_kept_plan_takes_each_calls_operands():
    # two matrix products with equal descriptors and different operand
    # buffers: the second call runs from the kept plan and must read its own
    # operands (a plan holds no array addresses)
    M, N, K = 256, 192, 128
    p = W.matmul_tilers(M, N, K)
    outs, refs = [], []
    for seed in (91, 92):
        a, b, _, _ = W.matmul_inputs(M, N, K, seed=seed)
        o = torch.full((M, N), float("nan"), device="cuda")
        rsm.run(p, [dev(a), dev(b)], o)
        outs.append(o)
        refs.append((a, b))
    for o, (a, b) in zip(outs, refs):
        r = oracle.run(p, [a, b])
        check_close(host(o), r.out, r.abs_sum, what="kept gemm plan")
