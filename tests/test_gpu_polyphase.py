"""GPU parity of weighted sums whose output pattern has several elements
(polyphase stages: one repetition reads a window and writes q outputs, each
with its own taps) against the FP64 oracle.

* forward and adjoint of single stages, taps along columns and along rows,
  on the polyphase kernels and on the generic kernels (FORCE_GENERIC), with
  windows that overlap and wrap at the borders and rows longer than one
  256-repetition chunk;
* the downscaler built from two such stages (1920x1080 -> 720x480 per frame)
  at its full size of 30 frames: every output of both stages against the
  oracle, the stage adjoints against the oracle's, and the chain through the
  autograd wrappers.

Tolerance: 1e-5 of each value's |term| sum (the oracle's), as for every FP32
task.
"""
import numpy as np
import pytest
import torch

import oracle
import rsm_workloads as W
from paper_1105_4424_amd import _abi, rsm

from .helpers import check_close, dev, host, say

pytestmark = pytest.mark.gpu


def _stage(A, taps, pave, q, origin, axis, seed):
    """One polyphase stage on a [F, H, W] array with taps along `axis`."""
    F, H, Wd = A
    rng = W.rng_for(seed)
    if axis == 2:
        t = W.h_stage(F, H, Wd, taps, pave, origin)
        rep = (F, H, -(-Wd // pave))
    else:
        t = W.v_stage(F, H, Wd, taps, pave, origin)
        rep = (F, -(-H // pave), Wd)
    c = W.phase_coeffs(rng, q, taps)
    x = rng.standard_normal(A).astype(np.float32)
    return W.Problem(rep, [t], W.phase_output(rep, axis, q), W.WSUM, c), x


def _forward_check(p, x, flags=0, what=""):
    ref = oracle.run(p, [x])
    out = torch.full(p.output.array_shape, float("nan"), device="cuda")
    rsm.run(p, [dev(x)], out, coeffs=dev(p.coeffs), flags=flags)
    check_close(host(out), ref.out, ref.abs_sum, what=what + " forward")
    return out


def _adjoint_check(p, x, gy, flags=0, what=""):
    a = oracle.adjoint(p, x, gy)
    gx = torch.full(p.inputs[0].array_shape, float("nan"), device="cuda")
    gc = torch.full(p.coeffs.shape, float("nan"), device="cuda")
    rsm.run_adjoint(p, dev(x), dev(gy), gx, gc, dev(p.coeffs), flags=flags)
    check_close(host(gx), a.gx, a.gx_abs, what=what + " gx")
    check_close(host(gc), a.gc, a.gc_abs, what=what + " gc")
    # accumulate adds onto the previous contents
    gx2, gc2 = gx.clone(), gc.clone()
    rsm.run_adjoint(p, dev(x), dev(gy), gx2, gc2, dev(p.coeffs), flags=flags | _abi.ACCUMULATE)
    check_close(host(gx2), 2 * a.gx, 2 * a.gx_abs, what=what + " gx accumulate")
    check_close(host(gc2), 2 * a.gc, 2 * a.gc_abs, what=what + " gc accumulate")


CASES = [
    # (array, taps, pave, q, origin, axis)
    ((2, 24, 200), 13, 8, 3, -2, 2),     # overlapping windows wrapping at both ends
    ((1, 5, 2100), 13, 8, 3, -6, 2),     # 263 repetitions per row: two chunks
    ((2, 7, 61), 5, 3, 2, 4, 2),         # ragged: 21 windows of step 3 over 61 columns
    ((1, 3, 40), 16, 4, 4, -7, 2),       # windows four steps long
    ((1, 4, 33), 32, 16, 8, 0, 2),       # the largest pattern and step the kernels take
    ((2, 72, 40), 14, 9, 4, -2, 1),      # taps along rows
    ((1, 50, 17), 7, 2, 3, -3, 1),
    ((1, 9, 8), 20, 3, 2, -11, 1),       # windows longer than the axis: several lifts
    ((1, 6, 48), 13, 4, 3, -5, 2),       # step 4: the phase form of the column adjoint
    ((1, 3, 36), 13, 3, 2, -1, 2),       # step 3 (not a power of two): the per-slot form
    ((1, 5, 64), 12, 4, 4, 0, 2),        # four outputs per window in registers
    ((2, 4, 12), 5, 4, 2, -3, 2),        # rows shorter than four vectors: every window wraps
]


def _vec_form(A, taps, pave, q, origin, axis):
    """Whether the columns form that reads windows as 16-byte vectors applies:
    steps and rows in whole vectors, the window inside four vectors from its
    phase, at most four outputs per repetition."""
    return axis == 2 and pave % 4 == 0 and A[2] % 4 == 0 and origin % 4 + taps <= 16 and q <= 4


@pytest.mark.parametrize("case", CASES, ids=[str(k) for k in range(len(CASES))])
@pytest.mark.parametrize("generic", [False, True], ids=["polyphase", "generic"])
def test_polyphase_stage_forward_and_adjoint(case, generic):
    A, taps, pave, q, origin, axis = case
    p, x = _stage(A, taps, pave, q, origin, axis, seed=600 + taps + pave)
    flags = _abi.FORCE_GENERIC if generic else 0
    fam = rsm.plan(p, flags=flags)
    if generic:
        want = "generic"
    elif axis == 1:
        want = "polyphase_rows"
    else:
        want = "polyphase_cols_vec" if _vec_form(*case) else "polyphase_cols"
    assert fam == want, fam
    say("polyphase", A, taps, pave, q, origin, axis, fam)
    _forward_check(p, x, flags, what=str(case))
    gy = W.rng_for(700 + taps).uniform(-1, 1, p.output.array_shape).astype(np.float32)
    _adjoint_check(p, x, gy, flags, what=str(case))


@pytest.mark.parametrize("case", [c for c in CASES if c[5] == 2], ids=lambda c: str(c))
def test_polyphase_columns_staged_form(case):
    # the LDS-staged columns kernel, requested by placement where the
    # vector form would be the default
    p, x = _stage(*case, seed=600 + case[1] + case[2])
    ref = oracle.run(p, [x])
    out = torch.full(p.output.array_shape, float("nan"), device="cuda")
    assert rsm.plan_placed(p, ["local", "any", "any"])[0] == "polyphase_cols"
    rsm.run_placed(p, [dev(x)], out, ["local", "any", "any"], coeffs=dev(p.coeffs))
    check_close(host(out), ref.out, ref.abs_sum, what=str(case) + " staged")


def test_vector_form_ignores_values_outside_the_windows():
    # 6 taps every 8 columns leave gaps of 2; infinities and NaNs there are
    # read by the vector form (inside its four vectors) but must not reach
    # any output
    A = (2, 9, 96)
    p, x = _stage(A, 6, 8, 3, 1, 2, seed=640)
    assert rsm.plan(p) == "polyphase_cols_vec"
    cols = np.arange(A[2])
    in_gap = ((cols - 1) % 8) >= 6
    x = x.copy()
    x[:, 0::2, in_gap] = np.inf
    x[:, 1::2, in_gap] = np.nan
    ref = oracle.run(p, [x])
    assert np.isfinite(ref.out).all()
    out = torch.full(p.output.array_shape, float("nan"), device="cuda")
    rsm.run(p, [dev(x)], out, coeffs=dev(p.coeffs))
    check_close(host(out), ref.out, ref.abs_sum, what="gaps holding inf/nan")


def test_input_off_a_16_byte_boundary():
    # the same stage on an input 4 bytes past a 16-byte boundary (the plan
    # kept for these descriptors and that alignment, which the vector form
    # does not meet)
    p, x = _stage((1, 6, 200), 13, 8, 3, -2, 2, seed=641)
    buf = torch.empty(x.size + 4, device="cuda")
    xd = buf[1:1 + x.size].view(x.shape)
    xd.copy_(dev(x))
    assert xd.data_ptr() % 16 == 4
    ref = oracle.run(p, [x])
    out = torch.full(p.output.array_shape, float("nan"), device="cuda")
    rsm.run(p, [xd], out, coeffs=dev(p.coeffs))
    check_close(host(out), ref.out, ref.abs_sum, what="misaligned input")
    assert rsm.plan(p) == "polyphase_cols_vec"   # an aligned array keeps the vector form


def test_polyphase_kernel_plan_names():
    # along columns both gradients come from one pass over row chunks
    p, _ = _stage((1, 8, 64), 13, 8, 3, -2, 2, seed=1)
    assert rsm.plan(p, flags=_abi.PLAN_ADJOINT) == "polyphase_adjoint_cols"
    # along rows: a gather for dL/dx, per-repetition partials for the weights
    pr, _ = _stage((1, 64, 8), 13, 8, 3, -2, 1, seed=1)
    assert rsm.plan(pr, flags=_abi.PLAN_ADJOINT) == "polyphase_adjoint_gather"
    p5, _ = _stage((1, 64, 8), 20, 8, 3, -2, 1, seed=1)   # 20 taps: weight gradient on the generic kernel
    assert rsm.plan(p5, flags=_abi.PLAN_ADJOINT) == "polyphase_adjoint_gather_generic_gc"
    # forward along columns: window and weights in registers
    assert rsm.plan(p) == "polyphase_cols_vec"
    assert [sp for sp, _ in rsm.plan_ports(p)] == ["private", "global", "private"]


# column adjoints on steps 4, 8 and 16, one to four outputs, one to three
# windows per column, gaps between windows, and rows that windows wrap
# around more than once (more repetitions than the row holds steps)
COL_ADJ_CASES = [
    # (array, taps, pave, q, origin, repetitions along the row or None)
    ((2, 5, 64), 13, 8, 1, -6, None),
    ((1, 4, 96), 6, 8, 2, 1, None),
    ((1, 3, 64), 16, 16, 4, 0, None),
    ((1, 3, 48), 9, 4, 4, -1, None),
    ((1, 2, 32), 13, 8, 3, -3, 6),
]


def _col_adj_stage(A, taps, pave, q, origin, reps, seed):
    F, H, Wd = A
    t = W.h_stage(F, H, Wd, taps, pave, origin)
    rep = (F, H, reps if reps else -(-Wd // pave))
    c = W.phase_coeffs(W.rng_for(seed), q, taps)
    x = W.rng_for(seed + 1).standard_normal(A).astype(np.float32)
    return W.Problem(rep, [t], W.phase_output(rep, 2, q), W.WSUM, c), x


@pytest.mark.parametrize("case", COL_ADJ_CASES, ids=[str(k) for k in range(len(COL_ADJ_CASES))])
def test_column_adjoint_phases_gaps_and_laps(case):
    p, x = _col_adj_stage(*case, seed=660 + case[1])
    fam = rsm.plan(p, flags=_abi.PLAN_ADJOINT)
    say("column adjoint", case, fam)
    assert fam != "generic_adjoint", fam
    gy = W.rng_for(670 + case[1]).uniform(-1, 1, p.output.array_shape).astype(np.float32)
    _adjoint_check(p, x, gy, what=str(case))
    # one gradient at a time
    a = oracle.adjoint(p, x, gy)
    gx = torch.full(p.inputs[0].array_shape, float("nan"), device="cuda")
    rsm.run_adjoint(p, dev(x), dev(gy), gx, None, dev(p.coeffs))
    check_close(host(gx), a.gx, a.gx_abs, what=str(case) + " gx only")
    gc = torch.full(p.coeffs.shape, float("nan"), device="cuda")
    rsm.run_adjoint(p, dev(x), dev(gy), None, gc, dev(p.coeffs))
    check_close(host(gc), a.gc, a.gc_abs, what=str(case) + " gc only")


def test_column_adjoint_keeps_other_windows_out():
    # infinities in dL/dy of one window must reach only the input columns
    # of that window
    p, x = _col_adj_stage((1, 4, 96), 6, 8, 2, 1, None, seed=680)
    gy = W.rng_for(681).uniform(-1, 1, p.output.array_shape).astype(np.float32)
    gy[0, 1, 2 * 5:2 * 5 + 2] = np.inf      # window 5 of row 1: columns 41 .. 46
    a = oracle.adjoint(p, x, gy)
    gx = torch.full(p.inputs[0].array_shape, float("nan"), device="cuda")
    rsm.run_adjoint(p, dev(x), dev(gy), gx, None, dev(p.coeffs))
    got, want = host(gx), a.gx
    assert np.array_equal(np.isinf(got), np.isinf(want)) and np.array_equal(np.isnan(got), np.isnan(want))
    fin = np.isfinite(want)
    assert fin.sum() > 0.9 * fin.size
    check_close(np.where(fin, got, 0), np.where(fin, want, 0), np.where(fin, a.gx_abs, 0),
                what="finite columns")


def test_polyphase_sum_task_rejected():
    p, x = _stage((1, 8, 64), 13, 8, 3, -2, 2, seed=2)
    ps = W.Problem(p.rep_shape, p.inputs, p.output, W.SUM)
    with pytest.raises(rsm.RsmError) as e:
        rsm.run(ps, [dev(x)], torch.empty(p.output.array_shape, device="cuda"))
    assert e.value.name == "RSM_E_SHAPE"


def _abs_problem(p):
    return W.Problem(p.rep_shape, p.inputs, p.output, p.task, np.abs(p.coeffs))


def test_polyphase_downscaler_full_size():
    say("polyphase downscaler 30 x 1080 x 1920")
    pp = W.polyphase_downscaler()
    x = dev(pp.x)
    ch, cv = dev(pp.c_h), dev(pp.c_v)
    mid = torch.full(pp.h.output.array_shape, float("nan"), device="cuda")
    out = torch.full(pp.v.output.array_shape, float("nan"), device="cuda")
    rsm.run(pp.h, [x], mid, coeffs=ch)
    rsm.run(pp.v, [mid], out, coeffs=cv)
    ref_h = oracle.run(pp.h, [pp.x])
    check_close(host(mid), ref_h.out, ref_h.abs_sum, what="full H")
    mid_h = host(mid)
    ref_v = oracle.run(pp.v, [mid_h])
    check_close(host(out), ref_v.out, ref_v.abs_sum, what="full V (on the GPU's H output)")
    # the chain call (stage by stage through the library's workspace) gives the same bits
    out2 = torch.full(pp.v.output.array_shape, float("nan"), device="cuda")
    rsm.run_chain([pp.h, pp.v], x, out2, [ch, cv])
    assert torch.equal(out2, out)
    # adjoints of both stages at full size
    rng = W.rng_for(808)
    gv = rng.uniform(-1, 1, pp.v.output.array_shape).astype(np.float32)
    say("polyphase adjoint V")
    _adjoint_full(pp.v, mid_h, gv, "full V")
    gh = rng.uniform(-1, 1, pp.h.output.array_shape).astype(np.float32)
    say("polyphase adjoint H")
    _adjoint_full(pp.h, pp.x, gh, "full H")


def _adjoint_full(p, x, gy, what):
    a = oracle.adjoint(p, x, gy)
    gx = torch.full(p.inputs[0].array_shape, float("nan"), device="cuda")
    gc = torch.full(p.coeffs.shape, float("nan"), device="cuda")
    rsm.run_adjoint(p, dev(x), dev(gy), gx, gc, dev(p.coeffs))
    check_close(host(gx), a.gx, a.gx_abs, what=what + " gx")
    check_close(host(gc), a.gc, a.gc_abs, what=what + " gc")


def test_polyphase_chain_autograd_matches_oracle():
    # loss sum(w * out^2) of the two-stage polyphase downscaler on 2 frames,
    # through rsm.TiledChain (the library runs the stages one by one and
    # recomputes the intermediate for the backward pass)
    pp = W.polyphase_downscaler(frames=2, rows=108, cols=192)
    w = W.loss_weights(pp.v.output.array_shape, seed=9)
    x = dev(pp.x).requires_grad_(True)
    ch = dev(pp.c_h).requires_grad_(True)
    cv = dev(pp.c_v).requires_grad_(True)
    out = rsm.TiledChain.apply(x, ch, cv, [pp.h, pp.v], True)
    loss = (dev(w) * out * out).sum()
    loss.backward()
    stages = [pp.h, pp.v]
    ref = oracle.chain_adjoint(stages, pp.x, w)
    absd = oracle.chain_adjoint([_abs_problem(s) for s in stages], np.abs(pp.x), np.abs(w))
    abs_out = oracle.chain_forward([_abs_problem(s) for s in stages], np.abs(pp.x))[-1].out
    check_close(host(out), ref.forward[-1].out, abs_out, what="chain out")
    check_close(host(x.grad), ref.gx, absd.gx, what="chain gx")
    check_close(host(ch.grad), ref.gc[0], absd.gc[0], what="chain gc_h")
    check_close(host(cv.grad), ref.gc[1], absd.gc[1], what="chain gc_v")
    # a single stage through rsm.TiledTask
    xs = dev(pp.x).requires_grad_(True)
    cs = dev(pp.c_h).requires_grad_(True)
    y = rsm.TiledTask.apply(xs, cs, pp.h)
    g = W.rng_for(10).uniform(-1, 1, pp.h.output.array_shape).astype(np.float32)
    (y * dev(g)).sum().backward()
    a = oracle.adjoint(pp.h, pp.x, g)
    check_close(host(xs.grad), a.gx, a.gx_abs, what="task gx")
    check_close(host(cs.grad), a.gc, a.gc_abs, what="task gc")


def test_polyphase_column_adjoint_rows_not_read_are_zero():
    # the column tiler reads every other row of a [1, 10, 64] array: dL/dx of
    # the rows no window reads must come out zero
    x = W.rng_for(909).standard_normal((1, 10, 64)).astype(np.float32)
    t = W.Tiler((1, 10, 64), [0, 1, -3], np.diag([1, 2, 8]), [[0], [0], [1]], (13,))
    rep = (1, 5, 8)
    c = W.phase_coeffs(W.rng_for(910), 3, 13)
    p = W.Problem(rep, [t], W.phase_output(rep, 2, 3), W.WSUM, c)
    assert rsm.plan(p, flags=_abi.PLAN_ADJOINT) == "polyphase_adjoint_cols"
    gy = W.rng_for(911).uniform(-1, 1, p.output.array_shape).astype(np.float32)
    _forward_check(p, x, 0, what="strided rows")
    _adjoint_check(p, x, gy, 0, what="strided rows")
