"""GPU parity of the adjoint kernels and the autograd wrappers.

* single stages (tap kernels and generic atomic path) against the oracle's
  adjoint on a seeded output gradient;
* the two-stage chain, fused and unfused, at full size (30 x 1080 x 1920);
* the loss sum(w * out^2) through torch autograd on the 32x32 crop against
  FP64 central differences (exact for this quadratic loss) and the oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import rsm_workloads as W
from paper_1105_4424_amd import _abi, rsm

from .helpers import check_close, dev, host, say

pytestmark = pytest.mark.gpu


def _abs_problem(p):
    return W.Problem(p.rep_shape, p.inputs, p.output, p.task,
                     None if p.coeffs is None else np.abs(p.coeffs))


def _adjoint_check(p, x, gy, flags=0, what=""):
    a = oracle.adjoint(p, x, gy)
    gx = torch.full(p.inputs[0].array_shape, float("nan"), device="cuda")
    gc = torch.full(p.inputs[0].pattern_shape, float("nan"), device="cuda") if p.task == W.WSUM else None
    rsm.run_adjoint(p, dev(x), dev(gy), gx, gc, dev(p.coeffs) if p.coeffs is not None else None,
                    flags=flags)
    check_close(host(gx), a.gx, a.gx_abs, what=what + " gx")
    if gc is not None:
        check_close(host(gc), a.gc, a.gc_abs, what=what + " gc")
        # the input gradient alone (x is not read) gives the same bits
        gx1 = torch.full(p.inputs[0].array_shape, float("nan"), device="cuda")
        rsm.run_adjoint(p, dev(x), dev(gy), gx1, None, dev(p.coeffs), flags=flags)
        assert torch.equal(gx1, gx), what + " gx without gc"
    # accumulate: adds onto the previous contents
    if gc is not None:
        gx2 = gx.clone()
        gc2 = gc.clone()
        rsm.run_adjoint(p, dev(x), dev(gy), gx2, gc2, dev(p.coeffs), flags=flags | _abi.ACCUMULATE)
        check_close(host(gx2), 2 * a.gx, 2 * a.gx_abs, what=what + " gx accumulate")
        check_close(host(gc2), 2 * a.gc, 2 * a.gc_abs, what=what + " gc accumulate")


@pytest.mark.parametrize("force_generic", [False, True])
def test_stage_adjoints_two_frames(force_generic):
    ts = W.two_stage_filter(frames=2)
    rng = W.rng_for(77)
    for st, name in ((ts.h, "h"), (ts.v, "v")):
        x = ts.x if name == "h" else oracle.run(ts.h, [ts.x]).out.astype(np.float32)
        gy = rng.uniform(-1, 1, st.rep_shape).astype(np.float32)
        say("adjoint", name, "generic" if force_generic else "fir")
        _adjoint_check(st, x, gy, _abi.FORCE_GENERIC if force_generic else 0, "stage " + name)


@pytest.mark.parametrize("taps,pave,ho,vo,rows,cols", [
    (8, 8, -3, -3, 64, 96),      # injective, wrapping: tap kernels
    (8, 8, -4, -5, 40, 64),      # 16-byte aligned windows, left border wraps: lane-pair kernel
    (8, 8, 4, 3, 40, 64),        # aligned, right border wraps
    (13, 8, -6, 0, 48, 80),      # overlapping reads: gather-form input gradient
    (5, 7, 0, -2, 31, 47),       # gaps between windows (elements never read get 0)
])
def test_stage_adjoint_variants(taps, pave, ho, vo, rows, cols):
    ts = W.two_stage_filter(frames=2, rows=rows, cols=cols, taps=taps, pave=pave, h_origin=ho,
                            v_origin=vo, seed=taps + rows)
    rng = W.rng_for(taps)
    for st, name in ((ts.h, "h"), (ts.v, "v")):
        x = ts.x if name == "h" else oracle.run(ts.h, [ts.x]).out.astype(np.float32)
        gy = rng.uniform(-1, 1, st.rep_shape).astype(np.float32)
        _adjoint_check(st, x, gy, 0, "variant %s %s" % (name, (taps, pave, ho, vo)))


def _random_window(rng):
    """A 1-D tap tiler on a 3-D array: taps along axis 1 or 2 with any step
    (overlapping, gapped or wrapping several times round the axis), the other
    two axes stepped without wrapping."""
    ax = int(rng.integers(1, 3))
    A = [int(rng.integers(1, 4)), int(rng.integers(1, 24)), int(rng.integers(1, 40))]
    T = int(rng.integers(1, 17))
    rep, o, p = [0, 0, 0], [0, 0, 0], [0, 0, 0]
    for d in range(3):
        if d == ax:
            p[d] = int(rng.integers(1, 9)) if rng.random() < 0.8 else int(rng.integers(9, 21))
            rep[d] = int(rng.integers(1, 12))
            o[d] = int(rng.integers(-30, 30))
        else:
            p[d] = int(rng.integers(1, 4))
            rep[d] = int(rng.integers(1, A[d] + 1))
            while p[d] * (rep[d] - 1) >= A[d]:
                rep[d] -= 1
            o[d] = int(rng.integers(0, A[d] - p[d] * (rep[d] - 1)))
    F = np.zeros((3, 1), np.int64)
    F[ax, 0] = 1
    t = W.Tiler(tuple(A), o, np.diag(p).astype(np.int64), F, (T,))
    c = rng.uniform(-1, 1, T).astype(np.float32)
    return W.Problem(tuple(rep), [t], W.identity_output(tuple(rep)), W.WSUM, c)


def test_gather_adjoint_random_windows():
    rng = W.rng_for(93)
    fams = {}
    for trial in range(80):
        p = _random_window(rng)
        fam = rsm.plan(p, flags=_abi.PLAN_ADJOINT)
        assert fam.startswith("fir_adjoint"), (trial, fam)
        fams[fam] = fams.get(fam, 0) + 1
        x = W.random_array(rng, p.inputs[0].array_shape)
        gy = rng.uniform(-1, 1, p.rep_shape).astype(np.float32)
        _adjoint_check(p, x, gy, 0, "window %d %s" % (trial, fam))
    say("families", fams)
    assert fams.get("fir_adjoint_gather", 0) >= 20 and fams.get("fir_adjoint_overlap_cols", 0) >= 20


# long rows: several 256-repetition chunks per row, and windows that go round
# a short row many times (every column has many lifts; the second chunk of
# each row owns no column, only repetitions)
@pytest.mark.parametrize("A,R,pave,taps,origin", [((2, 3, 5000), 700, 7, 13, -6),
                                                   ((1, 4, 3001), 300, 16, 16, 5),
                                                   ((3, 2, 50), 300, 3, 13, -7),
                                                   ((1, 1, 7), 1, 1, 16, -20)])
def test_overlap_cols_chunks_and_laps(A, R, pave, taps, origin):
    rng = W.rng_for(95 + R)
    t = W.Tiler(A, [0, 0, origin], np.diag([1, 1, pave]), [[0], [0], [1]], (taps,))
    rep = (A[0], A[1], R)
    c = rng.uniform(-1, 1, taps).astype(np.float32)
    p = W.Problem(rep, [t], W.identity_output(rep), W.WSUM, c)
    assert rsm.plan(p, flags=_abi.PLAN_ADJOINT) == "fir_adjoint_overlap_cols"
    x = W.random_array(rng, A)
    gy = rng.uniform(-1, 1, rep).astype(np.float32)
    _adjoint_check(p, x, gy, 0, "overlap cols %s R=%d p=%d T=%d o=%d" % (A, R, pave, taps, origin))


# taps along rows with whole rows of columns: the input gradient four
# columns per thread (16-byte dL/dy and dL/dx); frames the tiler skips (every
# other one), windows wrapping at both ends, one to four windows per element
@pytest.mark.parametrize("A,R,pave,taps,origin", [((4, 40, 64), 5, 8, 13, -6),
                                                   ((3, 24, 16), 6, 4, 16, -3),
                                                   ((2, 9, 12), 9, 1, 3, -1)])
def test_gather_adjoint_rows_four_columns(A, R, pave, taps, origin):
    rng = W.rng_for(97 + taps)
    rep = ((A[0] + 1) // 2, R, A[2])
    t = W.Tiler(A, [0, origin, 0], np.diag([2, pave, 1]), [[0], [1], [0]], (taps,))
    c = rng.uniform(-1, 1, taps).astype(np.float32)
    p = W.Problem(rep, [t], W.identity_output(rep), W.WSUM, c)
    assert rsm.plan(p, flags=_abi.PLAN_ADJOINT) == "fir_adjoint_gather"
    x = W.random_array(rng, A)
    gy = rng.uniform(-1, 1, rep).astype(np.float32)
    _adjoint_check(p, x, gy, 0, "rows, whole columns %s R=%d p=%d T=%d o=%d" % (A, R, pave, taps, origin))


@pytest.mark.parametrize("stage", ["h", "v"])
def test_gather_adjoint_overlapping_full_frames(stage):
    # 13 taps every 8 columns (rows), centred origin -6: windows overlap by 5
    # and wrap at both borders; 30 x 1080 x 1920
    ts = W.two_stage_filter(taps=13, pave=8, h_origin=-6, v_origin=-6)
    st = ts.h if stage == "h" else ts.v
    assert rsm.plan(st, flags=_abi.PLAN_ADJOINT) == ("fir_adjoint_overlap_cols" if stage == "h"
                                                     else "fir_adjoint_gather")
    x = ts.x if stage == "h" else oracle.run(ts.h, [ts.x]).out.astype(np.float32)
    gy = W.rng_for(94).uniform(-1, 1, st.rep_shape).astype(np.float32)
    say("oracle adjoint, overlapping", stage, x.shape)
    a = oracle.adjoint(st, x, gy)
    xd, gyd, cd = dev(x), dev(gy), dev(st.coeffs)
    runs = []
    for _ in range(2):
        gx = torch.full(x.shape, float("nan"), device="cuda")
        gc = torch.full((13,), float("nan"), device="cuda")
        rsm.run_adjoint(st, xd, gyd, gx, gc, cd)
        runs.append((gx, gc))
    check_close(host(runs[0][0]), a.gx, a.gx_abs, what="overlap %s gx" % stage)
    check_close(host(runs[0][1]), a.gc, a.gc_abs, what="overlap %s gc" % stage)
    # deterministic: no atomics anywhere on this path
    assert torch.equal(runs[0][0], runs[1][0]) and torch.equal(runs[0][1], runs[1][1])
    # input gradient alone (no weight gradient) gives the same bits
    gx1 = torch.full(x.shape, float("nan"), device="cuda")
    rsm.run_adjoint(st, xd, gyd, gx1, None, cd)
    assert torch.equal(gx1, runs[0][0])


def test_adjoint_random_tilers_generic():
    rng = W.rng_for(91)
    for trial in range(25):
        dr = int(rng.integers(1, 3))
        rep = tuple(int(v) for v in rng.integers(1, 6, dr))
        t = W.random_tiler(rng, dr, max_side=9, max_pattern_side=4)
        c = rng.uniform(-1, 1, t.pattern_shape).astype(np.float32)
        p = W.Problem(rep, [t], W.identity_output(rep), W.WSUM, c)
        x = W.random_array(rng, t.array_shape)
        gy = rng.uniform(-1, 1, rep).astype(np.float32)
        _adjoint_check(p, x, gy, 0, "random %d" % trial)


@pytest.mark.parametrize("fused", [True, False])
def test_chain_adjoint_full_size(fused):
    ts = W.two_stage_filter()
    stages = [ts.h, ts.v]
    gy = W.rng_for(12).uniform(-1, 1, ts.v.rep_shape).astype(np.float32)
    say("oracle chain adjoint, 30 frames")
    fw = oracle.chain_forward(stages, ts.x)
    av = oracle.adjoint(ts.v, fw[0].out, gy)
    ah = oracle.adjoint(ts.h, ts.x, av.gx)
    # |term| bounds through both stages: the oracle on absolute values
    abs_v = oracle.adjoint(_abs_problem(ts.v), np.abs(fw[0].out), np.abs(gy))
    abs_h = oracle.adjoint(_abs_problem(ts.h), np.abs(ts.x), abs_v.gx)
    x = dev(ts.x)
    gx = torch.full(ts.x.shape, float("nan"), device="cuda")
    gch = torch.full((8,), float("nan"), device="cuda")
    gcv = torch.full((8,), float("nan"), device="cuda")
    mids = None
    if not fused:
        mid = torch.empty(ts.h.rep_shape, device="cuda")
        rsm.run(ts.h, [x], mid, coeffs=dev(ts.c_h))
        mids = [mid]
    rsm.run_chain_adjoint(stages, x, dev(gy), gx, [gch, gcv], [dev(ts.c_h), dev(ts.c_v)], mids=mids,
                          flags=0 if fused else _abi.NO_FUSE)
    check_close(host(gx), ah.gx, abs_h.gx, what="chain gx fused=%s" % fused)
    check_close(host(gch), ah.gc, abs_h.gc, what="chain gc_h fused=%s" % fused)
    check_close(host(gcv), av.gc, abs_v.gc, what="chain gc_v fused=%s" % fused)


# (8, 8, 0): the workload's exact paving; (13, 8, -6): windows overlapping by
# five and wrapping round the 32-element crop on both axes (the adjoint then
# runs stage by stage, recomputing the intermediate when fused=True)
@pytest.mark.parametrize("taps,pave,origin", [(8, 8, 0), (13, 8, -6)])
@pytest.mark.parametrize("fused", [True, False])
def test_crop_loss_autograd_vs_finite_differences(fused, taps, pave, origin):
    """32x32 crop of frame 0 as its own [1,32,32] array; loss sum(w out^2)."""
    ts = W.two_stage_filter(frames=1, rows=32, cols=32, taps=taps, pave=pave, h_origin=origin,
                            v_origin=origin)
    w = W.loss_weights((1, 4, 4))
    stages = [ts.h, ts.v]
    x = dev(ts.x).requires_grad_(True)
    ch = dev(ts.c_h).requires_grad_(True)
    cv = dev(ts.c_v).requires_grad_(True)
    out = rsm.TiledChain.apply(x, ch, cv, stages, fused)
    loss = (dev(w) * out * out).sum()
    loss.backward()
    # FP64 central differences of the oracle forward (exact: L is quadratic in
    # every coordinate), step 2^-4
    h = 2.0 ** -4
    x64 = ts.x.astype(np.float64)
    w64 = w.astype(np.float64)

    def L(xv, chv, cvv):
        sh = W.Problem(ts.h.rep_shape, ts.h.inputs, ts.h.output, W.WSUM, chv)
        sv = W.Problem(ts.v.rep_shape, ts.v.inputs, ts.v.output, W.WSUM, cvv)
        o = oracle.chain_forward([sh, sv], xv)[-1].out
        return float(np.sum(w64 * o * o))

    ch64, cv64 = ts.c_h.astype(np.float64), ts.c_v.astype(np.float64)
    flat = x64.reshape(-1)
    fd = np.zeros_like(flat)
    for j in range(flat.size):
        xp, xm = flat.copy(), flat.copy()
        xp[j] += h
        xm[j] -= h
        fd[j] = (L(xp.reshape(x64.shape), ch64, cv64) - L(xm.reshape(x64.shape), ch64, cv64)) / (2 * h)
    fdc = []
    for which in range(2):
        g = np.zeros(taps)
        for k in range(taps):
            cp = [ch64.copy(), cv64.copy()]
            cm = [ch64.copy(), cv64.copy()]
            cp[which][k] += h
            cm[which][k] -= h
            g[k] = (L(x64, *cp) - L(x64, *cm)) / (2 * h)
        fdc.append(g)
    ref = oracle.chain_adjoint(stages, ts.x, w)
    # |term| bound: the oracle adjoint on absolute values of everything
    absd = oracle.chain_adjoint([_abs_problem(s) for s in stages], np.abs(ts.x), np.abs(w))
    gx_bound = absd.gx
    check_close(host(x.grad).reshape(-1), fd, gx_bound.reshape(-1), what="gx vs FD")
    check_close(host(x.grad), ref.gx, gx_bound, what="gx vs oracle")
    for k, g in enumerate((ch.grad, cv.grad)):
        check_close(host(g), fdc[k], absd.gc[k], what="gc[%d] vs FD" % k)
        check_close(host(g), ref.gc[k], absd.gc[k], what="gc[%d] vs oracle" % k)


def test_tiled_task_autograd_single_stage():
    ts = W.two_stage_filter(frames=2, rows=64, cols=128)
    gy = W.rng_for(5).uniform(-1, 1, ts.h.rep_shape).astype(np.float32)
    x = dev(ts.x).requires_grad_(True)
    c = dev(ts.c_h).requires_grad_(True)
    y = rsm.TiledTask.apply(x, c, ts.h)
    y.backward(dev(gy))
    a = oracle.adjoint(ts.h, ts.x, gy)
    check_close(host(x.grad), a.gx, a.gx_abs, what="TiledTask gx")
    check_close(host(c.grad), a.gc, a.gc_abs, what="TiledTask gc")


def test_chains_without_intermediate_buffers():
    # an overlapping chain (13 taps every 8, wrapping): the adjoint cannot
    # fuse, so without d_mid it recomputes the intermediate in the workspace
    ts = W.two_stage_filter(frames=3, rows=96, cols=200, taps=13, pave=8, h_origin=-6, v_origin=-6,
                            seed=21)
    stages = [ts.h, ts.v]
    gy = W.rng_for(22).uniform(-1, 1, ts.v.rep_shape).astype(np.float32)
    fw = oracle.chain_forward(stages, ts.x)
    av = oracle.adjoint(ts.v, fw[0].out, gy)
    ah = oracle.adjoint(ts.h, ts.x, av.gx)
    abs_v = oracle.adjoint(_abs_problem(ts.v), np.abs(fw[0].out), np.abs(gy))
    abs_h = oracle.adjoint(_abs_problem(ts.h), np.abs(ts.x), abs_v.gx)
    x, c = dev(ts.x), [dev(ts.c_h), dev(ts.c_v)]
    res = {}
    for name, mids, flags in (("recomputed", None, 0), ("given", "mid", _abi.NO_FUSE)):
        mid = None
        if mids:
            mid = torch.empty(ts.h.rep_shape, device="cuda")
            rsm.run(ts.h, [x], mid, coeffs=c[0])
        gx = torch.full(ts.x.shape, float("nan"), device="cuda")
        gcs = [torch.full((13,), float("nan"), device="cuda") for _ in range(2)]
        rsm.run_chain_adjoint(stages, x, dev(gy), gx, gcs, c, mids=None if mid is None else [mid], flags=flags)
        check_close(host(gx), ah.gx, abs_h.gx, what=name + " gx")
        check_close(host(gcs[0]), ah.gc, abs_h.gc, what=name + " gc_h")
        check_close(host(gcs[1]), av.gc, abs_v.gc, what=name + " gc_v")
        res[name] = (gx, gcs)
    # the same kernels on the same intermediate: the same bits
    assert torch.equal(res["recomputed"][0], res["given"][0])
    # a chain the planner cannot fuse (both stages along columns), run
    # without intermediate buffers
    t1 = W.h_stage(2, 40, 96, taps=5, pave=3, origin=-2)
    r1 = (2, 40, 32)
    t2 = W.h_stage(2, 40, 32, taps=3, pave=2, origin=0)
    r2 = (2, 40, 16)
    rng = W.rng_for(23)
    c1, c2 = rng.uniform(-1, 1, 5).astype(np.float32), rng.uniform(-1, 1, 3).astype(np.float32)
    st2 = [W.Problem(r1, [t1], W.identity_output(r1), W.WSUM, c1),
           W.Problem(r2, [t2], W.identity_output(r2), W.WSUM, c2)]
    x2 = rng.uniform(-1, 1, (2, 40, 96)).astype(np.float32)
    out = torch.full(r2, float("nan"), device="cuda")
    rsm.run_chain(st2, dev(x2), out, [dev(c1), dev(c2)])
    want = oracle.chain_forward(st2, x2)
    bound = oracle.chain_forward([_abs_problem(q) for q in st2], np.abs(x2))[-1].out
    check_close(host(out), want[-1].out, bound, what="unfusable chain without intermediates")


def test_in_kernel_reduction_gives_the_same_bits():
    # RSM_REDUCE_IN_KERNEL: the last workgroup of the launch (completion
    # counter, agent-scope ordering) sums the partial rows in the same fixed
    # order as the second kernel; three calls in a row check that the
    # counter is left at zero
    ts = W.two_stage_filter(frames=3, rows=96, cols=256, seed=31)
    x = dev(ts.x)
    c = [dev(ts.c_h), dev(ts.c_v)]
    gy = dev(W.rng_for(32).uniform(-1, 1, ts.v.rep_shape).astype(np.float32))
    gyh = dev(W.rng_for(33).uniform(-1, 1, ts.h.rep_shape).astype(np.float32))
    res = {}
    for flag in (0, _abi.REDUCE_IN_KERNEL):
        runs = []
        for _ in range(3):
            gx = torch.empty_like(x)
            gcs = [torch.empty(8, device="cuda"), torch.empty(8, device="cuda")]
            rsm.run_chain_adjoint([ts.h, ts.v], x, gy, gx, gcs, c, flags=flag)
            g1 = torch.empty_like(x)
            gc1 = torch.empty(8, device="cuda")
            rsm.run_adjoint(ts.h, x, gyh, g1, gc1, c[0], flags=flag)
            runs.append([host(t) for t in (gx, gcs[0], gcs[1], g1, gc1)])
        for r in runs[1:]:
            for a_, b_ in zip(r, runs[0]):
                assert np.array_equal(a_, b_)
        res[flag] = runs[0]
    for a_, b_ in zip(res[0], res[_abi.REDUCE_IN_KERNEL]):
        assert np.array_equal(a_, b_)


def test_deterministic_weight_gradient():
    ts = W.two_stage_filter(frames=4)
    gy = dev(W.rng_for(6).uniform(-1, 1, ts.v.rep_shape).astype(np.float32))
    x = dev(ts.x)
    res = []
    for _ in range(2):
        gch = torch.empty(8, device="cuda")
        gcv = torch.empty(8, device="cuda")
        gx = torch.empty_like(x)
        rsm.run_chain_adjoint([ts.h, ts.v], x, gy, gx, [gch, gcv], [dev(ts.c_h), dev(ts.c_v)])
        res.append((host(gx), host(gch), host(gcv)))
    for a, b in zip(res[0], res[1]):
        assert np.array_equal(a, b)


def test_calls_on_two_streams_use_separate_workspaces():
    # Unfused chain adjoints keep intermediate gradients and weight-gradient
    # partial rows in the library workspace.  Issued on two streams with no
    # ordering between them, each must give what it gives alone.
    cases = []
    for seed in (31, 32):
        ts = W.two_stage_filter(frames=4, rows=256, cols=512, seed=seed)
        x = dev(ts.x)
        chain = rsm.Chain([ts.h, ts.v], [dev(ts.c_h), dev(ts.c_v)])
        gy = dev(W.rng_for(seed).uniform(-1, 1, ts.v.rep_shape).astype(np.float32))
        cases.append((chain, x, gy))
    want = []
    for chain, x, gy in cases:
        gx = torch.empty_like(x)
        gcs = [torch.empty(8, device="cuda") for _ in range(2)]
        chain.adjoint(x, gy, gx, gcs, flags=_abi.NO_FUSE)
        want.append((gx, gcs))
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    got = []
    for (chain, x, gy), s in zip(cases, streams):
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            gx = torch.full_like(x, float("nan"))
            gcs = [torch.full((8,), float("nan"), device="cuda") for _ in range(2)]
            got.append((gx, gcs))
    for _ in range(3):
        for (chain, x, gy), s, (gx, gcs) in zip(cases, streams, got):
            chain.adjoint(x, gy, gx, gcs, flags=_abi.NO_FUSE, stream=s)
    torch.cuda.synchronize()
    for (gx, gcs), (wx, wcs) in zip(got, want):
        assert torch.equal(gx, wx)
        assert torch.equal(gcs[0], wcs[0]) and torch.equal(gcs[1], wcs[1])
