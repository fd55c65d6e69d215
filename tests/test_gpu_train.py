"""The training step (rsm_run_chain_train) against the oracle.

Loss L = sum(w * out^2) of two chained stages: the two-stage 8-tap filter
(lane-pair kernel), pairs with other tap counts, origins and gaps (the
one-thread-per-output fused kernel), and chains run stage by stage
(overlapping windows, polyphase stages).  The fused kernel
forms dL/dout = 2 (w out) in registers; the separate path forms it as
(2 w) out in torch.  Doubling is exact, and the fused kernel keeps the
arithmetic order of the fused forward and adjoint kernels, so out, dL/dx and
the weight gradients equal the separate GPU path bit for bit; against the
FP64 oracle every result is held to 1e-5 of its |term| sum (the oracle run on
absolute values of the input, weights and loss weights).
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
    return W.Problem(p.rep_shape, [W.Tiler(t.array_shape, t.origin, t.paving, t.fitting, t.pattern_shape)
                                   for t in p.inputs], p.output, p.task,
                     None if p.coeffs is None else np.abs(p.coeffs))


def _case(frames, rows, cols, seed=1, h_origin=0, v_origin=0):
    ts = W.two_stage_filter(frames=frames, rows=rows, cols=cols, taps=8, seed=seed,
                            h_origin=h_origin, v_origin=v_origin)
    w = W.loss_weights(ts.v.rep_shape)
    return ts, w


def _train(ts, w, flags=0, gx=None, gcs=None):
    x, ch, cv = dev(ts.x), dev(ts.c_h), dev(ts.c_v)
    out = torch.full(ts.v.rep_shape, float("nan"), device="cuda")
    gx = torch.full(ts.x.shape, float("nan"), device="cuda") if gx is None else gx
    gcs = [torch.full((8,), float("nan"), device="cuda") for _ in range(2)] if gcs is None else gcs
    rsm.Chain([ts.h, ts.v], [ch, cv]).train(x, dev(w), out, gx, gcs, flags=flags)
    return out, gx, gcs


def _separate(ts, w):
    x, ch, cv = dev(ts.x), dev(ts.c_h), dev(ts.c_v)
    chain = rsm.Chain([ts.h, ts.v], [ch, cv])
    out = torch.empty(ts.v.rep_shape, device="cuda")
    chain.forward(x, out)
    gy = (2.0 * dev(w)) * out
    gx = torch.empty_like(x)
    gcs = [torch.empty(8, device="cuda") for _ in range(2)]
    chain.adjoint(x, gy, gx, gcs)
    return out, gx, gcs


def _check_oracle(ts, w, out, gx, gcs, what):
    stages = [ts.h, ts.v]
    ref = oracle.chain_adjoint(stages, ts.x, w)
    absd = oracle.chain_adjoint([_abs_problem(s) for s in stages], np.abs(ts.x), np.abs(w))
    abs_out = oracle.chain_forward([_abs_problem(s) for s in stages], np.abs(ts.x))[-1].out
    check_close(host(out), ref.forward[-1].out, abs_out, what=what + " out")
    check_close(host(gx), ref.gx, absd.gx, what=what + " gx")
    check_close(host(gcs[0]), ref.gc[0], absd.gc[0], what=what + " gc_h")
    check_close(host(gcs[1]), ref.gc[1], absd.gc[1], what=what + " gc_v")


def test_train_full_size_matches_oracle_and_separate_path():
    ts, w = _case(30, 1080, 1920)
    out, gx, gcs = _train(ts, w)
    _check_oracle(ts, w, out, gx, gcs, "full")
    so, sgx, sgcs = _separate(ts, w)
    assert torch.equal(out, so)
    assert torch.equal(gx, sgx)
    assert torch.equal(gcs[0], sgcs[0]) and torch.equal(gcs[1], sgcs[1])


# origins -4 (columns, keeps 16-byte window starts) and -5 (rows) make the
# windows wrap at the borders
@pytest.mark.parametrize("h_origin,v_origin,rows,cols", [(0, 0, 64, 128), (-4, 0, 64, 136),
                                                          (0, -5, 72, 128), (-4, -5, 80, 200)])
def test_train_wrapping_and_ragged(h_origin, v_origin, rows, cols):
    ts, w = _case(2, rows, cols, seed=11, h_origin=h_origin, v_origin=v_origin)
    out, gx, gcs = _train(ts, w)
    _check_oracle(ts, w, out, gx, gcs, "o=(%d,%d) %dx%d" % (h_origin, v_origin, rows, cols))


def test_train_accumulate_and_optional_outputs():
    ts, w = _case(2, 64, 128, seed=12)
    out, gx, gcs = _train(ts, w)
    out2, gx2, gcs2 = _train(ts, w, flags=_abi.ACCUMULATE, gx=gx.clone(), gcs=[g.clone() for g in gcs])
    assert torch.equal(out2, out)
    assert torch.allclose(gx2, 2 * gx, rtol=0, atol=0)
    assert torch.allclose(gcs2[0], 2 * gcs[0], rtol=1e-6, atol=0)
    # without dL/dx and weight gradients only the forward output is written
    x = dev(ts.x)
    out3 = torch.empty(ts.v.rep_shape, device="cuda")
    rsm.Chain([ts.h, ts.v], [dev(ts.c_h), dev(ts.c_v)]).train(x, dev(w), out3, None, None)
    assert torch.equal(out3, out)


# chains the single-pass kernels do not take as lane pairs: any tap count,
# windows off 16-byte boundaries, gaps between windows (one thread per
# output, still one pass over x); and chains they cannot fuse at all
# (overlapping windows, multi-element output patterns), which run stage by
# stage through the workspace
GENERAL = [
    # (taps, pave, h_origin, v_origin, rows, cols)
    (5, 5, 0, 0, 40, 120),
    (8, 8, -3, 0, 64, 128),
    (6, 8, 2, -1, 48, 96),
    (16, 16, -5, 7, 64, 160),
    (13, 8, -6, -6, 72, 200),     # overlapping windows: stage by stage
]


def _general_case(taps, pave, ho, vo, rows, cols, seed):
    ts = W.two_stage_filter(frames=2, rows=rows, cols=cols, taps=taps, seed=seed, h_origin=ho,
                            v_origin=vo, pave=pave)
    w = W.loss_weights(ts.v.rep_shape)
    return ts, w


def _train_n(ts, w, taps, flags=0):
    x, ch, cv = dev(ts.x), dev(ts.c_h), dev(ts.c_v)
    out = torch.full(ts.v.rep_shape, float("nan"), device="cuda")
    gx = torch.full(ts.x.shape, float("nan"), device="cuda")
    gcs = [torch.full((taps,), float("nan"), device="cuda") for _ in range(2)]
    rsm.Chain([ts.h, ts.v], [ch, cv]).train(x, dev(w), out, gx, gcs, flags=flags)
    return out, gx, gcs


def _separate_n(ts, w, taps):
    x, ch, cv = dev(ts.x), dev(ts.c_h), dev(ts.c_v)
    chain = rsm.Chain([ts.h, ts.v], [ch, cv])
    out = torch.empty(ts.v.rep_shape, device="cuda")
    chain.forward(x, out)
    gy = (2.0 * dev(w)) * out
    gx = torch.empty_like(x)
    gcs = [torch.empty(taps, device="cuda") for _ in range(2)]
    chain.adjoint(x, gy, gx, gcs)
    return out, gx, gcs


@pytest.mark.parametrize("case", GENERAL, ids=[str(c[:4]) for c in GENERAL])
def test_train_general_pairs(case):
    taps, pave, ho, vo, rows, cols = case
    ts, w = _general_case(taps, pave, ho, vo, rows, cols, seed=40 + taps)
    out, gx, gcs = _train_n(ts, w, taps)
    _check_oracle(ts, w, out, gx, gcs, str(case))
    # the same kernels as the separate forward, 2 w y and adjoint calls
    so, sgx, sgcs = _separate_n(ts, w, taps)
    assert torch.equal(out, so)
    assert torch.equal(gx, sgx)
    assert torch.equal(gcs[0], sgcs[0]) and torch.equal(gcs[1], sgcs[1])
    # accumulate adds onto the previous gradients
    out2 = torch.empty_like(out)
    gx2, gc2 = gx.clone(), [g.clone() for g in gcs]
    rsm.Chain([ts.h, ts.v], [dev(ts.c_h), dev(ts.c_v)]).train(dev(ts.x), dev(w), out2, gx2, gc2,
                                                              flags=_abi.ACCUMULATE)
    assert torch.equal(out2, out)
    assert torch.equal(gx2, 2 * gx)


def test_train_forced_stage_by_stage_matches_fused():
    ts, w = _general_case(8, 8, 0, 0, 64, 128, seed=51)
    fused = _train_n(ts, w, 8)
    staged = _train_n(ts, w, 8, flags=_abi.NO_FUSE)
    _check_oracle(ts, w, *staged, "staged")
    torch.testing.assert_close(staged[0], fused[0], rtol=0, atol=1e-6)


def test_train_overlapping_pair_full_size():
    # 13 taps every 8 columns and rows, centred (origin -6): the windows
    # overlap by 5 and wrap at every border; 30 frames of 1080 x 1920
    say("training step, overlapping 13/8 pair, 30 x 1080 x 1920")
    ts2 = W.two_stage_filter(frames=30, rows=1080, cols=1920, taps=13, seed=53, h_origin=-6,
                             v_origin=-6, pave=8)
    w2 = W.loss_weights(ts2.v.rep_shape)
    out, gx, gcs = _train_n(ts2, w2, 13)
    _check_oracle(ts2, w2, out, gx, gcs, "13/8 full")


def test_train_polyphase_chain():
    # two polyphase stages (3 outputs per 13-tap window, then 4 per 14-tap
    # window): multi-element output patterns, stage by stage
    pp = W.polyphase_downscaler(frames=2, rows=108, cols=192)
    w = W.loss_weights(pp.v.output.array_shape, seed=21)
    x, ch, cv = dev(pp.x), dev(pp.c_h), dev(pp.c_v)
    out = torch.full(pp.v.output.array_shape, float("nan"), device="cuda")
    gx = torch.full(pp.x.shape, float("nan"), device="cuda")
    gcs = [torch.full(pp.c_h.shape, float("nan"), device="cuda"),
           torch.full(pp.c_v.shape, float("nan"), device="cuda")]
    rsm.Chain([pp.h, pp.v], [ch, cv]).train(x, dev(w), out, gx, gcs)
    stages = [pp.h, pp.v]
    ref = oracle.chain_adjoint(stages, pp.x, w)
    absd = oracle.chain_adjoint([_abs_problem(s) for s in stages], np.abs(pp.x), np.abs(w))
    abs_out = oracle.chain_forward([_abs_problem(s) for s in stages], np.abs(pp.x))[-1].out
    check_close(host(out), ref.forward[-1].out, abs_out, what="polyphase out")
    check_close(host(gx), ref.gx, absd.gx, what="polyphase gx")
    check_close(host(gcs[0]), ref.gc[0], absd.gc[0], what="polyphase gc_h")
    check_close(host(gcs[1]), ref.gc[1], absd.gc[1], what="polyphase gc_v")


def test_train_rejects_chains_of_other_lengths():
    ts = W.two_stage_filter(frames=1, rows=40, cols=128, seed=13)
    w = W.loss_weights(ts.h.rep_shape)
    x = dev(ts.x)
    with pytest.raises(rsm.RsmError) as e:
        rsm.Chain([ts.h], [dev(ts.c_h)]).train(x, dev(w), torch.empty(ts.h.rep_shape, device="cuda"),
                                               None, None)
    assert e.value.name == "RSM_E_UNSUPPORTED"
