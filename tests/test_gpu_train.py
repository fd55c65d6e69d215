"""The fused training step (rsm_run_chain_train) against the oracle.

Loss L = sum(w * out^2) of the two-stage 8-tap filter.  The fused kernel
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

from .helpers import check_close, dev, host

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


@pytest.mark.parametrize("taps,h_origin", [(5, 0), (8, -3)])
def test_train_rejects_unsupported_chain(taps, h_origin):
    # 5 taps per stage; 8 taps whose windows start off 16-byte boundaries
    ts = W.two_stage_filter(frames=1, rows=40, cols=120, taps=taps, seed=13, h_origin=h_origin)
    w = W.loss_weights(ts.v.rep_shape)
    with pytest.raises(rsm.RsmError) as e:
        _train(ts, w)
    assert e.value.name == "RSM_E_UNSUPPORTED"
