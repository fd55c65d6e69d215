"""GPU parity of the two-stage downscaler filter (tap kernels and the fused chain).

Full-size case: 30 frames of 1080x1920, 8-tap horizontal then 8-tap
vertical weighted sums, paving 8 (exact cover); the oracle evaluates it whole.
Variants exercise the modular wrap (centred origin, 13 overlapping taps) and
ragged shapes that leave the vector path.
"""
import numpy as np
import pytest
import torch

import oracle
import rsm_workloads as W
from paper_1105_4424_amd import _abi, rsm

from .helpers import check_close, dev, host, say

pytestmark = pytest.mark.gpu


def _abs_chain(stages, x):
    """|term| bound of the composed stages: the oracle on |x| and |c|."""
    ab = [W.Problem(s.rep_shape, s.inputs, s.output, s.task, np.abs(s.coeffs)) for s in stages]
    return oracle.chain_forward(ab, np.abs(x))


def _stage_check(ts, frames_label):
    for st, name in ((ts.h, "h"), (ts.v, "v")):
        x = ts.x if name == "h" else oracle.run(ts.h, [ts.x]).out.astype(np.float32)
        c = st.coeffs
        out = torch.full(st.rep_shape, float("nan"), device="cuda")
        rsm.run(st, [dev(x)], out, coeffs=dev(c))
        r = oracle.run(st, [x])
        say(frames_label, name, rsm.plan(st))
        check_close(host(out), r.out, r.abs_sum, what="%s stage %s" % (frames_label, name))


def test_stages_reduced_frames():
    _stage_check(W.two_stage_filter(frames=2), "2 frames")


@pytest.mark.parametrize("fused", [True, False])
def test_chain_full_size(fused):
    ts = W.two_stage_filter()          # 30 x 1080 x 1920
    say("oracle chain, 30 frames")
    fw = oracle.chain_forward([ts.h, ts.v], ts.x)
    bound = _abs_chain([ts.h, ts.v], ts.x)
    x = dev(ts.x)
    out = torch.full(ts.v.rep_shape, float("nan"), device="cuda")
    mids = None
    if not fused:
        mids = [torch.full(ts.h.rep_shape, float("nan"), device="cuda")]
    rsm.run_chain([ts.h, ts.v], x, out, [dev(ts.c_h), dev(ts.c_v)], mids=mids,
                  flags=0 if fused else _abi.NO_FUSE)
    if not fused:
        check_close(host(mids[0]), fw[0].out, fw[0].abs_sum, what="mid")
    check_close(host(out), fw[1].out, bound[1].out, what="chain fused=%s" % fused)


@pytest.mark.parametrize("taps,pave,ho,vo,rows,cols", [
    (8, 8, -3, -3, 64, 96),       # centred taps: windows wrap at both borders
    (8, 8, -4, -5, 40, 64),       # 16-byte aligned windows (lane-pair kernels), left border wraps
    (8, 8, 4, 3, 40, 64),         # aligned, right border wraps
    (13, 8, -6, 0, 48, 80),       # overlapping taps with wrap
    (8, 8, 0, 0, 40, 52),         # ragged: 52 columns (not a multiple of 8 after paving -> 7 cols)
    (4, 4, 2, 1, 33, 68),         # origin not a multiple of 4: scalar path
    (5, 3, 0, -2, 31, 47),        # taps > paving, odd sizes
])
def test_stage_variants(taps, pave, ho, vo, rows, cols):
    ts = W.two_stage_filter(frames=3, rows=rows, cols=cols, taps=taps, pave=pave,
                            h_origin=ho, v_origin=vo, seed=taps * 100 + cols)
    _stage_check(ts, "variant %s" % ((taps, pave, ho, vo, rows, cols),))
    fw = oracle.chain_forward([ts.h, ts.v], ts.x)
    bound = _abs_chain([ts.h, ts.v], ts.x)
    for flags in (0, _abi.NO_FUSE, _abi.FORCE_GENERIC):
        out = torch.full(ts.v.rep_shape, float("nan"), device="cuda")
        mids = None if flags == 0 else [torch.empty(ts.h.rep_shape, device="cuda")]
        rsm.run_chain([ts.h, ts.v], dev(ts.x), out, [dev(ts.c_h), dev(ts.c_v)], mids=mids, flags=flags)
        check_close(host(out), fw[1].out, bound[1].out, what="chain flags=%d" % flags)


def test_generic_and_fir_agree_full_frame():
    ts = W.two_stage_filter(frames=1)
    a = torch.empty(ts.h.rep_shape, device="cuda")
    b = torch.empty(ts.h.rep_shape, device="cuda")
    rsm.run(ts.h, [dev(ts.x)], a, coeffs=dev(ts.c_h))
    rsm.run(ts.h, [dev(ts.x)], b, coeffs=dev(ts.c_h), flags=_abi.FORCE_GENERIC)
    r = oracle.run(ts.h, [ts.x])
    check_close(host(a), r.out, r.abs_sum, what="fir")
    check_close(host(b), r.out, r.abs_sum, what="generic")


def test_misaligned_input_leaves_vector_path():
    # an input that starts 4 bytes into an allocation is not 16-byte aligned
    ts = W.two_stage_filter(frames=1, rows=16, cols=64)
    base = torch.zeros(ts.x.size + 1, device="cuda")
    base[1:] = dev(ts.x).reshape(-1)
    x = base[1:].view(ts.x.shape)
    out = torch.empty(ts.h.rep_shape, device="cuda")
    rsm.run(ts.h, [x], out, coeffs=dev(ts.c_h))
    r = oracle.run(ts.h, [ts.x])
    check_close(host(out), r.out, r.abs_sum, what="misaligned")
