"""The kernel timing hook (rsm_time_next_kernel) on the GPU.

Armed events bracket the fused chain kernel of the next chain call only: a
fused call records them around its kernel, the hook is then disarmed, and an
unfused call disarms it without recording.
"""
import pytest
import torch

import rsm_workloads as W
from paper_1105_4424_amd import _abi, rsm

pytestmark = pytest.mark.gpu


def _chain():
    ts = W.two_stage_filter(frames=2, rows=64, cols=128, taps=8, seed=1)
    x = torch.from_numpy(ts.x).cuda()
    ch = torch.from_numpy(ts.c_h).cuda()
    cv = torch.from_numpy(ts.c_v).cuda()
    out = torch.empty(ts.v.rep_shape, device="cuda")
    mid = torch.empty(ts.h.rep_shape, device="cuda")
    return rsm.Chain([ts.h, ts.v], [ch, cv]), x, out, mid


def test_hook_brackets_one_fused_call():
    chain, x, out, _ = _chain()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rsm.time_next_kernel(a, b)
    chain.forward(x, out)
    torch.cuda.synchronize()
    first = a.elapsed_time(b)
    assert 0.0 < first < 100.0
    # disarmed: further calls leave the events where they are
    chain.forward(x, out)
    torch.cuda.synchronize()
    assert a.elapsed_time(b) == first


def test_unfused_call_disarms_without_recording():
    chain, x, out, mid = _chain()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rsm.time_next_kernel(a, b)           # records both once (creation), then arms
    torch.cuda.synchronize()
    before = a.elapsed_time(b)
    chain.forward(x, out, mids=[mid], flags=_abi.NO_FUSE)
    chain.forward(x, out)                # hook already disarmed by the unfused call
    torch.cuda.synchronize()
    assert a.elapsed_time(b) == before
