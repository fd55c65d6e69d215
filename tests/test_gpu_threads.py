"""Calls from several host threads at once, each on its own stream (the
library keeps one workspace per stream and its kept plans per thread):
every thread's results equal the same calls made one after another on one
stream, bit for bit, and match the oracle."""
import threading

import numpy as np
import pytest
import torch

import oracle
import rsm_workloads as W
from paper_1105_4424_amd import rsm

from .helpers import check_close, dev, host, say

pytestmark = pytest.mark.gpu


def _work(ts, x, c, gy, stream, n):
    """n rounds of forward + adjoint of one stage (the adjoint's weight
    gradient goes through the stream's workspace); the last round's results."""
    out = torch.empty(ts.h.rep_shape, device="cuda")
    gx = torch.empty_like(x)
    gc = torch.empty(8, device="cuda")
    with torch.cuda.stream(stream):
        for _ in range(n):
            rsm.run(ts.h, [x], out, coeffs=c, stream=stream)
            rsm.run_adjoint(ts.h, x, gy, gx, gc, c, stream=stream)
    stream.synchronize()
    return out, gx, gc


def test_threads_on_own_streams_match_serial_calls():
    cases = []
    for k in range(3):
        # different shapes and origins: the threads plan different descriptors
        ts = W.two_stage_filter(frames=2, rows=32 + 8 * k, cols=128 + 64 * k, taps=8, seed=90 + k,
                                h_origin=-4 * k)
        gy = W.rng_for(95 + k).uniform(-1, 1, ts.h.rep_shape).astype(np.float32)
        cases.append((ts, dev(ts.x), dev(ts.c_h), dev(gy), gy))
    torch.cuda.synchronize()
    serial = [_work(ts, x, c, g, torch.cuda.current_stream(), 1) for ts, x, c, g, _ in cases]
    streams = [torch.cuda.Stream() for _ in cases]
    results = [None] * len(cases)
    errors = []

    def body(i):
        try:
            ts, x, c, g, _ = cases[i]
            results[i] = _work(ts, x, c, g, streams[i], 20)
        except Exception as e:   # reported below, in the main thread
            errors.append(repr(e))

    say("3 threads, 20 rounds each")
    th = [threading.Thread(target=body, args=(i,)) for i in range(len(cases))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    assert not errors, errors
    for i, (ts, x, c, g, gy) in enumerate(cases):
        for a, b in zip(results[i], serial[i]):
            assert torch.equal(a, b), i
        ref = oracle.run(ts.h, [ts.x])
        check_close(host(results[i][0]), ref.out, ref.abs_sum, what="thread %d forward" % i)
        adj = oracle.adjoint(ts.h, ts.x, gy)
        check_close(host(results[i][1]), adj.gx, adj.gx_abs, what="thread %d gx" % i)
        check_close(host(results[i][2]), adj.gc, adj.gc_abs, what="thread %d gc" % i)
