"""GPU parity of the 2-D window filters and the batched persistent launch.

Instances follow the batched workload's recipe (sides log-uniform in
[32, 2048], k in {3,5,7,9}, stride in {1,2,4}, centred origin so windows wrap
on every border).  Small batches are checked whole against the oracle; the
full 512-instance batch on every tile's corners and centre and on every
border output of every instance, and the batched
launch must equal the plain launches (same kernels, same tile shapes) bit for
bit, on every graph replay.
"""
import json
import os

import numpy as np
import pytest
import torch

import oracle
import rsm_workloads as W
from paper_1105_4424_amd import rsm

from .helpers import check_close, dev, host, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("k", [3, 5, 7, 9])
@pytest.mark.parametrize("s", [1, 2, 4])
def test_filter2d_single_problem_ragged(k, s):
    rng = W.rng_for(100 * k + s)
    for H, Wd in [(37, 53), (130, 67), (17, 200)]:
        c = (rng.uniform(-1, 1, (k, k)) / (k * k)).astype(np.float32)
        p = W.filter2d_problem(H, Wd, k, s, c)
        assert rsm.plan(p) == "filter2d_k%d_s%d" % (k, s)
        x = rng.standard_normal((H, Wd)).astype(np.float32)
        out = torch.full(p.rep_shape, float("nan"), device="cuda")
        rsm.run(p, [dev(x)], out, coeffs=dev(c))
        r = oracle.run(p, [x])
        check_close(host(out), r.out, r.abs_sum, what="k%d s%d %dx%d" % (k, s, H, Wd))


def test_filter2d_frames_and_origin():
    # three frames, an off-centre origin and a tiny array the window wraps several times
    rng = W.rng_for(7)
    for (F, H, Wd, k, s, o) in [(3, 45, 70, 5, 2, (-7, 3)), (2, 4, 5, 9, 1, (-4, -4))]:
        c = rng.uniform(-1, 1, (k, k)).astype(np.float32)
        rep = (F, -(-H // s), -(-Wd // s))
        t = W.Tiler((F, H, Wd), [0, o[0], o[1]], np.diag([1, s, s]),
                    [[0, 0], [1, 0], [0, 1]], (k, k))
        p = W.Problem(rep, [t], W.identity_output(rep), W.WSUM, c)
        assert rsm.plan(p).startswith("filter2d")
        x = rng.standard_normal((F, H, Wd)).astype(np.float32)
        out = torch.full(rep, float("nan"), device="cuda")
        rsm.run(p, [dev(x)], out, coeffs=dev(c))
        r = oracle.run(p, [x])
        check_close(host(out), r.out, r.abs_sum, what="frames %s" % ((F, H, Wd, k, s, o),))


def _make_batch(insts, tune_cache=None):
    xs = [dev(i.x) for i in insts]
    cs = [dev(i.coeffs) for i in insts]
    outs = [torch.full(i.out_shape, float("nan"), device="cuda") for i in insts]
    probs = [i.problem() for i in insts]
    b = rsm.Batch(probs, xs, outs, cs, tune_cache=tune_cache)
    return b, probs, xs, outs


def test_small_batch_whole_against_oracle(tmp_path):
    insts = W.filter_batch(24, seed=11, side_hi=300)
    b, probs, xs, outs = _make_batch(insts, tune_cache=str(tmp_path / "tune.json"))
    info = b.info()
    assert info["n_persistent"] == 24 and info["tuned_classes"] > 0
    b.run()
    for j, inst in enumerate(insts):
        r = oracle.run(probs[j], [inst.x])
        check_close(host(outs[j]), r.out, r.abs_sum, what="batched instance %d" % j)
    batched = [host(o).copy() for o in outs]
    for o in outs:
        o.fill_(float("nan"))
    b.run_plain()
    for j in range(len(insts)):
        assert np.array_equal(host(outs[j]), batched[j]), j
    b.close()


def test_tuning_cache_round_trip(tmp_path):
    path = str(tmp_path / "tune.json")
    insts = W.filter_batch(12, seed=5, side_hi=200)
    b1, _, _, _ = _make_batch(insts, tune_cache=path)
    i1 = b1.info()
    b1.close()
    doc = json.load(open(path))
    assert doc["arch"].startswith("gfx9") and len(doc["choices"]) == i1["tuned_classes"]
    b2, _, _, _ = _make_batch(insts, tune_cache=path)
    i2 = b2.info()
    assert i2["tuned_classes"] == 0 and i2["cached_classes"] == i1["tuned_classes"]
    tiles1 = [b2.tile(k) for k in range(len(insts))]
    b2.close()
    # a corrupt cache is ignored and rewritten
    open(path, "w").write("{not json")
    b3, _, _, _ = _make_batch(insts, tune_cache=path)
    assert b3.info()["tuned_classes"] == i1["tuned_classes"]
    assert all(t[0] > 0 and t[1] > 0 for t in tiles1)
    b3.close()
    json.load(open(path))


def _tile_samples(out_shape, tile):
    """Flat output indices: the four corners and the centre of every tile of
    the problem's tiling (tile = (rows, cols) of outputs per tile), plus the
    whole first and last output row and column (whose windows wrap)."""
    R, C = out_shape
    tr, tc = tile
    assert tr > 0 and tc > 0
    r0 = np.arange(0, R, tr)
    c0 = np.arange(0, C, tc)
    r1 = np.minimum(r0 + tr, R) - 1
    c1 = np.minimum(c0 + tc, C) - 1
    rm, cm = (r0 + r1) // 2, (c0 + c1) // 2
    pts = []
    for rr, cc in ((r0, c0), (r0, c1), (r1, c0), (r1, c1), (rm, cm)):
        pts.append((rr[:, None] * C + cc[None, :]).reshape(-1))
    pts += [np.arange(C), (R - 1) * C + np.arange(C), np.arange(R) * C, np.arange(R) * C + C - 1]
    return np.unique(np.concatenate(pts))


def test_full_batch_stratified_and_replays_bit_identical():
    say("generating 512 instances")
    insts = W.filter_batch(512)
    b, probs, xs, outs = _make_batch(insts)
    info = b.info()
    say("batch info", info)
    assert info["n_persistent"] == 512
    b.run()
    torch.cuda.synchronize()
    first = [host(o).copy() for o in outs]
    say("stratified oracle check: every tile's corners and centre, every border output")
    n_checked = 0
    for j, inst in enumerate(insts):
        sel = _tile_samples(inst.out_shape, b.tile(j))
        y, ya = oracle.run_sample(probs[j], [inst.x], sel)
        check_close(first[j].reshape(-1)[sel], y[:, 0], ya[:, 0], what="instance %d" % j)
        assert np.all(np.isfinite(first[j])), j
        n_checked += sel.size
    say("%d outputs checked against the oracle" % n_checked)
    # graph replays, with eager work in between, reproduce the first result bit for bit
    for rep in range(3):
        for o in outs:
            o.zero_()
        torch.cuda.synchronize()
        b.run()
        torch.cuda.synchronize()
        for j in range(len(insts)):
            assert np.array_equal(host(outs[j]), first[j]), (rep, j)
    # plain launches with the same tile shapes agree bit for bit
    for o in outs:
        o.fill_(float("nan"))
    b.run_plain()
    torch.cuda.synchronize()
    for j in range(len(insts)):
        assert np.array_equal(host(outs[j]), first[j]), ("plain", j)
    b.close()
