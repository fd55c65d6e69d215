"""GPU parity: index tables, the generic gather kernel and small patterns.

Every expected value comes from the CPU oracle on the same seeded inputs.
Index tables and COPY are compared bit for bit; FP32 reductions within
1e-5 of the |term| sum (helpers.check_close).
"""
import numpy as np
import pytest
import torch

import oracle
import rsm_workloads as W
from paper_1105_4424_amd import _abi, rsm

from .helpers import bf16_dev, check_close, dev, host, say

pytestmark = pytest.mark.gpu


def _rep(rng, lo=0, hi=3, side=5):
    dr = int(rng.integers(lo, hi + 1))
    return tuple(int(v) for v in rng.integers(1, side + 1, dr))


# ---------------------------------------------------------------------------
# index generation: bit-exact
# ---------------------------------------------------------------------------

def test_indices_bit_exact_random_tilers():
    rng = W.rng_for(31)
    for trial in range(150):
        rep = _rep(rng)
        t = W.random_tiler(rng, len(rep), max_side=9, max_origin=40)
        got = host(rsm.indices(rep, t))
        assert np.array_equal(got, oracle.indices(rep, t)), (trial, rep, t)


def test_indices_bit_exact_workload_tilers():
    x, p = W.small_sum()
    assert np.array_equal(host(rsm.indices(p.rep_shape, p.inputs[0])),
                          oracle.indices(p.rep_shape, p.inputs[0]))
    # full-resolution frames, 2 of them: 4.1 M indices per stage table
    ts = W.two_stage_filter(frames=2, rows=1080, cols=1920)
    for st in (ts.h, ts.v):
        say("indices", st.rep_shape)
        assert np.array_equal(host(rsm.indices(st.rep_shape, st.inputs[0])),
                              oracle.indices(st.rep_shape, st.inputs[0]))
    # centred windows with wrap on every border
    f = W.filter2d_problem(37, 53, 7, 2)
    assert np.array_equal(host(rsm.indices(f.rep_shape, f.inputs[0])),
                          oracle.indices(f.rep_shape, f.inputs[0]))


def test_indices_rank8_and_scalar_pattern():
    rng = W.rng_for(8)
    for trial in range(20):
        rep = tuple(int(v) for v in rng.integers(1, 3, 5))
        t = W.random_tiler(rng, 5, max_rank=8, max_side=3, pattern_rank=int(rng.integers(0, 4)),
                           max_pattern_side=2)
        assert np.array_equal(host(rsm.indices(rep, t)), oracle.indices(rep, t)), trial


# ---------------------------------------------------------------------------
# COPY: bit-exact gather and scatter
# ---------------------------------------------------------------------------

def _stacked_output(rep, pattern):
    """B[r..., i...] = y(r)[i]: array shape rep + pattern."""
    dr, dp = len(rep), len(pattern)
    P = np.zeros((dr + dp, dr), np.int64)
    F = np.zeros((dr + dp, dp), np.int64)
    P[:dr, :dr] = np.eye(dr, dtype=np.int64)
    F[dr:, :] = np.eye(dp, dtype=np.int64)
    return W.Tiler(tuple(rep) + tuple(pattern), np.zeros(dr + dp), P, F, tuple(pattern))


@pytest.mark.parametrize("dtype", [np.float32, np.float64, np.int64, "bf16"])
def test_copy_bit_exact_random_tilers(dtype):
    rng = W.rng_for(41)
    for trial in range(40):
        rep = _rep(rng, lo=1)
        t = W.random_tiler(rng, len(rep), max_side=9, max_origin=30)
        out_t = _stacked_output(rep, t.pattern_shape)
        p = W.Problem(rep, [t], out_t, W.COPY)
        if dtype == "bf16":
            bits = rng.integers(0, 1 << 16, t.array_shape).astype(np.uint16)
            out = torch.zeros(out_t.array_shape, dtype=torch.bfloat16, device="cuda")
            rsm.run(p, [bf16_dev(bits)], out)
            got = host(out.view(torch.int16)).view(np.uint16)
            want = bits.reshape(-1)[oracle.indices(rep, t).reshape(-1)].reshape(out_t.array_shape)
            assert np.array_equal(got, want), trial
            continue
        if dtype == np.int64:
            x = rng.integers(-(1 << 62), 1 << 62, t.array_shape, dtype=np.int64)
        else:
            x = rng.standard_normal(t.array_shape).astype(dtype)
        out = torch.zeros(out_t.array_shape, dtype=dev(x).dtype, device="cuda")
        rsm.run(p, [dev(x)], out)
        if dtype == np.int64:
            want = x.reshape(-1)[oracle.indices(rep, t).reshape(-1)].reshape(out_t.array_shape)
            assert np.array_equal(host(out), want), trial
        else:
            r = oracle.run(p, [x])
            assert np.all(r.hits == 1)
            assert np.array_equal(host(out).astype(np.float64), r.out), trial


def test_indices_beyond_2_31():
    # an array of 2^31 + 8191 FP32 elements (8.6 GB) holding x[i] = i mod 65536,
    # so every expected value follows from the tiler definition itself; the
    # tilers wrap past the end of the array (64-bit index path)
    N = (1 << 31) + 8191
    x = (torch.arange(N, dtype=torch.int64, device="cuda") % 65536).to(torch.float32)
    torch.cuda.synchronize()
    R = 1000
    o = N - 3000
    # COPY of every 7th element from 3000 before the end, wrapping round
    tc = W.Tiler((N,), [o], [[7]], np.zeros((1, 0)), ())
    pc = W.Problem((R,), [tc], W.identity_output((R,)), W.COPY)
    want_idx = (o + 7 * np.arange(R, dtype=np.int64)) % N
    out = torch.full((R,), -1.0, device="cuda")
    rsm.run(pc, [x], out)
    assert np.array_equal(host(out), (want_idx % 65536).astype(np.float32))
    idx = rsm.indices(pc.rep_shape, tc)
    assert np.array_equal(host(idx)[:, 0], want_idx)
    # SUM of three elements 10^9 apart from each repetition's start
    ts = W.Tiler((N,), [o], [[7]], [[10 ** 9]], (3,))
    ps = W.Problem((R,), [ts], W.identity_output((R,)), W.SUM)
    assert rsm.plan(ps) in ("generic", "pattern_reduce")
    out = torch.full((R,), -1.0, device="cuda")
    rsm.run(ps, [x], out)
    e = (o + 7 * np.arange(R, dtype=np.int64)[:, None] + 10 ** 9 * np.arange(3)[None, :]) % N
    want = (e % 65536).astype(np.float64).sum(1)
    assert np.array_equal(host(out).astype(np.float64), want)   # integers below 2^24: exact
    del x
    torch.cuda.empty_cache()


def test_uncovered_output_elements_untouched():
    x = np.arange(6, dtype=np.float32)
    tin = W.Tiler((6,), [0], [[1]], np.zeros((1, 0)), ())
    tout = W.Tiler((12,), [1], [[2]], np.zeros((1, 0)), ())
    p = W.Problem((6,), [tin], tout, W.COPY)
    out = torch.full((12,), -7.0, device="cuda")
    rsm.run(p, [dev(x)], out)
    want = oracle.run(p, [x], prior=np.full(12, -7.0)).out
    assert np.array_equal(host(out).astype(np.float64), want)


def test_empty_repetition_space():
    t = W.Tiler((8,), [0], [[1]], [[1]], (2,))
    p = W.Problem((0,), [t], W.Tiler((3,), [0], [[1]], np.zeros((1, 0)), ()), W.SUM)
    out = torch.full((3,), 5.0, device="cuda")
    rsm.run(p, [dev(np.ones(8, np.float32))], out)
    torch.cuda.synchronize()
    assert host(out).tolist() == [5.0, 5.0, 5.0]


# ---------------------------------------------------------------------------
# reductions on random tilers (generic kernel and small-pattern kernel)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind", [W.SUM, W.WSUM])
@pytest.mark.parametrize("force_generic", [False, True])
def test_sum_wsum_random_tilers(kind, force_generic):
    rng = W.rng_for(51 + kind + 10 * force_generic)
    for trial in range(40):
        rep = _rep(rng, lo=1, side=6)
        t = W.random_tiler(rng, len(rep), max_side=9, max_origin=30, max_pattern_side=6)
        c = rng.uniform(-1, 1, t.pattern_shape).astype(np.float32)
        p = W.Problem(rep, [t], W.identity_output(rep), kind, c if kind == W.WSUM else None)
        x = W.random_array(rng, t.array_shape)
        out = torch.full(rep, float("nan"), device="cuda")
        rsm.run(p, [dev(x)], out, coeffs=dev(c) if kind == W.WSUM else None,
                flags=_abi.FORCE_GENERIC if force_generic else 0)
        r = oracle.run(p, [x])
        check_close(host(out), r.out, r.abs_sum, what="trial %d" % trial)


def _scattered_output(rng, rep):
    """A single-assignment output tiler that is not the identity: each
    repetition axis goes to a different array axis (a random permutation),
    with a random stride s >= 1 and direction and a random origin, on an
    array s times longer along that axis (modular), so the strided writes
    are distinct and the elements between them are never written."""
    d = len(rep)
    perm = rng.permutation(d)
    stride = rng.integers(1, 4, d)
    sign = rng.choice([-1, 1], d)
    shape = tuple(int(stride[k] * rep[perm[k]]) for k in range(d))
    P = np.zeros((d, d), np.int64)
    for k in range(d):
        P[k, perm[k]] = sign[k] * stride[k]
    origin = [int(rng.integers(-20, 20)) for _ in range(d)]
    return W.Tiler(shape, origin, P, np.zeros((d, 0), np.int64), ())


@pytest.mark.parametrize("kind", [W.SUM, W.WSUM])
def test_sum_wsum_scattered_outputs(kind):
    # reductions written through permuted, strided, reversed output tilers:
    # covered elements match the oracle, the others keep their prior value
    rng = W.rng_for(57 + kind)
    for trial in range(30):
        rep = _rep(rng, lo=1, side=6)
        t = W.random_tiler(rng, len(rep), max_side=9, max_origin=30, max_pattern_side=5)
        out_t = _scattered_output(rng, rep)
        c = rng.uniform(-1, 1, t.pattern_shape).astype(np.float32)
        p = W.Problem(rep, [t], out_t, kind, c if kind == W.WSUM else None)
        x = W.random_array(rng, t.array_shape)
        prior = np.full(out_t.array_shape, -7.0, np.float32)
        out = dev(prior)
        rsm.run(p, [dev(x)], out, coeffs=dev(c) if kind == W.WSUM else None)
        r = oracle.run(p, [x], prior=prior)
        assert np.all(r.hits <= 1)
        got = host(out)
        cov = r.hits == 1
        assert np.all(got[~cov] == -7.0), trial
        check_close(got[cov], r.out[cov], r.abs_sum[cov], what="trial %d" % trial)


def test_adjoint_scattered_outputs():
    # the adjoint reads dL/dy through the same non-identity output tiler
    rng = W.rng_for(59)
    for trial in range(20):
        rep = _rep(rng, lo=1, side=6)
        t = W.random_tiler(rng, len(rep), max_side=9, max_origin=30, max_pattern_side=5)
        out_t = _scattered_output(rng, rep)
        c = rng.uniform(-1, 1, t.pattern_shape).astype(np.float32)
        p = W.Problem(rep, [t], out_t, W.WSUM, c)
        x = W.random_array(rng, t.array_shape)
        gy = rng.uniform(-1, 1, out_t.array_shape).astype(np.float32)
        a = oracle.adjoint(p, x, gy)
        gx = torch.full(t.array_shape, float("nan"), device="cuda")
        gc = torch.full(t.pattern_shape, float("nan"), device="cuda")
        rsm.run_adjoint(p, dev(x), dev(gy), gx, gc, dev(c))
        check_close(host(gx), a.gx, a.gx_abs, what="trial %d gx" % trial)
        check_close(host(gc), a.gc, a.gc_abs, what="trial %d gc" % trial)


def test_dot_random_tilers_f32_bf16_f64():
    rng = W.rng_for(61)
    for trial in range(30):
        rep = _rep(rng, lo=1, side=5)
        t1 = W.random_tiler(rng, len(rep), max_side=8, pattern_rank=2, max_pattern_side=5)
        n = int(np.prod(t1.pattern_shape))
        t2 = W.random_tiler(rng, len(rep), max_side=8, pattern_rank=1)
        t2 = W.Tiler(t2.array_shape, t2.origin, t2.paving, t2.fitting[:, :1], (n,))
        p = W.Problem(rep, [t1, t2], W.identity_output(rep), W.DOT)
        a = W.random_array(rng, t1.array_shape)
        b = W.random_array(rng, t2.array_shape)
        r = oracle.run(p, [a, b])
        out = torch.zeros(rep, device="cuda")
        rsm.run(p, [dev(a), dev(b)], out)
        check_close(host(out), r.out, r.abs_sum, what="f32 trial %d" % trial)
        # BF16 arrays: products exact in FP32, so the same FP32 bound holds
        ab, bb = W.f32_to_bf16_bits(a), W.f32_to_bf16_bits(b)
        rb = oracle.run(p, [ab, bb])
        p.compute = "bf16"
        outb = torch.zeros(rep, device="cuda")
        rsm.run(p, [bf16_dev(ab), bf16_dev(bb)], outb)
        check_close(host(outb), rb.out, rb.abs_sum, what="bf16 trial %d" % trial)
        p.compute = "f32"
        out64 = torch.zeros(rep, dtype=torch.float64, device="cuda")
        rsm.run(p, [dev(a.astype(np.float64)), dev(b.astype(np.float64))], out64)
        check_close(host(out64), r.out, r.abs_sum, tol=1e-13, what="f64 trial %d" % trial)


def test_long_pattern_generic_accuracy():
    # 16384-element sums: the FP32 bound must hold with the kernel's blocked accumulation
    rng = W.rng_for(71)
    t = W.Tiler((64, 16384), [0, 0], [[1], [0]], [[0], [1]], (16384,))
    p = W.Problem((64,), [t], W.identity_output((64,)), W.SUM)
    x = rng.uniform(-1, 1, (64, 16384)).astype(np.float32)
    out = torch.zeros(64, device="cuda")
    rsm.run(p, [dev(x)], out)
    r = oracle.run(p, [x])
    check_close(host(out), r.out, r.abs_sum, what="long sum")


# ---------------------------------------------------------------------------
# small plain task: 64x64 -> 16x16 sums of 4x4 patterns
# ---------------------------------------------------------------------------

def test_small_sum_pattern_reduce_and_generic():
    x, p = W.small_sum()
    assert rsm.plan(p) == "pattern_reduce"
    r = oracle.run(p, [x])
    for flags in (0, _abi.FORCE_GENERIC):
        out = torch.full((16, 16), float("nan"), device="cuda")
        rsm.run(p, [dev(x)], out, flags=flags)
        check_close(host(out), r.out, r.abs_sum, what="small sum flags=%d" % flags)


def test_pattern_reduce_ragged_and_wrapping():
    rng = W.rng_for(81)
    # 5x3 patterns (group of 16 lanes, 15 active), wrapping origin, ragged sizes
    t = W.Tiler((37, 29), [-7, 11], np.diag([3, 2]), [[1, 0], [0, -2]], (5, 3))
    rep = (23, 17)
    c = rng.uniform(-1, 1, (5, 3)).astype(np.float32)
    p = W.Problem(rep, [t], W.identity_output(rep), W.WSUM, c)
    assert rsm.plan(p) == "pattern_reduce"
    x = W.random_array(rng, t.array_shape)
    out = torch.zeros(rep, device="cuda")
    rsm.run(p, [dev(x)], out, coeffs=dev(c))
    r = oracle.run(p, [x])
    check_close(host(out), r.out, r.abs_sum, what="pattern_reduce wrap")
    # 64-element pattern, transposed output tiler
    t2 = W.Tiler((40, 40), [3, -5], np.diag([5, 5]), np.eye(2, dtype=np.int64), (8, 8))
    out_t = W.Tiler((8, 8), [0, 0], [[0, 1], [1, 0]], np.zeros((2, 0)), ())
    p2 = W.Problem((8, 8), [t2], out_t, W.SUM)
    x2 = W.random_array(rng, (40, 40))
    out2 = torch.zeros((8, 8), device="cuda")
    rsm.run(p2, [dev(x2)], out2)
    r2 = oracle.run(p2, [x2])
    check_close(host(out2), r2.out, r2.abs_sum, what="pattern_reduce transposed out")


def test_pattern_reduce_rank5_walk():
    # five repetition dimensions: past the 32-bit form's rank 4, so the
    # kernel walks the tilers in 64-bit arithmetic; wrapping origins
    rng = W.rng_for(88)
    F = np.zeros((5, 2), dtype=np.int64)
    F[3, 0] = 1
    F[4, 1] = 1
    t = W.Tiler((6, 5, 4, 3, 8), [1, -2, 0, 1, -3], np.diag([1, 1, 1, 1, 2]), F, (2, 4))
    rep = (6, 5, 4, 3, 4)
    c = rng.uniform(-1, 1, (2, 4)).astype(np.float32)
    p = W.Problem(rep, [t], W.identity_output(rep), W.WSUM, c)
    assert rsm.plan(p) == "pattern_reduce"
    x = W.random_array(rng, t.array_shape)
    out = torch.full(rep, float("nan"), device="cuda")
    rsm.run(p, [dev(x)], out, coeffs=dev(c))
    r = oracle.run(p, [x])
    check_close(host(out), r.out, r.abs_sum, what="pattern_reduce rank 5")
