"""Pins of the CPU oracle against facts that do not come from the oracle.

Each test below checks the oracle against something independent of its code:
a brute-force index walk that never uses a modulo, library routines
(NumPy's wrapping ravel, reshape/einsum sums, FFT circular correlation,
matrix products), invariants of exact-paving tilers, the adjoint identity and
central finite differences (exact for the quadratic loss used).  A plausible
slip in the oracle -- truncated instead of floored modulo, a transposed
paving or fitting matrix, a dropped origin/paving/fitting term, a swapped
weight, a wrong sign in the adjoint -- fails at least one of them (see
test_oracle_mutations.py, which plants such slips and checks they are caught).
"""
import itertools

import numpy as np
import pytest

import oracle
import rsm_workloads as W


# ---------------------------------------------------------------------------
# helpers that never use the oracle
# ---------------------------------------------------------------------------

def walk_indices(rep_shape, t):
    """Index table by incremental stepping: start at the origin, add paving /
    fitting columns while walking r and i in row-major order, and bring each
    coordinate back into [0, s) by repeated addition / subtraction of s."""
    s = np.array(t.array_shape, dtype=np.int64)
    da = len(s)

    def wrap(c):
        c = c.copy()
        for d in range(da):
            while c[d] < 0:
                c[d] += s[d]
            while c[d] >= s[d]:
                c[d] -= s[d]
        return c

    rows = []
    for r in itertools.product(*[range(n) for n in rep_shape]):
        base = np.array(t.origin, dtype=np.int64).copy()
        for k, rk in enumerate(r):
            for _ in range(rk):
                base = base + t.paving[:, k]
        row = []
        for i in itertools.product(*[range(n) for n in t.pattern_shape]):
            c = base.copy()
            for k, ik in enumerate(i):
                for _ in range(ik):
                    c = c + t.fitting[:, k]
            c = wrap(c)
            lin = 0
            for d in range(da):
                lin = lin * int(s[d]) + int(c[d])
            row.append(lin)
        rows.append(row)
    return np.array(rows, dtype=np.int64).reshape(
        int(np.prod(rep_shape)) if rep_shape else 1,
        int(np.prod(t.pattern_shape)) if t.pattern_shape else 1)


def numpy_indices(rep_shape, t):
    """Index table via NumPy's ravel_multi_index(mode='wrap')."""
    rg = np.stack(np.meshgrid(*[np.arange(n) for n in rep_shape], indexing="ij"), 0) \
        .reshape(len(rep_shape), -1) if rep_shape else np.zeros((0, 1), np.int64)
    pg = np.stack(np.meshgrid(*[np.arange(n) for n in t.pattern_shape], indexing="ij"), 0) \
        .reshape(len(t.pattern_shape), -1) if t.pattern_shape else np.zeros((0, 1), np.int64)
    base = t.origin[:, None] + (t.paving @ rg if rep_shape else 0)          # [da, nr]
    off = t.fitting @ pg if t.pattern_shape else np.zeros((len(t.array_shape), 1), np.int64)
    coords = base[:, :, None] + off[:, None, :]                              # [da, nr, np]
    return np.ravel_multi_index(tuple(coords.reshape(len(t.array_shape), -1)),
                                t.array_shape, mode="wrap").reshape(coords.shape[1], coords.shape[2])


# ---------------------------------------------------------------------------
# P1: brute force on tiny arrays
# ---------------------------------------------------------------------------

def test_indices_match_incremental_walk_random_tilers():
    rng = W.rng_for(1234)
    for trial in range(300):
        dr = int(rng.integers(0, 3))
        rep = tuple(int(v) for v in rng.integers(1, 5, dr))
        t = W.random_tiler(rng, dr)
        want = walk_indices(rep, t)
        got = oracle.indices(rep, t)
        assert np.array_equal(got, want), (trial, rep, t)


def test_indices_match_numpy_wrap_ravel_random_tilers():
    rng = W.rng_for(99)
    for trial in range(300):
        dr = int(rng.integers(1, 4))
        rep = tuple(int(v) for v in rng.integers(1, 6, dr))
        t = W.random_tiler(rng, dr, max_side=7, max_origin=50)
        assert np.array_equal(oracle.indices(rep, t), numpy_indices(rep, t)), (trial, t)


def test_indices_hand_example_negative_origin():
    # 1-D array of 5, origin -7, paving 3, fitting 2, pattern 3, 2 repetitions:
    # r=0: -7,-5,-3 -> 3,0,2 ; r=1: -4,-2,0 -> 1,3,0   (floored modulo 5)
    t = W.Tiler((5,), [-7], [[3]], [[2]], (3,))
    assert oracle.indices((2,), t).tolist() == [[3, 0, 2], [1, 3, 0]]


def test_indices_hand_example_2d_transposed_roles():
    # array [2,3]; rep [3]; paving (0,1) walks columns; fitting (1,0) walks rows
    t = W.Tiler((2, 3), [0, 0], [[0], [1]], [[1], [0]], (2,))
    # r = column c: elements (0,c), (1,c) -> offsets c, 3 + c
    assert oracle.indices((3,), t).tolist() == [[0, 3], [1, 4], [2, 5]]


# ---------------------------------------------------------------------------
# P2: exact cover of exact paving tilers; k^2 cover of stride-1 windows
# ---------------------------------------------------------------------------

def _hit_counts(rep, t):
    idx = oracle.indices(rep, t).reshape(-1)
    return np.bincount(idx, minlength=int(np.prod(t.array_shape)))


def test_exact_cover_small_sum_tiler():
    _, p = W.small_sum()
    t = p.inputs[0]
    assert np.prod(p.rep_shape) * np.prod(t.pattern_shape) == np.prod(t.array_shape)
    assert np.all(_hit_counts(p.rep_shape, t) == 1)


def test_exact_cover_two_stage_tilers_reduced():
    ts = W.two_stage_filter(frames=2, rows=16, cols=32)
    for p in (ts.h, ts.v):
        t = p.inputs[0]
        assert np.prod(p.rep_shape) * np.prod(t.pattern_shape) == np.prod(t.array_shape)
        assert np.all(_hit_counts(p.rep_shape, t) == 1)


@pytest.mark.parametrize("k", [3, 5, 7])
def test_stride1_window_covers_each_element_k2_times(k):
    p = W.filter2d_problem(11, 13, k, 1)
    assert np.all(_hit_counts(p.rep_shape, p.inputs[0]) == k * k)


def test_identity_output_tilers_single_assignment():
    for rep in [(16, 16), (3, 5, 7)]:
        t = W.identity_output(rep)
        assert np.all(_hit_counts(rep, t) == 1)


# ---------------------------------------------------------------------------
# P3: identity-tiler copy; transposing copy
# ---------------------------------------------------------------------------

def test_identity_copy_is_bit_exact():
    rng = W.rng_for(7)
    x = W.random_array(rng, (5, 6, 7))
    rep = x.shape
    tin = W.identity_output(rep)
    p = W.Problem(rep, [tin], W.identity_output(rep), W.COPY)
    r = oracle.run(p, [x])
    assert np.array_equal(r.out.astype(np.float32), x)
    assert np.all(r.hits == 1)


def test_copy_through_transposing_tiler():
    rng = W.rng_for(8)
    x = W.random_array(rng, (6, 9))
    # rep [9,6]: r=(c,r0) reads x[r0,c]; writes B[c,r0]  -> B = x.T
    tin = W.Tiler((6, 9), [0, 0], [[0, 1], [1, 0]], np.zeros((2, 0)), ())
    p = W.Problem((9, 6), [tin], W.identity_output((9, 6)), W.COPY)
    assert np.array_equal(oracle.run(p, [x]).out, x.T.astype(np.float64))


def test_copy_pattern_block_scatter():
    # each repetition copies a 2x3 block of x into a 2x3 block of B, blocks
    # transposed in position: B block (j, i) <- x block (i, j)
    rng = W.rng_for(9)
    x = W.random_array(rng, (4, 9))          # 2 x 3 blocks of 2x3
    tin = W.Tiler((4, 9), [0, 0], np.diag([2, 3]), np.eye(2, dtype=np.int64), (2, 3))
    tout = W.Tiler((6, 6), [0, 0], [[0, 2], [3, 0]], np.eye(2, dtype=np.int64), (2, 3))
    p = W.Problem((2, 3), [tin], tout, W.COPY)
    r = oracle.run(p, [x])
    want = np.zeros((6, 6))
    for i in range(2):
        for j in range(3):
            want[2 * j:2 * j + 2, 3 * i:3 * i + 3] = x[2 * i:2 * i + 2, 3 * j:3 * j + 3]
    assert np.array_equal(r.out, want)
    assert np.all(r.hits == 1)


def test_uncovered_output_keeps_prior():
    x = np.arange(4, dtype=np.float32)
    tin = W.Tiler((4,), [0], [[1]], np.zeros((1, 0)), ())
    tout = W.Tiler((8,), [1], [[2]], np.zeros((1, 0)), ())     # writes 1,3,5,7
    p = W.Problem((4,), [tin], tout, W.COPY)
    prior = np.full(8, -5.0)
    r = oracle.run(p, [x], prior=prior)
    assert r.out.tolist() == [-5, 0, -5, 1, -5, 2, -5, 3]
    assert r.hits.tolist() == [0, 1, 0, 1, 0, 1, 0, 1]


def test_overlapping_output_counts_hits():
    x = np.arange(6, dtype=np.float32)
    tin = W.Tiler((6,), [0], [[1]], np.zeros((1, 0)), ())
    tout = W.Tiler((3,), [0], [[1]], np.zeros((1, 0)), ())     # r and r+3 collide
    p = W.Problem((6,), [tin], tout, W.COPY)
    assert oracle.run(p, [x]).hits.tolist() == [2, 2, 2]


# ---------------------------------------------------------------------------
# P4: closed forms
# ---------------------------------------------------------------------------

def test_small_sum_equals_block_reshape_sum():
    x, p = W.small_sum()
    want = x.astype(np.float64).reshape(16, 4, 16, 4).sum(axis=(1, 3))
    r = oracle.run(p, [x])
    assert np.allclose(r.out, want, rtol=0, atol=1e-13)
    assert np.allclose(r.abs_sum, np.abs(x.astype(np.float64)).reshape(16, 4, 16, 4).sum((1, 3)))


def test_two_stage_equals_einsum():
    ts = W.two_stage_filter(frames=2, rows=24, cols=48)
    x = ts.x.astype(np.float64)
    mid = np.einsum("fhwk,k->fhw", x.reshape(2, 24, 6, 8), ts.c_h.astype(np.float64))
    out = np.einsum("fhkw,k->fhw", mid.reshape(2, 3, 8, 6), ts.c_v.astype(np.float64))
    fw = oracle.chain_forward([ts.h, ts.v], ts.x)
    assert np.allclose(fw[0].out, mid, rtol=0, atol=1e-14)
    assert np.allclose(fw[1].out, out, rtol=0, atol=1e-14)


def test_wrapped_fir_equals_roll():
    # centred 13-tap horizontal filter with paving 8 (overlapping, wraps at both
    # borders): y[f,h,w] = sum_k c[k] x[f,h,(8w - 6 + k) mod W]
    taps, pave, o = 13, 8, -6
    ts = W.two_stage_filter(frames=1, rows=3, cols=40, taps=taps, pave=pave, h_origin=o)
    x = ts.x.astype(np.float64)
    c = ts.c_h.astype(np.float64)
    want = np.zeros((1, 3, 5))
    for k in range(taps):
        want += c[k] * np.roll(x, -(o + k), axis=2)[:, :, ::pave]
    got = oracle.run(ts.h, [ts.x]).out
    assert np.allclose(got, want, rtol=0, atol=1e-14)


def _circular_filter_fft(x, c, o, s):
    H, W_ = x.shape
    k = c.shape[0]
    cp = np.zeros((H, W_))
    cp[:k, :k] = c
    corr = np.real(np.fft.ifft2(np.fft.fft2(x) * np.conj(np.fft.fft2(cp))))
    rows = (o + s * np.arange(-(-H // s))) % H
    cols = (o + s * np.arange(-(-W_ // s))) % W_
    return corr[np.ix_(rows, cols)]


@pytest.mark.parametrize("H,W_,k,s", [(17, 23, 3, 1), (32, 20, 5, 2), (19, 33, 7, 4),
                                      (40, 40, 9, 1), (9, 14, 9, 2)])
def test_filter2d_equals_fft_circular_correlation(H, W_, k, s):
    rng = W.rng_for(H * 1000 + W_)
    x = rng.standard_normal((H, W_)).astype(np.float32)
    c = (rng.uniform(-1, 1, (k, k)) / (k * k)).astype(np.float32)
    p = W.filter2d_problem(H, W_, k, s, c)
    want = _circular_filter_fft(x.astype(np.float64), c.astype(np.float64), -(k // 2), s)
    got = oracle.run(p, [x]).out
    assert np.allclose(got, want, rtol=0, atol=1e-12)


def _naive_matmul(a, b):
    M, K = a.shape
    N = b.shape[1]
    c = np.zeros((M, N))
    for m in range(M):
        for n in range(N):
            acc = 0.0
            for k in range(K):
                acc += float(a[m, k]) * float(b[k, n])
            c[m, n] = acc
    return c


def test_matmul_tilers_equal_naive_triple_loop():
    a, b, _, _ = W.matmul_inputs(12, 10, 16, seed=5)
    p = W.matmul_tilers(12, 10, 16)
    got = oracle.run(p, [a, b]).out
    assert np.allclose(got, _naive_matmul(a, b), rtol=0, atol=1e-12)


def test_matmul_tilers_equal_blas_and_transposed_layout():
    a, b, ab, bb = W.matmul_inputs(40, 24, 64, seed=6)
    p = W.matmul_tilers(40, 24, 64)
    assert np.allclose(oracle.run(p, [a, b]).out,
                       a.astype(np.float64) @ b.astype(np.float64), rtol=0, atol=1e-11)
    # BF16 bit patterns are widened exactly
    got = oracle.run(p, [ab, bb]).out
    want = W.bf16_bits_to_f32(ab).astype(np.float64) @ W.bf16_bits_to_f32(bb).astype(np.float64)
    assert np.allclose(got, want, rtol=0, atol=1e-11)
    # A stored transposed ([K, M]) : paving along columns, fitting along rows
    at = np.ascontiguousarray(a.T)
    ta = W.Tiler((64, 40), [0, 0], [[0, 0], [1, 0]], [[1], [0]], (64,))
    pt = W.Problem((40, 24), [ta, p.inputs[1]], p.output, W.DOT)
    assert np.allclose(oracle.run(pt, [at, b]).out,
                       a.astype(np.float64) @ b.astype(np.float64), rtol=0, atol=1e-11)


def test_run_sample_matches_run():
    a, b, _, _ = W.matmul_inputs(20, 30, 40, seed=11)
    p = W.matmul_tilers(20, 30, 40)
    full = oracle.run(p, [a, b])
    sel = np.array([0, 7, 599, 333, 42])
    y, ya = oracle.run_sample(p, [a, b], sel)
    assert np.array_equal(y[:, 0], full.out.reshape(-1)[sel])
    assert np.array_equal(ya[:, 0], full.abs_sum.reshape(-1)[sel])


# ---------------------------------------------------------------------------
# P5: adjoint identity <T x, g> = <x, T^T g>, and the weight gradient by
# linearity in the weights (forward with unit weights)
# ---------------------------------------------------------------------------

def test_adjoint_identity_random_tilers():
    rng = W.rng_for(2024)
    checked = 0
    while checked < 60:
        dr = int(rng.integers(1, 4))
        rep = tuple(int(v) for v in rng.integers(1, 5, dr))
        t = W.random_tiler(rng, dr, pattern_rank=int(rng.integers(0, 3)))
        c = rng.uniform(-1, 1, t.pattern_shape).astype(np.float32)
        p = W.Problem(rep, [t], W.identity_output(rep), W.WSUM, c)
        x = W.random_array(rng, t.array_shape)
        g = rng.uniform(-1, 1, rep)
        tx = oracle.run(p, [x]).out
        a = oracle.adjoint(p, x, g)
        lhs = float(np.sum(tx * g))
        rhs = float(np.sum(x.astype(np.float64) * a.gx))
        assert abs(lhs - rhs) <= 1e-12 * (1 + np.sum(np.abs(tx * g))), (lhs, rhs)
        # dL/dc_i of L = <T_c x, g> equals <T_{e_i} x, g>
        npat = c.size
        for i in range(npat):
            e = np.zeros(npat, np.float32)
            e[i] = 1.0
            pe = W.Problem(rep, [t], W.identity_output(rep), W.WSUM, e.reshape(c.shape))
            want = float(np.sum(oracle.run(pe, [x]).out * g))
            assert abs(a.gc.reshape(-1)[i] - want) <= 1e-12 * (1 + abs(want))
        checked += 1


def test_adjoint_of_sum_is_broadcast():
    x, p = W.small_sum()
    g = W.rng_for(3).uniform(-1, 1, (16, 16))
    a = oracle.adjoint(p, x, g)
    want = np.repeat(np.repeat(g, 4, axis=0), 4, axis=1)
    assert np.array_equal(a.gx, want)
    assert a.gc is None


# ---------------------------------------------------------------------------
# P4/P5 tolerance sums: every FP32 parity gate bounds an element's error by
# 1e-5 times the oracle's sum of |terms|.  Those sums are pinned here against
# index tables built without the oracle (NumPy's wrapping ravel) and against
# closed forms on |x| and |c|: a bound that drops the weight, takes |sum|
# instead of sum|.|, or is scaled, fails one of these.
# ---------------------------------------------------------------------------

def _abs_terms_by_table(rep, t, x, c):
    """sum_i |c_i| |x[e(r, i)]| per repetition, from the NumPy index table."""
    idx = numpy_indices(rep, t)
    xa = np.abs(x.astype(np.float64)).reshape(-1)
    ca = np.ones(idx.shape[1]) if c is None else np.abs(np.asarray(c, np.float64)).reshape(-1)
    return (xa[idx] * ca[None, :]).sum(axis=1)


def test_wsum_and_sum_abs_sums_match_index_table_random_tilers():
    rng = W.rng_for(4242)
    for trial in range(120):
        dr = int(rng.integers(1, 4))
        rep = tuple(int(v) for v in rng.integers(1, 5, dr))
        t = W.random_tiler(rng, dr, pattern_rank=int(rng.integers(0, 3)))
        x = W.random_array(rng, t.array_shape)
        weighted = trial % 3 != 0
        c = (rng.uniform(-2, 2, t.pattern_shape).astype(np.float32) if weighted else None)
        p = W.Problem(rep, [t], W.identity_output(rep), W.WSUM if weighted else W.SUM, c)
        want = _abs_terms_by_table(rep, t, x, c).reshape(rep)
        got = oracle.run(p, [x]).abs_sum
        assert np.allclose(got, want, rtol=1e-14, atol=0), (trial, t)
        ys, yas = oracle.run_sample(p, [x], np.arange(int(np.prod(rep)))[::2])
        assert np.allclose(yas[:, 0], want.reshape(-1)[::2], rtol=1e-14, atol=0), trial


def test_wsum_abs_sum_two_stage_closed_form():
    ts = W.two_stage_filter(frames=2, rows=24, cols=48)
    xa = np.abs(ts.x.astype(np.float64))
    ch, cv = np.abs(ts.c_h.astype(np.float64)), np.abs(ts.c_v.astype(np.float64))
    want_h = np.einsum("fhwk,k->fhw", xa.reshape(2, 24, 6, 8), ch)
    fh = oracle.run(ts.h, [ts.x])
    assert np.allclose(fh.abs_sum, want_h, rtol=1e-14, atol=0)
    mid = fh.out
    want_v = np.einsum("fhkw,k->fhw", np.abs(mid).reshape(2, 3, 8, 6), cv)
    assert np.allclose(oracle.run(ts.v, [mid]).abs_sum, want_v, rtol=1e-14, atol=0)


@pytest.mark.parametrize("H,W_,k,s", [(17, 23, 3, 1), (19, 33, 7, 4), (9, 14, 9, 2)])
def test_filter2d_abs_sum_equals_fft_of_absolutes(H, W_, k, s):
    rng = W.rng_for(H * 7 + W_)
    x = rng.standard_normal((H, W_)).astype(np.float32)
    c = (rng.uniform(-1, 1, (k, k)) / (k * k)).astype(np.float32)
    p = W.filter2d_problem(H, W_, k, s, c)
    want = _circular_filter_fft(np.abs(x.astype(np.float64)), np.abs(c.astype(np.float64)),
                                -(k // 2), s)
    assert np.allclose(oracle.run(p, [x]).abs_sum, want, rtol=1e-12, atol=1e-13)


def test_dot_abs_sum_equals_naive_loop_on_absolutes():
    a, b, _, _ = W.matmul_inputs(12, 10, 16, seed=15)
    p = W.matmul_tilers(12, 10, 16)
    want = _naive_matmul(np.abs(a), np.abs(b))
    r = oracle.run(p, [a, b])
    assert np.allclose(r.abs_sum, want, rtol=1e-14, atol=0)
    # the bound is never below |y| and is strictly above it where signs mix
    assert np.all(r.abs_sum >= np.abs(r.out))
    assert np.any(r.abs_sum > 1.5 * np.abs(r.out))


def test_dot_abs_sum_random_tiler_pairs():
    rng = W.rng_for(4343)
    for trial in range(60):
        dr = int(rng.integers(1, 3))
        rep = tuple(int(v) for v in rng.integers(1, 5, dr))
        dp = int(rng.integers(1, 3))
        t1 = W.random_tiler(rng, dr, pattern_rank=dp)
        t2 = W.random_tiler(rng, dr, pattern_rank=dp)
        t2 = W.Tiler(t2.array_shape, t2.origin, t2.paving,
                     rng.integers(-9, 10, (len(t2.array_shape), dp)), t1.pattern_shape)
        x1 = W.random_array(rng, t1.array_shape)
        x2 = W.random_array(rng, t2.array_shape)
        i1, i2 = numpy_indices(rep, t1), numpy_indices(rep, t2)
        v1, v2 = x1.astype(np.float64).reshape(-1)[i1], x2.astype(np.float64).reshape(-1)[i2]
        p = W.Problem(rep, [t1, t2], W.identity_output(rep), W.DOT)
        r = oracle.run(p, [x1, x2])
        assert np.allclose(r.out.reshape(-1), (v1 * v2).sum(1), rtol=0, atol=1e-13), trial
        assert np.allclose(r.abs_sum.reshape(-1), np.abs(v1 * v2).sum(1), rtol=1e-14, atol=0), trial


def test_copy_abs_sum_is_magnitude():
    rng = W.rng_for(17)
    x = W.random_array(rng, (5, 7))
    p = W.Problem((5, 7), [W.identity_output((5, 7))], W.identity_output((5, 7)), W.COPY)
    r = oracle.run(p, [x])
    assert np.array_equal(r.abs_sum, np.abs(x.astype(np.float64)))


def test_adjoint_abs_sums_match_index_table_random_tilers():
    rng = W.rng_for(4444)
    for trial in range(80):
        dr = int(rng.integers(1, 4))
        rep = tuple(int(v) for v in rng.integers(1, 5, dr))
        t = W.random_tiler(rng, dr, pattern_rank=int(rng.integers(0, 3)))
        c = rng.uniform(-2, 2, t.pattern_shape).astype(np.float32)
        p = W.Problem(rep, [t], W.identity_output(rep), W.WSUM, c)
        x = W.random_array(rng, t.array_shape)
        g = rng.uniform(-1, 1, rep)
        idx = numpy_indices(rep, t)                       # [nr, np]
        ca = np.abs(c.astype(np.float64)).reshape(-1)
        ga = np.abs(g).reshape(-1)
        xa = np.abs(x.astype(np.float64)).reshape(-1)
        want_gx = np.zeros(xa.size)
        np.add.at(want_gx, idx.reshape(-1), (ga[:, None] * ca[None, :]).reshape(-1))
        want_gc = (ga[:, None] * xa[idx]).sum(axis=0)
        a = oracle.adjoint(p, x, g)
        assert np.allclose(a.gx_abs.reshape(-1), want_gx, rtol=1e-14, atol=0), trial
        assert np.allclose(a.gc_abs.reshape(-1), want_gc, rtol=1e-14, atol=0), trial
        # the values themselves by the same tables (signed)
        gx = np.zeros(xa.size)
        np.add.at(gx, idx.reshape(-1), (g.reshape(-1)[:, None] * c.astype(np.float64).reshape(-1)[None, :]).reshape(-1))
        assert np.allclose(a.gx.reshape(-1), gx, rtol=0, atol=1e-13), trial


def test_adjoint_abs_sums_two_stage_closed_form():
    # exact paving: gx_abs[f,h,w] = |c_h[w mod 8]| |gy[f,h,w//8]| and
    # gc_abs[k] = sum_{f,h,q} |gy[f,h,q]| |x[f,h,8q+k]|
    ts = W.two_stage_filter(frames=2, rows=16, cols=40)
    g = W.rng_for(18).uniform(-1, 1, ts.h.rep_shape)
    a = oracle.adjoint(ts.h, ts.x, g)
    ch = np.abs(ts.c_h.astype(np.float64))
    want_gx = np.einsum("fhq,k->fhqk", np.abs(g), ch).reshape(ts.x.shape)
    want_gc = np.einsum("fhq,fhqk->k", np.abs(g), np.abs(ts.x.astype(np.float64)).reshape(2, 16, 5, 8))
    assert np.allclose(a.gx_abs, want_gx, rtol=1e-14, atol=0)
    assert np.allclose(a.gc_abs, want_gc, rtol=1e-14, atol=0)
    # unit weights (SUM): gx_abs is the broadcast of |gy|
    x, p = W.small_sum()
    g2 = W.rng_for(19).uniform(-1, 1, (16, 16))
    a2 = oracle.adjoint(p, x, g2)
    assert np.array_equal(a2.gx_abs, np.repeat(np.repeat(np.abs(g2), 4, 0), 4, 1))


# ---------------------------------------------------------------------------
# Weighted sums with an output pattern of q > 1 elements (polyphase stages):
# y(r)[j] = sum_i C[j, i] x[e(r, i)].  Along one axis, phase j of every row is
# the circular cross-correlation of the row with C[j], read at the window
# starts o + p r; the adjoint places the phase-j gradients at those starts
# and convolves with C[j].  Both are computed here with FFTs, a mechanism the
# oracle does not use.
# ---------------------------------------------------------------------------

def _corr_fft(x, c, axis):
    """corr[..., m, ...] = sum_i c[i] x[..., (m + i) mod n, ...] along axis."""
    n = x.shape[axis]
    cp = np.zeros(n)
    cp[:len(c)] = c
    shape = [1] * x.ndim
    shape[axis] = n
    fx = np.fft.fft(x, axis=axis)
    fc = np.conj(np.fft.fft(cp)).reshape(shape)
    return np.real(np.fft.ifft(fx * fc, axis=axis))


def _polyphase_fft(x, C, o, p, reps, axis):
    """Forward of a polyphase stage along `axis` by FFT correlation."""
    n = x.shape[axis]
    starts = (o + p * np.arange(reps)) % n
    q = C.shape[0]
    out_shape = list(x.shape)
    out_shape[axis] = reps * q
    out = np.zeros(out_shape)
    for j in range(q):
        cj = np.take(_corr_fft(x, C[j], axis), starts, axis=axis)
        sl = [slice(None)] * x.ndim
        sl[axis] = slice(j, reps * q, q)
        out[tuple(sl)] = cj
    return out


def _polyphase_adjoint_fft(x, g, C, o, p, axis):
    """(gx, gc) of a polyphase stage along `axis` by FFT convolution /
    correlation of the phase gradients placed at the window starts."""
    n = x.shape[axis]
    q, T = C.shape
    reps = g.shape[axis] // q
    starts = (o + p * np.arange(reps)) % n
    gx = np.zeros(x.shape)
    gc = np.zeros((q, T))
    shape = [1] * x.ndim
    shape[axis] = n
    for j in range(q):
        sl = [slice(None)] * g.ndim
        sl[axis] = slice(j, reps * q, q)
        gj = g[tuple(sl)]
        u = np.zeros(x.shape)
        usl = [slice(None)] * x.ndim
        for r in range(reps):      # starts are distinct when p r < n
            usl[axis] = starts[r]
            gsl = [slice(None)] * g.ndim
            gsl[axis] = r
            u[tuple(usl)] += gj[tuple(gsl)]
        cp = np.zeros(n)
        cp[:T] = C[j]
        fu = np.fft.fft(u, axis=axis)
        gx += np.real(np.fft.ifft(fu * np.fft.fft(cp).reshape(shape), axis=axis))
        cr = np.real(np.fft.ifft(np.conj(fu) * np.fft.fft(x, axis=axis), axis=axis))
        gc[j] = np.take(cr, np.arange(T) % n, axis=axis).sum(axis=tuple(a for a in range(x.ndim) if a != axis))
    return gx, gc


def test_polyphase_forward_equals_fft_correlation_per_phase():
    pp = W.polyphase_downscaler(frames=2, rows=40, cols=56)
    x = pp.x.astype(np.float64)
    ch = pp.c_h.astype(np.float64)
    cv = pp.c_v.astype(np.float64)
    fh = oracle.run(pp.h, [pp.x])
    want_h = _polyphase_fft(x, ch, -2, 8, pp.h.rep_shape[2], axis=2)
    assert np.allclose(fh.out, want_h, rtol=0, atol=1e-13)
    assert np.all(fh.hits == 1)
    want_abs = _polyphase_fft(np.abs(x), np.abs(ch), -2, 8, pp.h.rep_shape[2], axis=2)
    assert np.allclose(fh.abs_sum, want_abs, rtol=1e-12, atol=0)
    mid = fh.out.astype(np.float32)
    fv = oracle.run(pp.v, [mid])
    want_v = _polyphase_fft(mid.astype(np.float64), cv, -2, 9, pp.v.rep_shape[1], axis=1)
    assert np.allclose(fv.out, want_v, rtol=0, atol=1e-13)
    # run_sample gives whole output patterns per repetition
    y, ya = oracle.run_sample(pp.h, [pp.x], np.array([0, 5, 17]))
    flat = want_h.reshape(2 * 40, -1)
    for k, r in enumerate([0, 5, 17]):
        row, c = divmod(r, pp.h.rep_shape[2])
        assert np.allclose(y[k], flat[row, 3 * c:3 * c + 3], rtol=0, atol=1e-13)


def test_polyphase_one_hot_taps_select_samples():
    # C[j] = e_{s_j}: phase j of repetition r is x[(o + p r + s_j) mod n]
    # exactly (np.take with wrapping), for random geometries
    rng = W.rng_for(5151)
    for trial in range(30):
        n = int(rng.integers(5, 40))
        T = int(rng.integers(1, 9))
        p_ = int(rng.integers(1, 6))
        q = int(rng.integers(2, 5))
        o = int(rng.integers(-12, 12))
        reps = int(rng.integers(1, 8))
        sel = rng.integers(0, T, q)
        C = np.zeros((q, T), np.float32)
        C[np.arange(q), sel] = 1.0
        t = W.Tiler((n,), [o], [[p_]], [[1]], (T,))
        prob = W.Problem((reps,), [t], W.phase_output((reps,), 0, q), W.WSUM, C)
        x = rng.standard_normal(n).astype(np.float32)
        got = oracle.run(prob, [x]).out
        want = np.take(x, (o + p_ * np.arange(reps)[:, None] + sel[None, :]).reshape(-1), mode="wrap")
        assert np.array_equal(got, want.astype(np.float64)), trial


def test_polyphase_adjoint_equals_fft_and_adjoint_identity():
    pp = W.polyphase_downscaler(frames=2, rows=40, cols=56)
    rng = W.rng_for(5252)
    gh = rng.uniform(-1, 1, pp.h.output.array_shape)
    a = oracle.adjoint(pp.h, pp.x, gh)
    want_gx, want_gc = _polyphase_adjoint_fft(pp.x.astype(np.float64), gh, pp.c_h.astype(np.float64), -2, 8, axis=2)
    assert np.allclose(a.gx, want_gx, rtol=0, atol=1e-12)
    assert a.gc.shape == pp.c_h.shape
    assert np.allclose(a.gc, want_gc, rtol=0, atol=1e-11)
    # bounds: the same closed forms on absolute values
    abs_gx, abs_gc = _polyphase_adjoint_fft(np.abs(pp.x.astype(np.float64)), np.abs(gh),
                                            np.abs(pp.c_h.astype(np.float64)), -2, 8, axis=2)
    assert np.allclose(a.gx_abs, abs_gx, rtol=1e-11, atol=1e-13)
    assert np.allclose(a.gc_abs, abs_gc, rtol=1e-11, atol=0)
    # vertical stage: <T x, g> = <x, T^t g>, and gc[j, i] = <T_{E_ji} x, g>
    mid = oracle.run(pp.h, [pp.x]).out.astype(np.float32)
    gv = rng.uniform(-1, 1, pp.v.output.array_shape)
    av = oracle.adjoint(pp.v, mid, gv)
    tx = oracle.run(pp.v, [mid]).out
    lhs = float(np.sum(tx * gv))
    assert abs(lhs - float(np.sum(mid.astype(np.float64) * av.gx))) <= 1e-12 * np.sum(np.abs(tx * gv))
    q, T = pp.c_v.shape
    for j in range(q):
        for i in range(T):
            E = np.zeros((q, T), np.float32)
            E[j, i] = 1.0
            pe = W.Problem(pp.v.rep_shape, pp.v.inputs, pp.v.output, W.WSUM, E)
            want = float(np.sum(oracle.run(pe, [mid]).out * gv))
            assert abs(av.gc[j, i] - want) <= 1e-12 * (1 + abs(want)), (j, i)


def test_polyphase_sum_task_needs_scalar_output():
    pp = W.polyphase_downscaler(frames=1, rows=18, cols=24)
    ps = W.Problem(pp.h.rep_shape, pp.h.inputs, pp.h.output, W.SUM)
    with pytest.raises(ValueError):
        oracle.run(ps, [pp.x])
    with pytest.raises(ValueError):
        oracle.adjoint(ps, pp.x, np.zeros(pp.h.output.array_shape))


def test_chain_bound_on_absolutes_equals_einsum():
    # the chain tolerance (both stages run on |x| with |c|) is the closed form
    # of the two einsums on absolute values
    ts = W.two_stage_filter(frames=1, rows=16, cols=32)
    absp = [W.Problem(s.rep_shape, s.inputs, s.output, s.task, np.abs(s.coeffs)) for s in (ts.h, ts.v)]
    got = oracle.chain_forward(absp, np.abs(ts.x))[-1].out
    xa = np.abs(ts.x.astype(np.float64))
    mid = np.einsum("fhwk,k->fhw", xa.reshape(1, 16, 4, 8), np.abs(ts.c_h.astype(np.float64)))
    want = np.einsum("fhkw,k->fhw", mid.reshape(1, 2, 8, 4), np.abs(ts.c_v.astype(np.float64)))
    assert np.allclose(got, want, rtol=1e-14, atol=0)


# ---------------------------------------------------------------------------
# P6: finite differences are exact for L = sum(w * out^2)
# ---------------------------------------------------------------------------

def _crop_problem():
    """32x32 crop of the two-stage filter, treated as its own [1,32,32] array."""
    ts = W.two_stage_filter(frames=1, rows=32, cols=32)
    w = W.loss_weights((1, 4, 4))
    return ts, w


def _loss(stages, x):
    fw = oracle.chain_forward(stages, x)
    return fw


def test_finite_differences_match_chain_adjoint():
    ts, w = _crop_problem()
    stages = [ts.h, ts.v]
    x64 = ts.x.astype(np.float64)
    adj = oracle.chain_adjoint(stages, x64, w)
    h = 2.0 ** -4

    def L(xv, ch, cv):
        sh = W.Problem(ts.h.rep_shape, ts.h.inputs, ts.h.output, W.WSUM, ch)
        sv = W.Problem(ts.v.rep_shape, ts.v.inputs, ts.v.output, W.WSUM, cv)
        out = oracle.chain_forward([sh, sv], xv)[-1].out
        return float(np.sum(w.astype(np.float64) * out * out))

    ch = ts.c_h.astype(np.float64)
    cv = ts.c_v.astype(np.float64)
    base = L(x64, ch, cv)
    assert abs(base - adj.loss) <= 1e-15 * abs(base)
    flat = x64.reshape(-1)
    gx_fd = np.zeros_like(flat)
    for j in range(flat.size):
        xp = flat.copy(); xp[j] += h
        xm = flat.copy(); xm[j] -= h
        gx_fd[j] = (L(xp.reshape(x64.shape), ch, cv) - L(xm.reshape(x64.shape), ch, cv)) / (2 * h)
    assert np.allclose(adj.gx.reshape(-1), gx_fd, rtol=0, atol=1e-13)
    for which, cvec in (("h", ch), ("v", cv)):
        for k in range(8):
            cp, cm = cvec.copy(), cvec.copy()
            cp[k] += h
            cm[k] -= h
            if which == "h":
                fd = (L(x64, cp, cv) - L(x64, cm, cv)) / (2 * h)
                got = adj.gc[0][k]
            else:
                fd = (L(x64, ch, cp) - L(x64, ch, cm)) / (2 * h)
                got = adj.gc[1][k]
            assert abs(got - fd) <= 1e-12 * (1 + abs(fd)), (which, k, got, fd)


def test_fused_closed_form_of_chain_gradient():
    # gx[f,h,w] = c_h[w mod 8] c_v[h mod 8] gy[f, h//8, w//8], gy = 2 w out
    ts = W.two_stage_filter(frames=2, rows=16, cols=24)
    w = W.loss_weights((2, 2, 3))
    adj = oracle.chain_adjoint([ts.h, ts.v], ts.x, w)
    out = adj.forward[-1].out
    gy = 2.0 * w.astype(np.float64) * out
    ch = ts.c_h.astype(np.float64)
    cv = ts.c_v.astype(np.float64)
    want = np.einsum("fhw,a,b->fhawb", gy, cv, ch).reshape(2, 16, 24)
    assert np.allclose(adj.gx, want, rtol=0, atol=1e-15)


# ---------------------------------------------------------------------------
# inputs recipe sanity (shapes and seeds are deterministic)
# ---------------------------------------------------------------------------

def test_filter_batch_recipe_is_deterministic_and_in_range():
    a = W.filter_batch(64, with_data=False)
    b = W.filter_batch(64, with_data=True)
    assert [(i.H, i.W, i.k, i.s) for i in a] == [(i.H, i.W, i.k, i.s) for i in b]
    for i in b:
        assert 32 <= i.H <= 2048 and 32 <= i.W <= 2048
        assert i.k in (3, 5, 7, 9) and i.s in (1, 2, 4)
        assert i.x.shape == (i.H, i.W) and i.coeffs.shape == (i.k, i.k)


def test_bf16_rounding_is_rne():
    v = np.array([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, -2.5], np.float32)
    r = W.bf16_bits_to_f32(W.f32_to_bf16_bits(v))
    # 1+2^-8 is a tie -> even (1.0); 1+3*2^-8 tie -> even (1+2^-6)
    assert r.tolist() == [1.0, 1.0, 1.0 + 2 ** -6, 1.0, -2.5]


# ---------------------------------------------------------------------------
# indirect tilers: sparse matrix-vector product
# ---------------------------------------------------------------------------

def test_csr_matches_scipy_and_dense():
    import scipy.sparse as sp
    rng = W.rng_for(404)
    for trial in range(20):
        nr, nc = int(rng.integers(1, 40)), int(rng.integers(1, 40))
        A = W.random_csr(rng, nr, nc)
        x = rng.uniform(-1, 1, nc)
        y, ya = oracle.run_csr(A, x)
        M = sp.csr_matrix((A.vals, A.col_idx, A.row_ptr), shape=(nr, nc))
        assert np.allclose(y, M @ x, rtol=0, atol=1e-13)
        assert np.allclose(y, M.toarray() @ x, rtol=0, atol=1e-13)
        Mabs = sp.csr_matrix((np.abs(A.vals), A.col_idx, A.row_ptr), shape=(nr, nc))
        assert np.allclose(ya, Mabs.toarray() @ np.abs(x), rtol=0, atol=1e-13)


def test_csr_empty_rows_and_duplicate_columns():
    A = W.Csr(3, np.array([0, 0, 3, 3], np.int32), np.array([1, 1, 0], np.int32),
              np.array([2.0, 3.0, -1.0]))
    y, _ = oracle.run_csr(A, np.array([10.0, 100.0]))
    assert y.tolist() == [0.0, 490.0, 0.0]


def test_stencil_matrix_structure_and_spd():
    # the case study's counts: N = 51^3, NNZ = (3*51-2)^3
    A = W.stencil27_csr(51)
    assert A.n == 132651 and A.nnz == 3442951
    import scipy.sparse as sp
    small = W.stencil27_csr(6)
    M = sp.csr_matrix((small.vals, small.col_idx, small.row_ptr), shape=(small.n, small.n)).toarray()
    assert np.array_equal(M, M.T)
    assert np.linalg.eigvalsh(M).min() > 0
    # interior rows have 27 entries, corners 8
    counts = np.diff(small.row_ptr)
    assert counts.max() == 27 and counts.min() == 8


# ---------------------------------------------------------------------------
# conjugate gradient (the case study's loop)
# ---------------------------------------------------------------------------

def _dense_to_csr(M):
    rows, cols = np.nonzero(M)
    row_ptr = np.zeros(M.shape[0] + 1, np.int32)
    np.add.at(row_ptr, rows + 1, 1)
    return W.Csr(M.shape[0], np.cumsum(row_ptr).astype(np.int32), cols.astype(np.int32),
                 M[rows, cols].astype(np.float64))


def _spd(rng, n, cond=50.0):
    """Dense SPD matrix with eigenvalues log-spaced in [1, cond]."""
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    return (Q * np.geomspace(1.0, cond, n)) @ Q.T


def test_cg_identity_takes_one_step():
    b = W.rng_for(500).uniform(-1, 1, 17)
    r = oracle.cg(_dense_to_csr(np.eye(17)), b)
    assert r.iters == 1
    assert np.allclose(r.x, b, rtol=0, atol=1e-15)
    assert r.alpha[0] == pytest.approx(1.0)


def test_cg_terminates_after_distinct_eigenvalue_count():
    # in exact arithmetic CG stops after as many steps as A has distinct
    # eigenvalues (here 3) on a right-hand side that excites all of them
    d = np.array([1.0, 1.0, 4.0, 4.0, 4.0, 9.0, 9.0])
    b = W.rng_for(501).uniform(0.5, 1.0, d.size)
    r = oracle.cg(_dense_to_csr(np.diag(d)), b, tol=1e-12)
    assert r.iters == 3
    assert np.allclose(r.x, b / d, rtol=1e-12, atol=0)


def test_cg_solution_matches_dense_solve():
    rng = W.rng_for(502)
    for n, cond in ((5, 3.0), (30, 50.0), (64, 1e3)):
        M = _spd(rng, n, cond)
        b = rng.uniform(-1, 1, n)
        r = oracle.cg(_dense_to_csr(M), b, tol=1e-12, max_iter=10 * n)
        x = np.linalg.solve(M, b)
        # forward error <= cond * relative residual (plus rounding)
        assert np.linalg.norm(r.x - x) <= 2 * cond * 1e-12 * np.linalg.norm(x) + 1e-13
        assert np.linalg.norm(b - M @ r.x) <= 1.01e-12 * np.linalg.norm(b) + 1e-14
        # from a nonzero start the same solution is reached
        r0 = oracle.cg(_dense_to_csr(M), b, tol=1e-12, max_iter=10 * n, x0=rng.uniform(-1, 1, n))
        assert np.linalg.norm(r0.x - x) <= 2 * cond * 1e-12 * np.linalg.norm(x) + 1e-13


def test_cg_iterates_match_scipy():
    # SciPy's cg runs the same recurrences; after k steps from x0 = 0 both
    # hold the same iterate up to rounding
    import scipy.sparse as sp
    from scipy.sparse.linalg import cg as scipy_cg
    rng = W.rng_for(503)
    M = _spd(rng, 40, 20.0)
    b = rng.uniform(-1, 1, 40)
    A = _dense_to_csr(M)
    S = sp.csr_matrix((A.vals, A.col_idx, A.row_ptr), shape=(40, 40))
    for k in (1, 2, 5, 9):
        ours = oracle.cg(A, b, tol=0.0, max_iter=k)
        ref, _ = scipy_cg(S, b, x0=np.zeros(40), rtol=0.0, atol=0.0, maxiter=k)
        assert ours.iters == k
        assert np.allclose(ours.x, ref, rtol=0, atol=1e-12 * np.linalg.norm(ref))


def test_cg_residuals_orthogonal_and_directions_conjugate():
    # Krylov properties: r_i . r_j = 0 and p_i . A p_j = 0 for i != j (checked
    # on residuals recomputed as b - A x_k from separate runs)
    rng = W.rng_for(504)
    n = 24
    M = _spd(rng, n, 10.0)
    b = rng.uniform(-1, 1, n)
    A = _dense_to_csr(M)
    xs = [np.zeros(n)] + [oracle.cg(A, b, tol=0.0, max_iter=k).x for k in range(1, 7)]
    rs = [b - M @ x for x in xs]
    ps = [xs[k + 1] - xs[k] for k in range(6)]        # alpha_k p_k
    for i in range(6):
        for j in range(i):
            assert abs(rs[i] @ rs[j]) <= 1e-10 * np.linalg.norm(rs[i]) * np.linalg.norm(rs[j])
            assert abs(ps[i] @ M @ ps[j]) <= 1e-10 * np.sqrt((ps[i] @ M @ ps[i]) * (ps[j] @ M @ ps[j]))
    # the recorded residual norms are those of b - A x_k
    full = oracle.cg(A, b, tol=0.0, max_iter=6)
    for k in range(7):
        assert full.res[k] == pytest.approx(np.linalg.norm(rs[k]), rel=1e-9, abs=1e-14)


def test_cg_stopping_rule_is_relative():
    # scaling b by a power of two scales every iterate exactly and leaves the
    # iteration count unchanged
    rng = W.rng_for(505)
    M = _spd(rng, 30, 100.0)
    b = rng.uniform(-1, 1, 30)
    A = _dense_to_csr(M)
    r1 = oracle.cg(A, b, tol=1e-8, max_iter=300)
    r2 = oracle.cg(A, 2.0 ** 20 * b, tol=1e-8, max_iter=300)
    assert r1.iters == r2.iters < 300
    assert np.array_equal(r2.x, 2.0 ** 20 * r1.x)
    assert r1.res[-1] <= 1e-8 * np.linalg.norm(b) < r1.res[-2]


def test_cg_rejects_indefinite():
    with pytest.raises(ValueError):
        oracle.cg(_dense_to_csr(np.diag([1.0, -2.0, 3.0])), np.ones(3))
