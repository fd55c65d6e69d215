"""GPU parity of the matrix product expressed through tilers (DOT task).

BF16 operands: products are exact in FP32 and accumulation is FP32, so the
result is held to the FP32 bound against the FP64 oracle on the BF16-rounded
inputs; the error against FP64 of the original FP32 inputs (input
quantisation) is reported, with a sanity gate of 1e-2 normwise.
FP32 operands: FP32 bound against the FP64 oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import rsm_workloads as W
from paper_1105_4424_amd import rsm

from .helpers import bf16_dev, check_close, dev, host, say

pytestmark = pytest.mark.gpu


def _layouts(M, N, K):
    """(name, A tiler, B tiler, A transform, B transform) for the four storage orders."""
    base = W.matmul_tilers(M, N, K)
    ta_n, tb_n = base.inputs
    ta_t = W.Tiler((K, M), [0, 0], [[0, 0], [1, 0]], [[1], [0]], (K,))
    tb_t = W.Tiler((N, K), [0, 0], [[0, 1], [0, 0]], [[0], [1]], (K,))
    ident = lambda a: a
    trans = lambda a: np.ascontiguousarray(a.T)
    return [("nn", ta_n, tb_n, ident, ident), ("tn", ta_t, tb_n, trans, ident),
            ("nt", ta_n, tb_t, ident, trans), ("tt", ta_t, tb_t, trans, trans)]


@pytest.mark.parametrize("M,N,K", [(256, 256, 256), (200, 136, 264), (130, 300, 72), (1, 33, 8)])
@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_gemm_ragged_all_layouts(M, N, K, dtype):
    a, b, ab, bb = W.matmul_inputs(M, N, K, seed=M + N + K)
    for name, ta, tb, fa, fb in _layouts(M, N, K):
        p = W.Problem((M, N), [ta, tb], W.identity_output((M, N)), W.DOT, compute=dtype)
        assert rsm.plan(p, dtypes=(torch.bfloat16 if dtype == "bf16" else torch.float32,)) \
            .startswith("gemm_mfma_" + dtype), name
        if dtype == "bf16":
            xa, xb = fa(ab), fb(bb)
            da, db = bf16_dev(xa), bf16_dev(xb)
        else:
            xa, xb = fa(a), fb(b)
            da, db = dev(xa), dev(xb)
        r = oracle.run(p, [xa, xb])
        out = torch.full((M, N), float("nan"), device="cuda")
        rsm.run(p, [da, db], out)
        check_close(host(out), r.out, r.abs_sum, what="%s %s %dx%dx%d" % (dtype, name, M, N, K))


def _block_samples(M, N, block=32, tile=256, per_block=1, seed=0):
    """Flat output indices: per_block outputs in every block x block MFMA
    block, at positions that run through all block x block offsets across
    the blocks (so every lane / register slot of the fragment layout is
    checked many times), plus the four corners of every tile x tile tile."""
    nbi, nbj = -(-M // block), -(-N // block)
    bi, bj = np.meshgrid(np.arange(nbi), np.arange(nbj), indexing="ij")
    b = (bi * nbj + bj).reshape(-1)
    out = []
    for q in range(per_block):
        pos = (b * 389 + q * 517 + seed) % (block * block)
        r = bi.reshape(-1) * block + pos // block
        c = bj.reshape(-1) * block + pos % block
        ok = (r < M) & (c < N)
        out.append(r[ok] * N + c[ok])
    ti, tj = np.meshgrid(np.arange(-(-M // tile)), np.arange(-(-N // tile)), indexing="ij")
    ti, tj = ti.reshape(-1), tj.reshape(-1)
    for r, c in ((ti * tile, tj * tile), (np.minimum(ti * tile + tile, M) - 1, tj * tile),
                 (ti * tile, np.minimum(tj * tile + tile, N) - 1),
                 (np.minimum(ti * tile + tile, M) - 1, np.minimum(tj * tile + tile, N) - 1)):
        out.append(r * N + c)
    return np.unique(np.concatenate(out))


def _edge_samples(M, N, tile=256, step=7):
    """Outputs along every tile edge (both sides of each boundary) and along
    the last row and column, every step-th element."""
    rows = sorted({v for t in range(0, M, tile) for v in (t - 1, t) if 0 <= v < M} | {M - 1})
    cols = sorted({v for t in range(0, N, tile) for v in (t - 1, t) if 0 <= v < N} | {N - 1})
    out = [np.array(rows)[:, None] * N + np.arange(0, N, step)[None, :],
           np.arange(0, M, step)[:, None] * N + np.array(cols)[None, :]]
    return np.unique(np.concatenate([o.reshape(-1) for o in out]))


def test_gemm_full_size_every_block_and_error_report():
    # the 4096^3 workload on the large-tile kernel the bench times: one output
    # in every 32 x 32 MFMA block of every 256 x 256 tile (16,384 blocks) plus
    # every tile's corners, against the FP64 oracle; BF16 also against FP64
    # of the FP32 inputs (quantisation error, reported)
    M = N = K = 4096
    say("generating 4096^3 inputs")
    a, b, ab, bb = W.matmul_inputs(M, N, K)
    p = W.matmul_tilers(M, N, K)
    sel = _block_samples(M, N)
    say("%d stratified samples" % sel.size)
    # BF16 on the matrix cores
    p.compute = "bf16"
    assert rsm.plan(p, dtypes=(torch.bfloat16,)).startswith("gemm_mfma_bf16")
    out = torch.full((M, N), float("nan"), device="cuda")
    rsm.run(p, [bf16_dev(ab), bf16_dev(bb)], out)
    full = host(out)
    assert np.all(np.isfinite(full))
    got = full.reshape(-1)[sel]
    y_q, ya_q = oracle.run_sample(p, [ab, bb], sel)            # FP64 on BF16-rounded inputs
    st = check_close(got, y_q[:, 0], ya_q[:, 0], what="bf16 4096^3 vs FP64(bf16 inputs)")
    sub = sel[::4]
    y_f, _ = oracle.run_sample(p, [a, b], sub)                 # FP64 on the FP32 inputs
    g_sub = full.reshape(-1)[sub]
    err_f = float(np.linalg.norm(g_sub - y_f[:, 0]) / np.linalg.norm(y_f[:, 0]))
    err_q = float(np.linalg.norm(got - y_q[:, 0]) / np.linalg.norm(y_q[:, 0]))
    say("bf16 normwise relative error: %.3e vs FP64 of the FP32 inputs, %.3e vs FP64 of the "
        "BF16-rounded inputs (worst element %.3g of the 1e-5 |term| bound)" % (err_f, err_q, st["max_ratio"]))
    assert err_f < 1e-2
    del out, full
    # FP32
    p.compute = "f32"
    out32 = torch.full((M, N), float("nan"), device="cuda")
    rsm.run(p, [dev(a), dev(b)], out32)
    full32 = host(out32)
    assert np.all(np.isfinite(full32))
    y32, ya32 = oracle.run_sample(p, [a, b], sel)
    check_close(full32.reshape(-1)[sel], y32[:, 0], ya32[:, 0], what="f32 4096^3")


# large enough for the 256 x 256 tiles (M N >= 200 of them); M, N and K all
# ragged (K not a multiple of the 64-element k-tile).  BF16 B stored [K][N]
# ("nn" / "tn") is read in place through transposing LDS reads when its rows
# are 16-byte aligned (N = 4504), and transposed into the workspace when
# they are not (N = 4500)
@pytest.mark.parametrize("dtype,N", [("bf16", 4504), ("bf16", 4500), ("f32", 4504)])
def test_gemm_large_ragged_all_layouts_sampled(dtype, N):
    M, K = 3000, 1000
    a, b, ab, bb = W.matmul_inputs(M, N, K, seed=77)
    # one output in every 32 x 32 block, every tile's corners, and every
    # tile edge (both sides of each boundary, the ragged last row / column)
    sel = np.unique(np.concatenate([_block_samples(M, N, seed=N), _edge_samples(M, N)]))
    for name, ta, tb, fa, fb in _layouts(M, N, K):
        p = W.Problem((M, N), [ta, tb], W.identity_output((M, N)), W.DOT, compute=dtype)
        if dtype == "bf16":
            xa, xb = fa(ab), fb(bb)
            da, db = bf16_dev(xa), bf16_dev(xb)
        else:
            xa, xb = fa(a), fb(b)
            da, db = dev(xa), dev(xb)
        out = torch.full((M, N), float("nan"), device="cuda")
        rsm.run(p, [da, db], out)
        full = host(out)
        assert np.all(np.isfinite(full)), name
        y, ya = oracle.run_sample(p, [xa, xb], sel)
        check_close(full.reshape(-1)[sel], y[:, 0], ya[:, 0], what="%s %s %dx%dx%d" % (dtype, name, M, N, K))
