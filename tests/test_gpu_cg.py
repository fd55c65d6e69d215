"""GPU parity of the conjugate-gradient loop (FP64) against the oracle.

The device loop computes the same recurrences in FP64 but sums inner
products and rows in another order, so the iterates differ from the oracle's
by rounding that CG then propagates.  Parity is therefore checked on what
does not depend on that order beyond rounding:

* the residual history ||r_k|| / ||r_0|| agrees to 1e-9 (absolute, on the
  normalised history) over the iterations both runs take on the
  diagonally dominant stencil matrices; on random SPD matrices that are
  ill-conditioned relative to their size, finite-precision CG loses
  orthogonality and two summation orders drift apart, so there only the
  stable prefix (below) is compared pointwise and the iteration counts may
  differ by max(1, 5 %);
* the step scalars alpha_k, beta_k of the stable prefix -- the first (up to
  ten) steps whose residual stays above 1e-6 ||r_0|| -- agree to 1e-9
  relative;
* on the stencils the iteration count equals the oracle's, or differs by one
  only where the two residuals at the disputed step straddle the threshold;
* the GPU's final iterate meets the stopping rule on the TRUE residual
  b - A x (computed by the oracle's sparse product) within 2 tol ||b||.

Edge cases: b = 0, x0 = exact solution, max_iter = 0 and a small max_iter,
every check cadence giving identical bits, repeated calls identical, an
indefinite matrix reported as a breakdown, malformed indices rejected.
"""
import numpy as np
import pytest
import torch

import oracle
import rsm_workloads as W
from paper_1105_4424_amd import rsm

from .helpers import dev, host, say

pytestmark = pytest.mark.gpu


def _dev_csr(A):
    return dev(A.row_ptr), dev(A.col_idx), dev(A.vals, torch.float64)


def _solve(A, b, x0=None, **kw):
    rp, ci, va = _dev_csr(A)
    x = dev(np.zeros(A.n) if x0 is None else x0, torch.float64)
    info = rsm.cg_solve(rp, ci, va, dev(b, torch.float64), x, history=True, **kw)
    return info, host(x)


def _check_against_oracle(A, b, tol, max_iter=None, x0=None, check_every=16, what="",
                          full_history=True):
    info, x = _solve(A, b, x0=x0, tol=tol, max_iter=max_iter, check_every=check_every)
    ref = oracle.cg(A, b, tol=tol, max_iter=max_iter, x0=x0)
    k_gpu, k_ref = info["iterations"], ref.iters
    say("%s: n=%d nnz=%d iterations gpu %d oracle %d" % (what, A.n, A.nnz, k_gpu, k_ref))
    bnorm = np.linalg.norm(b)
    assert info["rhs_norm"] == pytest.approx(bnorm, rel=1e-13)
    res = host(info["res"])
    r0 = ref.res[0] if ref.res[0] > 0 else 1.0
    m = min(k_gpu, k_ref) + 1
    # the stable prefix: steps before the residual falls to 1e-6 ||r0|| (at
    # most ten), where loss of orthogonality has not yet amplified rounding
    q = 0
    while q < min(10, m - 1) and ref.res[q + 1] > 1e-6 * r0:
        q += 1
    hist = m if full_history else q + 1
    assert np.max(np.abs(res[:hist] - ref.res[:hist])) / r0 <= 1e-9, what
    if q > 0:
        assert np.allclose(host(info["alpha"])[:q], ref.alpha[:q], rtol=1e-9, atol=0), what
        assert np.allclose(host(info["beta"])[:q], ref.beta[:q], rtol=1e-9, atol=0), what
    if full_history:
        if k_gpu != k_ref:
            # a near-tie: at the disputed step the two residuals (held within
            # 1e-9 ||r0|| of each other) lie on opposite sides of the threshold
            assert abs(k_gpu - k_ref) == 1, what
            j = min(k_gpu, k_ref)
            assert (res[j] - tol * bnorm) * (ref.res[j] - tol * bnorm) <= 0, what
    else:
        assert abs(k_gpu - k_ref) <= max(1, int(np.ceil(0.05 * k_ref))), what
    limit = A.n if max_iter is None else max_iter
    if info["converged"]:
        true_res = np.linalg.norm(b - oracle.run_csr(A, x)[0])
        assert true_res <= 2 * tol * bnorm + 1e-300, (what, true_res, tol * bnorm)
        assert info["residual_norm"] <= tol * bnorm
    else:
        assert k_gpu == limit
    return info, x, ref


@pytest.mark.parametrize("n,cond,density", [(7, 5.0, 1.0), (150, 100.0, 1.0), (333, 50.0, 0.03),
                                            (1000, 300.0, 0.01)])
def test_random_spd(n, cond, density):
    rng = W.rng_for(600 + n)
    A = W.spd_csr(rng, n, cond, density)
    b = rng.uniform(-1, 1, n)
    # ill-conditioned relative to n: finite-precision CG loses orthogonality,
    # so only the stable prefix of the history is compared pointwise
    _check_against_oracle(A, b, 1e-10, max_iter=20 * n, what="spd n=%d" % n, full_history=False)


def test_stencil_small_and_nonzero_start():
    A = W.stencil27_csr(12, seed=5)
    b = W.cg_rhs(A.n, seed=6)
    _check_against_oracle(A, b, 1e-10, what="stencil 12^3")
    x0 = W.rng_for(601).uniform(-1, 1, A.n)
    _check_against_oracle(A, b, 1e-10, x0=x0, what="stencil 12^3, x0 != 0")


def test_stencil_case_study_size():
    # N = 51^3 = 132651, NNZ = 3442951: the case study's counts; tol 1e-10
    A = W.stencil27_csr(51, seed=5)
    b = W.cg_rhs(A.n, seed=6)
    info, x, ref = _check_against_oracle(A, b, 1e-10, what="stencil 51^3")
    assert info["converged"]


def test_edge_cases():
    A = W.stencil27_csr(6, seed=5)
    n = A.n
    # b = 0: ||r0|| = 0 is not above tol * 0, so no iteration runs
    info, x = _solve(A, np.zeros(n), tol=1e-10)
    assert info["iterations"] == 0 and info["converged"] and np.all(x == 0)
    # x0 = exact solution of A x = b (b formed by the oracle's product)
    xs = W.rng_for(602).uniform(-1, 1, n)
    b = oracle.run_csr(A, xs)[0]
    info, x = _solve(A, b, x0=xs, tol=1e-10)
    assert info["iterations"] == 0 and info["converged"]
    assert np.array_equal(x, xs)
    # max_iter = 0 and a small max_iter
    b = W.cg_rhs(n, seed=6)
    info, x = _solve(A, b, tol=1e-10, max_iter=0)
    assert info["iterations"] == 0 and not info["converged"] and np.all(x == 0)
    _check_against_oracle(A, b, 1e-14, max_iter=5, what="max_iter 5")


def test_cadence_and_repeat_give_identical_bits():
    A = W.stencil27_csr(10, seed=5)
    b = W.cg_rhs(A.n, seed=6)
    runs = [_solve(A, b, tol=1e-10, check_every=c) for c in (1, 3, 16, 1000)]
    runs.append(_solve(A, b, tol=1e-10, check_every=16))
    k0, x0 = runs[0][0]["iterations"], runs[0][1]
    for info, x in runs[1:]:
        assert info["iterations"] == k0
        assert np.array_equal(x, x0)
        assert np.array_equal(host(info["res"]), host(runs[0][0]["res"]))


def test_graph_replays_match_direct_launches():
    # the iteration batches replay a captured graph (kept while the call's
    # arguments repeat); every replay, with other GPU work and host
    # synchronisations in between, gives the bits of direct launches
    A = W.stencil27_csr(12, seed=5)
    b = W.cg_rhs(A.n, seed=6)
    rp, ci, va = _dev_csr(A)
    bd = dev(b, torch.float64)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")

    def solve(graph):
        x.zero_()
        info = rsm.cg_solve(rp, ci, va, bd, x, tol=1e-10, check_every=3, history=True, graph=graph)
        return info["iterations"], host(x), host(info["res"]), host(info["alpha"])

    ref = solve(False)
    y = torch.empty(A.n, dtype=torch.float64, device="cuda")
    for rep in range(3):
        got = solve(True)
        assert got[0] == ref[0], rep
        for g, r in zip(got[1:], ref[1:]):
            assert np.array_equal(g, r), rep
        rsm.run_csr(rp, ci, va, x, y)        # other work between replays
        torch.cuda.synchronize()
    # new arguments (another tolerance) capture a new graph
    x.zero_()
    info = rsm.cg_solve(rp, ci, va, bd, x, tol=1e-6, check_every=3)
    x2 = torch.zeros_like(x)
    info2 = rsm.cg_solve(rp, ci, va, bd, x2, tol=1e-6, check_every=3, graph=False)
    assert info["iterations"] == info2["iterations"] and torch.equal(x, x2)


def test_indefinite_matrix_reports_breakdown():
    A = W.dense_csr(np.diag([1.0, -2.0, 3.0, 4.0]))
    b = np.ones(4)
    with pytest.raises(ValueError):
        oracle.cg(A, b)
    info, x = _solve(A, b, tol=1e-10)
    assert info["breakdown"] and not info["converged"]
    assert np.all(np.isfinite(x))


def test_malformed_indices_rejected_when_checked():
    A = W.stencil27_csr(4, seed=5)
    ci = A.col_idx.copy()
    ci[5] = A.n + 3
    bad = W.Csr(A.n, A.row_ptr, ci, A.vals)
    rp, cidx, va = _dev_csr(bad)
    x = torch.zeros(A.n, dtype=torch.float64, device="cuda")
    with pytest.raises(rsm.RsmError) as e:
        rsm.cg_solve(rp, cidx, va, torch.ones(A.n, dtype=torch.float64, device="cuda"), x,
                     check_indices=True)
    assert e.value.name == "RSM_E_INVALID"
