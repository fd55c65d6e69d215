"""GPU parity of the sparse matrix-vector product (indirect tilers).

FP64 results are held to 1e-12 of the |term| sum, FP32 to 1e-5, against the
FP64 oracle on the same seeded matrices: random sparsity with empty rows,
repeated and unsorted columns, and the 27-point stencil matrix with the case
study's N = 132651 and NNZ = 3442951.
"""
import numpy as np
import pytest
import torch

import oracle
import rsm_workloads as W
from paper_1105_4424_amd import rsm

from .helpers import check_close, dev, host

pytestmark = pytest.mark.gpu


def _run(A, x, dtype):
    y = torch.full((A.n,), float("nan"), dtype=dtype, device="cuda")
    rsm.run_csr(dev(A.row_ptr), dev(A.col_idx), dev(A.vals, dtype), dev(x, dtype), y)
    return host(y)


@pytest.mark.parametrize("dtype,tol", [(torch.float64, 1e-12), (torch.float32, 1e-5)])
def test_random_csr(dtype, tol):
    rng = W.rng_for(505)
    for trial in range(30):
        nr, nc = int(rng.integers(1, 3000)), int(rng.integers(1, 500))
        A = W.random_csr(rng, nr, nc, max_per_row=int(rng.integers(1, 80)))
        x = rng.uniform(-1, 1, nc)
        if dtype == torch.float32:
            A = W.Csr(A.n, A.row_ptr, A.col_idx, A.vals.astype(np.float32).astype(np.float64))
            x = x.astype(np.float32).astype(np.float64)
        y, ya = oracle.run_csr(A, x)
        check_close(_run(A, x, dtype), y, ya, tol=tol, what="trial %d" % trial)


def test_stencil_case_study_size():
    A = W.stencil27_csr(51)
    x = W.rng_for(6).uniform(-1, 1, A.n)
    y, ya = oracle.run_csr(A, x)
    check_close(_run(A, x, torch.float64), y, ya, tol=1e-12, what="stencil 51^3")


def test_index_checks_and_guards():
    A = W.Csr(3, np.array([0, 2, 1, 3], np.int32), np.array([0, 1, 5], np.int32), np.ones(3))
    x = np.ones(2)
    y = torch.zeros(3, dtype=torch.float64, device="cuda")
    with pytest.raises(rsm.RsmError, match="RSM_E_INVALID"):
        rsm.run_csr(dev(A.row_ptr), dev(A.col_idx), dev(A.vals), dev(x), y, check_indices=True)
    # without the host check, an out-of-range column contributes nothing
    B = W.Csr(2, np.array([0, 2, 3], np.int32), np.array([0, 7, 1], np.int32), np.array([1.0, 5.0, 2.0]))
    got = _run(B, np.array([3.0, 4.0]), torch.float64)
    assert got.tolist() == [3.0, 8.0]
