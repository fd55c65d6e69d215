"""Shared test helpers: device transfer and the FP32 tolerance check.

Tolerance for FP32 tasks: per element |y_gpu - y_64| <= 1e-5 * sum_i |term_i|
(the oracle's |term| sum), the standard backward-error form of "1e-5
relative" that stays meaningful where a sum cancels to nearly zero.
"""
import sys

import numpy as np
import torch

FP32_TOL = 1e-5


def dev(a, dtype=None) -> torch.Tensor:
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def bf16_dev(bits: np.ndarray) -> torch.Tensor:
    """BF16 tensor on the GPU holding exactly the given bit patterns."""
    return torch.from_numpy(np.ascontiguousarray(bits).view(np.int16)).view(torch.bfloat16).cuda()


def host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def check_close(got, want, abs_sum, tol=FP32_TOL, what="", floor=0.0):
    got = np.asarray(got, dtype=np.float64).reshape(-1)
    want = np.asarray(want, dtype=np.float64).reshape(-1)
    abs_sum = np.asarray(abs_sum, dtype=np.float64).reshape(-1)
    assert got.shape == want.shape, (what, got.shape, want.shape)
    assert np.all(np.isfinite(got)), "%s: non-finite values" % what
    err = np.abs(got - want)
    bound = tol * abs_sum + floor
    bad = err > bound
    ratio = float(np.max(err / np.maximum(bound, 1e-300))) if err.size else 0.0
    norm = float(np.linalg.norm(got - want) / max(np.linalg.norm(want), 1e-300)) if err.size else 0.0
    assert not bad.any(), ("%s: %d of %d elements beyond %.1e * |terms| (worst ratio %.3g, "
                           "normwise rel err %.3g)" % (what, int(bad.sum()), bad.size, tol, ratio, norm))
    return {"max_ratio": ratio, "normwise": norm}


def say(*args):
    """Progress line for long GPU tests (flushed so a hang names its case)."""
    print(*args, flush=True)
    sys.stdout.flush()
