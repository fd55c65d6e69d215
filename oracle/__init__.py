"""CPU oracle of the RSM repetitive task (FP64, plain definition).

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg, never by the GPU library.  It shares no code
with the GPU path; the only module both use is the seeded input generator
(``rsm_workloads``), which holds data, not arithmetic.

The arithmetic lives in ``rsm_oracle.c`` (plain C99, FP64, built with gcc -O2,
no fast-math).  This wrapper only marshals arrays and, for the composition of
two stages and for batches, calls the C functions stage by stage / instance
by instance in list order.

Functions and the definition they follow (MARTE RSM / Array-OL tilers, the
repetitive tasks of the paper's Sec. 3, Sec. 6.1 and Sec. 7):
  indices      e(r,i) = (o + P r + F i) mod s, linearised row-major
  run          gather -> elementary task (COPY/SUM/WSUM/DOT) -> scatter
  run_sample   y(r) for selected repetitions only
  adjoint      transposed gather of the weighted sum, and its weight gradient
  chain_forward / chain_adjoint   two stages composed, loss sum(w * out^2)
  batch_run    independent tasks in list order
  run_csr      indirect tilers: the sparse matrix-vector product (Sec. 7)
  cg           the conjugate-gradient loop built from those tasks (Sec. 7,
               stopping rule of Table 1)
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import List, Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rsm_oracle.c")
_LIB = os.path.join(_HERE, "librsm_oracle.so")
_MAXR = 8

COPY, SUM, WSUM, DOT = 0, 1, 2, 3


class _OrTiler(ctypes.Structure):
    _fields_ = [
        ("arr_rank", ctypes.c_int32),
        ("pat_rank", ctypes.c_int32),
        ("shape", ctypes.c_int64 * _MAXR),
        ("origin", ctypes.c_int64 * _MAXR),
        ("paving", ctypes.c_int64 * (_MAXR * _MAXR)),
        ("fitting", ctypes.c_int64 * (_MAXR * _MAXR)),
        ("pat_shape", ctypes.c_int64 * _MAXR),
    ]


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-fPIC", "-shared",
                               "-fno-fast-math", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _bind(lib):
    """Declare the C signatures on a loaded oracle library."""
    P = ctypes.POINTER
    i64p = P(ctypes.c_int64)
    f64p = P(ctypes.c_double)
    tp = P(_OrTiler)
    lib.oracle_indices.argtypes = [ctypes.c_int32, i64p, tp, i64p]
    lib.oracle_run.argtypes = [ctypes.c_int32, i64p, ctypes.c_int32, tp, P(f64p),
                               tp, f64p, i64p, f64p, ctypes.c_int32, f64p]
    lib.oracle_run_sample.argtypes = [ctypes.c_int32, i64p, ctypes.c_int32, tp, P(f64p),
                                      ctypes.c_int64, ctypes.c_int32, f64p,
                                      ctypes.c_int64, i64p, f64p, f64p]
    lib.oracle_adjoint.argtypes = [ctypes.c_int32, i64p, tp, f64p, tp, f64p, f64p,
                                   f64p, f64p, f64p, f64p]
    i32p = P(ctypes.c_int32)
    lib.oracle_run_csr.argtypes = [ctypes.c_int64, i32p, i32p, f64p, f64p, f64p, f64p]
    for f in (lib.oracle_indices, lib.oracle_run, lib.oracle_run_sample, lib.oracle_adjoint,
              lib.oracle_run_csr):
        f.restype = ctypes.c_int
    lib.oracle_cg.argtypes = [ctypes.c_int64, i32p, i32p, f64p, f64p, f64p, ctypes.c_double,
                              ctypes.c_int64, f64p, f64p, f64p]
    lib.oracle_cg.restype = ctypes.c_int64
    return lib


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        _lib = _bind(ctypes.CDLL(_LIB))
    return _lib


# ---------------------------------------------------------------------------
# marshalling
# ---------------------------------------------------------------------------

def _tiler(t) -> _OrTiler:
    s = _OrTiler()
    shape = tuple(int(v) for v in t.array_shape)
    pshape = tuple(int(v) for v in t.pattern_shape)
    da, dp = len(shape), len(pshape)
    P = np.asarray(t.paving, dtype=np.int64).reshape(da, -1) if da else np.zeros((0, 0), np.int64)
    F = np.asarray(t.fitting, dtype=np.int64).reshape(da, dp)
    s.arr_rank, s.pat_rank = da, dp
    for d in range(da):
        s.shape[d] = shape[d]
        s.origin[d] = int(np.asarray(t.origin).reshape(-1)[d])
    dr = P.shape[1]
    for d in range(da):
        for k in range(dr):
            s.paving[d * dr + k] = int(P[d, k])
        for k in range(dp):
            s.fitting[d * dp + k] = int(F[d, k])
    for k in range(dp):
        s.pat_shape[k] = pshape[k]
    return s


def widen(a) -> np.ndarray:
    """Exact widening to FP64: float32/float64 as is; uint16 taken as BF16 bits."""
    a = np.asarray(a)
    if a.dtype == np.uint16:
        a = (a.astype(np.uint32) << np.uint32(16)).view(np.float32)
    return np.ascontiguousarray(a, dtype=np.float64)


def _i64(v) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(v, dtype=np.int64).reshape(-1))


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


# ---------------------------------------------------------------------------
# public functions
# ---------------------------------------------------------------------------

def indices(rep_shape: Sequence[int], tiler) -> np.ndarray:
    """Linear element offsets e(r, i), int64 [|rep|, |pattern|]."""
    lib = _load()
    rs = _i64(rep_shape if len(rep_shape) else [1])
    nr = int(np.prod(rep_shape)) if len(rep_shape) else 1
    npat = int(np.prod(tiler.pattern_shape)) if len(tiler.pattern_shape) else 1
    out = np.zeros((nr, npat), np.int64)
    rc = lib.oracle_indices(len(rep_shape), _ptr(rs, ctypes.c_int64),
                            ctypes.byref(_tiler(tiler)), _ptr(out, ctypes.c_int64))
    assert rc == 0
    return out


class RunResult:
    def __init__(self, out, hits, abs_sum):
        self.out = out          # FP64, output-array shaped
        self.hits = hits        # int64 write count per output element
        self.abs_sum = abs_sum  # FP64 sum of |terms| of the written value


def run(problem, inputs: List[np.ndarray], prior: Optional[np.ndarray] = None) -> RunResult:
    """Whole repetitive task in FP64.  `prior` = output contents before the
    task (default NaN, so uncovered elements show)."""
    lib = _load()
    xs = [widen(a).reshape(-1) for a in inputs]
    n_in = len(xs)
    tl = (_OrTiler * n_in)(*[_tiler(t) for t in problem.inputs])
    xp = (ctypes.POINTER(ctypes.c_double) * n_in)(*[_ptr(a, ctypes.c_double) for a in xs])
    oshape = tuple(problem.output.array_shape)
    out = (np.full(oshape, np.nan) if prior is None else widen(prior).copy()).reshape(-1)
    hits = np.zeros(out.size, np.int64)
    oabs = np.zeros(out.size, np.float64)
    c = widen(problem.coeffs).reshape(-1) if problem.coeffs is not None else np.zeros(1)
    rs = _i64(problem.rep_shape if len(problem.rep_shape) else [1])
    rc = lib.oracle_run(len(problem.rep_shape), _ptr(rs, ctypes.c_int64), n_in, tl, xp,
                        ctypes.byref(_tiler(problem.output)), _ptr(out, ctypes.c_double),
                        _ptr(hits, ctypes.c_int64), _ptr(oabs, ctypes.c_double),
                        int(problem.task), _ptr(c, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle: unsupported task / pattern combination")
    return RunResult(out.reshape(oshape), hits.reshape(oshape), oabs.reshape(oshape))


def run_sample(problem, inputs: List[np.ndarray], rep_flat: np.ndarray):
    """(y, abs_sum) for the listed flat repetition indices; [n, |out pattern|]."""
    lib = _load()
    xs = [widen(a).reshape(-1) for a in inputs]
    n_in = len(xs)
    tl = (_OrTiler * n_in)(*[_tiler(t) for t in problem.inputs])
    xp = (ctypes.POINTER(ctypes.c_double) * n_in)(*[_ptr(a, ctypes.c_double) for a in xs])
    n_out = int(np.prod(problem.output.pattern_shape)) if len(problem.output.pattern_shape) else 1
    rf = _i64(rep_flat)
    y = np.zeros((rf.size, n_out))
    ya = np.zeros((rf.size, n_out))
    c = widen(problem.coeffs).reshape(-1) if problem.coeffs is not None else np.zeros(1)
    rs = _i64(problem.rep_shape if len(problem.rep_shape) else [1])
    rc = lib.oracle_run_sample(len(problem.rep_shape), _ptr(rs, ctypes.c_int64), n_in, tl, xp,
                               n_out, int(problem.task), _ptr(c, ctypes.c_double),
                               rf.size, _ptr(rf, ctypes.c_int64),
                               _ptr(y, ctypes.c_double), _ptr(ya, ctypes.c_double))
    if rc != 0:
        raise ValueError("oracle: unsupported task / pattern combination")
    return y, ya


class AdjointResult:
    def __init__(self, gx, gx_abs, gc, gc_abs):
        self.gx, self.gx_abs, self.gc, self.gc_abs = gx, gx_abs, gc, gc_abs


def adjoint(problem, x: np.ndarray, gy: np.ndarray) -> AdjointResult:
    """Adjoint of a SUM task (scalar output pattern) or a WSUM task (any
    output pattern; weight gradient shaped like the coefficients, i.e.
    output pattern x input pattern, or the input pattern when scalar)."""
    lib = _load()
    t = problem.inputs[0]
    xw = widen(x).reshape(-1)
    gyw = widen(gy).reshape(-1)
    gx = np.zeros(xw.size)
    gxa = np.zeros(xw.size)
    npat = int(np.prod(t.pattern_shape)) if len(t.pattern_shape) else 1
    nq = int(np.prod(problem.output.pattern_shape)) if len(problem.output.pattern_shape) else 1
    gc = np.zeros(npat * nq)
    gca = np.zeros(npat * nq)
    weighted = problem.task == WSUM
    c = widen(problem.coeffs).reshape(-1) if weighted else None
    rs = _i64(problem.rep_shape if len(problem.rep_shape) else [1])
    null = ctypes.POINTER(ctypes.c_double)()
    rc = lib.oracle_adjoint(len(problem.rep_shape), _ptr(rs, ctypes.c_int64),
                            ctypes.byref(_tiler(t)), _ptr(xw, ctypes.c_double),
                            ctypes.byref(_tiler(problem.output)), _ptr(gyw, ctypes.c_double),
                            _ptr(c, ctypes.c_double) if weighted else null,
                            _ptr(gx, ctypes.c_double), _ptr(gxa, ctypes.c_double),
                            _ptr(gc, ctypes.c_double) if weighted else null,
                            _ptr(gca, ctypes.c_double) if weighted else null)
    if rc != 0:
        raise ValueError("oracle: the adjoint of SUM needs a scalar output pattern")
    shp = tuple(t.array_shape)
    cshape = tuple(t.pattern_shape) if nq == 1 else tuple(problem.output.pattern_shape) + tuple(t.pattern_shape)
    return AdjointResult(gx.reshape(shp), gxa.reshape(shp),
                         gc.reshape(cshape) if weighted else None,
                         gca.reshape(cshape) if weighted else None)


class ChainResult:
    pass


def chain_forward(stages, x: np.ndarray) -> List[RunResult]:
    """Stage k's output array is stage k+1's input array."""
    res, cur = [], x
    for st in stages:
        r = run(st, [cur])
        res.append(r)
        cur = r.out
    return res


def chain_adjoint(stages, x: np.ndarray, w: np.ndarray) -> ChainResult:
    """Loss L = sum(w * out^2) of the composed stages; dL/dout = 2 w out.
    The adjoint runs the stages in reverse, each stage's input gradient being
    the previous (later) stage's output gradient.  Returns the loss, the
    input gradient and every stage's weight gradient, with |term| sums."""
    fw = chain_forward(stages, x)
    out = fw[-1].out
    ww = widen(w)
    res = ChainResult()
    res.forward = fw
    res.loss = float(np.sum(ww * out * out))
    g = 2.0 * ww * out
    gcs, gcas = [None] * len(stages), [None] * len(stages)
    gx_abs = None
    for k in range(len(stages) - 1, -1, -1):
        xin = x if k == 0 else fw[k - 1].out
        a = adjoint(stages[k], xin, g)
        gcs[k], gcas[k] = a.gc, a.gc_abs
        g, gx_abs = a.gx, a.gx_abs
    res.gx, res.gx_abs, res.gc, res.gc_abs = g, gx_abs, gcs, gcas
    return res


def batch_run(problems, inputs) -> List[RunResult]:
    """Independent tasks in the order listed."""
    return [run(p, [x]) for p, x in zip(problems, inputs)]


def run_csr(csr, x: np.ndarray):
    """y = A x for a CSR matrix (row_ptr, col_idx, vals), FP64; returns (y, |terms| sums)."""
    lib = _load()
    rp = np.ascontiguousarray(csr.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(csr.col_idx, dtype=np.int32)
    va = widen(csr.vals).reshape(-1)
    xw = widen(x).reshape(-1)
    y = np.zeros(csr.n)
    ya = np.zeros(csr.n)
    rc = lib.oracle_run_csr(csr.n, _ptr(rp, ctypes.c_int32), _ptr(ci, ctypes.c_int32),
                            _ptr(va, ctypes.c_double), _ptr(xw, ctypes.c_double),
                            _ptr(y, ctypes.c_double), _ptr(ya, ctypes.c_double))
    assert rc == 0
    return y, ya


class CgResult:
    def __init__(self, x, iters, res, alpha, beta):
        self.x = x            # last iterate
        self.iters = iters    # iterations taken
        self.res = res        # ||r_k||, k = 0..iters
        self.alpha = alpha    # step lengths, k = 0..iters-1
        self.beta = beta      # direction updates, k = 0..iters-1


def cg(csr, b: np.ndarray, tol: float = 1e-10, max_iter: Optional[int] = None,
       x0: Optional[np.ndarray] = None) -> CgResult:
    """Conjugate gradient on a CSR matrix, FP64, from x0 (default zero) until
    ||r|| <= tol ||b|| or max_iter iterations (default n)."""
    lib = _load()
    n = int(csr.n)
    if max_iter is None:
        max_iter = n
    rp = np.ascontiguousarray(csr.row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(csr.col_idx, dtype=np.int32)
    va = widen(csr.vals).reshape(-1)
    bw = np.ascontiguousarray(widen(b).reshape(-1))
    x = np.zeros(n) if x0 is None else np.array(widen(x0).reshape(-1), dtype=np.float64)
    res = np.zeros(max_iter + 1)
    alpha = np.zeros(max(max_iter, 1))
    beta = np.zeros(max(max_iter, 1))
    k = lib.oracle_cg(n, _ptr(rp, ctypes.c_int32), _ptr(ci, ctypes.c_int32),
                      _ptr(va, ctypes.c_double), _ptr(bw, ctypes.c_double),
                      _ptr(x, ctypes.c_double), float(tol), int(max_iter),
                      _ptr(res, ctypes.c_double), _ptr(alpha, ctypes.c_double),
                      _ptr(beta, ctypes.c_double))
    if k < 0:
        raise ValueError("conjugate gradient broke down: matrix not positive definite")
    return CgResult(x, int(k), res[:k + 1].copy(), alpha[:k].copy(), beta[:k].copy())
