"""torch-facing wrappers over the C-ABI (marshalling only).

Tiler descriptions are duck-typed: any object with ``array_shape``,
``origin``, ``paving`` (d_a x d_r), ``fitting`` (d_a x d_p) and
``pattern_shape`` works (``rsm_workloads.Tiler`` is one).  A problem has
``rep_shape``, ``inputs`` (list of tilers), ``output`` (tiler) and ``task``
(0 copy, 1 sum, 2 weighted sum, 3 dot).  Arrays are contiguous torch
tensors on the GPU; weights are passed as device tensors.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import numpy as np
import torch

from . import _abi

_DTYPES = {torch.float32: _abi.F32, torch.bfloat16: _abi.BF16, torch.float64: _abi.F64,
           torch.int64: _abi.I64}
_COMPUTE = {"f32": _abi.F32, "bf16": _abi.BF16, "f64": _abi.F64}


class RsmError(RuntimeError):
    def __init__(self, status: int, detail: str):
        lib = _abi.load()
        name = lib.rsm_status_string(status).decode()
        super().__init__("%s: %s" % (name, detail))
        self.status = status
        self.name = name


def _check(status: int):
    if status != _abi.OK:
        raise RsmError(status, _abi.load().rsm_last_error().decode())


def _space(rep_shape: Sequence[int]) -> _abi.Space:
    s = _abi.Space()
    s.rank = len(rep_shape)
    for k, v in enumerate(list(rep_shape)[:_abi.MAX_RANK]):
        s.shape[k] = int(v)
    return s


def _tiler(t, dtype: int) -> _abi.Tiler:
    s = _abi.Tiler()
    shape = tuple(int(v) for v in t.array_shape)
    pshape = tuple(int(v) for v in t.pattern_shape)
    da, dp = len(shape), len(pshape)
    P = np.asarray(t.paving, dtype=np.int64).reshape(da, -1) if da else np.zeros((0, 0), np.int64)
    F = np.asarray(t.fitting, dtype=np.int64).reshape(da, dp)
    o = np.asarray(t.origin, dtype=np.int64).reshape(da)
    # ranks are passed as given (the library rejects ranks above 8); only the
    # entries that fit in the fixed-size arrays are copied
    s.array_rank, s.pattern_rank, s.dtype = da, dp, dtype
    M = _abi.MAX_RANK
    for d in range(min(da, M)):
        s.array_shape[d] = shape[d]
        s.origin[d] = int(o[d])
        for k in range(min(P.shape[1], M)):
            s.paving[d][k] = int(P[d, k])
        for k in range(min(dp, M)):
            s.fitting[d][k] = int(F[d, k])
    for k in range(min(dp, M)):
        s.pattern_shape[k] = pshape[k]
    return s


def _dcode(t: torch.Tensor) -> int:
    try:
        return _DTYPES[t.dtype]
    except KeyError:
        raise TypeError("unsupported dtype %s" % t.dtype)


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    if t.device.type != "cuda":
        raise ValueError("arrays must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("arrays must be contiguous (row-major)")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _task(kind: int, compute: int, coeffs: Optional[torch.Tensor]) -> _abi.Task:
    t = _abi.Task()
    t.kind, t.compute = int(kind), int(compute)
    t.coeffs = _ptr(coeffs).value if coeffs is not None else None
    return t


def _compute_for(problem, x: torch.Tensor) -> int:
    c = getattr(problem, "compute", "f32")
    if x.dtype == torch.float64:
        return _abi.F64
    return _COMPUTE.get(c, _abi.F32)


def _out_dtype_code(problem, x: torch.Tensor) -> int:
    if problem.task == _abi.TASK_COPY:
        return _dcode(x)
    return _abi.F64 if x.dtype == torch.float64 else _abi.F32


# ---------------------------------------------------------------------------
# plain calls
# ---------------------------------------------------------------------------

def validate(problem, dtypes: Sequence[torch.dtype] = (torch.float32,),
             check_single_assign: bool = False, compute: str = None):
    lib = _abi.load()
    codes = [_DTYPES[d] for d in dtypes]
    tin = (_abi.Tiler * len(problem.inputs))(*[_tiler(t, codes[min(i, len(codes) - 1)])
                                               for i, t in enumerate(problem.inputs)])
    c0 = codes[0]
    out_code = c0 if problem.task == _abi.TASK_COPY else (_abi.F64 if c0 == _abi.F64 else _abi.F32)
    comp = _COMPUTE[compute] if compute else (_abi.F64 if c0 == _abi.F64 else
                                              _COMPUTE.get(getattr(problem, "compute", "f32")))
    task = _abi.Task(problem.task, comp, ctypes.c_void_p(1).value)
    _check(lib.rsm_validate(ctypes.byref(_space(problem.rep_shape)), tin, len(problem.inputs),
                            ctypes.byref(_tiler(problem.output, out_code)), ctypes.byref(task),
                            _abi.CHECK_SINGLE_ASSIGN if check_single_assign else 0))


def plan_ports(problem, dtypes: Sequence[torch.dtype] = (torch.float32,), flags: int = 0):
    """Where the planned kernel keeps each port (inputs, output, then the
    coefficients of a weighted sum): a list of (space, bytes per workgroup)
    with space one of "global", "constant", "local", "private"."""
    lib = _abi.load()
    codes = [_DTYPES[d] for d in dtypes]
    tin = (_abi.Tiler * len(problem.inputs))(*[_tiler(t, codes[min(i, len(codes) - 1)])
                                               for i, t in enumerate(problem.inputs)])
    c0 = codes[0]
    out_code = c0 if problem.task == _abi.TASK_COPY else (_abi.F64 if c0 == _abi.F64 else _abi.F32)
    comp = _abi.F64 if c0 == _abi.F64 else _COMPUTE.get(getattr(problem, "compute", "f32"))
    task = _abi.Task(problem.task, comp, ctypes.c_void_p(1).value)
    ports = (_abi.PortPlacement * 8)()
    n = ctypes.c_int32(0)
    _check(lib.rsm_plan_ports(ctypes.byref(_space(problem.rep_shape)), tin, len(problem.inputs),
                              ctypes.byref(_tiler(problem.output, out_code)), ctypes.byref(task), flags,
                              ports, 8, ctypes.byref(n)))
    return [(_abi.MEM_SPACES[ports[k].space], int(ports[k].bytes_per_workgroup)) for k in range(n.value)]


def _spaces(spaces):
    """Placement request: a sequence of space names ("global", "constant",
    "local", "private", "any") or None, one per port (inputs, output,
    coefficients)."""
    if spaces is None:
        return None, 0
    arr = (ctypes.c_int32 * len(spaces))(*[_abi.MEM_CODES[s] for s in spaces])
    return arr, len(spaces)


def plan_placed(problem, spaces, dtypes: Sequence[torch.dtype] = (torch.float32,), flags: int = 0):
    """(family name, [(space, bytes per workgroup) per port]) of the kernel
    family that keeps the ports where `spaces` asks (host only); raises
    RsmError (RSM_E_UNSUPPORTED) when no family does."""
    lib = _abi.load()
    codes = [_DTYPES[d] for d in dtypes]
    tin = (_abi.Tiler * len(problem.inputs))(*[_tiler(t, codes[min(i, len(codes) - 1)])
                                               for i, t in enumerate(problem.inputs)])
    c0 = codes[0]
    out_code = c0 if problem.task == _abi.TASK_COPY else (_abi.F64 if c0 == _abi.F64 else _abi.F32)
    comp = _abi.F64 if c0 == _abi.F64 else _COMPUTE.get(getattr(problem, "compute", "f32"))
    task = _abi.Task(problem.task, comp, ctypes.c_void_p(1).value)
    sp, ns = _spaces(spaces)
    buf = ctypes.create_string_buffer(64)
    ports = (_abi.PortPlacement * 8)()
    n = ctypes.c_int32(0)
    _check(lib.rsm_plan_placed(ctypes.byref(_space(problem.rep_shape)), tin, len(problem.inputs),
                               ctypes.byref(_tiler(problem.output, out_code)), ctypes.byref(task), flags,
                               sp, ns, buf, 64, ports, 8, ctypes.byref(n)))
    return buf.value.decode(), [(_abi.MEM_SPACES[ports[k].space], int(ports[k].bytes_per_workgroup))
                                for k in range(n.value)]


def run_placed(problem, inputs: List[torch.Tensor], out: torch.Tensor, spaces, coeffs: torch.Tensor = None,
               flags: int = 0, stream=None) -> torch.Tensor:
    """run() by the kernel family that keeps the ports where `spaces` asks."""
    lib = _abi.load()
    n = len(inputs)
    tin = (_abi.Tiler * n)(*[_tiler(t, _dcode(x)) for t, x in zip(problem.inputs, inputs)])
    ptrs = (ctypes.c_void_p * n)(*[_ptr(x).value for x in inputs])
    task = _task(problem.task, _compute_for(problem, inputs[0]), coeffs)
    sp, ns = _spaces(spaces)
    _check(lib.rsm_run_placed(ctypes.byref(_space(problem.rep_shape)), tin, ptrs, n,
                              ctypes.byref(_tiler(problem.output, _dcode(out))), _ptr(out),
                              ctypes.byref(task), sp, ns, flags, _stream(stream)))
    return out


def plan(problem, dtypes: Sequence[torch.dtype] = (torch.float32,), flags: int = 0,
         compute: str = None) -> str:
    """Kernel family the planner picks (host only)."""
    lib = _abi.load()
    codes = [_DTYPES[d] for d in dtypes]
    tin = (_abi.Tiler * len(problem.inputs))(*[_tiler(t, codes[min(i, len(codes) - 1)])
                                               for i, t in enumerate(problem.inputs)])
    c0 = codes[0]
    out_code = c0 if problem.task == _abi.TASK_COPY else (_abi.F64 if c0 == _abi.F64 else _abi.F32)
    comp = _COMPUTE[compute] if compute else (_abi.F64 if c0 == _abi.F64 else
                                              _COMPUTE.get(getattr(problem, "compute", "f32")))
    task = _abi.Task(problem.task, comp, ctypes.c_void_p(1).value)
    buf = ctypes.create_string_buffer(64)
    _check(lib.rsm_plan(ctypes.byref(_space(problem.rep_shape)), tin, len(problem.inputs),
                        ctypes.byref(_tiler(problem.output, out_code)), ctypes.byref(task), flags,
                        buf, 64))
    return buf.value.decode()


def indices(rep_shape: Sequence[int], tiler, device="cuda", stream=None) -> torch.Tensor:
    """Index table e(r, i) (linear offsets), int64 [|s_r|, |s_p|], on the GPU."""
    lib = _abi.load()
    nr = int(np.prod(rep_shape)) if len(rep_shape) else 1
    np_ = int(np.prod(tiler.pattern_shape)) if len(tiler.pattern_shape) else 1
    out = torch.empty((nr, np_), dtype=torch.int64, device=device)
    _check(lib.rsm_indices(ctypes.byref(_space(rep_shape)), ctypes.byref(_tiler(tiler, _abi.F32)),
                           _ptr(out), _stream(stream)))
    return out


def run(problem, inputs: List[torch.Tensor], out: torch.Tensor, coeffs: torch.Tensor = None,
        flags: int = 0, stream=None, compute: str = None) -> torch.Tensor:
    lib = _abi.load()
    n = len(inputs)
    tin = (_abi.Tiler * n)(*[_tiler(t, _dcode(x)) for t, x in zip(problem.inputs, inputs)])
    ptrs = (ctypes.c_void_p * n)(*[_ptr(x).value for x in inputs])
    comp = _COMPUTE[compute] if compute else _compute_for(problem, inputs[0])
    task = _task(problem.task, comp, coeffs)
    _check(lib.rsm_run(ctypes.byref(_space(problem.rep_shape)), tin, ptrs, n,
                       ctypes.byref(_tiler(problem.output, _dcode(out))), _ptr(out),
                       ctypes.byref(task), flags, _stream(stream)))
    return out


def plan_cache_hits() -> int:
    """rsm_run calls on this thread launched from a kept plan (no validation
    or planning on the host)."""
    return int(_abi.load().rsm_plan_cache_hits())


class Prepared:
    """One task validated and planned once (rsm_prepare); run() passes only
    the arrays' addresses and the stream.  `dtypes` are the input arrays'
    dtypes (the output's follows from the task)."""

    def __init__(self, problem, dtypes: Sequence[torch.dtype] = (torch.float32,), flags: int = 0,
                 compute: str = None):
        lib = _abi.load()
        n = len(problem.inputs)
        self.in_dtypes = [dtypes[min(k, len(dtypes) - 1)] for k in range(n)]
        codes = [_DTYPES[d] for d in self.in_dtypes]
        tin = (_abi.Tiler * n)(*[_tiler(t, c) for t, c in zip(problem.inputs, codes)])
        c0 = codes[0]
        out_code = c0 if problem.task == _abi.TASK_COPY else (_abi.F64 if c0 == _abi.F64 else _abi.F32)
        self.out_dtype = {v: k for k, v in _DTYPES.items()}[out_code]
        comp = _COMPUTE[compute] if compute else (_abi.F64 if c0 == _abi.F64 else
                                                  _COMPUTE.get(getattr(problem, "compute", "f32")))
        task = _abi.Task(problem.task, comp, None)
        h = ctypes.c_void_p()
        _check(lib.rsm_prepare(ctypes.byref(_space(problem.rep_shape)), tin, n,
                               ctypes.byref(_tiler(problem.output, out_code)), ctypes.byref(task), flags,
                               ctypes.byref(h)))
        self._lib, self._h, self.n_in = lib, h, n
        self._ptrs = (ctypes.c_void_p * n)()
        buf = ctypes.create_string_buffer(64)
        _check(lib.rsm_prepared_name(h, buf, 64))
        self.name = buf.value.decode()

    def run(self, inputs: List[torch.Tensor], out: torch.Tensor, coeffs: torch.Tensor = None,
            stream=None) -> torch.Tensor:
        if self._h is None:
            raise RuntimeError("prepared task is closed")
        if len(inputs) != self.n_in:
            raise ValueError("expected %d input arrays" % self.n_in)
        for k, x in enumerate(inputs):
            if x.dtype != self.in_dtypes[k]:
                raise TypeError("input %d is %s, prepared for %s" % (k, x.dtype, self.in_dtypes[k]))
            self._ptrs[k] = _ptr(x).value
        if out.dtype != self.out_dtype:
            raise TypeError("output is %s, prepared for %s" % (out.dtype, self.out_dtype))
        _check(self._lib.rsm_run_prepared(self._h, self._ptrs, _ptr(out), _ptr(coeffs), _stream(stream)))
        return out

    def close(self):
        if self._h is not None:
            self._lib.rsm_prepared_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _stages(stages, coeffs, x_dtype=torch.float32):
    n = len(stages)
    arr = (_abi.Stage * n)()
    for k, st in enumerate(stages):
        arr[k].rep = _space(st.rep_shape)
        arr[k].in_ = _tiler(st.inputs[0], _DTYPES[x_dtype])
        arr[k].out = _tiler(st.output, _abi.F64 if x_dtype == torch.float64 else _abi.F32)
        c = coeffs[k] if coeffs is not None else None
        arr[k].task = _task(st.task, _abi.F64 if x_dtype == torch.float64 else _abi.F32, c)
    return arr


def run_chain(stages, x: torch.Tensor, out: torch.Tensor, coeffs: Sequence[torch.Tensor],
              mids: Optional[Sequence[torch.Tensor]] = None, flags: int = 0, stream=None):
    lib = _abi.load()
    arr = _stages(stages, coeffs, x.dtype)
    mp = None
    if mids is not None:
        mp = (ctypes.c_void_p * len(mids))(*[_ptr(m).value for m in mids])
    _check(lib.rsm_run_chain(arr, len(stages), _ptr(x), mp, _ptr(out), flags, _stream(stream)))
    return out


def run_adjoint(problem, x: Optional[torch.Tensor], gy: torch.Tensor,
                gx: Optional[torch.Tensor] = None, gc: Optional[torch.Tensor] = None,
                coeffs: Optional[torch.Tensor] = None, flags: int = 0, stream=None):
    lib = _abi.load()
    task = _task(problem.task, _abi.F32, coeffs)
    _check(lib.rsm_run_adjoint(ctypes.byref(_space(problem.rep_shape)),
                               ctypes.byref(_tiler(problem.inputs[0], _abi.F32)), _ptr(x),
                               ctypes.byref(_tiler(problem.output, _abi.F32)), _ptr(gy),
                               ctypes.byref(task), _ptr(gx), _ptr(gc), flags, _stream(stream)))


def run_chain_adjoint(stages, x: torch.Tensor, gy: torch.Tensor, gx: Optional[torch.Tensor],
                      gcs: Optional[Sequence[Optional[torch.Tensor]]], coeffs: Sequence[torch.Tensor],
                      mids: Optional[Sequence[torch.Tensor]] = None, flags: int = 0, stream=None):
    lib = _abi.load()
    arr = _stages(stages, coeffs)
    mp = None
    if mids is not None:
        mp = (ctypes.c_void_p * len(mids))(*[_ptr(m).value for m in mids])
    gp = None
    if gcs is not None:
        gp = (ctypes.c_void_p * len(stages))(*[(_ptr(g).value if g is not None else None) for g in gcs])
    _check(lib.rsm_run_chain_adjoint(arr, len(stages), _ptr(x), mp, _ptr(gy), _ptr(gx), gp, flags,
                                     _stream(stream)))


def run_chain_train(stages, x: torch.Tensor, w: torch.Tensor, out: torch.Tensor, gx: Optional[torch.Tensor],
                    coeffs: Sequence[torch.Tensor], gcs=None, flags: int = 0, stream=None) -> torch.Tensor:
    """Forward, dL/dout = 2 w out and the adjoint of a two-stage chain in one
    pass (loss sum(w * out^2)); see Chain.train."""
    return Chain(stages, coeffs).train(x, w, out, gx, gcs, flags=flags, stream=stream)


def run_csr(row_ptr: torch.Tensor, col_idx: torch.Tensor, vals: torch.Tensor, x: torch.Tensor,
            y: torch.Tensor, check_indices: bool = False, stream=None) -> torch.Tensor:
    """y = A x for a CSR matrix (indirect tilers; int32 indices on the GPU)."""
    lib = _abi.load()
    if row_ptr.dtype != torch.int32 or col_idx.dtype != torch.int32:
        raise TypeError("row_ptr and col_idx must be int32")
    if not (vals.dtype == x.dtype == y.dtype):
        raise TypeError("vals, x and y must share a dtype")
    _check(lib.rsm_run_csr(y.numel(), x.numel(), col_idx.numel(), _ptr(row_ptr), _ptr(col_idx),
                           _ptr(vals), _ptr(x), _ptr(y), _dcode(vals),
                           _abi.CHECK_INDICES if check_indices else 0, _stream(stream)))
    return y


def time_next_kernel(start: "torch.cuda.Event", stop: "torch.cuda.Event") -> None:
    """Arm the measurement hook: the next chain call on this thread records
    `start` / `stop` (timing events) immediately around its fused kernel."""
    lib = _abi.load()
    for ev in (start, stop):
        if not ev.cuda_event:   # torch creates the event on its first record
            ev.record()
    _check(lib.rsm_time_next_kernel(ctypes.c_void_p(start.cuda_event), ctypes.c_void_p(stop.cuda_event)))


def cg_solve(row_ptr: torch.Tensor, col_idx: torch.Tensor, vals: torch.Tensor, b: torch.Tensor,
             x: torch.Tensor, tol: float = 1e-10, max_iter: Optional[int] = None, check_every: int = 16,
             history: bool = False, check_indices: bool = False, graph: bool = True, stream=None) -> dict:
    """Conjugate gradient on an SPD CSR matrix, FP64, in place on x (x0 in,
    last iterate out).  Blocking: the host reads the device state every
    check_every iterations.  Returns the iteration count, final residual
    norm, ||b||, converged / breakdown flags and, with history=True, device
    tensors res (||r_k||), alpha and beta."""
    lib = _abi.load()
    if row_ptr.dtype != torch.int32 or col_idx.dtype != torch.int32:
        raise TypeError("row_ptr and col_idx must be int32")
    if not (vals.dtype == b.dtype == x.dtype == torch.float64):
        raise TypeError("vals, b and x must be float64")
    n = b.numel()
    if x.numel() != n or row_ptr.numel() != n + 1:
        raise ValueError("shape mismatch: b, x need n entries and row_ptr n + 1")
    if max_iter is None:
        max_iter = n
    res = alpha = beta = None
    if history:
        res = torch.zeros(max_iter + 1, dtype=torch.float64, device=b.device)
        alpha = torch.zeros(max(max_iter, 1), dtype=torch.float64, device=b.device)
        beta = torch.zeros(max(max_iter, 1), dtype=torch.float64, device=b.device)
    info = _abi.CgInfo()
    _check(lib.rsm_cg_solve(n, col_idx.numel(), _ptr(row_ptr), _ptr(col_idx), _ptr(vals), _ptr(b),
                            _ptr(x), float(tol), int(max_iter), int(check_every),
                            (_abi.CHECK_INDICES if check_indices else 0) | (0 if graph else _abi.NO_GRAPH),
                            _ptr(res) if res is not None else None,
                            _ptr(alpha) if alpha is not None else None,
                            _ptr(beta) if beta is not None else None, ctypes.byref(info), _stream(stream)))
    out = {"iterations": int(info.iterations), "residual_norm": float(info.residual_norm),
           "rhs_norm": float(info.rhs_norm), "converged": bool(info.converged),
           "breakdown": bool(info.breakdown)}
    if history:
        k = out["iterations"]
        out["res"], out["alpha"], out["beta"] = res[:k + 1], alpha[:k], beta[:k]
    return out


# ---------------------------------------------------------------------------
# autograd
# ---------------------------------------------------------------------------

class TiledTask(torch.autograd.Function):
    """y = T_c(x) for a single-input SUM / WSUM task; backward runs the
    adjoint kernels (transposed-tiler scatter-add for x, pattern reduction
    for the weights)."""

    @staticmethod
    def forward(ctx, x, coeffs, problem, flags=0):
        out = torch.zeros(tuple(problem.output.array_shape), device=x.device, dtype=torch.float32)
        run(problem, [x], out, coeffs=coeffs, flags=flags)
        ctx.save_for_backward(x, coeffs)
        ctx.problem, ctx.flags = problem, flags
        return out

    @staticmethod
    def backward(ctx, gy):
        x, coeffs = ctx.saved_tensors
        gy = gy.contiguous()
        gx = torch.empty_like(x) if ctx.needs_input_grad[0] else None
        gc = torch.empty_like(coeffs) if (coeffs is not None and ctx.needs_input_grad[1]) else None
        if gx is not None or gc is not None:
            run_adjoint(ctx.problem, x, gy, gx, gc, coeffs, ctx.flags & _abi.FORCE_GENERIC)
        return gx, gc, None, None


class TiledChain(torch.autograd.Function):
    """out = V(H(x)) for two chained weighted-sum stages.  fuse=True keeps the
    intermediate on chip (forward) and recomputes it in the fused adjoint."""

    @staticmethod
    def forward(ctx, x, ch, cv, stages, fuse=True):
        out = torch.empty(tuple(stages[1].output.array_shape), device=x.device, dtype=torch.float32)
        if fuse:
            run_chain(stages, x, out, [ch, cv])
            mid = None
        else:
            mid = torch.empty(tuple(stages[0].output.array_shape), device=x.device, dtype=torch.float32)
            run_chain(stages, x, out, [ch, cv], mids=[mid], flags=_abi.NO_FUSE)
        ctx.save_for_backward(x, ch, cv)
        ctx.stages, ctx.mid, ctx.fuse = stages, mid, fuse
        return out

    @staticmethod
    def backward(ctx, gy):
        x, ch, cv = ctx.saved_tensors
        gy = gy.contiguous()
        gx = torch.empty_like(x) if ctx.needs_input_grad[0] else None
        gch = torch.empty_like(ch) if ctx.needs_input_grad[1] else None
        gcv = torch.empty_like(cv) if ctx.needs_input_grad[2] else None
        run_chain_adjoint(ctx.stages, x, gy, gx, [gch, gcv], [ch, cv],
                          mids=None if ctx.fuse else [ctx.mid],
                          flags=0 if ctx.fuse else _abi.NO_FUSE)
        return gx, gch, gcv, None, None


# ---------------------------------------------------------------------------
# batches
# ---------------------------------------------------------------------------

class Batch:
    """Many independent single-input tasks run by one persistent launch
    (captured once into a HIP graph, replayed by later calls)."""

    def __init__(self, problems, inputs: Sequence[torch.Tensor], outputs: Sequence[torch.Tensor],
                 coeffs: Sequence[Optional[torch.Tensor]], tune_cache: Optional[str] = None,
                 flags: int = 0, stream=None):
        lib = _abi.load()
        n = len(problems)
        arr = (_abi.Problem * n)()
        for k, p in enumerate(problems):
            arr[k].rep = _space(p.rep_shape)
            arr[k].in_ = _tiler(p.inputs[0], _dcode(inputs[k]))
            arr[k].out = _tiler(p.output, _dcode(outputs[k]))
            arr[k].task = _task(p.task, _compute_for(p, inputs[k]), coeffs[k])
            arr[k].d_in = _ptr(inputs[k]).value
            arr[k].d_out = _ptr(outputs[k]).value
        # the handle uses these buffers on every run: keep them alive
        self._keep = (list(inputs), list(outputs), list(coeffs))
        self._h = ctypes.c_void_p()
        _check(lib.rsm_batch_create(arr, n, tune_cache.encode() if tune_cache else None, flags,
                                    _stream(stream), ctypes.byref(self._h)))
        self.n = n

    def run(self, stream=None):
        _check(_abi.load().rsm_batch_run(self._h, _stream(stream)))

    def run_plain(self, stream=None):
        """Same problems and tile shapes, one launch per problem (no graph)."""
        _check(_abi.load().rsm_batch_run_plain(self._h, _stream(stream)))

    def info(self) -> dict:
        i = _abi.BatchInfo()
        _check(_abi.load().rsm_batch_query(self._h, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in _abi.BatchInfo._fields_}

    def tile(self, k: int):
        r, c = ctypes.c_int32(), ctypes.c_int32()
        _check(_abi.load().rsm_batch_tile(self._h, k, ctypes.byref(r), ctypes.byref(c)))
        return r.value, c.value

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            _abi.load().rsm_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Chain:
    """A chain whose descriptors are marshalled once; forward() and adjoint()
    then cost one C call each (for tight loops)."""

    def __init__(self, stages, coeffs: Sequence[torch.Tensor]):
        self.stages = stages
        self._coeffs = list(coeffs)
        self._arr = _stages(stages, coeffs)
        self._n = len(stages)
        self._lib = _abi.load()

    def forward(self, x, out, mids=None, flags: int = 0, stream=None):
        mp = None
        if mids is not None:
            mp = (ctypes.c_void_p * len(mids))(*[_ptr(m).value for m in mids])
        _check(self._lib.rsm_run_chain(self._arr, self._n, _ptr(x), mp, _ptr(out), flags,
                                       _stream(stream)))
        return out

    def adjoint(self, x, gy, gx, gcs, mids=None, flags: int = 0, stream=None):
        mp = None
        if mids is not None:
            mp = (ctypes.c_void_p * len(mids))(*[_ptr(m).value for m in mids])
        gp = None
        if gcs is not None:
            gp = (ctypes.c_void_p * self._n)(*[(_ptr(g).value if g is not None else None) for g in gcs])
        _check(self._lib.rsm_run_chain_adjoint(self._arr, self._n, _ptr(x), mp, _ptr(gy), _ptr(gx),
                                               gp, flags, _stream(stream)))

    def train(self, x, w, out, gx, gcs, flags: int = 0, stream=None):
        """One fused training step under the loss sum(w * out^2): writes out,
        gx (may be None) and the weight gradients gcs (list, entries may be
        None) in one pass over x."""
        gp = None
        if gcs is not None:
            gp = (ctypes.c_void_p * self._n)(*[(_ptr(g).value if g is not None else None) for g in gcs])
        _check(self._lib.rsm_run_chain_train(self._arr, self._n, _ptr(x), _ptr(w), _ptr(out), _ptr(gx), gp,
                                             flags, _stream(stream)))
        return out

    def train_noalloc(self, x, w, out, gx, gcs, flags: int = 0, stream=None):
        """train() through rsm_run_chain_train_noalloc: the library allocates
        nothing (its partial rows live in a fixed per-device array, shared by
        every such call on the device)."""
        gp = None
        if gcs is not None:
            gp = (ctypes.c_void_p * self._n)(*[(_ptr(g).value if g is not None else None) for g in gcs])
        _check(self._lib.rsm_run_chain_train_noalloc(self._arr, self._n, _ptr(x), _ptr(w), _ptr(out), _ptr(gx),
                                                     gp, flags, _stream(stream)))
        return out
