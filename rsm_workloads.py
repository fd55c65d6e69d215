"""Seeded synthetic inputs and tiler descriptions for RSM repetitive tasks.

This module is shared by the CPU oracle's tests, the GPU path's tests and the
benchmark.  It holds *data only*: array generators (NumPy PCG64, one seed per
workload) and plain tiler descriptions (origin, paving, fitting, shapes).  It
contains none of the tiler arithmetic (no index evaluation, no modular
reduction, no gather/compute/scatter); both sides marshal these descriptions
into their own structures.

Notation (MARTE Repetitive Structure Modeling, the package the paper relies on
for its repetitive tasks, Sec. 3 and Sec. 6.1): a tiler on an array of shape
``s`` has an origin ``o``, a paving matrix ``P`` (array rank x repetition
rank) and a fitting matrix ``F`` (array rank x pattern rank) plus a pattern
shape ``s_p``.  Column k of ``P`` is the array step of repetition dimension k,
column k of ``F`` the array step of pattern dimension k.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np

# Task kinds (the elementary task applied once per repetition).
COPY, SUM, WSUM, DOT = 0, 1, 2, 3
TASK_NAMES = {COPY: "copy", SUM: "sum", WSUM: "wsum", DOT: "dot"}


@dataclass
class Tiler:
    """A tiler on one array: pure description, no behaviour."""

    array_shape: Tuple[int, ...]
    origin: np.ndarray            # int64 [d_a]
    paving: np.ndarray            # int64 [d_a, d_r]
    fitting: np.ndarray           # int64 [d_a, d_p]
    pattern_shape: Tuple[int, ...]

    def __post_init__(self):
        self.array_shape = tuple(int(v) for v in self.array_shape)
        self.pattern_shape = tuple(int(v) for v in self.pattern_shape)
        da = len(self.array_shape)
        self.origin = np.asarray(self.origin, dtype=np.int64).reshape(da)
        self.paving = np.asarray(self.paving, dtype=np.int64).reshape(da, -1) \
            if da else np.zeros((0, 0), np.int64)
        dp = len(self.pattern_shape)
        self.fitting = np.asarray(self.fitting, dtype=np.int64).reshape(da, dp)

    @property
    def rep_rank(self) -> int:
        return self.paving.shape[1]


@dataclass
class Problem:
    """One repetitive task: repetition space, input tilers, output tiler, task."""

    rep_shape: Tuple[int, ...]
    inputs: List[Tiler]
    output: Tiler
    task: int
    coeffs: Optional[np.ndarray] = None     # float32 (WSUM): input-pattern shaped, or
                                            # [output pattern, input pattern] when the
                                            # output pattern has several elements
    compute: str = "f32"                    # "f32" or "bf16" (DOT only)
    note: str = ""


def identity_output(rep_shape: Sequence[int]) -> Tiler:
    """Output tiler writing y(r) to B[r]: origin 0, paving I, scalar pattern."""
    d = len(rep_shape)
    return Tiler(tuple(rep_shape), np.zeros(d), np.eye(d, dtype=np.int64),
                 np.zeros((d, 0)), ())


def rng_for(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def f32_to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """Round float32 to bfloat16 (round to nearest, ties to even); uint16 bits.

    Input preparation for the BF16 contraction: done once, outside any timed
    region.  NaN inputs are not produced by the generators.
    """
    u = np.ascontiguousarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)
    return r.astype(np.uint16)


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint16).astype(np.uint32) << np.uint32(16)).view(np.float32)


# ---------------------------------------------------------------------------
# Small plain task: 64x64 sum over 4x4 patterns
# ---------------------------------------------------------------------------

def small_sum(seed: int = 0, n: int = 64, b: int = 4):
    """x ~ U[-1,1] FP32 [n,n]; repetition [n/b, n/b]; pattern [b,b];
    origin 0; paving diag(b,b); fitting I; task SUM; identity output."""
    x = rng_for(seed).uniform(-1.0, 1.0, size=(n, n)).astype(np.float32)
    r = n // b
    t = Tiler((n, n), [0, 0], np.diag([b, b]), np.eye(2, dtype=np.int64), (b, b))
    return x, Problem((r, r), [t], identity_output((r, r)), SUM)


# ---------------------------------------------------------------------------
# Two-stage downscaler-style filter (horizontal 8 taps, then vertical 8 taps)
# ---------------------------------------------------------------------------

def normalised_coeffs(rng: np.random.Generator, n: int) -> np.ndarray:
    """c = u / sum(u), u ~ U[0,1) drawn in FP64, then cast to FP32."""
    u = rng.random(n)
    return (u / u.sum()).astype(np.float32)


def h_stage(frames: int, rows: int, cols: int, taps: int = 8, pave: int = None,
            origin: int = 0, step: int = 1) -> Tiler:
    """Horizontal stage tiler on [frames, rows, cols]: pattern [taps] along
    columns (fitting (0,0,step)), repetition [frames, rows, cols/pave] with
    paving diag(1, 1, pave)."""
    pave = taps if pave is None else pave
    return Tiler((frames, rows, cols), [0, 0, origin],
                 np.diag([1, 1, pave]), [[0], [0], [step]], (taps,))


def v_stage(frames: int, rows: int, cols: int, taps: int = 8, pave: int = None,
            origin: int = 0, step: int = 1) -> Tiler:
    """Vertical stage tiler on [frames, rows, cols]: pattern [taps] along rows
    (fitting (0,step,0)), repetition [frames, rows/pave, cols] with paving
    diag(1, pave, 1)."""
    pave = taps if pave is None else pave
    return Tiler((frames, rows, cols), [0, origin, 0],
                 np.diag([1, pave, 1]), [[0], [step], [0]], (taps,))


def rep_of(t: Tiler, axis: int, n_rep: int) -> Tuple[int, ...]:
    s = list(t.array_shape)
    s[axis] = n_rep
    return tuple(s)


@dataclass
class TwoStage:
    x: np.ndarray
    c_h: np.ndarray
    c_v: np.ndarray
    h: Problem
    v: Problem


def two_stage_filter(frames: int = 30, rows: int = 1080, cols: int = 1920,
                     taps: int = 8, seed: int = 1, h_origin: int = 0,
                     v_origin: int = 0, pave: int = None) -> TwoStage:
    """Downscaler-style filter.  x ~ U[0,1) FP32 [frames, rows, cols];
    c_h, c_v normalised from the same seed stream (after x).  With the default
    taps = paving = 8 the stages pave their arrays exactly."""
    pave = taps if pave is None else pave
    rng = rng_for(seed)
    x = rng.random((frames, rows, cols), dtype=np.float32)
    c_h = normalised_coeffs(rng, taps)
    c_v = normalised_coeffs(rng, taps)
    wc = -(-cols // pave)
    hr = -(-rows // pave)
    th = h_stage(frames, rows, cols, taps, pave, h_origin)
    rep_h = (frames, rows, wc)
    tv = v_stage(frames, rows, wc, taps, pave, v_origin)
    rep_v = (frames, hr, wc)
    hp = Problem(rep_h, [th], identity_output(rep_h), WSUM, c_h)
    vp = Problem(rep_v, [tv], identity_output(rep_v), WSUM, c_v)
    return TwoStage(x, c_h, c_v, hp, vp)


# ---------------------------------------------------------------------------
# Polyphase (multi-output) stages: one repetition reads a window of `taps`
# elements and writes `phases` consecutive outputs, each with its own taps
# (a weighted sum whose output pattern has `phases` elements)
# ---------------------------------------------------------------------------

def phase_output(rep_shape: Sequence[int], axis: int, phases: int) -> Tiler:
    """Output tiler writing y(r)[j] to B[..., phases * r_axis + j, ...]:
    origin 0, paving diag with `phases` on `axis`, pattern [phases] along it."""
    d = len(rep_shape)
    shape = list(rep_shape)
    shape[axis] *= phases
    pav = np.eye(d, dtype=np.int64)
    pav[axis, axis] = phases
    fit = np.zeros((d, 1), np.int64)
    fit[axis, 0] = 1
    return Tiler(tuple(shape), np.zeros(d), pav, fit, (phases,))


def phase_coeffs(rng: np.random.Generator, phases: int, taps: int) -> np.ndarray:
    """[phases, taps] FP32, each row normalised like normalised_coeffs."""
    return np.stack([normalised_coeffs(rng, taps) for _ in range(phases)])


@dataclass
class Polyphase:
    x: np.ndarray
    c_h: np.ndarray      # [phases_h, taps_h]
    c_v: np.ndarray      # [phases_v, taps_v]
    h: Problem
    v: Problem


def polyphase_downscaler(frames: int = 30, rows: int = 1080, cols: int = 1920,
                         taps_h: int = 13, pave_h: int = 8, phases_h: int = 3, origin_h: int = -2,
                         taps_v: int = 14, pave_v: int = 9, phases_v: int = 4, origin_v: int = -2,
                         seed: int = 5) -> Polyphase:
    """Downscaler built from two polyphase stages (1920x1080 -> 720x480 per
    frame with the defaults): horizontally every 8 columns a 13-tap window
    (origin -2, overlapping its neighbours by 5 and wrapping at both borders)
    gives 3 outputs, then vertically every 9 rows a 14-tap window (origin -2)
    gives 4 outputs.  x ~ U[0,1) FP32; coefficient rows normalised, from the
    same seed stream after x."""
    rng = rng_for(seed)
    x = rng.random((frames, rows, cols), dtype=np.float32)
    c_h = phase_coeffs(rng, phases_h, taps_h)
    c_v = phase_coeffs(rng, phases_v, taps_v)
    rc = -(-cols // pave_h)
    rep_h = (frames, rows, rc)
    th = h_stage(frames, rows, cols, taps_h, pave_h, origin_h)
    hp = Problem(rep_h, [th], phase_output(rep_h, 2, phases_h), WSUM, c_h)
    mid_cols = rc * phases_h
    rr = -(-rows // pave_v)
    rep_v = (frames, rr, mid_cols)
    tv = v_stage(frames, rows, mid_cols, taps_v, pave_v, origin_v)
    vp = Problem(rep_v, [tv], phase_output(rep_v, 1, phases_v), WSUM, c_v)
    return Polyphase(x, c_h, c_v, hp, vp)


def loss_weights(shape: Sequence[int], seed: int = 4) -> np.ndarray:
    """w ~ U[0,1) FP32 for the loss sum(w * out**2)."""
    return rng_for(seed).random(tuple(shape), dtype=np.float32)


# ---------------------------------------------------------------------------
# Matrix product expressed through tilers
# ---------------------------------------------------------------------------

def matmul_tilers(M: int, N: int, K: int) -> Problem:
    """C[m,n] = sum_k A[m,k] B[k,n] as a repetitive DOT task.

    Repetition [M, N]; A [M,K] with paving [[1,0],[0,0]] and fitting [[0],[1]];
    B [K,N] with paving [[0,0],[0,1]] and fitting [[1],[0]]; pattern [K]."""
    ta = Tiler((M, K), [0, 0], [[1, 0], [0, 0]], [[0], [1]], (K,))
    tb = Tiler((K, N), [0, 0], [[0, 0], [0, 1]], [[1], [0]], (K,))
    return Problem((M, N), [ta, tb], identity_output((M, N)), DOT)


def matmul_inputs(M: int, N: int, K: int, seed: int = 2):
    """A, B ~ N(0,1) FP32; also their BF16 (RNE) bit patterns."""
    rng = rng_for(seed)
    a = rng.standard_normal((M, K), dtype=np.float32)
    b = rng.standard_normal((K, N), dtype=np.float32)
    return a, b, f32_to_bf16_bits(a), f32_to_bf16_bits(b)


# ---------------------------------------------------------------------------
# Batched uneven 2D filters
# ---------------------------------------------------------------------------

@dataclass
class FilterInstance:
    H: int
    W: int
    k: int
    s: int
    x: np.ndarray = field(repr=False)
    coeffs: np.ndarray = field(repr=False)

    @property
    def out_shape(self):
        return (-(-self.H // self.s), -(-self.W // self.s))

    def problem(self) -> Problem:
        return filter2d_problem(self.H, self.W, self.k, self.s, self.coeffs)


def filter2d_problem(H: int, W: int, k: int, s: int, coeffs=None) -> Problem:
    """k x k window, stride s in both dimensions, centred origin
    (-floor(k/2), -floor(k/2)) so windows wrap on every border; fitting I;
    repetition [ceil(H/s), ceil(W/s)]; identity output."""
    rep = (-(-H // s), -(-W // s))
    c = -(k // 2)
    t = Tiler((H, W), [c, c], np.diag([s, s]), np.eye(2, dtype=np.int64), (k, k))
    return Problem(rep, [t], identity_output(rep), WSUM, coeffs)


def filter_batch(n: int = 512, seed: int = 3, side_lo: int = 32,
                 side_hi: int = 2048, with_data: bool = True) -> List[FilterInstance]:
    """Uneven instances: H, W = round(exp(U[ln lo, ln hi])) independently;
    k uniform in {3,5,7,9}; s uniform in {1,2,4}; coefficients U[-1,1]/k^2
    (FP32); inputs N(0,1) FP32.  Shapes are drawn first for all instances,
    then data instance by instance, so shapes do not depend on with_data."""
    rng = rng_for(seed)
    lo, hi = math.log(side_lo), math.log(side_hi)
    H = np.rint(np.exp(rng.uniform(lo, hi, n))).astype(np.int64)
    W = np.rint(np.exp(rng.uniform(lo, hi, n))).astype(np.int64)
    K = rng.choice(np.array([3, 5, 7, 9]), n)
    S = rng.choice(np.array([1, 2, 4]), n)
    out = []
    for j in range(n):
        k = int(K[j])
        if with_data:
            c = (rng.uniform(-1.0, 1.0, (k, k)) / (k * k)).astype(np.float32)
            x = rng.standard_normal((int(H[j]), int(W[j])), dtype=np.float32)
        else:
            c = np.zeros((k, k), np.float32)
            x = np.zeros((0, 0), np.float32)
        out.append(FilterInstance(int(H[j]), int(W[j]), k, int(S[j]), x, c))
    return out


# ---------------------------------------------------------------------------
# Random tilers for property tests
# ---------------------------------------------------------------------------

def random_tiler(rng: np.random.Generator, rep_rank: int, max_rank: int = 3,
                 max_side: int = 8, max_step: int = 9, max_origin: int = 20,
                 pattern_rank: Optional[int] = None,
                 max_pattern_side: int = 4) -> Tiler:
    da = int(rng.integers(1, max_rank + 1))
    dp = int(rng.integers(0, 3)) if pattern_rank is None else pattern_rank
    shape = tuple(int(v) for v in rng.integers(1, max_side + 1, da))
    o = rng.integers(-max_origin, max_origin + 1, da)
    P = rng.integers(-max_step, max_step + 1, (da, rep_rank))
    F = rng.integers(-max_step, max_step + 1, (da, dp))
    sp = tuple(int(v) for v in rng.integers(1, max_pattern_side + 1, dp))
    return Tiler(shape, o, P, F, sp)


def random_array(rng: np.random.Generator, shape, dtype=np.float32) -> np.ndarray:
    return rng.uniform(-1.0, 1.0, size=tuple(shape)).astype(dtype)


# ---------------------------------------------------------------------------
# Sparse matrix of the conjugate-gradient case study (Sec. 7): N = 132651,
# NNZ = 3442951.  These are exactly the counts of a 27-point stencil on a
# 51^3 grid (N = 51^3, NNZ = (3*51 - 2)^3), so the stand-in is that stencil
# with seeded symmetric weights and a dominant diagonal (symmetric positive
# definite, as the method requires).
# ---------------------------------------------------------------------------

@dataclass
class Csr:
    n: int
    row_ptr: np.ndarray   # int32 [n + 1]
    col_idx: np.ndarray   # int32 [nnz]
    vals: np.ndarray      # float64 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.col_idx.size)


def stencil27_csr(side: int = 51, seed: int = 5) -> Csr:
    """27-point stencil on a side^3 grid, row-major grid numbering.
    Off-diagonal weights -(1 + 0.5 u), u ~ U[0,1) per undirected edge (so the
    matrix is symmetric); diagonal = sum of |off-diagonal| of the row + 0.25."""
    rng = rng_for(seed)
    n = side ** 3
    g = np.arange(n, dtype=np.int64).reshape(side, side, side)
    offs = [(a, b, c) for a in (-1, 0, 1) for b in (-1, 0, 1) for c in (-1, 0, 1)]
    # edge weights: one draw per (node, positive-direction offset), mirrored
    pos = [o for o in offs if o > (0, 0, 0)]
    wpos = {}
    for o in pos:
        wpos[o] = -(1.0 + 0.5 * rng.random((side, side, side)))
    rows, cols, vals = [], [], []
    for o in offs:
        if o == (0, 0, 0):
            continue
        a, b, c = o
        src = g[max(0, -a):side - max(0, a), max(0, -b):side - max(0, b), max(0, -c):side - max(0, c)]
        dst = g[max(0, a):side - max(0, -a), max(0, b):side - max(0, -b), max(0, c):side - max(0, -c)]
        if o in wpos:
            w = wpos[o][max(0, -a):side - max(0, a), max(0, -b):side - max(0, b), max(0, -c):side - max(0, c)]
        else:
            m = (-a, -b, -c)
            # weight of the mirrored edge, indexed at its source (= this dst)
            w = wpos[m][max(0, a):side - max(0, -a), max(0, b):side - max(0, -b), max(0, c):side - max(0, -c)]
        rows.append(src.reshape(-1))
        cols.append(dst.reshape(-1))
        vals.append(w.reshape(-1))
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate(vals)
    diag = np.zeros(n)
    np.add.at(diag, rows, np.abs(vals))
    rows = np.concatenate([rows, np.arange(n)])
    cols = np.concatenate([cols, np.arange(n)])
    vals = np.concatenate([vals, diag + 0.25])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    row_ptr = np.zeros(n + 1, np.int64)
    np.add.at(row_ptr, rows + 1, 1)
    row_ptr = np.cumsum(row_ptr)
    return Csr(n, row_ptr.astype(np.int32), cols.astype(np.int32), vals.astype(np.float64))


def random_csr(rng: np.random.Generator, n_rows: int, n_cols: int, max_per_row: int = 9,
               allow_empty: bool = True) -> Csr:
    """Random sparsity (rows may be empty), values U[-1,1), unsorted columns allowed."""
    counts = rng.integers(0 if allow_empty else 1, max_per_row + 1, n_rows)
    row_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    col_idx = rng.integers(0, n_cols, int(row_ptr[-1])).astype(np.int32)
    vals = rng.uniform(-1.0, 1.0, int(row_ptr[-1]))
    return Csr(n_rows, row_ptr, col_idx, vals)


def dense_csr(M: np.ndarray) -> Csr:
    """CSR form of a dense matrix (its nonzero entries, row-major order)."""
    rows, cols = np.nonzero(M)
    counts = np.bincount(rows, minlength=M.shape[0])
    row_ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int32)
    return Csr(M.shape[0], row_ptr, cols.astype(np.int32), M[rows, cols].astype(np.float64))


def spd_csr(rng: np.random.Generator, n: int, cond: float = 50.0, density: float = 1.0) -> Csr:
    """Random symmetric positive definite matrix: Q diag(eigenvalues) Q^T with
    eigenvalues log-spaced in [1, cond]; with density < 1, a sparse SPD matrix
    instead (random symmetric pattern, diagonal dominance margin from cond)."""
    if density >= 1.0:
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        return dense_csr((Q * np.geomspace(1.0, cond, n)) @ Q.T)
    mask = np.triu(rng.random((n, n)) < density, 1)
    off = np.where(mask, -rng.uniform(0.5, 1.5, (n, n)), 0.0)
    off = off + off.T
    M = off + np.diag(np.abs(off).sum(1) + np.abs(off).sum(1).max() / cond + 1e-3)
    return dense_csr(M)


def cg_rhs(n: int, seed: int = 6) -> np.ndarray:
    """Right-hand side for the conjugate-gradient workload: U[-1, 1)."""
    return rng_for(seed).uniform(-1.0, 1.0, n)
