// k_window.hip -- kernels for axis-aligned tilers (weighted / plain sums).
//
//  * pattern_reduce: small patterns (<= 64 elements) on any affine tiler.  One
//    lane per pattern element, a group of 2^k lanes per repetition, and a
//    butterfly reduction across the group with wavefront shuffles.
//  * fir:            1-D taps along one axis of a [B, R, C] view.  One output
//    per thread per loop trip; taps along the contiguous axis are read as
//    16-byte vectors, taps along rows are coalesced across the wavefront.
//    Windows that cross a border take a modular path.
//  * fir_chain:      two FIR stages (columns, then rows) fused: the
//    intermediate array is never written; each thread reads the block of
//    input the output depends on, exactly once.
//  * fir_adjoint / fir_chain_adjoint: transposed tilers written as gathers
//    (each input element is read by at most one repetition, so the
//    scatter-add is a plain store) plus per-block weight-gradient partials.
#include <hip/hip_runtime.h>

#include "rsm_internal.h"

namespace rsm {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxTaps = 16;   // taps held in registers by the adjoint kernels

__device__ __forceinline__ int wrap_mod(int64_t v, int n) {
  int64_t q = v % n;
  return int(q < 0 ? q + n : q);
}

// The lane-pair adjoint and training-step kernels touch every element of x
// and dL/dx once per launch, and nothing after them reads x again the way a
// forward pass is followed by its adjoint.  They load x and store dL/dx with
// the nontemporal cache policy, which streams the data past the caches
// instead of filling lines (or leaving dirty ones to be written back during
// the next kernel): the training step runs 8-9 % faster.  The forward kernel
// keeps ordinary loads, so an adjoint that follows it can still find x in
// the 256 MB last-level cache.
typedef float stream4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float4 load_stream4(const float* p) {
  const stream4_t v = __builtin_nontemporal_load(reinterpret_cast<const stream4_t*>(p));
  return make_float4(v.x, v.y, v.z, v.w);
}

__device__ __forceinline__ void store_stream4(float* p, const float4& w) {
  const stream4_t v = {w.x, w.y, w.z, w.w};
  __builtin_nontemporal_store(v, reinterpret_cast<stream4_t*>(p));
}

__device__ __forceinline__ void store_stream(float* p, float w) { __builtin_nontemporal_store(w, p); }

// ---------------------------------------------------------------------------
// pattern_reduce
// ---------------------------------------------------------------------------
template <int R>
__global__ void __launch_bounds__(kBlock) pattern_reduce_kernel(PatternReduceArgs a) {
  const int G = 1 << a.group_log2;
  const int lane = threadIdx.x & (G - 1);
  const int64_t groups_total = (int64_t(gridDim.x) * kBlock) >> a.group_log2;
  const int64_t group0 = (int64_t(blockIdx.x) * kBlock + threadIdx.x) >> a.group_log2;

  // pattern offset of this lane: (F i) mod s, i = lane's pattern multi-index
  int64_t off[R];
  {
    int64_t i[R];
    int64_t f = lane;
#pragma unroll
    for (int k = R - 1; k >= 0; --k) {
      if (k < a.in.pat_rank) {
        i[k] = f % a.in.pat_shape[k];
        f /= a.in.pat_shape[k];
      } else {
        i[k] = 0;
      }
    }
#pragma unroll
    for (int d = 0; d < R; ++d) {
      off[d] = 0;
      if (d < a.in.arr_rank) {
        int64_t v = 0;
#pragma unroll
        for (int k = 0; k < R; ++k)
          if (k < a.in.pat_rank) v += a.in.fit[d][k] * i[k];
        off[d] = v % a.in.shape[d];
      }
    }
  }
  const bool active = lane < a.n_pat;
  const float coef = (active && a.c) ? a.c[lane] : 1.0f;

  for (int64_t rf = group0; rf < a.n_rep; rf += groups_total) {
    int64_t r[R];
    {
      int64_t f = rf;
#pragma unroll
      for (int k = R - 1; k >= 0; --k) {
        if (k < a.rep_rank) {
          r[k] = f % a.rep_shape[k];
          f /= a.rep_shape[k];
        } else {
          r[k] = 0;
        }
      }
    }
    float v = 0.0f;
    if (active) {
      int64_t lin = 0;
#pragma unroll
      for (int d = 0; d < R; ++d) {
        if (d < a.in.arr_rank) {
          const int64_t s = a.in.shape[d];
          int64_t c = a.in.origin[d];
#pragma unroll
          for (int k = 0; k < R; ++k) {
            if (k < a.rep_rank) {
              c += (a.in.pav[d][k] * r[k]) % s;
              if (c >= s) c -= s;
            }
          }
          c += off[d];
          if (c >= s) c -= s;
          lin = lin * s + c;
        }
      }
      v = a.x[lin] * coef;
    }
    // butterfly across the group (G divides 64, groups never straddle a wave)
    for (int m = G >> 1; m > 0; m >>= 1) v += __shfl_xor(v, m);
    if (lane == 0) {
      int64_t lin = 0;
#pragma unroll
      for (int d = 0; d < R; ++d) {
        if (d < a.out.arr_rank) {
          const int64_t s = a.out.shape[d];
          int64_t c = a.out.origin[d];
#pragma unroll
          for (int k = 0; k < R; ++k) {
            if (k < a.rep_rank) {
              c += (a.out.pav[d][k] * r[k]) % s;
              if (c >= s) c -= s;
            }
          }
          lin = lin * s + c;
        }
      }
      a.y[lin] = v;
    }
  }
}

// ---------------------------------------------------------------------------
// FIR helpers
// ---------------------------------------------------------------------------
struct OutPos {
  int b, r, c;  // repetition coordinates
};

__device__ __forceinline__ OutPos decode(uint32_t o, const Win3& w, const FastDiv& drc,
                                         const FastDiv& drr) {
  const uint32_t row = fdiv(o, drc);
  OutPos p;
  p.c = int(o - row * uint32_t(w.rep[2]));
  const uint32_t b = fdiv(row, drr);
  p.r = int(row - b * uint32_t(w.rep[1]));
  p.b = int(b);
  return p;
}

// Sum_k c[k] * x[row_base + (start + k) mod n] along the contiguous axis
// (element step 1).  `row_base` is the offset of the row's first element.
template <bool VEC, int TT>
__device__ __forceinline__ float taps_contig(const float* __restrict__ x, int row_base, int start,
                                             int n, int taps, const float* __restrict__ c) {
  float acc = 0.0f;
  if (start >= 0 && start + taps <= n) {
    const float* p = x + row_base + start;
    if (VEC) {
      const int nv = (TT ? TT : taps) / 4;
#pragma unroll
      for (int q = 0; q < nv; ++q) {
        const float4 v = *reinterpret_cast<const float4*>(p + 4 * q);
        acc = fmaf(c[4 * q + 0], v.x, acc);
        acc = fmaf(c[4 * q + 1], v.y, acc);
        acc = fmaf(c[4 * q + 2], v.z, acc);
        acc = fmaf(c[4 * q + 3], v.w, acc);
      }
    } else {
      const int nt = TT ? TT : taps;
#pragma unroll 8
      for (int k = 0; k < nt; ++k) acc = fmaf(c[k], p[k], acc);
    }
  } else {
    int col = wrap_mod(start, n);
    const int nt = TT ? TT : taps;
    for (int k = 0; k < nt; ++k) {
      acc = fmaf(c[k], x[row_base + col], acc);
      if (++col == n) col = 0;
    }
  }
  return acc;
}

// Sum_k c[k] * x[plane + ((start + k) mod n) * row_stride + col] along rows.
template <int TT>
__device__ __forceinline__ float taps_rows(const float* __restrict__ x, int plane, int start,
                                           int n, int row_stride, int col, int taps,
                                           const float* __restrict__ c) {
  float acc = 0.0f;
  const int nt = TT ? TT : taps;
  if (start >= 0 && start + nt <= n) {
    const float* p = x + plane + start * row_stride + col;
#pragma unroll 8
    for (int k = 0; k < nt; ++k) acc = fmaf(c[k], p[k * row_stride], acc);
  } else {
    int row = wrap_mod(start, n);
    for (int k = 0; k < nt; ++k) {
      acc = fmaf(c[k], x[plane + row * row_stride + col], acc);
      if (++row == n) row = 0;
    }
  }
  return acc;
}

// ---------------------------------------------------------------------------
// FIR forward
// ---------------------------------------------------------------------------
template <int AX, bool VEC, int TT>
__global__ void __launch_bounds__(kBlock) fir_kernel(FirArgs a) {
  const Win3& w = a.w;
  const uint32_t stride = gridDim.x * kBlock;
  for (uint32_t o = blockIdx.x * kBlock + threadIdx.x; o < a.n_out; o += stride) {
    const OutPos q = decode(o, w, a.div_rc, a.div_rr);
    const int ib = w.o[0] + w.p[0] * q.b;
    float acc;
    if (AX == 2) {
      const int ir = w.o[1] + w.p[1] * q.r;
      const int row_base = (ib * w.A[1] + ir) * w.A[2];
      acc = taps_contig<VEC, TT>(a.x, row_base, w.o[2] + w.p[2] * q.c, w.A[2], w.taps, a.c);
    } else {
      const int ic = w.o[2] + w.p[2] * q.c;
      acc = taps_rows<TT>(a.x, ib * w.A[1] * w.A[2], w.o[1] + w.p[1] * q.r, w.A[1], w.A[2], ic,
                          w.taps, a.c);
    }
    a.y[o] = acc;
  }
}

// 8 taps along columns, 16-byte aligned windows: lanes 2m and 2m+1 share one
// output and load four taps each, so every load instruction covers 1 KiB of
// contiguous input; the half sums (taps 0-3 + taps 4-7, each accumulated in
// tap order) meet through a lane shuffle, the order the fused chain uses for
// its first stage.  A window that crosses the border takes the modular path.
__global__ void __launch_bounds__(kBlock) fir_pair_kernel(FirArgs a) {
  const Win3& w = a.w;
  const int hh = threadIdx.x & 1;
  float c4[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) c4[e] = a.c[4 * hh + e];
  const uint32_t n_half = 2u * a.n_out;
  const uint32_t stride = gridDim.x * kBlock;
  const int n = w.A[2];
  for (uint32_t gi = blockIdx.x * kBlock + threadIdx.x; gi < n_half; gi += stride) {
    const uint32_t o = gi >> 1;
    const OutPos q = decode(o, w, a.div_rc, a.div_rr);
    const int ib = w.o[0] + w.p[0] * q.b;
    const int row_base = (ib * w.A[1] + w.o[1] + w.p[1] * q.r) * n;
    const int pos = w.o[2] + w.p[2] * q.c;
    float part;
    if (pos >= 0 && pos + 8 <= n) {
      const float4 xv = *reinterpret_cast<const float4*>(a.x + row_base + pos + 4 * hh);
      part = c4[0] * xv.x;
      part = fmaf(c4[1], xv.y, part);
      part = fmaf(c4[2], xv.z, part);
      part = fmaf(c4[3], xv.w, part);
    } else {
      int e = wrap_mod(int64_t(pos) + 4 * hh, n);
      part = c4[0] * a.x[row_base + e];
#pragma unroll
      for (int k = 1; k < 4; ++k) {
        if (++e == n) e = 0;
        part = fmaf(c4[k], a.x[row_base + e], part);
      }
    }
    const float other = __shfl_xor(part, 1);
    if (hh == 0) a.y[o] = part + other;
  }
}

// ---------------------------------------------------------------------------
// fused chain: out = V(H(x))
// ---------------------------------------------------------------------------
// Offsets of the T1 input rows an output of the fused chain reads, when
// neither stage's window wraps (the common, interior case); false otherwise.
template <int T0, int T1>
__device__ __forceinline__ bool chain_rows(const Win3& h, const Win3& v, const OutPos& q,
                                           int (&off)[T1]) {
  const int mb = v.o[0] + v.p[0] * q.b;          // intermediate frame
  const int mc = v.o[2] + v.p[2] * q.c;          // intermediate column
  const int xb = h.o[0] + h.p[0] * mb;           // input frame
  const int xstart = h.o[2] + h.p[2] * mc;       // first input column of the window
  const int mr0 = v.o[1] + v.p[1] * q.r;         // first intermediate row
  const bool inside = xstart >= 0 && xstart + T0 <= h.A[2] && mr0 >= 0 && mr0 + T1 <= v.A[1];
#pragma unroll
  for (int j = 0; j < T1; ++j) off[j] = (xb * h.A[1] + h.o[1] + h.p[1] * (mr0 + j)) * h.A[2] + xstart;
  return inside;
}

template <bool VEC, int T0, int T1>
__global__ void __launch_bounds__(kBlock) fir_chain_kernel(FirChainArgs a) {
  const Win3& h = a.h;
  const Win3& v = a.v;
  const uint32_t stride = gridDim.x * kBlock;
  const int t1 = T1 ? T1 : v.taps;
  for (uint32_t o = blockIdx.x * kBlock + threadIdx.x; o < a.n_out; o += stride) {
    const OutPos q = decode(o, v, a.div_rc, a.div_rr);
    if constexpr (VEC && T0 > 0 && T1 > 0) {
      // interior: issue every 16-byte load of the T1 x T0 input block first
      int off[T1];
      if (chain_rows<T0, T1>(h, v, q, off)) {
        float4 blk[T1][T0 / 4];
#pragma unroll
        for (int j = 0; j < T1; ++j)
#pragma unroll
          for (int u = 0; u < T0 / 4; ++u) blk[j][u] = *reinterpret_cast<const float4*>(a.x + off[j] + 4 * u);
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < T1; ++j) {
          float mid = 0.0f;
#pragma unroll
          for (int u = 0; u < T0 / 4; ++u) {
            mid = fmaf(a.ch[4 * u + 0], blk[j][u].x, mid);
            mid = fmaf(a.ch[4 * u + 1], blk[j][u].y, mid);
            mid = fmaf(a.ch[4 * u + 2], blk[j][u].z, mid);
            mid = fmaf(a.ch[4 * u + 3], blk[j][u].w, mid);
          }
          acc = fmaf(a.cv[j], mid, acc);
        }
        a.y[o] = acc;
        continue;
      }
    }
    // general case: any window position, modular wrap along both tap axes
    const int mb = v.o[0] + v.p[0] * q.b;
    const int mc = v.o[2] + v.p[2] * q.c;
    const int xb = h.o[0] + h.p[0] * mb;
    const int xstart = h.o[2] + h.p[2] * mc;
    int mr = wrap_mod(int64_t(v.o[1]) + int64_t(v.p[1]) * q.r, v.A[1]);
    float acc = 0.0f;
    for (int j = 0; j < t1; ++j) {
      const int xr = h.o[1] + h.p[1] * mr;
      const int row_base = (xb * h.A[1] + xr) * h.A[2];
      const float mid = taps_contig<VEC, T0>(a.x, row_base, xstart, h.A[2], h.taps, a.ch);
      acc = fmaf(a.cv[j], mid, acc);
      if (++mr == v.A[1]) mr = 0;
    }
    a.y[o] = acc;
  }
}

// ---------------------------------------------------------------------------
// fused chain, 8 column taps, lane pairs
//
// Lanes 2m and 2m+1 share one output: each loads one 16-byte half of the
// 8-tap window of every row, so consecutive lanes read consecutive 16-byte
// chunks and every load instruction covers 1 KiB of contiguous input.  The
// two half sums of a row are combined with a lane shuffle.  A lane's half
// (its parity) never changes inside the grid-stride loop (the stride is even).
// ---------------------------------------------------------------------------
template <int T1>
struct FwdPairBlock {
  uint32_t o;
  int off[T1];
  float4 x[T1];
  bool fast;
};

template <int T1>
__device__ __forceinline__ void fwd_pair_fetch(const FirChainArgs& a, uint32_t gidx, int hh,
                                               FwdPairBlock<T1>& b) {
  b.o = gidx >> 1;
  const OutPos q = decode(b.o, a.v, a.div_rc, a.div_rr);
  b.fast = chain_rows<8, T1>(a.h, a.v, q, b.off);
  if (b.fast) {
#pragma unroll
    for (int j = 0; j < T1; ++j) b.x[j] = *reinterpret_cast<const float4*>(a.x + b.off[j] + 4 * hh);
  }
}

// Software-pipelined: the next output's loads are issued before the current
// output is reduced and stored.
template <int T1>
__global__ void __launch_bounds__(kBlock) fir_chain_pair_kernel(FirChainArgs a) {
  const Win3& h = a.h;
  const Win3& v = a.v;
  const uint32_t n_half = 2u * a.n_out;
  const uint32_t stride = gridDim.x * kBlock;
  const int hh = threadIdx.x & 1;
  float c4[4], cv[T1];
#pragma unroll
  for (int e = 0; e < 4; ++e) c4[e] = a.ch[4 * hh + e];
#pragma unroll
  for (int j = 0; j < T1; ++j) cv[j] = a.cv[j];
  uint32_t gi = blockIdx.x * kBlock + threadIdx.x;
  FwdPairBlock<T1> cur;
  if (gi < n_half) fwd_pair_fetch<T1>(a, gi, hh, cur);
  while (gi < n_half) {
    const uint32_t gn = gi + stride;
    FwdPairBlock<T1> nxt;
    if (gn < n_half) fwd_pair_fetch<T1>(a, gn, hh, nxt);
    if (cur.fast) {
      float acc = 0.0f;
#pragma unroll
      for (int j = 0; j < T1; ++j) {
        float part = c4[0] * cur.x[j].x;
        part = fmaf(c4[1], cur.x[j].y, part);
        part = fmaf(c4[2], cur.x[j].z, part);
        part = fmaf(c4[3], cur.x[j].w, part);
        // lane 2m holds taps 0-3, lane 2m+1 taps 4-7: add them in that order
        const float other = __shfl_xor(part, 1);
        const float mid = hh ? other + part : part + other;
        acc = fmaf(cv[j], mid, acc);
      }
      if (hh == 0) a.y[cur.o] = acc;
    } else if (hh == 0) {
      // window wraps: the even lane evaluates the output on the modular path
      const OutPos q = decode(cur.o, v, a.div_rc, a.div_rr);
      const int mb = v.o[0] + v.p[0] * q.b;
      const int mc = v.o[2] + v.p[2] * q.c;
      const int xb = h.o[0] + h.p[0] * mb;
      const int xstart = h.o[2] + h.p[2] * mc;
      int mr = wrap_mod(int64_t(v.o[1]) + int64_t(v.p[1]) * q.r, v.A[1]);
      float acc = 0.0f;
      for (int j = 0; j < T1; ++j) {
        const int row_base = (xb * h.A[1] + h.o[1] + h.p[1] * mr) * h.A[2];
        acc = fmaf(cv[j], taps_contig<false, 8>(a.x, row_base, xstart, h.A[2], 8, a.ch), acc);
        if (++mr == v.A[1]) mr = 0;
      }
      a.y[cur.o] = acc;
    }
    cur = nxt;
    gi = gn;
  }
}

// ---------------------------------------------------------------------------
// weight-gradient reduction inside the adjoint kernels
//
// Each workgroup reduces its per-thread partial vectors (wavefront butterfly,
// then across the 4 waves in LDS) and stores one row of partials.  The
// workgroup that arrives last at the completion counter sums the rows in a
// fixed order and writes the gradient, so the result does not depend on
// scheduling.  Rows are written and read with agent-scope atomic accesses and
// the counter is updated with acquire-release ordering, which keeps the
// exchange coherent across the XCDs' separate L2 caches.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void store_agent(float* p, float v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ float load_agent(const float* p) {
  return __hip_atomic_load(const_cast<float*>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int N>
__device__ __forceinline__ void block_reduce_store(float (&v)[N], int n, float* out_row, bool coherent) {
  __shared__ float sm[kBlock / 64][N];
#pragma unroll
  for (int i = 0; i < N; ++i) {
    float t = v[i];
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) t += __shfl_xor(t, m);
    v[i] = t;
  }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int i = 0; i < N; ++i) sm[wave][i] = v[i];
  }
  __syncthreads();
  if (int(threadIdx.x) < n) {
    float t = 0.0f;
#pragma unroll
    for (int wv = 0; wv < kBlock / 64; ++wv) t += sm[wv][threadIdx.x];
    if (coherent)
      store_agent(out_row + threadIdx.x, t);
    else
      out_row[threadIdx.x] = t;
  }
}

// True in the last workgroup to arrive (all rows of partials are then visible).
__device__ __forceinline__ bool arrive_last(uint32_t* counter) {
  __shared__ int last;
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t prev =
        __hip_atomic_fetch_add(counter, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
    last = prev == gridDim.x - 1;
  }
  __syncthreads();
  return last != 0;
}

// out[j] (=|+=) sum over rows b < n_rows of partial[b * row + col0 + j], j < count
__device__ __forceinline__ void reduce_rows_fixed(const float* partial, int n_rows, int row,
                                                  int col0, int count, float* out, int accumulate) {
  __shared__ float red[kBlock / 64];
  for (int j = 0; j < count; ++j) {
    // rows t, t + kBlock, ... added in that order, loads issued eight at a time
    const float* col = partial + col0 + j;
    float acc = 0.0f;
    int b = threadIdx.x;
    for (; b + 7 * kBlock < n_rows; b += 8 * kBlock) {
      float v[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) v[u] = load_agent(col + int64_t(b + u * kBlock) * row);
#pragma unroll
      for (int u = 0; u < 8; ++u) acc += v[u];
    }
    for (; b < n_rows; b += kBlock) acc += load_agent(col + int64_t(b) * row);
    // the order of the second-kernel reduction: a butterfly inside each
    // wavefront, then the four wavefront sums in order
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) acc += __shfl_xor(acc, m);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      const float tot = ((red[0] + red[1]) + red[2]) + red[3];
      out[j] = accumulate ? out[j] + tot : tot;
    }
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// adjoint of one injective FIR stage
// ---------------------------------------------------------------------------
template <int AX, bool VEC, int TT>
__global__ void __launch_bounds__(kBlock) fir_adjoint_kernel(FirAdjArgs a) {
  const Win3& w = a.w;
  const int taps = TT ? TT : w.taps;
  float gc[kMaxTaps];
#pragma unroll
  for (int k = 0; k < kMaxTaps; ++k) gc[k] = 0.0f;
  float cr[kMaxTaps];
#pragma unroll
  for (int k = 0; k < kMaxTaps; ++k) cr[k] = k < taps ? a.c[k] : 0.0f;

  const uint32_t stride = gridDim.x * kBlock;
  for (uint32_t o = blockIdx.x * kBlock + threadIdx.x; o < a.n_rep; o += stride) {
    const OutPos q = decode(o, w, a.div_rc, a.div_rr);
    const float g = a.gy[o];
    const int ib = w.o[0] + w.p[0] * q.b;
    int base, step, pos, n;
    if (AX == 2) {
      base = (ib * w.A[1] + w.o[1] + w.p[1] * q.r) * w.A[2];
      pos = w.o[2] + w.p[2] * q.c;
      step = 1;
      n = w.A[2];
    } else {
      base = ib * w.A[1] * w.A[2] + w.o[2] + w.p[2] * q.c;
      pos = w.o[1] + w.p[1] * q.r;
      step = w.A[2];
      n = w.A[1];
    }
    const bool inside = pos >= 0 && pos + taps <= n;
    // loads first (all taps), then the weight-gradient arithmetic, then stores
    float xs[kMaxTaps];
    if (AX == 2 && VEC && inside) {
      if (a.x) {
        const float* xp = a.x + base + pos;
#pragma unroll
        for (int q4 = 0; q4 < (TT ? TT : kMaxTaps) / 4; ++q4) {
          if (4 * q4 >= taps) break;
          const float4 xv = *reinterpret_cast<const float4*>(xp + 4 * q4);
          xs[4 * q4 + 0] = xv.x; xs[4 * q4 + 1] = xv.y;
          xs[4 * q4 + 2] = xv.z; xs[4 * q4 + 3] = xv.w;
        }
#pragma unroll
        for (int k = 0; k < (TT ? TT : kMaxTaps); ++k) {
          if (k >= taps) break;
          gc[k] = fmaf(g, xs[k], gc[k]);
        }
      }
      if (a.gx) {
        float* gxp = a.gx + base + pos;
#pragma unroll
        for (int q4 = 0; q4 < (TT ? TT : kMaxTaps) / 4; ++q4) {
          if (4 * q4 >= taps) break;
          float4 gv = make_float4(cr[4 * q4 + 0] * g, cr[4 * q4 + 1] * g, cr[4 * q4 + 2] * g,
                                  cr[4 * q4 + 3] * g);
          float4* dst = reinterpret_cast<float4*>(gxp + 4 * q4);
          if (a.accumulate) {
            const float4 old = *dst;
            gv.x += old.x; gv.y += old.y; gv.z += old.z; gv.w += old.w;
          }
          *dst = gv;
        }
      }
    } else {
      int offs[kMaxTaps];
      int e = inside ? pos : wrap_mod(pos, n);
#pragma unroll
      for (int k = 0; k < (TT ? TT : kMaxTaps); ++k) {
        if (k >= taps) break;
        offs[k] = base + e * step;
        if (++e == n) e = 0;
      }
      if (a.x) {
#pragma unroll
        for (int k = 0; k < (TT ? TT : kMaxTaps); ++k) {
          if (k >= taps) break;
          xs[k] = a.x[offs[k]];
        }
#pragma unroll
        for (int k = 0; k < (TT ? TT : kMaxTaps); ++k) {
          if (k >= taps) break;
          gc[k] = fmaf(g, xs[k], gc[k]);
        }
      }
      if (a.gx) {
#pragma unroll
        for (int k = 0; k < (TT ? TT : kMaxTaps); ++k) {
          if (k >= taps) break;
          const float gv = cr[k] * g;
          a.gx[offs[k]] = a.accumulate ? a.gx[offs[k]] + gv : gv;
        }
      }
    }
  }
  if (a.partial) {
    block_reduce_store<kMaxTaps>(gc, taps, a.partial + int64_t(blockIdx.x) * taps, a.counter != nullptr);
    if (a.counter && arrive_last(a.counter)) {
      reduce_rows_fixed(a.partial, gridDim.x, taps, 0, taps, a.gc, a.accumulate);
      if (threadIdx.x == 0) __hip_atomic_store(a.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// 8 taps along columns, 16-byte aligned windows: lanes 2m and 2m+1 share one
// repetition and take four taps each, so every load and store instruction of
// a wavefront covers 1 KiB of contiguous x or dL/dx (one lane per repetition
// leaves each instruction every other 16 bytes of its span).  Interior
// windows stream x and dL/dx with the nontemporal policy; a window that
// crosses the border takes the modular path, four taps per lane.  Lane 2m
// accumulates the weight gradient of taps 0-3, lane 2m+1 of taps 4-7.
__global__ void __launch_bounds__(kBlock) fir_adjoint_pair_kernel(FirAdjArgs a) {
  const Win3& w = a.w;
  const int hh = threadIdx.x & 1;
  float c4[4], g4[4];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    c4[e] = a.c[4 * hh + e];
    g4[e] = 0.0f;
  }
  const uint32_t n_half = 2u * a.n_rep;
  const uint32_t stride = gridDim.x * kBlock;
  const int n = w.A[2];
  for (uint32_t gi = blockIdx.x * kBlock + threadIdx.x; gi < n_half; gi += stride) {
    const uint32_t o = gi >> 1;
    const OutPos q = decode(o, w, a.div_rc, a.div_rr);
    const float g = a.gy[o];
    const int ib = w.o[0] + w.p[0] * q.b;
    const int base = (ib * w.A[1] + w.o[1] + w.p[1] * q.r) * n;
    const int pos = w.o[2] + w.p[2] * q.c;
    if (pos >= 0 && pos + 8 <= n) {
      const int at = base + pos + 4 * hh;
      if (a.x) {
        const float4 xv = load_stream4(a.x + at);
        g4[0] = fmaf(g, xv.x, g4[0]);
        g4[1] = fmaf(g, xv.y, g4[1]);
        g4[2] = fmaf(g, xv.z, g4[2]);
        g4[3] = fmaf(g, xv.w, g4[3]);
      }
      if (a.gx) {
        float4 gv = make_float4(c4[0] * g, c4[1] * g, c4[2] * g, c4[3] * g);
        if (a.accumulate) {
          const float4 old = *reinterpret_cast<const float4*>(a.gx + at);
          gv.x += old.x; gv.y += old.y; gv.z += old.z; gv.w += old.w;
        }
        store_stream4(a.gx + at, gv);
      }
    } else {
      int e = wrap_mod(int64_t(pos) + 4 * hh, n);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int off = base + e;
        if (a.x) g4[k] = fmaf(g, a.x[off], g4[k]);
        if (a.gx) {
          const float gv = c4[k] * g;
          a.gx[off] = a.accumulate ? a.gx[off] + gv : gv;
        }
        if (++e == n) e = 0;
      }
    }
  }
  if (a.partial) {
    float packed[8];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      packed[e] = hh ? 0.0f : g4[e];
      packed[4 + e] = hh ? g4[e] : 0.0f;
    }
    block_reduce_store<8>(packed, 8, a.partial + int64_t(blockIdx.x) * 8, a.counter != nullptr);
    if (a.counter && arrive_last(a.counter)) {
      reduce_rows_fixed(a.partial, gridDim.x, 8, 0, 8, a.gc, a.accumulate);
      if (threadIdx.x == 0) __hip_atomic_store(a.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint of the fused chain (both stages injective)
// ---------------------------------------------------------------------------
template <bool VEC, int T0, int T1>
__global__ void __launch_bounds__(kBlock) fir_chain_adjoint_kernel(FirChainAdjArgs a) {
  const Win3& h = a.h;
  const Win3& v = a.v;
  const int t0 = T0 ? T0 : h.taps;
  const int t1 = T1 ? T1 : v.taps;
  float ch[kMaxTaps], cv[kMaxTaps], gp[2 * kMaxTaps];
#pragma unroll
  for (int k = 0; k < kMaxTaps; ++k) {
    ch[k] = k < t0 ? a.ch[k] : 0.0f;
    cv[k] = k < t1 ? a.cv[k] : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < 2 * kMaxTaps; ++k) gp[k] = 0.0f;

  const uint32_t stride = gridDim.x * kBlock;
  for (uint32_t o = blockIdx.x * kBlock + threadIdx.x; o < a.n_out; o += stride) {
    const OutPos q = decode(o, v, a.div_rc, a.div_rr);
    const float g = a.gy[o];
    if constexpr (VEC && T0 > 0 && T1 > 0) {
      // interior: all loads of the T1 x T0 input block, then arithmetic, then stores
      int off[T1];
      if (chain_rows<T0, T1>(h, v, q, off)) {
        float4 blk[T1][T0 / 4];
#pragma unroll
        for (int j = 0; j < T1; ++j)
#pragma unroll
          for (int u = 0; u < T0 / 4; ++u) blk[j][u] = *reinterpret_cast<const float4*>(a.x + off[j] + 4 * u);
#pragma unroll
        for (int j = 0; j < T1; ++j) {
          const float gm = cv[j] * g;
          float mid = 0.0f;
#pragma unroll
          for (int u = 0; u < T0 / 4; ++u) {
            const float xv[4] = {blk[j][u].x, blk[j][u].y, blk[j][u].z, blk[j][u].w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
              mid = fmaf(ch[4 * u + e], xv[e], mid);
              gp[4 * u + e] = fmaf(gm, xv[e], gp[4 * u + e]);
            }
          }
          gp[kMaxTaps + j] = fmaf(g, mid, gp[kMaxTaps + j]);
        }
        if (a.gx) {
#pragma unroll
          for (int j = 0; j < T1; ++j) {
            const float gm = cv[j] * g;
#pragma unroll
            for (int u = 0; u < T0 / 4; ++u) {
              float4 gv = make_float4(ch[4 * u + 0] * gm, ch[4 * u + 1] * gm, ch[4 * u + 2] * gm,
                                      ch[4 * u + 3] * gm);
              float4* d4 = reinterpret_cast<float4*>(a.gx + off[j] + 4 * u);
              if (a.accumulate) {
                const float4 old = *d4;
                gv.x += old.x; gv.y += old.y; gv.z += old.z; gv.w += old.w;
              }
              *d4 = gv;
            }
          }
        }
        continue;
      }
    }
    const int mb = v.o[0] + v.p[0] * q.b;
    const int mc = v.o[2] + v.p[2] * q.c;
    const int xb = h.o[0] + h.p[0] * mb;
    const int xstart = h.o[2] + h.p[2] * mc;
    const bool inside = xstart >= 0 && xstart + t0 <= h.A[2];
    int mr = wrap_mod(int64_t(v.o[1]) + int64_t(v.p[1]) * q.r, v.A[1]);
#pragma unroll
    for (int j = 0; j < (T1 ? T1 : kMaxTaps); ++j) {
      if (j >= t1) break;
      const int row_base = (xb * h.A[1] + h.o[1] + h.p[1] * mr) * h.A[2];
      const float gm = cv[j] * g;          // gradient of this intermediate element
      float xs[kMaxTaps];
      if (VEC && inside) {
        const float* xp = a.x + row_base + xstart;
#pragma unroll
        for (int q4 = 0; q4 < (T0 ? T0 : kMaxTaps) / 4; ++q4) {
          if (4 * q4 >= t0) break;
          const float4 xv = *reinterpret_cast<const float4*>(xp + 4 * q4);
          xs[4 * q4 + 0] = xv.x; xs[4 * q4 + 1] = xv.y;
          xs[4 * q4 + 2] = xv.z; xs[4 * q4 + 3] = xv.w;
        }
      } else {
        int e = inside ? xstart : wrap_mod(xstart, h.A[2]);
#pragma unroll
        for (int k = 0; k < (T0 ? T0 : kMaxTaps); ++k) {
          if (k >= t0) break;
          xs[k] = a.x[row_base + e];
          if (++e == h.A[2]) e = 0;
        }
      }
      float mid = 0.0f;
#pragma unroll
      for (int k = 0; k < (T0 ? T0 : kMaxTaps); ++k) {
        if (k >= t0) break;
        mid = fmaf(ch[k], xs[k], mid);
        gp[k] = fmaf(gm, xs[k], gp[k]);                 // d/dch[k]
      }
      gp[kMaxTaps + j] = fmaf(g, mid, gp[kMaxTaps + j]);  // d/dcv[j]
      if (a.gx) {
        if (VEC && inside) {
          float* dst = a.gx + row_base + xstart;
#pragma unroll
          for (int q4 = 0; q4 < (T0 ? T0 : kMaxTaps) / 4; ++q4) {
            if (4 * q4 >= t0) break;
            float4 gv = make_float4(ch[4 * q4 + 0] * gm, ch[4 * q4 + 1] * gm,
                                    ch[4 * q4 + 2] * gm, ch[4 * q4 + 3] * gm);
            float4* d4 = reinterpret_cast<float4*>(dst + 4 * q4);
            if (a.accumulate) {
              const float4 old = *d4;
              gv.x += old.x; gv.y += old.y; gv.z += old.z; gv.w += old.w;
            }
            *d4 = gv;
          }
        } else {
          int e = inside ? xstart : wrap_mod(xstart, h.A[2]);
#pragma unroll
          for (int k = 0; k < (T0 ? T0 : kMaxTaps); ++k) {
            if (k >= t0) break;
            const float gv = ch[k] * gm;
            float* d = a.gx + row_base + e;
            *d = a.accumulate ? *d + gv : gv;
            if (++e == h.A[2]) e = 0;
          }
        }
      }
      if (++mr == v.A[1]) mr = 0;
    }
  }
  if (a.partial) {
    // pack [ch grads (t0) | cv grads (t1)] contiguously
    float packed[2 * kMaxTaps];
#pragma unroll
    for (int k = 0; k < 2 * kMaxTaps; ++k) packed[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < kMaxTaps; ++k) {
      if (k < t0) packed[k] = gp[k];
    }
#pragma unroll
    for (int k = 0; k < kMaxTaps; ++k) {
      if (k < t1) packed[t0 + k] = gp[kMaxTaps + k];
    }
    block_reduce_store<2 * kMaxTaps>(packed, t0 + t1, a.partial + int64_t(blockIdx.x) * (t0 + t1),
                                     a.counter != nullptr);
    if (a.counter && arrive_last(a.counter)) {
      if (a.gch) reduce_rows_fixed(a.partial, gridDim.x, t0 + t1, 0, t0, a.gch, a.accumulate);
      if (a.gcv) reduce_rows_fixed(a.partial, gridDim.x, t0 + t1, t0, t1, a.gcv, a.accumulate);
      if (threadIdx.x == 0) __hip_atomic_store(a.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------
// adjoint of the fused chain, 8 column taps, lane pairs, software-pipelined:
// the loads of a thread's next output are issued before the stores of the
// current one, so stores retire while the next block streams in.
// ---------------------------------------------------------------------------
template <int T1>
struct PairBlock {
  uint32_t o;
  int off[T1];
  float4 x[T1];
  float g;
  bool fast;
};

template <int T1>
__device__ __forceinline__ void pair_fetch(const FirChainAdjArgs& a, uint32_t gidx, int hh,
                                           PairBlock<T1>& b) {
  b.o = gidx >> 1;
  const OutPos q = decode(b.o, a.v, a.div_rc, a.div_rr);
  b.fast = chain_rows<8, T1>(a.h, a.v, q, b.off);
  b.g = a.gy[b.o];
  if (b.fast) {
#pragma unroll
    for (int j = 0; j < T1; ++j) b.x[j] = load_stream4(a.x + b.off[j] + 4 * hh);
  }
}

template <int T1>
__global__ void __launch_bounds__(kBlock) fir_chain_adjoint_pair_kernel(FirChainAdjArgs a) {
  const Win3& h = a.h;
  const Win3& v = a.v;
  const uint32_t n_half = 2u * a.n_out;
  const uint32_t stride = gridDim.x * kBlock;
  const int hh = threadIdx.x & 1;
  float c4[4], cv[T1], g4[4], gv[T1];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    c4[e] = a.ch[4 * hh + e];
    g4[e] = 0.0f;
  }
#pragma unroll
  for (int j = 0; j < T1; ++j) {
    cv[j] = a.cv[j];
    gv[j] = 0.0f;
  }
  uint32_t gi = blockIdx.x * kBlock + threadIdx.x;
  PairBlock<T1> cur;
  if (gi < n_half) pair_fetch<T1>(a, gi, hh, cur);
  while (gi < n_half) {
    const uint32_t gn = gi + stride;
    PairBlock<T1> nxt;
    if (gn < n_half) pair_fetch<T1>(a, gn, hh, nxt);
    const float g = cur.g;
    if (cur.fast) {
#pragma unroll
      for (int j = 0; j < T1; ++j) {
        const float gm = cv[j] * g;
        float part = c4[0] * cur.x[j].x;
        part = fmaf(c4[1], cur.x[j].y, part);
        part = fmaf(c4[2], cur.x[j].z, part);
        part = fmaf(c4[3], cur.x[j].w, part);
        const float other = __shfl_xor(part, 1);
        const float mid = hh ? other + part : part + other;
        if (hh == 0) gv[j] = fmaf(g, mid, gv[j]);
        g4[0] = fmaf(gm, cur.x[j].x, g4[0]);
        g4[1] = fmaf(gm, cur.x[j].y, g4[1]);
        g4[2] = fmaf(gm, cur.x[j].z, g4[2]);
        g4[3] = fmaf(gm, cur.x[j].w, g4[3]);
      }
      if (a.gx) {
#pragma unroll
        for (int j = 0; j < T1; ++j) {
          const float gm = cv[j] * g;
          float4 w4 = make_float4(c4[0] * gm, c4[1] * gm, c4[2] * gm, c4[3] * gm);
          float4* d4 = reinterpret_cast<float4*>(a.gx + cur.off[j] + 4 * hh);
          if (a.accumulate) {
            const float4 old = *d4;
            w4.x += old.x; w4.y += old.y; w4.z += old.z; w4.w += old.w;
          }
          store_stream4(reinterpret_cast<float*>(d4), w4);
        }
      }
    } else {
      // window wraps: each lane handles its own four taps on the modular path
      const OutPos q = decode(cur.o, v, a.div_rc, a.div_rr);
      const int mb = v.o[0] + v.p[0] * q.b;
      const int mc = v.o[2] + v.p[2] * q.c;
      const int xb = h.o[0] + h.p[0] * mb;
      const int xstart = h.o[2] + h.p[2] * mc;
      int mr = wrap_mod(int64_t(v.o[1]) + int64_t(v.p[1]) * q.r, v.A[1]);
      for (int j = 0; j < T1; ++j) {
        const int row_base = (xb * h.A[1] + h.o[1] + h.p[1] * mr) * h.A[2];
        const float gm = cv[j] * g;
        int col = wrap_mod(int64_t(xstart) + 4 * hh, h.A[2]);
        float xs[4];
        int cols[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          cols[e] = col;
          xs[e] = a.x[row_base + col];
          if (++col == h.A[2]) col = 0;
        }
        float part = c4[0] * xs[0];
        part = fmaf(c4[1], xs[1], part);
        part = fmaf(c4[2], xs[2], part);
        part = fmaf(c4[3], xs[3], part);
        const float other = __shfl_xor(part, 1);
        const float mid = hh ? other + part : part + other;
        if (hh == 0) gv[j] = fmaf(g, mid, gv[j]);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          g4[e] = fmaf(gm, xs[e], g4[e]);
          if (a.gx) {
            float* d = a.gx + row_base + cols[e];
            *d = a.accumulate ? *d + c4[e] * gm : c4[e] * gm;
          }
        }
        if (++mr == v.A[1]) mr = 0;
      }
    }
    cur = nxt;
    gi = gn;
  }
  if (a.partial) {
    // [d/dch (8) | d/dcv (T1)]: a lane owns half of the ch slots
    float packed[8 + T1];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      packed[e] = hh ? 0.0f : g4[e];
      packed[4 + e] = hh ? g4[e] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < T1; ++j) packed[8 + j] = gv[j];
    block_reduce_store<8 + T1>(packed, 8 + T1, a.partial + int64_t(blockIdx.x) * (8 + T1),
                               a.counter != nullptr);
    if (a.counter && arrive_last(a.counter)) {
      if (a.gch) reduce_rows_fixed(a.partial, gridDim.x, 8 + T1, 0, 8, a.gch, a.accumulate);
      if (a.gcv) reduce_rows_fixed(a.partial, gridDim.x, 8 + T1, 8, T1, a.gcv, a.accumulate);
      if (threadIdx.x == 0) __hip_atomic_store(a.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

// ---------------------------------------------------------------------------
// training step of the fused chain under the loss L = sum_o wl[o] y[o]^2:
// one pass over x computes y (stored), dL/dy = 2 wl y in registers, and the
// adjoint (dL/dx stored, weight-gradient partials), so the step reads x once
// instead of twice and never writes or reads dL/dy.  Same lane-pair layout
// and software pipeline as the adjoint kernel; the stage-1 sums of the
// forward are the ones the weight gradient of stage 2 needs.
// ---------------------------------------------------------------------------
template <int T1>
__device__ __forceinline__ void train_fetch(const FirChainAdjArgs& a, uint32_t gidx, int hh, PairBlock<T1>& b) {
  b.o = gidx >> 1;
  const OutPos q = decode(b.o, a.v, a.div_rc, a.div_rr);
  b.fast = chain_rows<8, T1>(a.h, a.v, q, b.off);
  b.g = a.wl[b.o];
  if (b.fast) {
#pragma unroll
    for (int j = 0; j < T1; ++j) b.x[j] = load_stream4(a.x + b.off[j] + 4 * hh);
  }
}

template <int T1>
__global__ void __launch_bounds__(kBlock) fir_chain_train_pair_kernel(FirChainAdjArgs a) {
  const Win3& h = a.h;
  const Win3& v = a.v;
  const uint32_t n_half = 2u * a.n_out;
  const uint32_t stride = gridDim.x * kBlock;
  const int hh = threadIdx.x & 1;
  float c4[4], cv[T1], g4[4], gv[T1];
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    c4[e] = a.ch[4 * hh + e];
    g4[e] = 0.0f;
  }
#pragma unroll
  for (int j = 0; j < T1; ++j) {
    cv[j] = a.cv[j];
    gv[j] = 0.0f;
  }
  uint32_t gi = blockIdx.x * kBlock + threadIdx.x;
  PairBlock<T1> cur;
  if (gi < n_half) train_fetch<T1>(a, gi, hh, cur);
  while (gi < n_half) {
    const uint32_t gn = gi + stride;
    PairBlock<T1> nxt;
    if (gn < n_half) train_fetch<T1>(a, gn, hh, nxt);
    if (cur.fast) {
      // forward: stage-1 sums per row (lane 2m: taps 0-3, lane 2m+1: 4-7,
      // added in that order on both lanes), then the stage-2 sum
      float mid[T1];
      float y = 0.0f;
#pragma unroll
      for (int j = 0; j < T1; ++j) {
        float part = c4[0] * cur.x[j].x;
        part = fmaf(c4[1], cur.x[j].y, part);
        part = fmaf(c4[2], cur.x[j].z, part);
        part = fmaf(c4[3], cur.x[j].w, part);
        const float other = __shfl_xor(part, 1);
        mid[j] = hh ? other + part : part + other;
        y = fmaf(cv[j], mid[j], y);
      }
      if (hh == 0) store_stream(a.y + cur.o, y);
      const float g = 2.0f * (cur.g * y);
#pragma unroll
      for (int j = 0; j < T1; ++j) {
        const float gm = cv[j] * g;
        if (hh == 0) gv[j] = fmaf(g, mid[j], gv[j]);
        g4[0] = fmaf(gm, cur.x[j].x, g4[0]);
        g4[1] = fmaf(gm, cur.x[j].y, g4[1]);
        g4[2] = fmaf(gm, cur.x[j].z, g4[2]);
        g4[3] = fmaf(gm, cur.x[j].w, g4[3]);
      }
      if (a.gx) {
#pragma unroll
        for (int j = 0; j < T1; ++j) {
          const float gm = cv[j] * g;
          float4 w4 = make_float4(c4[0] * gm, c4[1] * gm, c4[2] * gm, c4[3] * gm);
          float4* d4 = reinterpret_cast<float4*>(a.gx + cur.off[j] + 4 * hh);
          if (a.accumulate) {
            const float4 old = *d4;
            w4.x += old.x; w4.y += old.y; w4.z += old.z; w4.w += old.w;
          }
          store_stream4(reinterpret_cast<float*>(d4), w4);
        }
      }
    } else {
      // window wraps: each lane reads its own four taps of every row on the
      // modular path, keeps them for the adjoint, and both lanes form y
      const OutPos q = decode(cur.o, v, a.div_rc, a.div_rr);
      const int mb = v.o[0] + v.p[0] * q.b;
      const int mc = v.o[2] + v.p[2] * q.c;
      const int xb = h.o[0] + h.p[0] * mb;
      const int xstart = h.o[2] + h.p[2] * mc;
      const int mr0 = wrap_mod(int64_t(v.o[1]) + int64_t(v.p[1]) * q.r, v.A[1]);
      const int col0 = wrap_mod(int64_t(xstart) + 4 * hh, h.A[2]);
      float xs[T1][4], mid[T1];
      float y = 0.0f;
      int mr = mr0;
#pragma unroll
      for (int j = 0; j < T1; ++j) {
        const int row_base = (xb * h.A[1] + h.o[1] + h.p[1] * mr) * h.A[2];
        int col = col0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          xs[j][e] = a.x[row_base + col];
          if (++col == h.A[2]) col = 0;
        }
        float part = c4[0] * xs[j][0];
        part = fmaf(c4[1], xs[j][1], part);
        part = fmaf(c4[2], xs[j][2], part);
        part = fmaf(c4[3], xs[j][3], part);
        const float other = __shfl_xor(part, 1);
        mid[j] = hh ? other + part : part + other;
        y = fmaf(cv[j], mid[j], y);
        if (++mr == v.A[1]) mr = 0;
      }
      if (hh == 0) a.y[cur.o] = y;
      const float g = 2.0f * (cur.g * y);
      mr = mr0;
#pragma unroll
      for (int j = 0; j < T1; ++j) {
        const int row_base = (xb * h.A[1] + h.o[1] + h.p[1] * mr) * h.A[2];
        const float gm = cv[j] * g;
        if (hh == 0) gv[j] = fmaf(g, mid[j], gv[j]);
        int col = col0;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          g4[e] = fmaf(gm, xs[j][e], g4[e]);
          if (a.gx) {
            float* d = a.gx + row_base + col;
            *d = a.accumulate ? *d + c4[e] * gm : c4[e] * gm;
          }
          if (++col == h.A[2]) col = 0;
        }
        if (++mr == v.A[1]) mr = 0;
      }
    }
    cur = nxt;
    gi = gn;
  }
  if (a.partial) {
    float packed[8 + T1];
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      packed[e] = hh ? 0.0f : g4[e];
      packed[4 + e] = hh ? g4[e] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < T1; ++j) packed[8 + j] = gv[j];
    block_reduce_store<8 + T1>(packed, 8 + T1, a.partial + int64_t(blockIdx.x) * (8 + T1), false);
  }
}

// ---------------------------------------------------------------------------
// training step of a fused injective pair with any tap counts (up to 16 per
// stage) and any window alignment: one thread per output.  The forward sums
// are formed as in fir_chain_kernel (taps in order, then the stage-2 sum),
// dL/dy = 2 wl y, and the adjoint follows fir_chain_adjoint_kernel; x is read
// twice per output, the second time from the cache the first read filled.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) fir_chain_train_kernel(FirChainAdjArgs a) {
  const Win3& h = a.h;
  const Win3& v = a.v;
  const int t0 = h.taps, t1 = v.taps;
  float ch[kMaxTaps], cv[kMaxTaps], gp[2 * kMaxTaps];
#pragma unroll
  for (int k = 0; k < kMaxTaps; ++k) {
    ch[k] = k < t0 ? a.ch[k] : 0.0f;
    cv[k] = k < t1 ? a.cv[k] : 0.0f;
  }
#pragma unroll
  for (int k = 0; k < 2 * kMaxTaps; ++k) gp[k] = 0.0f;
  const uint32_t stride = gridDim.x * kBlock;
  for (uint32_t o = blockIdx.x * kBlock + threadIdx.x; o < a.n_out; o += stride) {
    const OutPos q = decode(o, v, a.div_rc, a.div_rr);
    const int mb = v.o[0] + v.p[0] * q.b;
    const int mc = v.o[2] + v.p[2] * q.c;
    const int xb = h.o[0] + h.p[0] * mb;
    const int xstart = h.o[2] + h.p[2] * mc;
    const bool inside = xstart >= 0 && xstart + t0 <= h.A[2];
    const int col0 = inside ? xstart : wrap_mod(xstart, h.A[2]);
    const int mr0 = wrap_mod(int64_t(v.o[1]) + int64_t(v.p[1]) * q.r, v.A[1]);
    // forward
    float mid[kMaxTaps];
    float y = 0.0f;
    int mr = mr0;
#pragma unroll
    for (int j = 0; j < kMaxTaps; ++j) {
      mid[j] = 0.0f;
      if (j >= t1) break;
      const int row_base = (xb * h.A[1] + h.o[1] + h.p[1] * mr) * h.A[2];
      float m = 0.0f;
      int e = col0;
#pragma unroll
      for (int k = 0; k < kMaxTaps; ++k) {
        if (k >= t0) break;
        m = fmaf(ch[k], a.x[row_base + e], m);
        if (++e == h.A[2]) e = 0;
      }
      mid[j] = m;
      y = fmaf(cv[j], m, y);
      if (++mr == v.A[1]) mr = 0;
    }
    a.y[o] = y;
    const float g = 2.0f * (a.wl[o] * y);
    // adjoint
    mr = mr0;
#pragma unroll
    for (int j = 0; j < kMaxTaps; ++j) {
      if (j >= t1) break;
      const int row_base = (xb * h.A[1] + h.o[1] + h.p[1] * mr) * h.A[2];
      const float gm = cv[j] * g;
      gp[kMaxTaps + j] = fmaf(g, mid[j], gp[kMaxTaps + j]);
      int e = col0;
#pragma unroll
      for (int k = 0; k < kMaxTaps; ++k) {
        if (k >= t0) break;
        gp[k] = fmaf(gm, a.x[row_base + e], gp[k]);
        if (a.gx) {
          float* d = a.gx + row_base + e;
          const float gv = ch[k] * gm;
          *d = a.accumulate ? *d + gv : gv;
        }
        if (++e == h.A[2]) e = 0;
      }
      if (++mr == v.A[1]) mr = 0;
    }
  }
  if (a.partial) {
    // [ch grads (t0) | cv grads (t1)] contiguously
    float packed[2 * kMaxTaps];
#pragma unroll
    for (int k = 0; k < 2 * kMaxTaps; ++k) packed[k] = 0.0f;
#pragma unroll
    for (int k = 0; k < kMaxTaps; ++k)
      if (k < t0) packed[k] = gp[k];
#pragma unroll
    for (int k = 0; k < kMaxTaps; ++k)
      if (k < t1) packed[t0 + k] = gp[kMaxTaps + k];
    block_reduce_store<2 * kMaxTaps>(packed, t0 + t1, a.partial + int64_t(blockIdx.x) * (t0 + t1), false);
  }
}

int stream_grid(uint32_t work, int waves_per_cu = 8) {
  // enough resident blocks to cover the chip several times, grid-stride beyond
  const int cap = 256 * waves_per_cu;
  const uint32_t need = (work + kBlock - 1) / kBlock;
  return int(need < uint32_t(cap) ? (need ? need : 1) : cap);
}

}  // namespace

hipError_t launch_pattern_reduce(const PatternReduceArgs& a, int max_rank, hipStream_t st) {
  const int64_t lanes = a.n_rep << a.group_log2;
  int64_t grid = (lanes + kBlock - 1) / kBlock;
  if (grid < 1) grid = 1;
  if (grid > 16384) grid = 16384;
  if (max_rank <= 4)
    pattern_reduce_kernel<4><<<unsigned(grid), kBlock, 0, st>>>(a);
  else
    pattern_reduce_kernel<kMaxRank><<<unsigned(grid), kBlock, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_fir(const FirArgs& a, bool vec4, hipStream_t st) {
  const int grid = stream_grid(a.n_out, 16);
  if (a.w.ax == 2) {
    if (vec4 && a.w.taps == 8 && a.n_out < (1u << 30))
      fir_pair_kernel<<<stream_grid(2u * a.n_out, 16), kBlock, 0, st>>>(a);
    else if (vec4 && a.w.taps == 8)
      fir_kernel<2, true, 8><<<grid, kBlock, 0, st>>>(a);
    else if (vec4)
      fir_kernel<2, true, 0><<<grid, kBlock, 0, st>>>(a);
    else if (a.w.taps == 8)
      fir_kernel<2, false, 8><<<grid, kBlock, 0, st>>>(a);
    else
      fir_kernel<2, false, 0><<<grid, kBlock, 0, st>>>(a);
  } else {
    if (a.w.taps == 8)
      fir_kernel<1, false, 8><<<grid, kBlock, 0, st>>>(a);
    else
      fir_kernel<1, false, 0><<<grid, kBlock, 0, st>>>(a);
  }
  return hipGetLastError();
}

hipError_t launch_fir_chain(const FirChainArgs& a, bool vec4, hipStream_t st) {
  if (vec4 && a.h.taps == 8 && a.v.taps == 8) {
    fir_chain_pair_kernel<8><<<stream_grid(2u * a.n_out, 8), kBlock, 0, st>>>(a);
    return hipGetLastError();
  }
  const int grid = stream_grid(a.n_out, 16);
  if (vec4)
    fir_chain_kernel<true, 0, 0><<<grid, kBlock, 0, st>>>(a);
  else
    fir_chain_kernel<false, 0, 0><<<grid, kBlock, 0, st>>>(a);
  return hipGetLastError();
}

// sized for two lanes per repetition (the lane-pair kernel); the other
// variants run one lane per repetition over the same grid
int fir_adjoint_grid(const FirAdjArgs& a) { return stream_grid(2u * a.n_rep, 8); }

hipError_t launch_fir_adjoint(const FirAdjArgs& a, bool vec4, int* grid_out, hipStream_t st) {
  const int grid = fir_adjoint_grid(a);
  if (grid_out) *grid_out = grid;
  if (a.w.ax == 2) {
    if (vec4 && a.w.taps == 8)
      fir_adjoint_pair_kernel<<<grid, kBlock, 0, st>>>(a);
    else if (vec4)
      fir_adjoint_kernel<2, true, 0><<<grid, kBlock, 0, st>>>(a);
    else
      fir_adjoint_kernel<2, false, 0><<<grid, kBlock, 0, st>>>(a);
  } else {
    if (a.w.taps == 8)
      fir_adjoint_kernel<1, false, 8><<<grid, kBlock, 0, st>>>(a);
    else
      fir_adjoint_kernel<1, false, 0><<<grid, kBlock, 0, st>>>(a);
  }
  return hipGetLastError();
}

static bool chain_adjoint_uses_pairs(const FirChainAdjArgs& a, bool vec4) {
  return vec4 && a.h.taps == 8 && a.v.taps == 8;
}

int fir_chain_adjoint_grid(const FirChainAdjArgs& a, bool vec4) {
  return chain_adjoint_uses_pairs(a, vec4) ? stream_grid(2u * a.n_out, 8) : stream_grid(a.n_out, 8);
}

int fir_chain_adjoint_partial_width(const FirChainAdjArgs& a, bool vec4) {
  return chain_adjoint_uses_pairs(a, vec4) ? 8 + a.v.taps : a.h.taps + a.v.taps;
}

hipError_t launch_fir_chain_adjoint(const FirChainAdjArgs& a, bool vec4, hipStream_t st) {
  const int grid = fir_chain_adjoint_grid(a, vec4);
  if (chain_adjoint_uses_pairs(a, vec4))
    fir_chain_adjoint_pair_kernel<8><<<grid, kBlock, 0, st>>>(a);
  else if (vec4)
    fir_chain_adjoint_kernel<true, 0, 0><<<grid, kBlock, 0, st>>>(a);
  else
    fir_chain_adjoint_kernel<false, 0, 0><<<grid, kBlock, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_fir_chain_train(const FirChainAdjArgs& a, hipStream_t st) {
  fir_chain_train_pair_kernel<8><<<fir_chain_adjoint_grid(a, true), kBlock, 0, st>>>(a);
  return hipGetLastError();
}

int fir_chain_train_generic_grid(const FirChainAdjArgs& a) { return stream_grid(a.n_out, 8); }

hipError_t launch_fir_chain_train_generic(const FirChainAdjArgs& a, hipStream_t st) {
  fir_chain_train_kernel<<<fir_chain_train_generic_grid(a), kBlock, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace rsm
