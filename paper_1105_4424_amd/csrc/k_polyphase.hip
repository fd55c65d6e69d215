// k_polyphase.hip -- weighted sums whose output pattern has q > 1 elements
// along the tap axis (polyphase stages): repetition r reads the window
// x[(o + p r + i) mod A], i < T, and writes q consecutive outputs
//
//     y[q r + j] = sum_i c[j T + i] x[(o + p r + i) mod A],   j < q
//
// (rows of the q x T coefficient matrix are the taps of each phase).  The
// two outer axes of the [B, R, C] view are single points of each window and
// do not wrap.
//
//  * poly_cols_kernel: taps along columns.  One workgroup per (row, chunk of
//    256 repetitions): the chunk's input segment (p (n - 1) + T columns,
//    wrapped at the borders) is staged in LDS with coalesced loads, each
//    thread forms the q outputs of one repetition from its window in LDS,
//    and the chunk's q n outputs leave through LDS as one contiguous run.
//  * poly_rows_kernel: taps along rows.  One thread per repetition, lanes
//    along the contiguous column axis, so every load and store of a
//    wavefront is one contiguous 256-byte run.
//  * poly_gx_gather_kernel: input gradient as a gather, one thread per input
//    element: the (repetition, tap) pairs that reach the element are found
//    by lifting its index to the unwrapped window positions, and each pair
//    adds sum_j c[j T + i] gy[q r + j] in a fixed order (no atomics).
//  * poly_gc_kernel: weight gradient, one thread per repetition, q x T
//    partial sums per thread reduced per workgroup in a fixed order; a
//    second kernel sums the workgroups' rows in a fixed order.
#include <hip/hip_runtime.h>

#include "rsm_internal.h"

namespace rsm {
namespace {

constexpr int kBlock = 256;
constexpr int kChunk = 256;          // repetitions per workgroup item (columns kernel)
constexpr int kMaxP = 16;            // paving step along the tap axis
constexpr int kMaxT = 32;            // taps
constexpr int kMaxQ = 8;             // outputs per repetition
constexpr int kSeg = kMaxP * (kChunk - 1) + kMaxT;   // staged input floats per item

__device__ __forceinline__ int wrap_mod(int64_t v, int n) {
  int64_t q = v % n;
  return int(q < 0 ? q + n : q);
}

// ---------------------------------------------------------------------------
// forward, taps along columns
// ---------------------------------------------------------------------------
template <int KT>
__global__ void __launch_bounds__(kBlock) poly_cols_kernel(PolyArgs a) {
  __shared__ float xs[kSeg];
  __shared__ float ys[kMaxQ * kChunk];
  __shared__ float cs[kMaxQ * kMaxT];
  const Win3& w = a.w;
  const int T = w.taps, q = a.q, p = w.p[2];
  const int t = int(threadIdx.x);
  if (t < q * T) cs[t] = a.c[t];
  const uint32_t item = blockIdx.x;
  const uint32_t row = fdiv(item, a.div_chunks);            // (b, r) of the outer axes
  const int chunk = int(item - row * uint32_t(a.n_chunks));
  const uint32_t b = fdiv(row, a.div_rr);
  const int r1 = int(row - b * uint32_t(w.rep[1]));
  const int xb = w.o[0] + w.p[0] * int(b);
  const int xr = w.o[1] + w.p[1] * r1;
  const float* __restrict__ xrow = a.x + (int64_t(xb) * w.A[1] + xr) * w.A[2];
  const int c0 = chunk * kChunk;
  const int n = min(kChunk, w.rep[2] - c0);
  const int L = p * (n - 1) + T;
  const int64_t s0 = int64_t(w.o[2]) + int64_t(p) * c0;
  if (s0 >= 0 && s0 + L <= w.A[2]) {
    const float* src = xrow + s0;
    for (int e = t; e < L; e += kBlock) xs[e] = src[e];
  } else {
    int col = wrap_mod(s0 + t, w.A[2]);
    const int step = kBlock % w.A[2];
    for (int e = t; e < L; e += kBlock) {
      xs[e] = xrow[col];
      col += step;
      if (col >= w.A[2]) col -= w.A[2];
    }
  }
  __syncthreads();
  if (t < n) {
    float win[KT];
#pragma unroll
    for (int i = 0; i < KT; ++i) win[i] = i < T ? xs[p * t + i] : 0.0f;
#pragma unroll
    for (int j = 0; j < kMaxQ; ++j) {
      if (j < q) {
        float acc = 0.0f;
#pragma unroll
        for (int i = 0; i < KT; ++i)
          if (i < T) acc = fmaf(cs[j * T + i], win[i], acc);
        ys[q * t + j] = acc;
      }
    }
  }
  __syncthreads();
  float* __restrict__ yrow = a.y + int64_t(row) * (int64_t(w.rep[2]) * q) + int64_t(c0) * q;
  for (int e = t; e < q * n; e += kBlock) yrow[e] = ys[e];
}

// ---------------------------------------------------------------------------
// forward, taps along rows
// ---------------------------------------------------------------------------
template <int KT>
__global__ void __launch_bounds__(kBlock) poly_rows_kernel(PolyArgs a) {
  __shared__ float cs[kMaxQ * kMaxT];
  const Win3& w = a.w;
  const int T = w.taps, q = a.q;
  if (int(threadIdx.x) < q * T) cs[threadIdx.x] = a.c[threadIdx.x];
  __syncthreads();
  const uint32_t stride = gridDim.x * kBlock;
  for (uint32_t o = blockIdx.x * kBlock + threadIdx.x; o < a.n_items; o += stride) {
    const uint32_t rowi = fdiv(o, a.div_rc);
    const int c = int(o - rowi * uint32_t(w.rep[2]));
    const uint32_t b = fdiv(rowi, a.div_rr);
    const int r = int(rowi - b * uint32_t(w.rep[1]));
    const int xb = w.o[0] + w.p[0] * int(b);
    const int xc = w.o[2] + w.p[2] * c;
    const float* __restrict__ plane = a.x + int64_t(xb) * w.A[1] * w.A[2] + xc;
    const int64_t start = int64_t(w.o[1]) + int64_t(w.p[1]) * r;
    float win[KT];
    if (start >= 0 && start + T <= w.A[1]) {
#pragma unroll
      for (int i = 0; i < KT; ++i) win[i] = i < T ? plane[(start + i) * w.A[2]] : 0.0f;
    } else {
      int xr = wrap_mod(start, w.A[1]);
#pragma unroll
      for (int i = 0; i < KT; ++i) {
        win[i] = i < T ? plane[int64_t(xr) * w.A[2]] : 0.0f;
        if (++xr == w.A[1]) xr = 0;
      }
    }
    float* __restrict__ dst = a.y + (int64_t(b) * w.rep[1] * q + int64_t(q) * r) * w.rep[2] + c;
#pragma unroll
    for (int j = 0; j < kMaxQ; ++j) {
      if (j < q) {
        float acc = 0.0f;
#pragma unroll
        for (int i = 0; i < KT; ++i)
          if (i < T) acc = fmaf(cs[j * T + i], win[i], acc);
        dst[int64_t(j) * w.rep[2]] = acc;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// input gradient as a gather (either tap axis)
// ---------------------------------------------------------------------------
// Repetition index along a non-tap axis for array index a_d, or -1 if no
// repetition reads it.
__device__ __forceinline__ int outer_rep(int a_d, int o, int p, int rep, const FastDiv& dp) {
  const int v = a_d - o;
  if (v < 0) return -1;
  if (rep == 1) return v == 0 ? 0 : -1;
  const int k = int(fdiv(uint32_t(v), dp));
  return (k * p == v && k < rep) ? k : -1;
}

template <int AX>
__global__ void __launch_bounds__(kBlock) poly_gx_gather_kernel(PolyGatherArgs a) {
  __shared__ float cs[kMaxQ * kMaxT];
  const Win3& w = a.w;
  const int T = w.taps, q = a.q;
  if (int(threadIdx.x) < q * T) cs[threadIdx.x] = a.c[threadIdx.x];
  __syncthreads();
  const int n_ax = w.A[AX], R = w.rep[AX], p = w.p[AX];
  const int span = p * (R - 1) + T;   // unwrapped positions covered, v in [0, span)
  const uint32_t stride = gridDim.x * kBlock;
  for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < a.n_arr; e += stride) {
    const uint32_t rowi = fdiv(e, a.div_a2);
    const int ac = int(e - rowi * uint32_t(w.A[2]));
    const uint32_t bb = fdiv(rowi, a.div_a1);
    const int ar = int(rowi - bb * uint32_t(w.A[1]));
    const int rb = outer_rep(int(bb), w.o[0], w.p[0], w.rep[0], a.div_p[0]);
    int ro, at;
    if (AX == 2) {
      ro = outer_rep(ar, w.o[1], w.p[1], w.rep[1], a.div_p[1]);
      at = ac;
    } else {
      ro = outer_rep(ac, w.o[2], w.p[2], w.rep[2], a.div_p[2]);
      at = ar;
    }
    float acc = 0.0f;
    if (rb >= 0 && ro >= 0) {
      // gy offset of (repetition r, phase j) along the tap axis: g0 + r gs + j gj
      int64_t g0, gs, gj;
      if (AX == 2) {
        g0 = (int64_t(rb) * w.rep[1] + ro) * (int64_t(R) * q);
        gs = q;
        gj = 1;
      } else {
        g0 = int64_t(rb) * (int64_t(R) * q) * w.rep[2] + ro;
        gs = int64_t(q) * w.rep[2];
        gj = w.rep[2];
      }
      int v = at - a.o_mod;   // first lift: v = (a - o) mod A
      if (v < 0) v += n_ax;
      for (; v < span; v += n_ax) {
        int r = int(fdiv(uint32_t(v), a.div_p[AX]));
        if (r > R - 1) r = R - 1;
        for (int i = v - p * r; r >= 0 && i < T; --r, i += p) {
          const float* g = a.gy + g0 + r * gs;
          for (int j = 0; j < q; ++j) acc = fmaf(cs[j * T + i], g[j * gj], acc);
        }
      }
    }
    a.gx[e] = a.accumulate ? a.gx[e] + acc : acc;
  }
}

// ---------------------------------------------------------------------------
// weight gradient: gc[j][i] = sum_r gy[q r + j] x[(o + p r + i) mod A]
// ---------------------------------------------------------------------------
template <int AX>
__global__ void __launch_bounds__(kBlock) poly_gc_kernel(PolyArgs a) {
  constexpr int KT = 16, QT = 4;
  __shared__ float sm[kBlock / 64][QT * KT];
  const Win3& w = a.w;
  const int T = w.taps, q = a.q;
  float gp[QT][KT];
#pragma unroll
  for (int j = 0; j < QT; ++j)
#pragma unroll
    for (int i = 0; i < KT; ++i) gp[j][i] = 0.0f;
  const uint32_t stride = gridDim.x * kBlock;
  for (uint32_t o = blockIdx.x * kBlock + threadIdx.x; o < a.n_items; o += stride) {
    const uint32_t rowi = fdiv(o, a.div_rc);
    const int c = int(o - rowi * uint32_t(w.rep[2]));
    const uint32_t b = fdiv(rowi, a.div_rr);
    const int r = int(rowi - b * uint32_t(w.rep[1]));
    const int xb = w.o[0] + w.p[0] * int(b);
    float win[KT], g[QT];
    if (AX == 2) {
      const int xr = w.o[1] + w.p[1] * r;
      const float* __restrict__ xrow = a.x + (int64_t(xb) * w.A[1] + xr) * w.A[2];
      int col = wrap_mod(int64_t(w.o[2]) + int64_t(w.p[2]) * c, w.A[2]);
#pragma unroll
      for (int i = 0; i < KT; ++i) {
        win[i] = i < T ? xrow[col] : 0.0f;
        if (++col == w.A[2]) col = 0;
      }
      const float* gr = a.gy + int64_t(rowi) * (int64_t(w.rep[2]) * q) + int64_t(q) * c;
#pragma unroll
      for (int j = 0; j < QT; ++j) g[j] = j < q ? gr[j] : 0.0f;
    } else {
      const int xc = w.o[2] + w.p[2] * c;
      const float* __restrict__ plane = a.x + int64_t(xb) * w.A[1] * w.A[2] + xc;
      int xr = wrap_mod(int64_t(w.o[1]) + int64_t(w.p[1]) * r, w.A[1]);
#pragma unroll
      for (int i = 0; i < KT; ++i) {
        win[i] = i < T ? plane[int64_t(xr) * w.A[2]] : 0.0f;
        if (++xr == w.A[1]) xr = 0;
      }
      const float* gr = a.gy + (int64_t(b) * w.rep[1] * q + int64_t(q) * r) * w.rep[2] + c;
#pragma unroll
      for (int j = 0; j < QT; ++j) g[j] = j < q ? gr[int64_t(j) * w.rep[2]] : 0.0f;
    }
#pragma unroll
    for (int j = 0; j < QT; ++j)
#pragma unroll
      for (int i = 0; i < KT; ++i) gp[j][i] = fmaf(g[j], win[i], gp[j][i]);
  }
  // per workgroup: butterfly inside each wavefront, then the four wavefront
  // sums in order; one row of q T partials per workgroup
#pragma unroll
  for (int j = 0; j < QT; ++j)
#pragma unroll
    for (int i = 0; i < KT; ++i) {
      float v = gp[j][i];
#pragma unroll
      for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
      gp[j][i] = v;
    }
  const int wave = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) {
#pragma unroll
    for (int j = 0; j < QT; ++j)
#pragma unroll
      for (int i = 0; i < KT; ++i) sm[wave][j * KT + i] = gp[j][i];
  }
  __syncthreads();
  const int k = int(threadIdx.x);
  if (k < q * T) {
    const int j = k / T, i = k - j * T;
    const int s = j * KT + i;
    a.partial[int64_t(blockIdx.x) * (q * T) + k] = ((sm[0][s] + sm[1][s]) + sm[2][s]) + sm[3][s];
  }
}

}  // namespace

bool poly_supported(const Win3& w, int q) {
  if (w.ax == 2 && (w.p[2] < 1 || w.p[2] > kMaxP)) return false;
  return w.taps >= 1 && w.taps <= kMaxT && q >= 1 && q <= kMaxQ;
}

bool poly_gc_supported(const Win3& w, int q) { return w.taps <= 16 && q <= 4; }

int poly_chunks(const Win3& w) { return (w.rep[2] + kChunk - 1) / kChunk; }

hipError_t launch_poly(const PolyArgs& a, hipStream_t st) {
  const int T = a.w.taps;
  if (a.w.ax == 2) {
    const unsigned grid = a.n_items;
    if (T <= 8)
      poly_cols_kernel<8><<<grid, kBlock, 0, st>>>(a);
    else if (T <= 16)
      poly_cols_kernel<16><<<grid, kBlock, 0, st>>>(a);
    else
      poly_cols_kernel<32><<<grid, kBlock, 0, st>>>(a);
  } else {
    const uint32_t need = (a.n_items + kBlock - 1) / kBlock;
    const int grid = int(need < 256u * 16u ? (need ? need : 1) : 256u * 16u);
    if (T <= 8)
      poly_rows_kernel<8><<<grid, kBlock, 0, st>>>(a);
    else if (T <= 16)
      poly_rows_kernel<16><<<grid, kBlock, 0, st>>>(a);
    else
      poly_rows_kernel<32><<<grid, kBlock, 0, st>>>(a);
  }
  return hipGetLastError();
}

hipError_t launch_poly_gx_gather(const PolyGatherArgs& a, hipStream_t st) {
  const uint32_t need = (a.n_arr + kBlock - 1) / kBlock;
  const int grid = int(need < 256u * 16u ? (need ? need : 1) : 256u * 16u);
  if (a.w.ax == 2)
    poly_gx_gather_kernel<2><<<grid, kBlock, 0, st>>>(a);
  else
    poly_gx_gather_kernel<1><<<grid, kBlock, 0, st>>>(a);
  return hipGetLastError();
}

int poly_gc_grid(uint32_t n_rep) {
  const uint32_t need = (n_rep + kBlock - 1) / kBlock;
  return int(need < 256u * 8u ? (need ? need : 1) : 256u * 8u);
}

hipError_t launch_poly_gc(const PolyArgs& a, hipStream_t st) {
  const int grid = poly_gc_grid(a.n_items);
  if (a.w.ax == 2)
    poly_gc_kernel<2><<<grid, kBlock, 0, st>>>(a);
  else
    poly_gc_kernel<1><<<grid, kBlock, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace rsm
