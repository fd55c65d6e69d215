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
//  * poly_cols_kernel: taps along columns.  Items are (row, chunk of 256
//    repetitions); a resident grid walks them, each workgroup staging an
//    item's input segment (p (n - 1) + T columns, wrapped at the borders) in
//    LDS from registers that were loaded, coalesced, while it computed the
//    previous items (two items in flight); each thread forms and stores the
//    q outputs of one repetition from its window in LDS.
//  * poly_cols_vec_kernel: taps along columns, one thread per repetition,
//    its window read as four 16-byte vectors (p and A[2] multiples of four,
//    o mod 4 + T <= 16, q <= 4).
//  * poly_rows_kernel: taps along rows.  One thread per repetition, lanes
//    along the contiguous column axis, so every load and store of a
//    wavefront is one contiguous 256-byte run; poly_rows_vec_kernel gives a
//    thread four adjacent repetitions (16-byte loads and stores) where the
//    columns allow it.
//  * poly_gx_gather_kernel: input gradient as a gather, one thread per input
//    element: the (repetition, tap) pairs that reach the element are found
//    by lifting its index to the unwrapped window positions, and each pair
//    adds sum_j c[j T + i] gy[q r + j] in a fixed order (no atomics).
//  * poly_gc_kernel: weight gradient, one thread per repetition, q x T
//    partial sums per thread reduced per workgroup in a fixed order; a
//    second kernel sums the workgroups' rows in a fixed order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <mutex>
#include <utility>
#include <vector>

#include "rsm_internal.h"

namespace rsm {
namespace {

constexpr int kBlock = 256;
constexpr int kChunk = 256;          // repetitions per workgroup item (columns kernel)
constexpr int kMaxP = 16;            // paving step along the tap axis
constexpr int kMaxT = 32;            // taps
constexpr int kMaxQ = 8;             // outputs per repetition
constexpr int kSeg = kMaxP * (kChunk - 1) + kMaxT;   // staged input floats per item
static_assert(kMaxQ * kMaxT == kBlock, "one coefficient slot per thread");

__device__ __forceinline__ int wrap_mod(int64_t v, int n) {
  int64_t q = v % n;
  return int(q < 0 ? q + n : q);
}

// ---------------------------------------------------------------------------
// forward, taps along columns
// ---------------------------------------------------------------------------
// Geometry of one (row, chunk) item.
struct ColItem {
  const float* xrow;   // the input row
  float* yrow;         // the chunk's first output
  int64_t s0;          // first input column of the chunk's segment (unwrapped)
  int n;               // repetitions in the chunk
  int L;               // segment length p (n - 1) + T
  bool interior;       // the segment does not wrap
};

__device__ __forceinline__ ColItem col_item(const PolyArgs& a, uint32_t item) {
  const Win3& w = a.w;
  ColItem it;
  const uint32_t row = fdiv(item, a.div_chunks);            // (b, r) of the outer axes
  const int chunk = int(item - row * uint32_t(a.n_chunks));
  const uint32_t b = fdiv(row, a.div_rr);
  const int r1 = int(row - b * uint32_t(w.rep[1]));
  const int xb = w.o[0] + w.p[0] * int(b);
  const int xr = w.o[1] + w.p[1] * r1;
  it.xrow = a.x + (int64_t(xb) * w.A[1] + xr) * w.A[2];
  const int c0 = chunk * kChunk;
  it.n = min(kChunk, w.rep[2] - c0);
  it.L = w.p[2] * (it.n - 1) + w.taps;
  it.s0 = int64_t(w.o[2]) + int64_t(w.p[2]) * c0;
  it.interior = it.s0 >= 0 && it.s0 + it.L <= w.A[2];
  it.yrow = a.y + int64_t(row) * (int64_t(w.rep[2]) * a.q) + int64_t(c0) * a.q;
  return it;
}

// Issue the loads of an item's input segment into registers: element
// e = t + 256 m of the segment goes to thread t.
template <int PF>
__device__ __forceinline__ void col_fetch(const ColItem& it, int A2, float (&v)[PF]) {
  const int t = int(threadIdx.x);
  if (it.interior) {
    const float* src = it.xrow + it.s0;
#pragma unroll
    for (int m = 0; m < PF; ++m) {
      const int e = t + kBlock * m;
      v[m] = e < it.L ? src[e] : 0.0f;
    }
  } else {
    int col = wrap_mod(it.s0 + t, A2);
    const int step = kBlock % A2;
#pragma unroll
    for (int m = 0; m < PF; ++m) {
      const int e = t + kBlock * m;
      v[m] = e < it.L ? it.xrow[col] : 0.0f;
      col += step;
      if (col >= A2) col -= A2;
    }
  }
}

// One item: its segment (fetched into v earlier) goes to LDS, the loads of
// the item two places further on go out into the same registers, and each
// thread forms the q outputs of one repetition.  A window whose start is a
// multiple of four floats (p % 4 == 0) is read as 16-byte vectors.  With
// q > 1 the outputs of a wavefront (64 q consecutive floats) pass through a
// per-wavefront LDS slice so that every store instruction writes 256
// contiguous bytes (a wavefront's LDS accesses stay in order, so no barrier
// is needed for that).
template <int KT, int PF, int QT>
__device__ __forceinline__ void col_step(const PolyArgs& a, const ColItem& it, float (&v)[PF], uint32_t ahead,
                                         float* xs, const float* cs, float* ws) {
  const Win3& w = a.w;
  const int T = w.taps, q = a.q, p = w.p[2];
  const int t = int(threadIdx.x);
  __syncthreads();   // the previous item's readers of xs are done
#pragma unroll
  for (int m = 0; m < PF; ++m) {
    const int e = t + kBlock * m;
    if (e < it.L) xs[e] = v[m];
  }
  __syncthreads();
  if (ahead < a.n_items) col_fetch<PF>(col_item(a, ahead), w.A[2], v);
  float win[KT];
  if ((p & 3) == 0) {
#pragma unroll
    for (int u = 0; u < KT / 4; ++u) {
      if (4 * u < T) {
        const float4 f = *reinterpret_cast<const float4*>(xs + p * t + 4 * u);
        win[4 * u + 0] = f.x; win[4 * u + 1] = f.y; win[4 * u + 2] = f.z; win[4 * u + 3] = f.w;
      } else {
        win[4 * u + 0] = win[4 * u + 1] = win[4 * u + 2] = win[4 * u + 3] = 0.0f;
      }
    }
  } else {
#pragma unroll
    for (int i = 0; i < KT; ++i) win[i] = i < T ? xs[p * t + i] : 0.0f;
  }
  // coefficient rows padded with zeros to kMaxT floats: read as 16-byte
  // broadcasts; taps past T multiply zeros and are skipped
  float y[QT];
#pragma unroll
  for (int j = 0; j < QT; ++j) {
    y[j] = 0.0f;
    if (j < q) {
#pragma unroll
      for (int u = 0; u < KT / 4; ++u) {
        if (4 * u < T) {
          const float4 c4 = *reinterpret_cast<const float4*>(cs + j * kMaxT + 4 * u);
          const float cc[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
          for (int e = 0; e < 4; ++e)
            if (4 * u + e < T) y[j] = fmaf(cc[e], win[4 * u + e], y[j]);
        }
      }
    }
  }
  if (q == 1) {
    if (t < it.n) it.yrow[t] = y[0];
    return;
  }
  const int lane = t & 63, wave = t >> 6;
  float* wsl = ws + wave * (64 * kMaxQ);
#pragma unroll
  for (int j = 0; j < QT; ++j)
    if (j < q) wsl[q * lane + j] = y[j];
  // this wavefront's repetitions 64 wave + 0..63 own outputs [64 q wave, 64 q (wave + 1))
  const int nw = min(64, it.n - 64 * wave);   // repetitions of the chunk this wavefront holds
  float* dst = it.yrow + 64 * q * wave;
#pragma unroll
  for (int j = 0; j < QT; ++j)
    if (j < q && 64 * j + lane < q * nw) dst[64 * j + lane] = wsl[64 * j + lane];
}

// Persistent: workgroup b takes items b, b + grid, ...; two items' segments
// are in flight in registers while it computes the current one from LDS.
template <int KT, int PF, int QT>
__global__ void __launch_bounds__(kBlock) poly_cols_kernel(PolyArgs a) {
  __shared__ __align__(16) float xs[PF * kBlock + 32];
  __shared__ __align__(16) float cs[kMaxQ * kMaxT];
  __shared__ float ws[kBlock * kMaxQ];
  const Win3& w = a.w;
  const int t = int(threadIdx.x);
  const uint32_t g = gridDim.x;
  uint32_t item = blockIdx.x;
  if (item >= a.n_items) return;
  {
    const int j = t / kMaxT, i = t - j * kMaxT;   // 256 threads = kMaxQ rows of kMaxT
    cs[t] = (j < a.q && i < w.taps) ? a.c[j * w.taps + i] : 0.0f;
  }
  float v0[PF], v1[PF];
  col_fetch<PF>(col_item(a, item), w.A[2], v0);
  if (item + g < a.n_items) col_fetch<PF>(col_item(a, item + g), w.A[2], v1);
  while (true) {
    col_step<KT, PF, QT>(a, col_item(a, item), v0, item + 2 * g, xs, cs, ws);
    item += g;
    if (item >= a.n_items) break;
    col_step<KT, PF, QT>(a, col_item(a, item), v1, item + 2 * g, xs, cs, ws);
    item += g;
    if (item >= a.n_items) break;
  }
}

// One thread per repetition with the window in registers, read as 16-byte
// vectors straight from memory.  With p and A[2] multiples of four, every
// window start o + p r lies the same distance off = o mod 4 past a 16-byte
// boundary, so taps 0 .. T-1 are floats off .. off+T-1 of the four aligned
// vectors at o + p r - off (off + T <= 16).  The weights, shifted by off and
// zero outside the taps, are read once per thread into vector registers.
// Floats of the 16 outside
// the window are zeroed before the products (they may hold non-finite
// values that the window does not contain), so each output adds its taps in
// ascending order to zero, like the staged kernel.  Neighbouring windows
// share half of their vectors; the second read mostly comes from the L1 or
// L2 cache (1.03-1.06 x the input from memory).  Windows that cross the
// row's border read each float with the wrap.
template <int QT>
__global__ void __launch_bounds__(kBlock) poly_cols_vec_kernel(PolyArgs a) {
  const Win3& w = a.w;
  const int T = w.taps, p = w.p[2], A2 = w.A[2], R = w.rep[2];
  const int off = ((w.o[2] % 4) + 4) % 4;
  // the shifted weights in vector registers (16 q of them: in scalar
  // registers they spill for q >= 3); lane0 is zero on every lane but not
  // known to be uniform, so the loads are vector loads
  const int lane0 = int(__builtin_amdgcn_mbcnt_lo(0u, 0u));
  float cv[QT][16];
#pragma unroll
  for (int j = 0; j < QT; ++j)
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const int k = i - off;
      const int kc = k < 0 ? 0 : (k >= T ? T - 1 : k);   // an address inside the weights
      const float v = a.c[j * T + kc + lane0];
      cv[j][i] = (k >= 0 && k < T) ? v : 0.0f;
    }
  const uint32_t stride = gridDim.x * kBlock;
  for (uint32_t it = blockIdx.x * kBlock + threadIdx.x; it < a.n_items; it += stride) {
    const uint32_t row = fdiv(it, a.div_rc);
    const int c = int(it - row * uint32_t(R));
    const uint32_t b = fdiv(row, a.div_rr);
    const int r1 = int(row - b * uint32_t(w.rep[1]));
    const float* xrow = a.x + (int64_t(w.o[0] + w.p[0] * int(b)) * w.A[1] + (w.o[1] + w.p[1] * r1)) * A2;
    const int base = w.o[2] + p * c - off;   // a multiple of 4
    float win[16];
    if (base >= 0 && base + 16 <= A2) {
      const float4* src = reinterpret_cast<const float4*>(xrow + base);
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const float4 f = src[u];
        win[4 * u + 0] = f.x; win[4 * u + 1] = f.y; win[4 * u + 2] = f.z; win[4 * u + 3] = f.w;
      }
    } else {
      int col = wrap_mod(base, A2);
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        win[i] = xrow[col];
        if (++col == A2) col = 0;
      }
    }
#pragma unroll
    for (int i = 0; i < 16; ++i)
      if (i < off || i >= off + T) win[i] = 0.0f;
    float* dst = a.y + (int64_t(row) * R + c) * QT;
#pragma unroll
    for (int j = 0; j < QT; ++j) {
      float acc = 0.0f;
#pragma unroll
      for (int i = 0; i < 16; ++i) acc = fmaf(cv[j][i], win[i], acc);
      dst[j] = acc;
    }
  }
}

// ---------------------------------------------------------------------------
// forward, taps along rows
// ---------------------------------------------------------------------------
template <int KT>
__global__ void __launch_bounds__(kBlock) poly_rows_kernel(PolyArgs a) {
  __shared__ __align__(16) float cs[kMaxQ * kMaxT];
  const Win3& w = a.w;
  const int T = w.taps, q = a.q;
  {
    const int t = int(threadIdx.x);
    const int j = t / kMaxT, i = t - j * kMaxT;   // rows padded with zeros to kMaxT
    cs[t] = (j < q && i < T) ? a.c[j * T + i] : 0.0f;
  }
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
        for (int u = 0; u < KT / 4; ++u) {
          if (4 * u < T) {
            const float4 c4 = *reinterpret_cast<const float4*>(cs + j * kMaxT + 4 * u);
            const float cc[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
            for (int e = 0; e < 4; ++e)
              if (4 * u + e < T) acc = fmaf(cc[e], win[4 * u + e], acc);
          }
        }
        dst[int64_t(j) * w.rep[2]] = acc;
      }
    }
  }
}


// The same with V adjacent repetitions along the column axis per thread
// (column step 1, rows of a multiple of V repetitions starting on a 4V-byte
// boundary, the launcher checks): every load and store moves 4V bytes and
// each coefficient read serves V windows.
template <int V>
struct VecF;
template <>
struct VecF<2> {
  typedef float2 T;
};
template <>
struct VecF<4> {
  typedef float4 T;
};

template <int KT, int QT, int V>
__global__ void __launch_bounds__(kBlock) poly_rows_vec_kernel(PolyArgs a) {
  typedef typename VecF<V>::T vec;
  __shared__ __align__(16) float cs[kMaxQ * kMaxT];
  const Win3& w = a.w;
  const int T = w.taps, q = a.q;
  {
    const int t = int(threadIdx.x);
    const int j = t / kMaxT, i = t - j * kMaxT;   // rows padded with zeros to kMaxT
    cs[t] = (j < q && i < T) ? a.c[j * T + i] : 0.0f;
  }
  __syncthreads();
  const uint32_t nv = a.n_items / V;
  const uint32_t stride = gridDim.x * kBlock;
  // workgroups are dealt to the 8 XCDs round-robin; give each XCD a
  // contiguous band of the launch (the grid is a multiple of 8), so that the
  // windows one step further down a column, taken one output row of threads
  // later, usually run on the same XCD and find their shared rows in its L2
  const uint32_t band = gridDim.x / 8;
  const uint32_t lb = (blockIdx.x % 8) * band + blockIdx.x / 8;
  for (uint32_t ov = lb * kBlock + threadIdx.x; ov < nv; ov += stride) {
    const uint32_t o = V * ov;
    const uint32_t rowi = fdiv(o, a.div_rc);
    const int c = int(o - rowi * uint32_t(w.rep[2]));   // a multiple of V
    const uint32_t b = fdiv(rowi, a.div_rr);
    const int r = int(rowi - b * uint32_t(w.rep[1]));
    const int xb = w.o[0] + w.p[0] * int(b);
    const float* __restrict__ plane = a.x + int64_t(xb) * w.A[1] * w.A[2] + w.o[2] + c;
    const int64_t start = int64_t(w.o[1]) + int64_t(w.p[1]) * r;
    float win[KT][V];
    int xr = start >= 0 && start < w.A[1] ? int(start) : wrap_mod(start, w.A[1]);
#pragma unroll
    for (int i = 0; i < KT; ++i) {
      if (i < T) {
        const vec v = *reinterpret_cast<const vec*>(plane + int64_t(xr) * w.A[2]);
        const float* f = reinterpret_cast<const float*>(&v);
#pragma unroll
        for (int e = 0; e < V; ++e) win[i][e] = f[e];
      } else {
#pragma unroll
        for (int e = 0; e < V; ++e) win[i][e] = 0.0f;
      }
      if (++xr == w.A[1]) xr = 0;
    }
    float* __restrict__ dst = a.y + (int64_t(b) * w.rep[1] * q + int64_t(q) * r) * w.rep[2] + c;
#pragma unroll
    for (int j = 0; j < QT; ++j) {
      if (j < q) {
        float acc[V];
#pragma unroll
        for (int e = 0; e < V; ++e) acc[e] = 0.0f;
#pragma unroll
        for (int u = 0; u < KT / 4; ++u) {
          if (4 * u < T) {
            const float4 c4 = *reinterpret_cast<const float4*>(cs + j * kMaxT + 4 * u);
            const float cc[4] = {c4.x, c4.y, c4.z, c4.w};
#pragma unroll
            for (int k = 0; k < 4; ++k)
              if (4 * u + k < T) {
#pragma unroll
                for (int e = 0; e < V; ++e) acc[e] = fmaf(cc[k], win[4 * u + k][e], acc[e]);
              }
          }
        }
        vec out;
        float* of = reinterpret_cast<float*>(&out);
#pragma unroll
        for (int e = 0; e < V; ++e) of[e] = acc[e];
        *reinterpret_cast<vec*>(dst + int64_t(j) * w.rep[2]) = out;
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

// ---------------------------------------------------------------------------
// both gradients of a polyphase stage along columns, one pass
//
// Items are (row, chunk of 256 repetitions); the chunk owns the columns a
// whose first lift v = (a - o) mod A lies in [256 p c, 256 p (c + 1)) (the
// same ownership as the forward chunks, so every column is written by
// exactly one item).  A workgroup stages the dL/dy of the repetitions those
// columns can meet (the chunk's, and the K - 1 before it, K = ceil(T / p))
// and, for the weight gradient, the input segment of the chunk's own
// repetitions.  Then
//  * each thread forms dL/dx at its columns (positions v = 256 p c + t +
//    256 m): the pairs (r, i) with p r + i = v, r from min(R - 1, v / p)
//    down while i < T, each adding sum_j c[j T + i] dL/dy[q r + j]; pairs of
//    further lifts (windows that go round the row) follow, from LDS when the
//    row is one chunk, from memory otherwise;
//  * thread t < G q T (G = floor(256 / (q T)) groups) keeps one weight
//    slot s = t mod q T, (j, i) = (s / T, s mod T), and adds
//    dL/dy[q r + j] x[(o + p r + i) mod A] over its group's share of the
//    chunk's repetitions, in order.
// Nothing is atomic: dL/dx is a plain store per element and the weight
// slots are reduced per workgroup (groups in order), then across
// workgroups, in a fixed order.
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(kBlock) poly_adj_cols_kernel(PolyAdjArgs a) {
  __shared__ __align__(16) float xs[kSeg + 32];
  __shared__ float gys[kMaxQ * (kChunk + kMaxT)];
  __shared__ __align__(16) float cs[kMaxQ * kMaxT];
  __shared__ float red[kBlock];
  const Win3& w = a.w;
  const int T = w.taps, q = a.q, p = w.p[2], A2 = w.A[2], R = w.rep[2];
  const int K = (T + p - 1) / p;
  const int span = p * (R - 1) + T;
  const int t = int(threadIdx.x);
  {
    const int j = t / kMaxT, i = t - j * kMaxT;   // rows padded with zeros to kMaxT
    cs[t] = (j < q && i < T) ? a.c[j * T + i] : 0.0f;
  }
  const int nslot = q * T;
  const int G = kBlock / nslot;                    // groups of weight slots
  const int slot = t % nslot, grp = t / nslot;
  const int sj = slot / T, si = slot - sj * T;
  float gacc = 0.0f;
  for (uint32_t item = blockIdx.x; item < a.n_items; item += gridDim.x) {
    const uint32_t row = fdiv(item, a.div_chunks);
    const int chunk = int(item - row * uint32_t(a.n_chunks));
    const uint32_t b = fdiv(row, a.div_rr);
    const int r1 = int(row - b * uint32_t(w.rep[1]));
    const int xb = w.o[0] + w.p[0] * int(b);
    const int xr = w.o[1] + w.p[1] * r1;
    const int64_t xoff = (int64_t(xb) * w.A[1] + xr) * A2;
    const float* __restrict__ gyrow = a.gy + int64_t(row) * (int64_t(R) * q);
    const int c0 = chunk * kChunk;
    const int n = max(0, min(kChunk, R - c0));     // the chunk's own repetitions
    const int rs = c0 - (K - 1);                   // first staged repetition
    const int ng = min(kChunk + K - 1, R - rs);    // staged repetitions
    __syncthreads();   // the previous item's readers of xs and gys are done
    const int e_lo = rs < 0 ? -rs * q : 0;        // repetition rs + e / q >= 0
    for (int e = t; e < q * ng; e += kBlock) gys[e] = e >= e_lo ? gyrow[int64_t(rs) * q + e] : 0.0f;
    const int L = n > 0 ? p * (n - 1) + T : 0;
    if (a.partial && L > 0) {
      const float* xrow = a.x + xoff;
      const int64_t s0 = int64_t(w.o[2]) + int64_t(p) * c0;
      if (s0 >= 0 && s0 + L <= A2) {
        for (int e = t; e < L; e += kBlock) xs[e] = xrow[s0 + e];
      } else {
        int col = wrap_mod(s0 + t, A2);
        const int step = kBlock % A2;
        for (int e = t; e < L; e += kBlock) {
          xs[e] = xrow[col];
          col += step;
          if (col >= A2) col -= A2;
        }
      }
    }
    __syncthreads();
    // input gradient at the chunk's columns
    if (a.gx) {
      float* __restrict__ gxrow = a.gx + xoff;
      const int v_end = min(p * (c0 + kChunk), A2);
      for (int v = p * c0 + t; v < v_end; v += kBlock) {
        float acc = 0.0f;
        int r = int(fdiv(uint32_t(v), a.div_p));
        if (r > R - 1) r = R - 1;
        for (int i = v - p * r; r >= 0 && i < T; --r, i += p) {
          const float* g = gys + (r - rs) * q;
          for (int j = 0; j < q; ++j) acc = fmaf(cs[j * kMaxT + i], g[j], acc);
        }
        for (int u = v + A2; u < span; u += A2) {
          r = int(fdiv(uint32_t(u), a.div_p));
          if (r > R - 1) r = R - 1;
          for (int i = u - p * r; r >= 0 && i < T; --r, i += p) {
            const float* g = a.n_chunks == 1 ? gys + (r - rs) * q : gyrow + int64_t(r) * q;
            for (int j = 0; j < q; ++j) acc = fmaf(cs[j * kMaxT + i], g[j], acc);
          }
        }
        int col = a.o_mod + v;
        if (col >= A2) col -= A2;
        gxrow[col] = a.accumulate ? gxrow[col] + acc : acc;
      }
    }
    // weight slots: this group's share of the chunk's repetitions
    if (a.partial && grp < G) {
      const int per = (n + G - 1) / G;
      const int t0 = grp * per, t1 = min(n, t0 + per);
      const float* g = gys + (t0 + K - 1) * q + sj;
      const float* xv = xs + p * t0 + si;
      for (int tt = t0; tt < t1; ++tt) {
        gacc = fmaf(*g, *xv, gacc);
        g += q;
        xv += p;
      }
    }
  }
  if (!a.partial) return;
  // per workgroup: slot s is the sum of groups 0, 1, ... in order
  __syncthreads();
  red[t] = grp < G ? gacc : 0.0f;
  __syncthreads();
  if (t < nslot) {
    float sum = 0.0f;
    for (int gg = 0; gg < G; ++gg) sum += red[gg * nslot + t];
    a.partial[int64_t(blockIdx.x) * nslot + t] = sum;
  }
}

// ---------------------------------------------------------------------------
// both gradients along columns, phase form: when p divides 256 and the row
// length, a thread's positions v = 256 p c + t + 256 m all have the same
// phase i0 = v mod p, and every pair (r, i) that reaches one of them -- first
// lift or further lifts -- has a tap i = i0 + k p with k < K.  The thread
// keeps c[j][i0 + k p] in registers and adds gy[q r + j] x[v] into weight
// slot (k, j) as it forms dL/dx[v]; slots of equal phase are summed over the
// workgroup's threads in a fixed order at the end.  The item staging is the
// same as above, x taken at the owned positions (one value per position).
// ---------------------------------------------------------------------------
// Geometry of one adjoint item.
struct AdjItem {
  int64_t xoff;          // offset of the input row (x and dL/dx)
  const float* gyrow;    // dL/dy row
  int c0, rs, ng;        // first repetition of the chunk, first staged repetition, staged count
  int v0, nv;            // first owned position, owned positions
  int col0;              // column of position v0
};

__device__ __forceinline__ AdjItem adj_item(const PolyAdjArgs& a, uint32_t item, int K) {
  const Win3& w = a.w;
  AdjItem it;
  const uint32_t row = fdiv(item, a.div_chunks);
  const int chunk = int(item - row * uint32_t(a.n_chunks));
  const uint32_t b = fdiv(row, a.div_rr);
  const int r1 = int(row - b * uint32_t(w.rep[1]));
  const int xb = w.o[0] + w.p[0] * int(b);
  const int xr = w.o[1] + w.p[1] * r1;
  it.xoff = (int64_t(xb) * w.A[1] + xr) * w.A[2];
  it.gyrow = a.gy + int64_t(row) * (int64_t(w.rep[2]) * a.q);
  it.c0 = chunk * kChunk;
  it.rs = it.c0 - (K - 1);
  it.ng = min(kChunk + K - 1, w.rep[2] - it.rs);
  it.v0 = w.p[2] * it.c0;
  it.nv = max(0, min(w.p[2] * kChunk, w.A[2] - it.v0));
  it.col0 = a.o_mod + it.v0;
  if (it.col0 >= w.A[2]) it.col0 -= w.A[2];
  return it;
}

// Loads of an item's staged values into registers: x at the owned positions
// (element e = t + 256 m) and dL/dy of the staged repetitions.
template <int XF, int GF>
__device__ __forceinline__ void adj_fetch(const PolyAdjArgs& a, const AdjItem& it, float (&xv)[XF], float (&gv)[GF]) {
  const int t = int(threadIdx.x);
  const int A2 = a.w.A[2], q = a.q;
  // staged value e belongs to repetition rs + e / q, which exists from
  // e >= -rs q on (rs < 0 only in a row's first chunk): no division
  const int e_lo = it.rs < 0 ? -it.rs * q : 0, e_hi = q * it.ng;
#pragma unroll
  for (int m = 0; m < GF; ++m) {
    const int e = t + kBlock * m;
    gv[m] = (e < e_hi && e >= e_lo) ? it.gyrow[int64_t(it.rs) * q + e] : 0.0f;
  }
  if (!a.partial) return;
  const float* xrow = a.x + it.xoff;
  if (it.col0 + it.nv <= A2) {
#pragma unroll
    for (int m = 0; m < XF; ++m) {
      const int e = t + kBlock * m;
      xv[m] = e < it.nv ? xrow[it.col0 + e] : 0.0f;
    }
  } else {
    int col = it.col0 + t;
    while (col >= A2) col -= A2;
    const int step = kBlock % A2;
#pragma unroll
    for (int m = 0; m < XF; ++m) {
      const int e = t + kBlock * m;
      xv[m] = e < it.nv ? xrow[col] : 0.0f;
      col += step;
      if (col >= A2) col -= A2;
    }
  }
}

template <int KM, int QM, int XF, int GF>
__device__ __forceinline__ void adj_step(const PolyAdjArgs& a, const AdjItem& it, float (&xv)[XF],
                                         float (&gv)[GF], uint32_t ahead, float* xs, float* gys,
                                         const float (&cr)[KM][QM], float (&ga)[KM][QM]) {
  const Win3& w = a.w;
  const int T = w.taps, q = a.q, p = w.p[2], A2 = w.A[2], R = w.rep[2];
  const int K = (T + p - 1) / p;
  const int span = p * (R - 1) + T;
  const int t = int(threadIdx.x);
  const int lp = 31 - __builtin_clz(uint32_t(p));   // p = 2^lp
  const int i0 = t & (p - 1);
  const int per_m = kBlock >> lp;                  // repetitions between a thread's positions
  __syncthreads();   // the previous item's readers of xs and gys are done
#pragma unroll
  for (int m = 0; m < GF; ++m) gys[t + kBlock * m] = gv[m];
  if (a.partial) {
#pragma unroll
    for (int m = 0; m < XF; ++m) xs[t + kBlock * m] = xv[m];
  }
  __syncthreads();
  if (ahead < a.n_items) adj_fetch<XF, GF>(a, adj_item(a, ahead, K), xv, gv);   // travels meanwhile
  float* __restrict__ gxrow = a.gx ? a.gx + it.xoff : nullptr;
  const float* __restrict__ gyrow = it.gyrow;
  const int rs = it.rs;
  int r_hi = it.c0 + (t >> lp);
  for (int e = t; e < it.nv; e += kBlock, r_hi += per_m) {
    const int v = it.v0 + e;
    const float x1 = a.partial ? xs[e] : 0.0f;
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      const int r = r_hi - k;
      if (k < K && r >= 0 && r <= R - 1 && i0 + k * p < T) {
        const float* g = gys + (r - rs) * q;
#pragma unroll
        for (int j = 0; j < QM; ++j)
          if (j < q) {
            const float g1 = g[j];
            acc = fmaf(cr[k][j], g1, acc);
            ga[k][j] = fmaf(g1, x1, ga[k][j]);
          }
      }
    }
    // further lifts: u = v + m A, r = u / p - k, the same taps (A % p == 0)
    for (int u = v + A2, rr = r_hi + (A2 >> lp); u < span; u += A2, rr += (A2 >> lp)) {
#pragma unroll
      for (int k = 0; k < KM; ++k) {
        const int r = rr - k;
        if (k < K && r >= 0 && r <= R - 1 && i0 + k * p < T) {
          const float* g = a.n_chunks == 1 ? gys + (r - rs) * q : gyrow + int64_t(r) * q;
#pragma unroll
          for (int j = 0; j < QM; ++j)
            if (j < q) {
              const float g1 = g[j];
              acc = fmaf(cr[k][j], g1, acc);
              ga[k][j] = fmaf(g1, x1, ga[k][j]);
            }
        }
      }
    }
    if (gxrow) {
      int col = it.col0 + e;
      if (col >= A2) col -= A2;
      gxrow[col] = a.accumulate ? gxrow[col] + acc : acc;
    }
  }
}

// Persistent over items, two items' loads in flight in registers.  Bounded
// to 72 registers so that seven waves share a SIMD instead of six (one
// register and a few scalars spill; 166 -> 160 us back to back on the
// 30 x 1080 x 1920 stage).
template <int KM, int QM, int XF, int GF>
__global__ void __launch_bounds__(kBlock, 7) poly_adj_phase_kernel(PolyAdjArgs a) {
  __shared__ float xs[XF * kBlock];
  __shared__ float gys[GF * kBlock];
  __shared__ float red[kBlock];
  const Win3& w = a.w;
  const int T = w.taps, q = a.q, p = w.p[2];
  const int K = (T + p - 1) / p;
  const int t = int(threadIdx.x);
  const int i0 = t & (p - 1);
  float cr[KM][QM], ga[KM][QM];
#pragma unroll
  for (int k = 0; k < KM; ++k)
#pragma unroll
    for (int j = 0; j < QM; ++j) {
      const int i = i0 + k * p;
      cr[k][j] = (k < K && j < q && i < T) ? a.c[j * T + i] : 0.0f;
      ga[k][j] = 0.0f;
    }
  const uint32_t g = gridDim.x;
  uint32_t item = blockIdx.x;
  if (item < a.n_items) {
    float x0[XF], x1[XF], g0[GF], g1[GF];
    adj_fetch<XF, GF>(a, adj_item(a, item, K), x0, g0);
    if (item + g < a.n_items) adj_fetch<XF, GF>(a, adj_item(a, item + g, K), x1, g1);
    while (true) {
      adj_step<KM, QM, XF, GF>(a, adj_item(a, item, K), x0, g0, item + 2 * g, xs, gys, cr, ga);
      item += g;
      if (item >= a.n_items) break;
      adj_step<KM, QM, XF, GF>(a, adj_item(a, item, K), x1, g1, item + 2 * g, xs, gys, cr, ga);
      item += g;
      if (item >= a.n_items) break;
    }
  }
  if (!a.partial) return;
  // weight (j, i0 + k p): the slots (k, j) of the threads of phase i0, added
  // in ascending thread order
#pragma unroll
  for (int k = 0; k < KM; ++k)
#pragma unroll
    for (int j = 0; j < QM; ++j) {
      if (k >= K || j >= q) continue;
      __syncthreads();
      red[t] = ga[k][j];
      __syncthreads();
      if (t < p && t + k * p < T) {
        float sum = 0.0f;
        for (int l = t; l < kBlock; l += p) sum += red[l];
        a.partial[int64_t(blockIdx.x) * (q * T) + j * T + t + k * p] = sum;
      }
    }
}

}  // namespace

bool poly_supported(const Win3& w, int q) {
  if (w.ax == 2 && (w.p[2] < 1 || w.p[2] > kMaxP)) return false;
  return w.taps >= 1 && w.taps <= kMaxT && q >= 1 && q <= kMaxQ;
}

bool poly_gc_supported(const Win3& w, int q) { return w.taps <= 16 && q <= 4; }

int poly_chunks(const Win3& w) { return (w.rep[2] + kChunk - 1) / kChunk; }

namespace {
// Workgroups of the columns kernel resident on the whole device.
int poly_cols_resident() {
  static const int resident = [] {
    int per_cu = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, poly_cols_kernel<16, 9, 4>, kBlock, 0) != hipSuccess ||
        per_cu < 1) {
      (void)hipGetLastError();   // a failed query must not surface as a launch error
      per_cu = 4;
    }
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
      (void)hipGetLastError();
      cus = 256;
    }
    return per_cu * cus;
  }();
  return resident;
}
}  // namespace

namespace {
template <int KT, int PF>
void launch_cols_q(const PolyArgs& a, int qt, int grid, hipStream_t st) {
  if (qt == 1)
    poly_cols_kernel<KT, PF, 1><<<grid, kBlock, 0, st>>>(a);
  else if (qt == 4)
    poly_cols_kernel<KT, PF, 4><<<grid, kBlock, 0, st>>>(a);
  else
    poly_cols_kernel<KT, PF, 8><<<grid, kBlock, 0, st>>>(a);
}

template <int KT>
void launch_cols_pf(const PolyArgs& a, int pf, int qt, int grid, hipStream_t st) {
  if (pf == 9)
    launch_cols_q<KT, 9>(a, qt, grid, st);
  else
    launch_cols_q<KT, 17>(a, qt, grid, st);
}

void launch_cols(const PolyArgs& a, int kt, int pf, int qt, int grid, hipStream_t st) {
  if (kt == 8)
    launch_cols_pf<8>(a, pf, qt, grid, st);
  else if (kt == 16)
    launch_cols_pf<16>(a, pf, qt, grid, st);
  else
    launch_cols_pf<32>(a, pf, qt, grid, st);
}
}  // namespace

hipError_t launch_poly(const PolyArgs& a, hipStream_t st) {
  const int T = a.w.taps;
  if (a.w.ax == 2) {
    // one resident wave of workgroups, at most one per item
    const int grid = int(std::min<uint32_t>(a.n_items, uint32_t(poly_cols_resident())));
    const bool small_step = a.w.p[2] <= 8;   // segments of at most 2072 floats: 9 per thread
    const int qt = a.q == 1 ? 1 : a.q <= 4 ? 4 : 8;
    launch_cols(a, T <= 8 ? 8 : T <= 16 ? 16 : 32, small_step ? 9 : 17, qt, grid, st);
  } else {
    // four repetitions per thread where the columns allow 16-byte accesses
    // (30 x 1080 x 720 -> 480 rows, 14 taps every 9 rows, 4 outputs: 43.9 ->
    // 31.3 us; two per thread with 8-byte accesses 33.4 us)
    const uintptr_t xy = reinterpret_cast<uintptr_t>(a.x) | reinterpret_cast<uintptr_t>(a.y);
    if (a.w.p[2] == 1 && a.w.o[2] >= 0 && a.w.o[2] + a.w.rep[2] <= a.w.A[2] && T <= 16 && a.w.rep[2] % 4 == 0 &&
        a.w.A[2] % 4 == 0 && a.w.o[2] % 4 == 0 && !(xy & 15)) {
      const uint32_t need = (a.n_items / 4 + kBlock - 1) / kBlock;
      const int grid = int(((need < 256u * 16u ? need : 256u * 16u) + 7) / 8 * 8);   // a multiple of 8
      if (T <= 8 && a.q <= 4)
        poly_rows_vec_kernel<8, 4, 4><<<grid, kBlock, 0, st>>>(a);
      else if (T <= 8)
        poly_rows_vec_kernel<8, 8, 4><<<grid, kBlock, 0, st>>>(a);
      else if (a.q <= 4)
        poly_rows_vec_kernel<16, 4, 4><<<grid, kBlock, 0, st>>>(a);
      else
        poly_rows_vec_kernel<16, 8, 4><<<grid, kBlock, 0, st>>>(a);
      return hipGetLastError();
    }
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

bool poly_cols_vec_ok(const Win3& w, int q, const void* x) {
  if (w.ax != 2 || q < 1 || q > 4 || w.p[2] % 4 || w.A[2] % 4) return false;
  if (((w.o[2] % 4) + 4) % 4 + w.taps > 16) return false;
  if (int64_t(w.rep[0]) * w.rep[1] * w.rep[2] >= (int64_t(1) << 31)) return false;   // item index + stride in 32 bits
  // window starts in 32-bit arithmetic
  if (std::abs(int64_t(w.o[2])) + int64_t(w.p[2]) * w.rep[2] + 16 >= (int64_t(1) << 31)) return false;
  return x == nullptr || (reinterpret_cast<uintptr_t>(x) & 15) == 0;
}

hipError_t launch_poly_cols_vec(const PolyArgs& args, hipStream_t st) {
  PolyArgs a = args;
  a.n_items = uint32_t(int64_t(a.w.rep[0]) * a.w.rep[1] * a.w.rep[2]);
  if (a.n_items == 0) return hipSuccess;
  const uint32_t need = (a.n_items + kBlock - 1) / kBlock;
  const int grid = int(need < 256u * 32u ? need : 256u * 32u);
  switch (a.q) {
    case 1: poly_cols_vec_kernel<1><<<grid, kBlock, 0, st>>>(a); break;
    case 2: poly_cols_vec_kernel<2><<<grid, kBlock, 0, st>>>(a); break;
    case 3: poly_cols_vec_kernel<3><<<grid, kBlock, 0, st>>>(a); break;
    default: poly_cols_vec_kernel<4><<<grid, kBlock, 0, st>>>(a); break;
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

bool poly_adj_cols_supported(const Win3& w, int q) {
  return w.ax == 2 && w.p[2] >= 1 && w.p[2] <= kMaxP && w.taps <= kMaxT && q * w.taps <= kBlock && w.A[2] < (1 << 28) &&
         int64_t(w.p[2]) * (w.rep[2] - 1) + w.taps < (int64_t(1) << 30);
}

bool poly_adj_phase_ok(const Win3& w, int q) {
  const int p = w.p[2];
  return (p & (p - 1)) == 0 && (kBlock % p) == 0 && (w.A[2] % p) == 0 && (w.taps + p - 1) / p <= 4 && q <= 4;
}

namespace {
using PolyAdjKernel = void (*)(PolyAdjArgs);

// The columns adjoint for this stage: the phase form (GF = 5 registers hold
// q (256 + K - 1) <= 4 x 259 staged values; XF = p) or the general one.
PolyAdjKernel poly_adj_kernel_for(const Win3& w, int q) {
  if (!poly_adj_phase_ok(w, q)) return poly_adj_cols_kernel;
  const int K = (w.taps + w.p[2] - 1) / w.p[2];
  if (w.p[2] <= 8) return K <= 2 ? poly_adj_phase_kernel<2, 4, 8, 5> : poly_adj_phase_kernel<4, 4, 8, 5>;
  return K <= 2 ? poly_adj_phase_kernel<2, 4, 16, 5> : poly_adj_phase_kernel<4, 4, 16, 5>;
}

// Workgroups of a kernel resident on the whole device, from its own
// occupancy (cached per kernel).
int poly_adj_resident(PolyAdjKernel k) {
  static std::mutex mu;
  static std::vector<std::pair<PolyAdjKernel, int>> known;
  std::lock_guard<std::mutex> lock(mu);
  for (const auto& e : known)
    if (e.first == k) return e.second;
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k, kBlock, 0) != hipSuccess || per_cu < 1) {
    (void)hipGetLastError();   // a failed query must not surface as a launch error
    per_cu = 4;
  }
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1) {
    (void)hipGetLastError();
    cus = 256;
  }
  known.emplace_back(k, per_cu * cus);
  return per_cu * cus;
}
}  // namespace

int poly_adj_cols_grid(const Win3& w, int q, uint32_t n_items) {
  const uint32_t res = uint32_t(poly_adj_resident(poly_adj_kernel_for(w, q)));
  return int(n_items < res ? (n_items ? n_items : 1) : res);
}

hipError_t launch_poly_adj_cols(const PolyAdjArgs& a, hipStream_t st) {
  const int grid = poly_adj_cols_grid(a.w, a.q, a.n_items);
  hipLaunchKernelGGL(poly_adj_kernel_for(a.w, a.q), dim3(grid), dim3(kBlock), 0, st, a);
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
