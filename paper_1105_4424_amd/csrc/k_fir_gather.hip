// k_fir_gather.hip -- input gradient of a 1-D tap tiler whose windows
// overlap (pattern longer than the paving step) or wrap onto each other,
// written as a gather: one thread per input element.
//
// The transposed tiler sends c_i gy[r] to element (o + p r + i) mod A along
// the tap axis (the tiler's index function, origin o, paving p, fitting 1).
// For an element a the pairs (r, i) that reach it are found by lifting a to
// the unwrapped positions u = a + m A that lie in [o, o + p (R - 1) + T - 1]
// (several lifts when the windows cover the axis more than once); for each
// lift, v = u - o = p r + i with 0 <= i < T, so r runs down from
// min(R - 1, floor(v / p)) while i = v - p r stays below T.  Every pair is
// visited exactly once, in a fixed order (lifts ascending, taps ascending),
// so the result is deterministic without atomics; elements that no window
// reads get zero.  The two outer axes do not wrap (their windows are single
// points): an element is read only if (a_d - o_d) is a non-negative multiple
// of p_d below p_d rep_d.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <utility>
#include <vector>

#include "rsm_internal.h"

namespace rsm {
namespace {

constexpr int kBlock = 256;
constexpr int kMaxTapsGather = 16;   // taps of a 1-D window on the tap paths

__device__ __forceinline__ int wrap_mod(int v, int n) {
  const int q = v % n;
  return q < 0 ? q + n : q;
}

// Repetition index along a non-tap axis for array index a_d, or -1 if no
// repetition reads it.
__device__ __forceinline__ int outer_rep(int a_d, int o, int p, int rep, const FastDiv& dp) {
  const int v = a_d - o;
  if (v < 0) return -1;
  if (rep == 1) return v == 0 ? 0 : -1;
  const int q = int(fdiv(uint32_t(v), dp));
  return (q * p == v && q < rep) ? q : -1;
}

// KM >= ceil(T / p): the taps of one lift that can meet an element.  Its
// pairs r = r0 - k, i = i0 + k p (k < KM) are tested and their dL/dy loads
// issued together, then added in the order of ascending tap (the order of
// a walk down from r0); the weights are read from LDS.
template <int AX, int KM>
__global__ void __launch_bounds__(kBlock) fir_gx_gather_kernel(FirGatherArgs a) {
  const Win3& w = a.w;
  const int n_ax = w.A[AX], R = w.rep[AX], p = w.p[AX], T = w.taps;
  const int span = p * (R - 1) + T;   // unwrapped positions covered, v in [0, span)
  __shared__ float cs[kMaxTapsGather];
  if (threadIdx.x < kMaxTapsGather) cs[threadIdx.x] = int(threadIdx.x) < T ? a.c[threadIdx.x] : 0.0f;
  __syncthreads();
  const uint32_t stride = gridDim.x * kBlock;
  for (uint32_t e = blockIdx.x * kBlock + threadIdx.x; e < a.n_arr; e += stride) {
    const uint32_t row = fdiv(e, a.div_a2);
    const int ac = int(e - row * uint32_t(w.A[2]));
    const uint32_t b = fdiv(row, a.div_a1);
    const int ar = int(row - b * uint32_t(w.A[1]));
    const int ab = int(b);
    const int rb = outer_rep(ab, w.o[0], w.p[0], w.rep[0], a.div_p[0]);
    int ro, at;   // the other outer axis' repetition; the tap-axis index
    if (AX == 2) {
      ro = outer_rep(ar, w.o[1], w.p[1], w.rep[1], a.div_p[1]);
      at = ac;
    } else {
      ro = outer_rep(ac, w.o[2], w.p[2], w.rep[2], a.div_p[2]);
      at = ar;
    }
    float acc = 0.0f;
    if (rb >= 0 && ro >= 0) {
      // gy offset of repetition r along the tap axis: g0 + r * gs
      const int g0 = AX == 2 ? (rb * w.rep[1] + ro) * w.rep[2] : rb * w.rep[1] * w.rep[2] + ro;
      const int gs = AX == 2 ? 1 : w.rep[2];
      int v = at - a.o_mod;   // first lift: v = (a - o) mod A
      if (v < 0) v += n_ax;
      for (; v < span; v += n_ax) {
        const int r0 = int(fdiv(uint32_t(v), a.div_p[AX]));
        const int i0 = v - p * r0;   // in [0, p)
        float g[KM];
        bool ok[KM];
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          const int r = r0 - k, i = i0 + k * p;
          ok[k] = r >= 0 && r <= R - 1 && i < T;
          g[k] = ok[k] ? a.gy[g0 + r * gs] : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          const int i = i0 + k * p;
          if (ok[k]) acc = fmaf(cs[i < kMaxTapsGather ? i : 0], g[k], acc);
        }
      }
    }
    a.gx[e] = a.accumulate ? a.gx[e] + acc : acc;
  }
}

// Taps along rows with the column axis taken whole (p[2] = 1, o[2] = 0,
// rep[2] = A[2], A[2] a multiple of 4, dL/dy and dL/dx 16-byte aligned):
// one thread per four adjacent columns of a row, which meet the same
// windows, so the index work is done once and dL/dy and dL/dx move as
// 16-byte vectors.  Each column adds its pairs in the order of the
// one-column kernel above.
template <int KM>
__global__ void __launch_bounds__(kBlock) fir_gx_gather_rows_vec_kernel(FirGatherArgs a) {
  const Win3& w = a.w;
  const int n_ax = w.A[1], R = w.rep[1], p = w.p[1], T = w.taps;
  const int span = p * (R - 1) + T;   // unwrapped positions covered, v in [0, span)
  __shared__ float cs[kMaxTapsGather];
  if (threadIdx.x < kMaxTapsGather) cs[threadIdx.x] = int(threadIdx.x) < T ? a.c[threadIdx.x] : 0.0f;
  __syncthreads();
  const uint32_t n4 = a.n_arr / 4;
  const uint32_t stride = gridDim.x * kBlock;
  for (uint32_t q4 = blockIdx.x * kBlock + threadIdx.x; q4 < n4; q4 += stride) {
    const uint32_t e = 4 * q4;
    const uint32_t row = fdiv(e, a.div_a2);
    const int ac = int(e - row * uint32_t(w.A[2]));
    const uint32_t b = fdiv(row, a.div_a1);
    const int ar = int(row - b * uint32_t(w.A[1]));
    const int rb = outer_rep(int(b), w.o[0], w.p[0], w.rep[0], a.div_p[0]);
    float acc[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (rb >= 0) {
      const int64_t g0 = int64_t(rb) * w.rep[1] * w.rep[2] + ac;
      const int gs = w.rep[2];
      int v = ar - a.o_mod;   // first lift: v = (a - o) mod A
      if (v < 0) v += n_ax;
      for (; v < span; v += n_ax) {
        const int r0 = int(fdiv(uint32_t(v), a.div_p[1]));
        const int i0 = v - p * r0;   // in [0, p)
        float4 g[KM];
        bool ok[KM];
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          const int r = r0 - k, i = i0 + k * p;
          ok[k] = r >= 0 && r <= R - 1 && i < T;
          g[k] = ok[k] ? *reinterpret_cast<const float4*>(a.gy + g0 + int64_t(r) * gs)
                       : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          if (!ok[k]) continue;
          const int i = i0 + k * p;
          const float c = cs[i < kMaxTapsGather ? i : 0];
          acc[0] = fmaf(c, g[k].x, acc[0]);
          acc[1] = fmaf(c, g[k].y, acc[1]);
          acc[2] = fmaf(c, g[k].z, acc[2]);
          acc[3] = fmaf(c, g[k].w, acc[3]);
        }
      }
    }
    float4* dst = reinterpret_cast<float4*>(a.gx + e);
    float4 out = make_float4(acc[0], acc[1], acc[2], acc[3]);
    if (a.accumulate) {
      const float4 old = *dst;
      out.x += old.x; out.y += old.y; out.z += old.z; out.w += old.w;
    }
    *dst = out;
  }
}

// ---------------------------------------------------------------------------
// Taps along columns with steps of at most 16: input gradient and weight
// gradient in one pass.  Work items are (array row, chunk of kRC repetitions
// along the row).  For each item a workgroup stages the chunk's gy values
// (with the K - 1 before it) in LDS; then each lane walks the positions v it
// owns, v = (a - o) mod A (the first lift of column a) in [chunk p kRC,
// (chunk + 1) p kRC), in steps of p (kBlock / p), so that its phase
// j = v mod p never changes.  At each position the pairs of the first lift
// are r = floor(v / p) - k, i = j + k p (k < K): the lane adds c_i gy[r]
// into dL/dx and x[a] gy[r] into its weight-gradient slot k, whose tap
// j + k p is fixed for the lane.  Pairs of further lifts (windows that go
// round the row more than once) take a per-lane loop: lane (li, lr) keeps
// tap li for the repetitions of the chunk whose pair lies past A.  x is read
// once, coalesced, and dL/dx written once; the partials of a tap are summed
// over fixed lanes in a fixed order, so nothing is atomic and every bit is
// reproducible.  The next item's gy values are loaded while the current
// item is computed.
// ---------------------------------------------------------------------------
constexpr int kRC = 256;        // repetitions per chunk
constexpr int kMaxTaps = 16;
constexpr uint32_t kBufferWord3 = 0x00020000;   // 32-bit data format, raw access
constexpr uint32_t kOutOfRange = 0x80000000u;   // a read here returns zero
constexpr int kPos = 16;        // positions per lane per item: ceil(256 p / (p floor(256 / p))) <= 16

// Work item -> array row, chunk, and the row's repetition offset in gy (-1 if
// no repetition reads the row).
__device__ __forceinline__ void overlap_item(const FirOverlapArgs& a, uint32_t item, int& row, int& chunk,
                                             int& g0) {
  const Win3& w = a.w;
  const uint32_t r = fdiv(item, a.div_chunks);
  row = int(r);
  chunk = int(item - r * uint32_t(a.n_chunks));
  const uint32_t b = fdiv(r, a.div_a1);
  const int ar = int(r - b * uint32_t(w.A[1]));
  const int rb = outer_rep(int(b), w.o[0], w.p[0], w.rep[0], a.div_p0);
  const int ro = outer_rep(ar, w.o[1], w.p[1], w.rep[1], a.div_p1);
  g0 = (rb >= 0 && ro >= 0) ? (rb * w.rep[1] + ro) * w.rep[2] : -1;
}

// This thread's staged gy values of an item (j = tid and tid + kBlock of
// repetition rs + j), loaded unconditionally: a repetition outside [0, R),
// or any repetition of a row nothing reads, reads zero.
__device__ __forceinline__ void overlap_fetch_gy(const FirOverlapArgs& a, int chunk, int g0, int K, float& g0v,
                                                 float& g1v) {
  const int R = a.w.rep[2];
  const bool read = g0 >= 0;
  const __amdgpu_buffer_rsrc_t rg = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(a.gy) + (read ? g0 : 0), short(0), read ? R * 4 : 0, int(kBufferWord3));
  const int rs = chunk * kRC - (K - 1);
  const int j0 = int(threadIdx.x), j1 = j0 + kBlock;
  const int q0 = rs + j0, q1 = rs + j1;
  const uint32_t o0 = (j0 < kRC + K - 1 && q0 >= 0 && q0 < R) ? uint32_t(q0) * 4u : kOutOfRange;
  const uint32_t o1 = (j1 < kRC + K - 1 && q1 >= 0 && q1 < R) ? uint32_t(q1) * 4u : kOutOfRange;
  g0v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rg, o0, 0, 0));
  g1v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rg, o1, 0, 0));
}

// KS: taps per lift K as a compile-time constant (1..4), or 0 for any K.
// GC: the weight gradient is wanted (a.partial set).
// KP: positions per lane per item, 8 when the step p is at most 8 (else 16):
// a form sized for 16 keeps 16 x values and 16 guarded loads per item where
// 8 are used (13 taps every 8 columns on 30 x 1080 x 1920: 128 -> 113 us,
// with the first-lift taps of a fixed tap count held in registers).
template <bool ACC, int KS, bool GC, int KP>
// at most 80 registers: six waves per SIMD instead of five (127-132 us
// against 132-136 us for the same workload, when every form held 16)
__global__ void __launch_bounds__(kBlock, 6) fir_adjoint_overlap_cols_kernel(FirOverlapArgs a) {
  const Win3& w = a.w;
  const int A2 = w.A[2], R = w.rep[2], p = w.p[2], T = w.taps;
  const int K = KS ? KS : (T + p - 1) / p;   // taps of one lift that can meet an element
  constexpr int KM = KS ? KS : kMaxTaps;
  const int span = p * (R - 1) + T;
  const int W = p * kRC;                     // positions owned by one chunk
  const int qstep = kBlock / p;              // repetitions per position step
  const int step = p * qstep;                // positions per step: a multiple of p
  // coefficients padded with zeros to 2 kMaxTaps: j + k p < K p <= T + p - 1
  // is always a valid index, so the tap loop needs no bound test
  __shared__ float cs[2 * kMaxTaps];
  __shared__ float gys[kRC + kMaxTaps];
  __shared__ float red[kBlock];
  const int t = int(threadIdx.x);
  if (t < 2 * kMaxTaps) cs[t] = t < T ? a.c[t] : 0.0f;
  const int jph = t % p;                     // this lane's position phase
  __syncthreads();
  // every position of this lane has phase jph: its first-lift taps are
  // jph + k p, the same for all of them, so a fixed tap count keeps them in
  // registers (the form for any tap count reads them from LDS)
  float cl[KS ? KS : 1];
#pragma unroll
  for (int k = 0; k < (KS ? KS : 1); ++k) cl[k] = cs[jph + k * p];
  const int per = kBlock / T;                // further-lift pairs: repetitions per pass
  const int li = t % T, lr = t / T;
  float gcl[KM];                             // first-lift slots: tap jph + k p
#pragma unroll
  for (int k = 0; k < KM; ++k) gcl[k] = 0.0f;
  float gext = 0.0f;                         // further-lift pairs: tap li

  uint32_t item = blockIdx.x;
  int row, chunk, g0;
  overlap_item(a, item, row, chunk, g0);
  float gv0, gv1;
  overlap_fetch_gy(a, chunk, g0, K, gv0, gv1);
  for (; item < a.n_items; item += gridDim.x) {
    const bool read = g0 >= 0;
    const int r0 = chunk * kRC, rs = r0 - (K - 1);
    // this item's x values at the lane's positions, all loads issued before
    // any is used (positions past the chunk, or rows nothing reads, read zero)
    float xr[KP];
    // a wave issuing an item's loads outranks the computing waves of the
    // other workgroups on its CU (125 against 132-138 us)
    __builtin_amdgcn_s_setprio(2);
    if (GC) {
      const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
          const_cast<float*>(a.x) + int64_t(row) * A2, short(0), read ? A2 * 4 : 0, int(kBufferWord3));
      const int v_end = min((chunk + 1) * W, A2);
#pragma unroll
      for (int m = 0; m < KP; ++m) {
        const int v = chunk * W + t + m * step;
        int e = a.o_mod + v;
        if (e >= A2) e -= A2;
        const uint32_t off = (t < step && v < v_end) ? uint32_t(e) * 4u : kOutOfRange;
        xr[m] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx, off, 0, 0));
      }
    }
    __builtin_amdgcn_s_setprio(0);
    __syncthreads();               // the previous item's readers of gys are done
    if (t < kRC + K - 1) gys[t] = gv0;
    if (t + kBlock < kRC + K - 1) gys[t + kBlock] = gv1;
    __syncthreads();
    const int cur_row = row, cur_chunk = chunk, cur_g0 = g0;
    const uint32_t nxt = item + gridDim.x;
    g0 = -1;
    if (nxt < a.n_items) overlap_item(a, nxt, row, chunk, g0);
    overlap_fetch_gy(a, chunk, g0, K, gv0, gv1);   // the next item's gy travels meanwhile

    const float* __restrict__ xrow = GC ? a.x + int64_t(cur_row) * A2 : nullptr;
    float* gxrow = a.gx ? a.gx + int64_t(cur_row) * A2 : nullptr;
    const int v_end = min((cur_chunk + 1) * W, A2);
    const int v0 = cur_chunk * W + t;
    const int q0 = int(fdiv(uint32_t(v0), a.div_p));
#pragma unroll
    for (int m = 0; m < KP; ++m) {
      const int v = v0 + m * step;
      if (!(t < step && v < v_end && (gxrow || (GC && read)))) continue;
      const int q = q0 + m * qstep;
      {
        int e = a.o_mod + v;
        if (e >= A2) e -= A2;
        const float xv = GC ? xr[m] : 0.0f;
        float acc = 0.0f;
        // r = q - k: q - k - rs lies in [0, kRC + K - 1) for every owned v,
        // and the staged gy is zero for r outside [0, R)
#pragma unroll
        for (int k = 0; k < KM; ++k) {
          if (!KS && k >= K) break;
          const float g = gys[q - k - rs];
          acc = fmaf(KS ? cl[KS ? k : 0] : cs[jph + k * p], g, acc);
          if (GC) gcl[k] = fmaf(xv, g, gcl[k]);
        }
        if (gxrow) {
          if (read) {
            // further lifts: with one chunk per row every repetition is
            // staged in LDS, otherwise gy is read from memory
            if (a.n_chunks == 1) {
              for (int u = v + A2; u < span; u += A2) {
                int r = int(fdiv(uint32_t(u), a.div_p));
                if (r > R - 1) r = R - 1;
                for (int i = u - p * r; r >= 0 && i < T; --r, i += p) acc = fmaf(cs[i], gys[r - rs], acc);
              }
            } else {
              for (int u = v + A2; u < span; u += A2) {
                int r = int(fdiv(uint32_t(u), a.div_p));
                if (r > R - 1) r = R - 1;
                for (int i = u - p * r; r >= 0 && i < T; --r, i += p)
                  acc = fmaf(cs[i], a.gy[cur_g0 + r], acc);
              }
            }
          }
          if (ACC) acc += gxrow[e];
          gxrow[e] = acc;
        }
      }
    }
    if (GC && read && lr < per && span > A2) {
      // weight-gradient pairs past the row's end (u = p r + li >= A2) of
      // this chunk's repetitions: r >= ceil((A2 - li) / p)
      const int r_end = min(r0 + kRC, R);
      const int r_lo = (A2 - li + p - 1) / p;
      int r = r0 + lr;
      if (r < r_lo) r += ((r_lo - r + per - 1) / per) * per;
      for (; r < r_end; r += per) {
        const int e = (a.o_mod + p * r + li) % A2;
        gext = fmaf(gys[r - rs], xrow[e], gext);
      }
    }
  }
  if (GC) {
    // tap i = j + k p: slot k of the lanes of phase j, then the further-lift
    // sums of the lanes keeping tap i; each in ascending lane order
    float s = 0.0f;
    for (int k = 0; k < K; ++k) {
      __syncthreads();
      red[t] = t < step ? gcl[k] : 0.0f;
      __syncthreads();
      if (t < T && t / p == k)
        for (int l = t % p; l < step; l += p) s += red[l];
    }
    __syncthreads();
    red[t] = lr < per ? gext : 0.0f;
    __syncthreads();
    if (t < T) {
      for (int l = t; l < per * T; l += T) s += red[l];
      a.partial[int64_t(blockIdx.x) * T + t] = s;
    }
  }
}

}  // namespace

namespace {
typedef void (*OverlapKernel)(FirOverlapArgs);

template <bool GC, int KP>
OverlapKernel overlap_kernel_kp(int K, bool acc) {
  if (acc) return fir_adjoint_overlap_cols_kernel<true, 0, GC, KP>;
  switch (K) {
    case 1: return fir_adjoint_overlap_cols_kernel<false, 1, GC, KP>;
    case 2: return fir_adjoint_overlap_cols_kernel<false, 2, GC, KP>;
    case 3: return fir_adjoint_overlap_cols_kernel<false, 3, GC, KP>;
    case 4: return fir_adjoint_overlap_cols_kernel<false, 4, GC, KP>;
    default: return fir_adjoint_overlap_cols_kernel<false, 0, GC, KP>;
  }
}

// The kernel form for step p (positions per lane ceil(256 / floor(256 / p)):
// at most 8 for p <= 8), K taps per lift, accumulation, weight gradient.
OverlapKernel overlap_kernel(int p, int K, bool acc, bool gc) {
  if (p <= 8) return gc ? overlap_kernel_kp<true, 8>(K, acc) : overlap_kernel_kp<false, 8>(K, acc);
  return gc ? overlap_kernel_kp<true, kPos>(K, acc) : overlap_kernel_kp<false, kPos>(K, acc);
}

// Resident workgroups of a kernel form on the device (cached per form).
int overlap_resident(OverlapKernel k) {
  static std::mutex mu;
  static std::vector<std::pair<OverlapKernel, int>> known;
  std::lock_guard<std::mutex> lock(mu);
  for (const auto& e : known)
    if (e.first == k) return e.second;
  int per_cu = 0, dev = 0, cus = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(k), kBlock, 0) !=
          hipSuccess ||
      per_cu < 1) {
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

// One resident wave of workgroups of the form for any tap count (the one
// holding the most registers), at most one per item, whatever form runs:
// for 13 taps every 8 columns on 30 x 1080 x 1920 that is 6 workgroups per
// CU, and measured with 3 .. 8 per CU: 140, 119, 115, 114, 142, 131 us.  The
// weight-gradient workspace holds one partial row per workgroup, so the
// planner sizes it with this same function.
int fir_overlap_cols_grid(uint32_t n_items, int p) {
  const int resident = overlap_resident(overlap_kernel(p, 0, false, true));
  return int(n_items < uint32_t(resident) ? (n_items ? n_items : 1) : uint32_t(resident));
}

hipError_t launch_fir_adjoint_overlap_cols(const FirOverlapArgs& a, hipStream_t st) {
  const int p = a.w.p[2], K = (a.w.taps + p - 1) / p;
  const bool gc = a.partial != nullptr;
  const int grid = fir_overlap_cols_grid(a.n_items, p);
  hipLaunchKernelGGL(overlap_kernel(p, K, a.accumulate != 0, gc), dim3(grid), dim3(kBlock), 0, st, a);
  return hipGetLastError();
}

hipError_t launch_fir_gx_gather(const FirGatherArgs& a, hipStream_t st) {
  const uint32_t need = (a.n_arr + kBlock - 1) / kBlock;
  const int grid = int(need < 256u * 16u ? (need ? need : 1) : 256u * 16u);
  const int p = a.w.p[a.w.ax];
  const int K = p >= 1 ? (a.w.taps + p - 1) / p : a.w.taps;   // taps of one lift
  const uintptr_t al = reinterpret_cast<uintptr_t>(a.gy) | reinterpret_cast<uintptr_t>(a.gx);
  if (a.w.ax == 1 && a.w.p[2] == 1 && a.w.o[2] == 0 && a.w.rep[2] == a.w.A[2] && a.w.A[2] % 4 == 0 &&
      (al & 15) == 0 && K <= 4) {
    const uint32_t need4 = (a.n_arr / 4 + kBlock - 1) / kBlock;
    const int grid4 = int(need4 < 256u * 16u ? (need4 ? need4 : 1) : 256u * 16u);
    if (K <= 2)
      fir_gx_gather_rows_vec_kernel<2><<<grid4, kBlock, 0, st>>>(a);
    else
      fir_gx_gather_rows_vec_kernel<4><<<grid4, kBlock, 0, st>>>(a);
    return hipGetLastError();
  }
  if (a.w.ax == 2) {
    if (K <= 2) fir_gx_gather_kernel<2, 2><<<grid, kBlock, 0, st>>>(a);
    else if (K <= 4) fir_gx_gather_kernel<2, 4><<<grid, kBlock, 0, st>>>(a);
    else fir_gx_gather_kernel<2, kMaxTapsGather><<<grid, kBlock, 0, st>>>(a);
  } else {
    if (K <= 2) fir_gx_gather_kernel<1, 2><<<grid, kBlock, 0, st>>>(a);
    else if (K <= 4) fir_gx_gather_kernel<1, 4><<<grid, kBlock, 0, st>>>(a);
    else fir_gx_gather_kernel<1, kMaxTapsGather><<<grid, kBlock, 0, st>>>(a);
  }
  return hipGetLastError();
}

}  // namespace rsm
