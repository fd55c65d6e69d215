// k_generic.hip -- kernels that handle any affine tiler (int64 index arithmetic).
//
//  * index_table:   e(r, i) for every (r, i), evaluated directly per element
//  * generic_*:     gather -> task -> scatter for one repetition per thread,
//                   walking the pattern incrementally (add a fitting column,
//                   one conditional subtract; on a carry, rewind the column)
//  * generic adjoint: transposed gather as an atomic scatter-add, and the
//                   weight gradient as a two-pass fixed-order reduction
//
// These are the correctness floor for tilers the specialised kernels do not
// cover.  Storage of the tiler descriptor keeps origin / paving / fitting
// reduced into [0, s_d), so the walk never sees a negative coordinate.
#include <hip/hip_runtime.h>

#include "rsm_internal.h"

namespace rsm {
namespace {

constexpr int kBlock = 256;

// Loops over rank-bounded arrays unroll fully for ranks <= 4 (registers);
// the rank-8 variants keep rolled loops to bound code size and compile time.
#define RSM_UNROLL_R _Pragma("unroll (R <= 4 ? R : 1)")

__device__ __forceinline__ float bf16_to_f32(uint16_t b) {
  return __uint_as_float(uint32_t(b) << 16);
}

template <typename T, typename Acc>
__device__ __forceinline__ Acc load_as(const void* p, int64_t i);
template <>
__device__ __forceinline__ float load_as<float, float>(const void* p, int64_t i) {
  return static_cast<const float*>(p)[i];
}
template <>
__device__ __forceinline__ float load_as<uint16_t, float>(const void* p, int64_t i) {
  return bf16_to_f32(static_cast<const uint16_t*>(p)[i]);
}
template <>
__device__ __forceinline__ double load_as<double, double>(const void* p, int64_t i) {
  return static_cast<const double*>(p)[i];
}

template <int R>
__device__ __forceinline__ void unflatten(int64_t f, int rank, const int64_t* shape, int64_t* idx) {
RSM_UNROLL_R
  for (int k = R - 1; k >= 0; --k) {
    if (k < rank) {
      idx[k] = f % shape[k];
      f /= shape[k];
    } else {
      idx[k] = 0;
    }
  }
}

// Coordinates of the reference element e(r, 0) = (o + P r) mod s.
template <int R>
__device__ __forceinline__ void start_coords(const GTiler& t, int rep_rank, const int64_t* r,
                                             int64_t* cur) {
RSM_UNROLL_R
  for (int d = 0; d < R; ++d) {
    cur[d] = 0;
    if (d < t.arr_rank) {
      const int64_t s = t.shape[d];
      int64_t v = t.origin[d];
RSM_UNROLL_R
      for (int k = 0; k < R; ++k) {
        if (k < rep_rank) {
          v += (t.pav[d][k] * r[k]) % s;
          if (v >= s) v -= s;
        }
      }
      cur[d] = v;
    }
  }
}

template <int R>
__device__ __forceinline__ int64_t linear(const GTiler& t, const int64_t* cur) {
  int64_t lin = 0;
RSM_UNROLL_R
  for (int d = 0; d < R; ++d)
    if (d < t.arr_rank) lin = lin * t.shape[d] + cur[d];
  return lin;
}

// Advance the row-major pattern index by one and update the coordinates.
template <int R>
__device__ __forceinline__ void step_pattern(const GTiler& t, int64_t* pidx, int64_t* cur) {
RSM_UNROLL_R
  for (int kk = R - 1; kk >= 0; --kk) {
    if (kk >= t.pat_rank) continue;
    pidx[kk] += 1;
    if (pidx[kk] < t.pat_shape[kk]) {
RSM_UNROLL_R
      for (int d = 0; d < R; ++d) {
        if (d < t.arr_rank) {
          cur[d] += t.fit[d][kk];
          if (cur[d] >= t.shape[d]) cur[d] -= t.shape[d];
        }
      }
      return;
    }
    // carry: pattern index kk wraps to 0, undo its (pat_shape - 1) steps
    pidx[kk] = 0;
RSM_UNROLL_R
    for (int d = 0; d < R; ++d) {
      if (d < t.arr_rank) {
        const int64_t back = (t.fit[d][kk] * (t.pat_shape[kk] - 1)) % t.shape[d];
        cur[d] -= back;
        if (cur[d] < 0) cur[d] += t.shape[d];
      }
    }
  }
}

// ---------------------------------------------------------------------------
// index table: one thread per (r, i); direct evaluation with floored modulo
// ---------------------------------------------------------------------------
struct IndexArgs {
  GTiler t;
  int32_t rep_rank;
  int64_t rep_shape[kMaxRank];
  int64_t n_rep, n_pat;
  int64_t* out;
};

__global__ void __launch_bounds__(kBlock) index_table_kernel(IndexArgs a) {
  const int64_t total = a.n_rep * a.n_pat;
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t g = int64_t(blockIdx.x) * kBlock + threadIdx.x; g < total; g += stride) {
    const int64_t rf = g / a.n_pat;
    const int64_t pf = g - rf * a.n_pat;
    int64_t r[kMaxRank], i[kMaxRank];
    unflatten<kMaxRank>(rf, a.rep_rank, a.rep_shape, r);
    unflatten<kMaxRank>(pf, a.t.pat_rank, a.t.pat_shape, i);
    int64_t lin = 0;
    for (int d = 0; d < a.t.arr_rank; ++d) {
      const int64_t s = a.t.shape[d];
      int64_t v = a.t.origin[d];
      for (int k = 0; k < a.rep_rank; ++k) v = (v + (a.t.pav[d][k] * r[k]) % s) % s;
      for (int k = 0; k < a.t.pat_rank; ++k) v = (v + (a.t.fit[d][k] * i[k]) % s) % s;
      lin = lin * s + v;
    }
    a.out[g] = lin;
  }
}

int grid_for(int64_t work, int per_block = kBlock, int cap = 65536) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return int(g);
}

// ---------------------------------------------------------------------------
// generic gather -> task -> scatter, one repetition per thread
// ---------------------------------------------------------------------------
template <int R, typename Tin, typename Acc, typename Tout, int KIND, int NIN>
__global__ void __launch_bounds__(kBlock) generic_reduce_kernel(GenericArgs a) {
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t rf = int64_t(blockIdx.x) * kBlock + threadIdx.x; rf < a.n_rep; rf += stride) {
    int64_t r[R], c0[R], c1[R], p0[R], p1[R];
    unflatten<R>(rf, a.rep_rank, a.rep_shape, r);
    start_coords<R>(a.in[0], a.rep_rank, r, c0);
    if (NIN == 2) start_coords<R>(a.in[1], a.rep_rank, r, c1);
RSM_UNROLL_R
    for (int k = 0; k < R; ++k) { p0[k] = 0; p1[k] = 0; }
    Acc acc[4] = {Acc(0), Acc(0), Acc(0), Acc(0)};
    for (int64_t p = 0; p < a.n_pat; ++p) {
      Acc v = load_as<Tin, Acc>(a.x[0], linear<R>(a.in[0], c0));
      if (KIND == kWsum) v *= static_cast<const Acc*>(a.coeffs)[p];
      if (KIND == kDot) v *= load_as<Tin, Acc>(a.x[1], linear<R>(a.in[1], c1));
      acc[p & 3] += v;
      if (p + 1 < a.n_pat) {
        step_pattern<R>(a.in[0], p0, c0);
        if (NIN == 2) step_pattern<R>(a.in[1], p1, c1);
      }
    }
    int64_t co[R];
    start_coords<R>(a.out, a.rep_rank, r, co);
    static_cast<Tout*>(a.y)[linear<R>(a.out, co)] = Tout((acc[0] + acc[1]) + (acc[2] + acc[3]));
  }
}

// Weighted sum with an output pattern of n_q elements: output element j of
// repetition r is sum_p c[j n_pat + p] x[e_in(r, p)], written to e_out(r, j).
template <int R, typename Tin, typename Acc, typename Tout>
__global__ void __launch_bounds__(kBlock) generic_wsum_multi_kernel(GenericArgs a) {
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  const Acc* __restrict__ c = static_cast<const Acc*>(a.coeffs);
  for (int64_t rf = int64_t(blockIdx.x) * kBlock + threadIdx.x; rf < a.n_rep; rf += stride) {
    int64_t r[R], c0[R], p0[R], co[R], po[R];
    unflatten<R>(rf, a.rep_rank, a.rep_shape, r);
    start_coords<R>(a.out, a.rep_rank, r, co);
RSM_UNROLL_R
    for (int k = 0; k < R; ++k) po[k] = 0;
    for (int64_t j = 0; j < a.n_q; ++j) {
      start_coords<R>(a.in[0], a.rep_rank, r, c0);
RSM_UNROLL_R
      for (int k = 0; k < R; ++k) p0[k] = 0;
      Acc acc[4] = {Acc(0), Acc(0), Acc(0), Acc(0)};
      for (int64_t p = 0; p < a.n_pat; ++p) {
        acc[p & 3] += load_as<Tin, Acc>(a.x[0], linear<R>(a.in[0], c0)) * c[j * a.n_pat + p];
        if (p + 1 < a.n_pat) step_pattern<R>(a.in[0], p0, c0);
      }
      static_cast<Tout*>(a.y)[linear<R>(a.out, co)] = Tout((acc[0] + acc[1]) + (acc[2] + acc[3]));
      if (j + 1 < a.n_q) step_pattern<R>(a.out, po, co);
    }
  }
}

template <int R, typename E>
__global__ void __launch_bounds__(kBlock) generic_copy_kernel(GenericArgs a) {
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t rf = int64_t(blockIdx.x) * kBlock + threadIdx.x; rf < a.n_rep; rf += stride) {
    int64_t r[R], ci[R], co[R], pi[R], po[R];
    unflatten<R>(rf, a.rep_rank, a.rep_shape, r);
    start_coords<R>(a.in[0], a.rep_rank, r, ci);
    start_coords<R>(a.out, a.rep_rank, r, co);
RSM_UNROLL_R
    for (int k = 0; k < R; ++k) { pi[k] = 0; po[k] = 0; }
    for (int64_t p = 0; p < a.n_pat; ++p) {
      static_cast<E*>(a.y)[linear<R>(a.out, co)] =
          static_cast<const E*>(a.x[0])[linear<R>(a.in[0], ci)];
      if (p + 1 < a.n_pat) {
        step_pattern<R>(a.in[0], pi, ci);
        step_pattern<R>(a.out, po, co);
      }
    }
  }
}

template <int R>
hipError_t dispatch_generic(const GenericArgs& a, int in_dtype, int kind, int elem_bytes,
                            hipStream_t st) {
  const int grid = grid_for(a.n_rep);
  if (kind == kCopy) {
    switch (elem_bytes) {
      case 2: generic_copy_kernel<R, uint16_t><<<grid, kBlock, 0, st>>>(a); break;
      case 4: generic_copy_kernel<R, uint32_t><<<grid, kBlock, 0, st>>>(a); break;
      case 8: generic_copy_kernel<R, uint64_t><<<grid, kBlock, 0, st>>>(a); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
#define RSM_GEN(TIN, ACC, TOUT)                                                              \
  do {                                                                                       \
    if (kind == kWsum && a.n_q > 1)                                                          \
      generic_wsum_multi_kernel<R, TIN, ACC, TOUT><<<grid, kBlock, 0, st>>>(a);               \
    else if (kind == kSum)                                                                   \
      generic_reduce_kernel<R, TIN, ACC, TOUT, kSum, 1><<<grid, kBlock, 0, st>>>(a);          \
    else if (kind == kWsum)                                                                  \
      generic_reduce_kernel<R, TIN, ACC, TOUT, kWsum, 1><<<grid, kBlock, 0, st>>>(a);         \
    else if (kind == kDot)                                                                   \
      generic_reduce_kernel<R, TIN, ACC, TOUT, kDot, 2><<<grid, kBlock, 0, st>>>(a);          \
    else                                                                                     \
      return hipErrorInvalidValue;                                                           \
  } while (0)
  if (in_dtype == RSM_F32)
    RSM_GEN(float, float, float);
  else if (in_dtype == RSM_BF16)
    RSM_GEN(uint16_t, float, float);
  else if (in_dtype == RSM_F64)
    RSM_GEN(double, double, double);
  else
    return hipErrorInvalidValue;
#undef RSM_GEN
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// generic adjoint
// ---------------------------------------------------------------------------
template <int R>
__global__ void __launch_bounds__(kBlock) generic_adjoint_kernel(GenericAdjArgs a) {
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t rf = int64_t(blockIdx.x) * kBlock + threadIdx.x; rf < a.n_rep; rf += stride) {
    int64_t r[R], ci[R], co[R], pi[R], po[R];
    unflatten<R>(rf, a.rep_rank, a.rep_shape, r);
    start_coords<R>(a.out, a.rep_rank, r, co);
RSM_UNROLL_R
    for (int k = 0; k < R; ++k) po[k] = 0;
    // output element j of the repetition sends c[j n_pat + p] gy to input element p
    for (int64_t j = 0; j < a.n_q; ++j) {
      const float g = a.gy[linear<R>(a.out, co)];
      start_coords<R>(a.in, a.rep_rank, r, ci);
RSM_UNROLL_R
      for (int k = 0; k < R; ++k) pi[k] = 0;
      for (int64_t p = 0; p < a.n_pat; ++p) {
        const float c = a.c ? a.c[j * a.n_pat + p] : 1.0f;
        atomicAdd(a.gx + linear<R>(a.in, ci), c * g);
        if (p + 1 < a.n_pat) step_pattern<R>(a.in, pi, ci);
      }
      if (j + 1 < a.n_q) step_pattern<R>(a.out, po, co);
    }
  }
}

// partial[k][block] = sum over this block's repetitions of
// gy[e_out(r, j)] * x[e_in(r, p)], for weight k = j n_pat + p
template <int R>
__global__ void __launch_bounds__(kBlock) generic_coef_grad_kernel(GenericCoefGradArgs a) {
  __shared__ float red[kBlock];
  const int64_t r_begin = int64_t(blockIdx.x) * a.chunk;
  int64_t r_end = r_begin + a.chunk;
  if (r_end > a.n_rep) r_end = a.n_rep;
  for (int64_t kc = blockIdx.y; kc < a.n_q * a.n_pat; kc += gridDim.y) {
    const int64_t jq = kc / a.n_pat, p = kc - jq * a.n_pat;
    int64_t pidx[R], qidx[R];
    unflatten<R>(p, a.in.pat_rank, a.in.pat_shape, pidx);
    unflatten<R>(jq, a.out.pat_rank, a.out.pat_shape, qidx);
    float acc = 0.0f;
    for (int64_t rf = r_begin + threadIdx.x; rf < r_end; rf += kBlock) {
      int64_t r[R], ci[R], co[R];
      unflatten<R>(rf, a.rep_rank, a.rep_shape, r);
      start_coords<R>(a.in, a.rep_rank, r, ci);
RSM_UNROLL_R
      for (int d = 0; d < R; ++d) {
        if (d < a.in.arr_rank) {
          int64_t v = ci[d];
RSM_UNROLL_R
          for (int k = 0; k < R; ++k)
            if (k < a.in.pat_rank) v = (v + (a.in.fit[d][k] * pidx[k]) % a.in.shape[d]) % a.in.shape[d];
          ci[d] = v;
        }
      }
      start_coords<R>(a.out, a.rep_rank, r, co);
RSM_UNROLL_R
      for (int d = 0; d < R; ++d) {
        if (d < a.out.arr_rank) {
          int64_t v = co[d];
RSM_UNROLL_R
          for (int k = 0; k < R; ++k)
            if (k < a.out.pat_rank) v = (v + (a.out.fit[d][k] * qidx[k]) % a.out.shape[d]) % a.out.shape[d];
          co[d] = v;
        }
      }
      acc += a.gy[linear<R>(a.out, co)] * a.x[linear<R>(a.in, ci)];
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
      if (int(threadIdx.x) < s) red[threadIdx.x] += red[threadIdx.x + s];
      __syncthreads();
    }
    if (threadIdx.x == 0) a.partial[kc * int64_t(gridDim.x) + blockIdx.x] = red[0];
    __syncthreads();
  }
}

// Sum of src[j * stride] over j = t, t + kBlock, t + 2 kBlock, ... < n
// (t = threadIdx.x), added in that order.  The loads are issued eight at a
// time so that their latencies overlap; the order of the additions, and so
// the result, is that of the plain loop.
__device__ __forceinline__ float strided_sum(const float* src, int64_t n, int64_t stride) {
  float acc = 0.0f;
  int64_t j = threadIdx.x;
  for (; j + 7 * kBlock < n; j += 8 * kBlock) {
    float v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = src[(j + u * kBlock) * stride];
#pragma unroll
    for (int u = 0; u < 8; ++u) acc += v[u];
  }
  for (; j < n; j += kBlock) acc += src[j * stride];
  return acc;
}

// Sum over the workgroup of each thread's v, returned to thread 0: a
// butterfly inside each wavefront (every lane pairs the same operands), then
// the four wavefront sums in wavefront order.  The in-kernel weight-gradient
// reduction of the tap kernels uses the same order, so both give the same
// bits.
__device__ __forceinline__ float block_total(float v, float* red) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  return ((red[0] + red[1]) + red[2]) + red[3];
}
static_assert(kBlock == 256, "block_total adds four wavefront sums");

// out[i] (=|+=) sum_j src[i*si + j*sj], j < n, in a fixed order per i
__global__ void __launch_bounds__(kBlock) reduce_strided_kernel(const float* src, int64_t n,
                                                               int64_t si, int64_t sj,
                                                               float* out, int accumulate) {
  __shared__ float red[kBlock / 64];
  const int64_t i = blockIdx.x;
  const float tot = block_total(strided_sum(src + i * si, n, sj), red);
  if (threadIdx.x == 0) out[i] = accumulate ? out[i] + tot : tot;
}

// Two weight gradients from one partial table [n][row_stride]: column
// blockIdx.x < n0 goes to out0[blockIdx.x], the next n1 columns to out1.
// Each column is reduced in the same fixed order as reduce_strided_kernel.
__global__ void __launch_bounds__(kBlock) reduce_pair_kernel(const float* src, int64_t n, int64_t row_stride,
                                                             int n0, float* out0, float* out1, int accumulate) {
  __shared__ float red[kBlock / 64];
  const int i = int(blockIdx.x);
  const float tot = block_total(strided_sum(src + i, n, row_stride), red);
  if (threadIdx.x == 0) {
    float* o = i < n0 ? out0 + i : out1 + (i - n0);
    *o = accumulate ? *o + tot : tot;
  }
}

__global__ void __launch_bounds__(kBlock) loss_grad_kernel(const float* __restrict__ y, const float* __restrict__ w,
                                                          float* __restrict__ g, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n; i += stride) g[i] = 2.0f * (w[i] * y[i]);
}

__global__ void __launch_bounds__(kBlock) zero_kernel(uint32_t* p, int64_t n_words) {
  const int64_t stride = int64_t(gridDim.x) * kBlock;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < n_words; i += stride) p[i] = 0u;
}

__global__ void zero_bytes_kernel(uint8_t* p, int64_t n) {
  const int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// pattern_reduce in 32-bit arithmetic (conditions in PatternReduceSmallArgs):
// one lane per pattern element, groups of 2^group_log2 lanes per repetition
// summed by a butterfly of shuffles, as pattern_reduce_kernel (k_window.hip)
// does in 64-bit arithmetic; the index walk uses multiply-high divisions.
__device__ __forceinline__ uint32_t fmod32(uint32_t n, const FastDiv& f) { return n - fdiv(n, f) * f.d; }

__global__ void __launch_bounds__(kBlock) pattern_reduce_small_kernel(PatternReduceSmallArgs a) {
  const int G = 1 << a.group_log2;
  const int lane = threadIdx.x & (G - 1);
  const uint32_t groups_total = (gridDim.x * kBlock) >> a.group_log2;
  const uint32_t group0 = (blockIdx.x * kBlock + threadIdx.x) >> a.group_log2;

  // this lane's pattern element and its offset (F i) mod s per dimension
  uint32_t off[4] = {0, 0, 0, 0};
  {
    uint32_t i[4] = {0, 0, 0, 0};
    uint32_t f = uint32_t(lane);
#pragma unroll
    for (int k = 3; k >= 0; --k)
      if (k < a.pat_rank) {
        i[k] = f % a.pat_s[k];
        f /= a.pat_s[k];
      }
#pragma unroll
    for (int d = 0; d < 4; ++d)
      if (d < a.in_rank) {
        uint64_t v = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (k < a.pat_rank) v += uint64_t(a.in_f[d][k]) * i[k];
        off[d] = uint32_t(v % a.in_s[d]);
      }
  }
  const bool active = lane < a.n_pat;
  const float coef = (active && a.c) ? a.c[lane] : 1.0f;

  for (uint32_t rf = group0; rf < a.n_rep; rf += groups_total) {
    uint32_t r[4] = {0, 0, 0, 0};
    {
      uint32_t f = rf;
#pragma unroll
      for (int k = 3; k >= 0; --k)
        if (k < a.rep_rank) {
          const uint32_t q = fdiv(f, a.rep_div[k]);
          r[k] = f - q * a.rep_div[k].d;
          f = q;
        }
    }
    float v = 0.0f;
    if (active) {
      uint32_t lin = 0;
#pragma unroll
      for (int d = 0; d < 4; ++d)
        if (d < a.in_rank) {
          const uint32_t s = a.in_s[d];
          uint32_t c = a.in_o[d] + off[d];
          if (c >= s) c -= s;
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (k < a.rep_rank) {
              c += fmod32(a.in_p[d][k] * r[k], a.in_div[d]);
              if (c >= s) c -= s;
            }
          lin = lin * s + c;
        }
      v = a.x[lin] * coef;
    }
    for (int m = G >> 1; m > 0; m >>= 1) v += __shfl_xor(v, m);
    if (lane == 0) {
      uint32_t lin = 0;
#pragma unroll
      for (int d = 0; d < 4; ++d)
        if (d < a.out_rank) {
          const uint32_t s = a.out_s[d];
          uint32_t c = a.out_o[d];
#pragma unroll
          for (int k = 0; k < 4; ++k)
            if (k < a.rep_rank) {
              c += fmod32(a.out_p[d][k] * r[k], a.out_div[d]);
              if (c >= s) c -= s;
            }
          lin = lin * s + c;
        }
      a.y[lin] = v;
    }
  }
}

}  // namespace

hipError_t launch_indices(const GTiler& t, int rep_rank, const int64_t* rep_shape, int64_t n_rep,
                          int64_t n_pat, int64_t* d_idx, hipStream_t st) {
  IndexArgs a;
  a.t = t;
  a.rep_rank = rep_rank;
  for (int k = 0; k < kMaxRank; ++k) a.rep_shape[k] = k < rep_rank ? rep_shape[k] : 1;
  a.n_rep = n_rep;
  a.n_pat = n_pat;
  a.out = d_idx;
  index_table_kernel<<<grid_for(n_rep * n_pat), kBlock, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_generic(const GenericArgs& a, int max_rank, int in_dtype, int /*out_dtype*/,
                          int kind, int elem_bytes, hipStream_t st) {
  if (max_rank <= 4) return dispatch_generic<4>(a, in_dtype, kind, elem_bytes, st);
  return dispatch_generic<kMaxRank>(a, in_dtype, kind, elem_bytes, st);
}

hipError_t launch_generic_adjoint(const GenericAdjArgs& a, int max_rank, hipStream_t st) {
  const int grid = grid_for(a.n_rep);
  if (max_rank <= 4)
    generic_adjoint_kernel<4><<<grid, kBlock, 0, st>>>(a);
  else
    generic_adjoint_kernel<kMaxRank><<<grid, kBlock, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_generic_coef_grad(const GenericCoefGradArgs& a, int max_rank, int n_blocks,
                                    hipStream_t st) {
  const int64_t n_coef = a.n_q * a.n_pat;
  dim3 grid(n_blocks, unsigned(n_coef < 65535 ? n_coef : 65535));
  if (max_rank <= 4)
    generic_coef_grad_kernel<4><<<grid, kBlock, 0, st>>>(a);
  else
    generic_coef_grad_kernel<kMaxRank><<<grid, kBlock, 0, st>>>(a);
  return hipGetLastError();
}

hipError_t launch_reduce_rows(const float* partial, int64_t n_rows, int64_t n_cols, float* out,
                              int accumulate, hipStream_t st) {
  if (n_rows <= 0) return hipSuccess;
  reduce_strided_kernel<<<unsigned(n_rows), kBlock, 0, st>>>(partial, n_cols, n_cols, 1, out,
                                                             accumulate);
  return hipGetLastError();
}

// partial is [n_blocks][row_stride]; out0[j] = sum_b partial[b][j] for
// j < n0 and out1[j] = sum_b partial[b][n0 + j] for j < n1, in one launch
// (out0 or out1 may be null when its count is zero)
hipError_t launch_reduce_partial_pair(const float* partial, int n_blocks, int n0, float* out0, int n1,
                                      float* out1, int row_stride, int accumulate, hipStream_t st) {
  if (n0 + n1 <= 0) return hipSuccess;
  reduce_pair_kernel<<<unsigned(n0 + n1), kBlock, 0, st>>>(partial, n_blocks, row_stride, n0, out0, out1,
                                                            accumulate);
  return hipGetLastError();
}

// partial is [n_blocks][row_stride]; out[j] = sum_b partial[b][j] for j < n_coef
hipError_t launch_reduce_partials(const float* partial, int n_blocks, int n_coef, int row_stride,
                                  float* out, int accumulate, hipStream_t st) {
  if (n_coef <= 0) return hipSuccess;
  reduce_strided_kernel<<<unsigned(n_coef), kBlock, 0, st>>>(partial, n_blocks, 1, row_stride, out,
                                                             accumulate);
  return hipGetLastError();
}

hipError_t launch_loss_grad(const float* y, const float* w, float* g, int64_t n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  loss_grad_kernel<<<grid_for(n, kBlock, 16384), kBlock, 0, st>>>(y, w, g, n);
  return hipGetLastError();
}

// Clears device memory with a kernel (no memset node, so the call can sit in
// a captured graph).
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t st) {
  if (bytes <= 0) return hipSuccess;
  const uintptr_t addr = reinterpret_cast<uintptr_t>(p);
  if ((addr & 3) == 0 && (bytes & 3) == 0) {
    const int64_t words = bytes / 4;
    zero_kernel<<<grid_for(words, kBlock, 16384), kBlock, 0, st>>>(static_cast<uint32_t*>(p), words);
  } else {
    zero_bytes_kernel<<<unsigned((bytes + 255) / 256), 256, 0, st>>>(static_cast<uint8_t*>(p), bytes);
  }
  return hipGetLastError();
}

bool pattern_reduce_small_args(const PatternReduceArgs& a, PatternReduceSmallArgs* s) {
  const int64_t kMax31 = (int64_t(1) << 31) - 1;
  if (a.rep_rank > 4 || a.in.arr_rank > 4 || a.in.pat_rank > 4 || a.out.arr_rank > 4) return false;
  if (a.n_rep > kMax31 || a.n_pat > 64) return false;
  // the launch covers n_rep << group_log2 lanes; keep the counters in 32 bits
  if ((a.n_rep << a.group_log2) > kMax31) return false;
  int64_t n_in = 1, n_out = 1;
  for (int d = 0; d < a.in.arr_rank; ++d) n_in *= a.in.shape[d];
  for (int d = 0; d < a.out.arr_rank; ++d) n_out *= a.out.shape[d];
  if (n_in > kMax31 || n_out > kMax31) return false;
  *s = PatternReduceSmallArgs{};
  s->n_rep = uint32_t(a.n_rep);
  s->rep_rank = a.rep_rank;
  s->group_log2 = a.group_log2;
  s->n_pat = int32_t(a.n_pat);
  for (int k = 0; k < 4; ++k) s->rep_div[k] = make_fastdiv(uint32_t(k < a.rep_rank ? a.rep_shape[k] : 1));
  s->in_rank = a.in.arr_rank;
  s->pat_rank = a.in.pat_rank;
  s->out_rank = a.out.arr_rank;
  const uint64_t kMax32 = uint64_t(1) << 32;
  for (int d = 0; d < 4; ++d) {
    const bool di = d < a.in.arr_rank, dout = d < a.out.arr_rank;
    s->in_s[d] = uint32_t(di ? a.in.shape[d] : 1);
    s->in_o[d] = uint32_t(di ? a.in.origin[d] : 0);
    s->in_div[d] = make_fastdiv(s->in_s[d]);
    s->out_s[d] = uint32_t(dout ? a.out.shape[d] : 1);
    s->out_o[d] = uint32_t(dout ? a.out.origin[d] : 0);
    s->out_div[d] = make_fastdiv(s->out_s[d]);
    s->pat_s[d] = uint32_t(d < a.in.pat_rank ? a.in.pat_shape[d] : 1);
    for (int k = 0; k < 4; ++k) {
      s->in_p[d][k] = uint32_t(di && k < a.rep_rank ? a.in.pav[d][k] : 0);
      s->in_f[d][k] = uint32_t(di && k < a.in.pat_rank ? a.in.fit[d][k] : 0);
      s->out_p[d][k] = uint32_t(dout && k < a.rep_rank ? a.out.pav[d][k] : 0);
      // reduced steps times repetition indices must stay below 2^32
      if (k < a.rep_rank) {
        const uint64_t rk = uint64_t(a.rep_shape[k]);
        if (uint64_t(s->in_p[d][k]) * rk >= kMax32 || uint64_t(s->out_p[d][k]) * rk >= kMax32) return false;
      }
    }
  }
  s->x = a.x;
  s->y = a.y;
  s->c = a.c;
  return true;
}

hipError_t launch_pattern_reduce_small(const PatternReduceSmallArgs& a, hipStream_t st) {
  const int64_t lanes = int64_t(a.n_rep) << a.group_log2;
  int64_t grid = (lanes + kBlock - 1) / kBlock;
  if (grid < 1) grid = 1;
  if (grid > 16384) grid = 16384;
  pattern_reduce_small_kernel<<<unsigned(grid), kBlock, 0, st>>>(a);
  return hipGetLastError();
}

}  // namespace rsm
