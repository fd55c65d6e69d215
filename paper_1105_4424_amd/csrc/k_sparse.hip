// k_sparse.hip -- repetitive task with data-dependent (indirect) tilers: the
// sparse matrix-vector product in CSR form.
//
// A group of G lanes (G a power of two, chosen from the mean row length)
// handles two rows at a time: each lane takes entries lane, lane + G, ...,
// lane + 3 G of a row chunk (consecutive lanes read consecutive values and
// column indices, so those loads coalesce), issues every index and value
// load of both rows before gathering x through the column indices (x is
// small enough to stay in L2), and the group reduces with a butterfly of
// wavefront shuffles.  Row bounds are clamped into [0, nnz] and column
// indices outside [0, n_cols) contribute nothing, so malformed input cannot
// read out of bounds.
#include <hip/hip_runtime.h>

#include "rsm_internal.h"

namespace rsm {
namespace {

constexpr int kBlock = 256;

constexpr int kEntries = 4;   // entries per lane per row chunk

template <typename T, int G>
__global__ void __launch_bounds__(kBlock) csr_kernel(CsrArgs a) {
  constexpr int E = kEntries;
  const T* __restrict__ vals = static_cast<const T*>(a.vals);
  const T* __restrict__ x = static_cast<const T*>(a.x);
  T* __restrict__ y = static_cast<T*>(a.y);
  const int lane = threadIdx.x & (G - 1);
  const int64_t groups = int64_t(gridDim.x) * (kBlock / G);
  for (int64_t r0 = (int64_t(blockIdx.x) * kBlock + threadIdx.x) / G; r0 < a.n_rows; r0 += 2 * groups) {
    const int64_t r1 = r0 + groups;
    const bool has1 = r1 < a.n_rows;
    int64_t b0 = a.row_ptr[r0], e0 = a.row_ptr[r0 + 1];
    int64_t b1 = has1 ? a.row_ptr[r1] : 0, e1 = has1 ? a.row_ptr[r1 + 1] : 0;
    b0 = b0 < 0 ? 0 : (b0 > a.nnz ? a.nnz : b0);
    e0 = e0 < b0 ? b0 : (e0 > a.nnz ? a.nnz : e0);
    b1 = b1 < 0 ? 0 : (b1 > a.nnz ? a.nnz : b1);
    e1 = e1 < b1 ? b1 : (e1 > a.nnz ? a.nnz : e1);
    T acc0 = T(0), acc1 = T(0);
    for (int64_t k0 = b0 + lane, k1 = b1 + lane; k0 < e0 || k1 < e1; k0 += G * E, k1 += G * E) {
      int32_t c0[E], c1[E];
      T v0[E], v1[E];
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int64_t q0 = k0 + j * G, q1 = k1 + j * G;
        c0[j] = q0 < e0 ? a.col_idx[q0] : -1;
        v0[j] = q0 < e0 ? vals[q0] : T(0);
        c1[j] = q1 < e1 ? a.col_idx[q1] : -1;
        v1[j] = q1 < e1 ? vals[q1] : T(0);
      }
#pragma unroll
      for (int j = 0; j < E; ++j) {
        if (uint32_t(c0[j]) < uint32_t(a.n_cols)) acc0 += v0[j] * x[c0[j]];
        if (uint32_t(c1[j]) < uint32_t(a.n_cols)) acc1 += v1[j] * x[c1[j]];
      }
    }
#pragma unroll
    for (int m = G >> 1; m > 0; m >>= 1) {
      acc0 += __shfl_xor(acc0, m);
      acc1 += __shfl_xor(acc1, m);
    }
    if (lane == 0) {
      y[r0] = acc0;
      if (has1) y[r1] = acc1;
    }
  }
}

// The same walk with raw buffer loads (values, column indices and x each
// under 2 GiB): every load is issued unconditionally, an entry past its row
// reads a zero value and column and gathers a zero x (out-of-range offsets
// read zero), so the compiler can keep all of a chunk's loads in flight
// instead of waiting for each conditional one.  Rows are read at clamped
// indices.
constexpr uint32_t kBufferWord3 = 0x00020000;   // 32-bit data format, raw access
constexpr uint32_t kOutOfRange = 0x80000000u;

template <typename T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

template <typename T, int G>
__global__ void __launch_bounds__(kBlock) csr_buf_kernel(CsrArgs a) {
  constexpr int E = kEntries;
  constexpr uint32_t S = sizeof(T);
  const __amdgpu_buffer_rsrc_t rc = __builtin_amdgcn_make_buffer_rsrc(const_cast<int32_t*>(a.col_idx), short(0),
                                                                      int(a.nnz * 4), int(kBufferWord3));
  const __amdgpu_buffer_rsrc_t rv = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(a.vals), short(0),
                                                                      int(a.nnz * S), int(kBufferWord3));
  const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(a.x), short(0),
                                                                      int(a.n_cols * S), int(kBufferWord3));
  T* __restrict__ y = static_cast<T*>(a.y);
  const int lane = threadIdx.x & (G - 1);
  const int64_t groups = int64_t(gridDim.x) * (kBlock / G);
  for (int64_t r0 = (int64_t(blockIdx.x) * kBlock + threadIdx.x) / G; r0 < a.n_rows; r0 += 2 * groups) {
    const int64_t r1 = r0 + groups;
    const bool has1 = r1 < a.n_rows;
    const int64_t r1c = has1 ? r1 : r0;
    int64_t b0 = a.row_ptr[r0], e0 = a.row_ptr[r0 + 1];
    int64_t b1 = a.row_ptr[r1c], e1 = a.row_ptr[r1c + 1];
    if (!has1) e1 = b1;
    b0 = b0 < 0 ? 0 : (b0 > a.nnz ? a.nnz : b0);
    e0 = e0 < b0 ? b0 : (e0 > a.nnz ? a.nnz : e0);
    b1 = b1 < 0 ? 0 : (b1 > a.nnz ? a.nnz : b1);
    e1 = e1 < b1 ? b1 : (e1 > a.nnz ? a.nnz : e1);
    T acc0 = T(0), acc1 = T(0);
    for (int64_t k0 = b0 + lane, k1 = b1 + lane; k0 < e0 || k1 < e1; k0 += G * E, k1 += G * E) {
      int32_t c0[E], c1[E];
      T v0[E], v1[E];
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int64_t q0 = k0 + j * G, q1 = k1 + j * G;
        const bool in0 = q0 < e0, in1 = q1 < e1;
        c0[j] = int32_t(__builtin_amdgcn_raw_buffer_load_b32(rc, in0 ? uint32_t(q0) * 4u : kOutOfRange, 0, 0));
        v0[j] = buf_load<T>(rv, in0 ? uint32_t(q0) * S : kOutOfRange);
        c1[j] = int32_t(__builtin_amdgcn_raw_buffer_load_b32(rc, in1 ? uint32_t(q1) * 4u : kOutOfRange, 0, 0));
        v1[j] = buf_load<T>(rv, in1 ? uint32_t(q1) * S : kOutOfRange);
      }
      // every gather of the chunk before the first product
      T x0[E], x1[E];
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const bool ok0 = k0 + j * G < e0 && uint32_t(c0[j]) < uint32_t(a.n_cols);
        const bool ok1 = k1 + j * G < e1 && uint32_t(c1[j]) < uint32_t(a.n_cols);
        x0[j] = buf_load<T>(rx, ok0 ? uint32_t(c0[j]) * S : kOutOfRange);
        x1[j] = buf_load<T>(rx, ok1 ? uint32_t(c1[j]) * S : kOutOfRange);
      }
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        acc0 += v0[j] * x0[j];
        acc1 += v1[j] * x1[j];
      }
    }
#pragma unroll
    for (int m = G >> 1; m > 0; m >>= 1) {
      acc0 += __shfl_xor(acc0, m);
      acc1 += __shfl_xor(acc1, m);
    }
    if (lane == 0) {
      y[r0] = acc0;
      if (has1) y[r1] = acc1;
    }
  }
}

template <typename T>
hipError_t launch_t(const CsrArgs& a, int g, hipStream_t st) {
  const int64_t lanes = ((a.n_rows + 1) / 2) * g;
  int64_t grid = (lanes + kBlock - 1) / kBlock;
  if (grid > 8192) grid = 8192;
  if (grid < 1) grid = 1;
  // buffer offsets are 32-bit: values and x must stay under 2 GiB
  const int64_t lim = int64_t(1) << 31;
  const bool buf = a.nnz * int64_t(sizeof(T)) < lim && a.n_cols * int64_t(sizeof(T)) < lim;
  if (buf) {
    switch (g) {
      case 4: csr_buf_kernel<T, 4><<<unsigned(grid), kBlock, 0, st>>>(a); break;
      case 8: csr_buf_kernel<T, 8><<<unsigned(grid), kBlock, 0, st>>>(a); break;
      case 16: csr_buf_kernel<T, 16><<<unsigned(grid), kBlock, 0, st>>>(a); break;
      case 32: csr_buf_kernel<T, 32><<<unsigned(grid), kBlock, 0, st>>>(a); break;
      default: csr_buf_kernel<T, 64><<<unsigned(grid), kBlock, 0, st>>>(a); break;
    }
    return hipGetLastError();
  }
  switch (g) {
    case 4: csr_kernel<T, 4><<<unsigned(grid), kBlock, 0, st>>>(a); break;
    case 8: csr_kernel<T, 8><<<unsigned(grid), kBlock, 0, st>>>(a); break;
    case 16: csr_kernel<T, 16><<<unsigned(grid), kBlock, 0, st>>>(a); break;
    case 32: csr_kernel<T, 32><<<unsigned(grid), kBlock, 0, st>>>(a); break;
    default: csr_kernel<T, 64><<<unsigned(grid), kBlock, 0, st>>>(a); break;
  }
  return hipGetLastError();
}

}  // namespace

int csr_group_size(int64_t n_rows, int64_t nnz) {
  const double mean = n_rows > 0 ? double(nnz) / double(n_rows) : 0.0;
  int g = 4;
  while (g < 64 && g * kEntries < mean) g *= 2;
  return g;
}

hipError_t launch_csr(const CsrArgs& a, int dtype, hipStream_t st) {
  const int g = csr_group_size(a.n_rows, a.nnz);
  return dtype == RSM_F64 ? launch_t<double>(a, g, st) : launch_t<float>(a, g, st);
}

}  // namespace rsm
