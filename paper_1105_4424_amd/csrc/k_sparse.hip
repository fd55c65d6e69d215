// k_sparse.hip -- repetitive task with data-dependent (indirect) tilers: the
// sparse matrix-vector product in CSR form.
//
// A group of G lanes (G a power of two, chosen from the mean row length)
// handles one row: lanes stride through the row's entries (consecutive
// lanes read consecutive values and column indices, so those loads
// coalesce), gather x through the column indices (x is small enough to stay
// in L2), and reduce with a butterfly of wavefront shuffles.  Row bounds are
// clamped into [0, nnz] and column indices outside [0, n_cols) contribute
// nothing, so malformed input cannot read out of bounds.
#include <hip/hip_runtime.h>

#include "rsm_internal.h"

namespace rsm {
namespace {

constexpr int kBlock = 256;

template <typename T, int G>
__global__ void __launch_bounds__(kBlock) csr_kernel(CsrArgs a) {
  const T* __restrict__ vals = static_cast<const T*>(a.vals);
  const T* __restrict__ x = static_cast<const T*>(a.x);
  T* __restrict__ y = static_cast<T*>(a.y);
  const int lane = threadIdx.x & (G - 1);
  const int64_t groups = int64_t(gridDim.x) * (kBlock / G);
  for (int64_t r = (int64_t(blockIdx.x) * kBlock + threadIdx.x) / G; r < a.n_rows; r += groups) {
    int64_t b = a.row_ptr[r], e = a.row_ptr[r + 1];
    b = b < 0 ? 0 : (b > a.nnz ? a.nnz : b);
    e = e < b ? b : (e > a.nnz ? a.nnz : e);
    T acc = T(0);
    for (int64_t k = b + lane; k < e; k += G) {
      const int32_t c = a.col_idx[k];
      if (uint32_t(c) < uint32_t(a.n_cols)) acc += vals[k] * x[c];
    }
#pragma unroll
    for (int m = G >> 1; m > 0; m >>= 1) acc += __shfl_xor(acc, m);
    if (lane == 0) y[r] = acc;
  }
}

template <typename T>
hipError_t launch_t(const CsrArgs& a, int g, hipStream_t st) {
  const int64_t lanes = a.n_rows * g;
  int64_t grid = (lanes + kBlock - 1) / kBlock;
  if (grid > 8192) grid = 8192;
  if (grid < 1) grid = 1;
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
  while (g < 64 && g < mean) g *= 2;
  return g;
}

hipError_t launch_csr(const CsrArgs& a, int dtype, hipStream_t st) {
  const int g = csr_group_size(a.n_rows, a.nnz);
  return dtype == RSM_F64 ? launch_t<double>(a, g, st) : launch_t<float>(a, g, st);
}

}  // namespace rsm
