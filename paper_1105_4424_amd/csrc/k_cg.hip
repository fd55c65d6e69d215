// k_cg.hip -- the conjugate-gradient loop of the paper's case study (Sec. 7)
// on the device, FP64.
//
// Every step of the loop is a repetitive task: the sparse matrix-vector
// product (indirect tilers, one repetition per row), the inner products
// (a reduction over the element repetitions) and the vector updates
// (element-wise repetitions).  The paper runs the scalar steps on the CPU
// between launches; here they stay on the device so the loop never waits for
// the host.  One iteration k is two kernels:
//
//   cg_spmv  rho_k from the <r,r> partials; stop test; beta_{k-1} =
//            rho_k / rho_{k-1}; p_k = r_k + beta_{k-1} p_{k-1}, formed on
//            the fly for every gathered column and stored for the own rows;
//            q = A p_k; <p_k,q> partials
//   cg_xr    alpha = rho_k / <p_k,q>; x += alpha p_k; r -= alpha q;
//            <r,r> partials; k += 1
//
// The directions alternate between two buffers (p_k in P[k mod 2]), so the
// product reads p_{k-1} while it writes p_k.  Every workgroup rebuilds a
// scalar from the previous kernel's per-workgroup partials in one fixed
// order, so all workgroups hold the same bits and the loop is deterministic
// for a given launch shape; the iterates are those of the textbook order
// (p = r + beta p after the update of r) bit for bit.  The sparse product
// runs on a large grid (latency hiding); the vector kernel on at most 256
// workgroups, so the partials every workgroup re-sums stay few.  Each field
// of the state block is written by workgroup 0 of one kernel only and read
// by other kernels, never by the kernel that writes it: rho[k mod 2], done,
// k_spmv by cg_spmv; breakdown, k by cg_xr.  After the stop test has fired,
// every kernel writes what it wrote before or nothing, so surplus launched
// iterations change nothing.
#include <hip/hip_runtime.h>

#include "rsm_internal.h"

namespace rsm {
namespace {

constexpr int kBlock = 256;

// Sum of v over the workgroup in a fixed order, returned to every thread: a
// butterfly inside each wavefront (lane i adds lane i xor 32, 16, ..., 1, so
// every lane pairs the same operands and holds the same bits), then the four
// wavefront sums in wavefront order.  Two barriers instead of one per level
// of an LDS tree.
__device__ __forceinline__ double block_sum(double v, double* lds) {
#pragma unroll
  for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
  __syncthreads();
  const double s = ((lds[0] + lds[1]) + lds[2]) + lds[3];
  __syncthreads();   // lds is written again by the next call
  return s;
}
static_assert(kBlock == 256, "block_sum adds four wavefront sums");

// Sum of part[0..n) in a fixed order (thread t adds t, t + 256, ..., then the
// tree): identical bits in every workgroup.  The loads are issued eight at a
// time, so a workgroup waits for one round trip per 2048 partials instead of
// one per 256; the additions keep the order of the plain loop.
__device__ __forceinline__ double partial_sum(const double* part, int n, double* lds) {
  double s = 0.0;
  int i = threadIdx.x;
  for (; i + 7 * kBlock < n; i += 8 * kBlock) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = part[i + u * kBlock];
#pragma unroll
    for (int u = 0; u < 8; ++u) s += v[u];
  }
  for (; i < n; i += kBlock) s += part[i];
  return block_sum(s, lds);
}

__device__ __forceinline__ bool lead() { return blockIdx.x == 0 && threadIdx.x == 0; }

// y[r] = sum_k vals[k] v(col_idx[k]) for the rows of this group of G lanes,
// two rows at a time; calls f(r, y_r) on lane 0 of the group.  Each lane
// takes entries lane, lane + G, ..., lane + (E - 1) G of a row chunk and
// issues all index and value loads of both rows, then all gathers of v,
// before the first product, so a lane has 4 E loads in flight.  Row bounds
// are clamped into [0, nnz] and columns outside [0, n) contribute nothing.
// BUF (matrix and vectors under 2 GiB): raw buffer loads, all issued
// unconditionally; an entry past its row reads a zero value and column and
// gathers zero (v(c, false) must return 0), so no load waits on a branch.
constexpr int kEntries = 4;   // E
constexpr uint32_t kBufferWord3 = 0x00020000;   // 32-bit data format, raw access
constexpr uint32_t kOutOfRange = 0x80000000u;   // a read here returns zero

__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc(const void* p, int64_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), short(0), int(bytes), int(kBufferWord3));
}

__device__ __forceinline__ double load_f64(__amdgpu_buffer_rsrc_t r, int32_t c, bool ok) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, ok ? uint32_t(c) * 8u : kOutOfRange, 0, 0));
}

template <int G, bool BUF, typename V, typename F>
__device__ __forceinline__ void spmv_rows(const CgArgs& a, V v, F f) {
  constexpr int E = kEntries;
  const int lane = threadIdx.x & (G - 1);
  const int64_t groups = int64_t(gridDim.x) * (kBlock / G);
  const __amdgpu_buffer_rsrc_t rc = rsrc(a.col_idx, BUF ? a.nnz * 4 : 0);
  const __amdgpu_buffer_rsrc_t rv = rsrc(a.vals, BUF ? a.nnz * 8 : 0);
  for (int64_t r0 = (int64_t(blockIdx.x) * kBlock + threadIdx.x) / G; r0 < a.n; r0 += 2 * groups) {
    const int64_t r1 = r0 + groups;
    const bool has1 = r1 < a.n;
    const int64_t r1c = has1 ? r1 : r0;
    int64_t b0 = a.row_ptr[r0], e0 = a.row_ptr[r0 + 1];
    int64_t b1 = a.row_ptr[r1c], e1 = a.row_ptr[r1c + 1];
    if (!has1) e1 = b1;
    b0 = b0 < 0 ? 0 : (b0 > a.nnz ? a.nnz : b0);
    e0 = e0 < b0 ? b0 : (e0 > a.nnz ? a.nnz : e0);
    b1 = b1 < 0 ? 0 : (b1 > a.nnz ? a.nnz : b1);
    e1 = e1 < b1 ? b1 : (e1 > a.nnz ? a.nnz : e1);
    double acc0 = 0.0, acc1 = 0.0;
    for (int64_t k0 = b0 + lane, k1 = b1 + lane; k0 < e0 || k1 < e1; k0 += G * E, k1 += G * E) {
      int32_t c0[E], c1[E];
      double v0[E], v1[E];
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const int64_t q0 = k0 + j * G, q1 = k1 + j * G;
        if (BUF) {
          const bool in0 = q0 < e0, in1 = q1 < e1;
          c0[j] = int32_t(__builtin_amdgcn_raw_buffer_load_b32(rc, in0 ? uint32_t(q0) * 4u : kOutOfRange, 0, 0));
          v0[j] = __builtin_bit_cast(
              double, __builtin_amdgcn_raw_buffer_load_b64(rv, in0 ? uint32_t(q0) * 8u : kOutOfRange, 0, 0));
          c1[j] = int32_t(__builtin_amdgcn_raw_buffer_load_b32(rc, in1 ? uint32_t(q1) * 4u : kOutOfRange, 0, 0));
          v1[j] = __builtin_bit_cast(
              double, __builtin_amdgcn_raw_buffer_load_b64(rv, in1 ? uint32_t(q1) * 8u : kOutOfRange, 0, 0));
        } else {
          c0[j] = q0 < e0 ? a.col_idx[q0] : -1;
          v0[j] = q0 < e0 ? a.vals[q0] : 0.0;
          c1[j] = q1 < e1 ? a.col_idx[q1] : -1;
          v1[j] = q1 < e1 ? a.vals[q1] : 0.0;
        }
      }
      double x0[E], x1[E];
#pragma unroll
      for (int j = 0; j < E; ++j) {
        x0[j] = v(c0[j], k0 + j * G < e0 && uint32_t(c0[j]) < uint32_t(a.n));
        x1[j] = v(c1[j], k1 + j * G < e1 && uint32_t(c1[j]) < uint32_t(a.n));
      }
      if (BUF) __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int j = 0; j < E; ++j) {
        if (BUF || uint32_t(c0[j]) < uint32_t(a.n)) acc0 += v0[j] * x0[j];
        if (BUF || uint32_t(c1[j]) < uint32_t(a.n)) acc1 += v1[j] * x1[j];
      }
    }
#pragma unroll
    for (int m = G >> 1; m > 0; m >>= 1) {
      acc0 += __shfl_xor(acc0, m);
      acc1 += __shfl_xor(acc1, m);
    }
    if (lane == 0) {
      f(r0, acc0);
      if (has1) f(r1, acc1);
    }
  }
}

// r = b - A x0; P[1] = 0 (p_{-1}: p_0 = r_0 + 0 p_{-1}); partials of <r,r>
// and <b,b>.
template <int G, bool BUF>
__global__ void __launch_bounds__(kBlock) cg_init_kernel(CgArgs a) {
  __shared__ double lds[kBlock];
  double rr = 0.0, bb = 0.0;
  const double* __restrict__ x = a.x;
  const __amdgpu_buffer_rsrc_t rx = rsrc(x, BUF ? a.n * 8 : 0);
  auto gather = [&](int32_t c, bool ok) { return BUF ? load_f64(rx, c, ok) : (ok ? x[c] : 0.0); };
  spmv_rows<G, BUF>(a, gather, [&](int64_t r, double ax) {
    const double b = a.b[r];
    const double res = b - ax;
    a.r[r] = res;
    rr += res * res;
    bb += b * b;
  });
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < a.n; i += int64_t(gridDim.x) * kBlock)
    a.p1[i] = 0.0;
  rr = block_sum(rr, lds);
  bb = block_sum(bb, lds);
  if (threadIdx.x == 0) {
    a.part_rr[blockIdx.x] = rr;
    a.part_bb[blockIdx.x] = bb;
  }
}

// One workgroup: ||b||, a fresh state block, and the <r0,r0> partials of
// cg_init (one per row workgroup) folded into part_rr[0] with zeros after
// it, the layout cg_spmv reads (one per vector workgroup); adding zeros
// leaves the fixed-order sum unchanged.
__global__ void __launch_bounds__(kBlock) cg_start_kernel(CgArgs a) {
  __shared__ double lds[kBlock];
  const double bb = partial_sum(a.part_bb, a.grid_rows, lds);
  const double rr = partial_sum(a.part_rr, a.grid_rows, lds);
  for (int i = threadIdx.x; i < a.grid_vec; i += kBlock) a.part_rr[i] = i == 0 ? rr : 0.0;
  if (threadIdx.x == 0) {
    a.st->bnorm = sqrt(bb);
    a.st->rho[0] = 0.0;
    a.st->rho[1] = 0.0;
    a.st->k = 0;
    a.st->k_spmv = 0;
    a.st->done = 0;
    a.st->breakdown = 0;
  }
}

template <int G, bool BUF>
__global__ void __launch_bounds__(kBlock) cg_spmv_kernel(CgArgs a) {
  __shared__ double lds[kBlock];
  const double rho = partial_sum(a.part_rr, a.grid_vec, lds);
  const int64_t k = a.st->k;
  const bool stop = a.st->breakdown != 0 || k >= a.max_iter || !(sqrt(rho) > a.tol * a.st->bnorm);
  const double beta = k > 0 ? rho / a.st->rho[(k - 1) & 1] : 0.0;
  if (lead()) {
    a.st->rho[k & 1] = rho;
    a.st->k_spmv = k;
    a.st->done = stop ? 1 : 0;
    if (a.res) a.res[k] = sqrt(rho);
    if (k > 0 && a.beta) a.beta[k - 1] = beta;
  }
  if (stop) return;
  const double* __restrict__ r = a.r;
  const double* __restrict__ p_old = (k & 1) ? a.p0 : a.p1;
  double* __restrict__ p_new = (k & 1) ? a.p1 : a.p0;
  double pq = 0.0;
  const __amdgpu_buffer_rsrc_t rr_ = rsrc(r, BUF ? a.n * 8 : 0), rp_ = rsrc(p_old, BUF ? a.n * 8 : 0);
  auto gather = [&](int32_t c, bool ok) {
    return BUF ? fma(beta, load_f64(rp_, c, ok), load_f64(rr_, c, ok)) : (ok ? fma(beta, p_old[c], r[c]) : 0.0);
  };
  spmv_rows<G, BUF>(a, gather, [&](int64_t i, double q) {
    const double p = fma(beta, p_old[i], r[i]);
    p_new[i] = p;
    a.q[i] = q;
    pq += p * q;
  });
  pq = block_sum(pq, lds);
  if (threadIdx.x == 0) a.part_pq[blockIdx.x] = pq;
}

__global__ void __launch_bounds__(kBlock) cg_xr_kernel(CgArgs a) {
  __shared__ double lds[kBlock];
  if (a.st->done) return;
  const double pq = partial_sum(a.part_pq, a.grid_rows, lds);
  if (!(pq > 0.0)) {  // A is not positive definite along p
    if (lead()) a.st->breakdown = 1;
    return;
  }
  const int64_t k = a.st->k_spmv;
  const double alpha = a.st->rho[k & 1] / pq;
  if (lead() && a.alpha) a.alpha[k] = alpha;
  const double* __restrict__ p = (k & 1) ? a.p1 : a.p0;
  double rr = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kBlock + threadIdx.x; i < a.n; i += int64_t(gridDim.x) * kBlock) {
    a.x[i] += alpha * p[i];
    const double res = a.r[i] - alpha * a.q[i];
    a.r[i] = res;
    rr += res * res;
  }
  rr = block_sum(rr, lds);
  if (threadIdx.x == 0) a.part_rr[blockIdx.x] = rr;
  if (lead()) a.st->k = k + 1;
}

template <int G, bool BUF>
hipError_t launch_gb(const CgArgs& a, bool init, int iters, hipStream_t st) {
  const unsigned gr = unsigned(a.grid_rows), gv = unsigned(a.grid_vec);
  if (init) {
    cg_init_kernel<G, BUF><<<gr, kBlock, 0, st>>>(a);
    cg_start_kernel<<<1, kBlock, 0, st>>>(a);
  }
  for (int i = 0; i < iters; ++i) {
    cg_spmv_kernel<G, BUF><<<gr, kBlock, 0, st>>>(a);
    cg_xr_kernel<<<gv, kBlock, 0, st>>>(a);
  }
  return hipGetLastError();
}

// buffer offsets are 32-bit: values (8 B per entry) and vectors under 2 GiB
template <int G>
hipError_t launch_g(const CgArgs& a, bool init, int iters, hipStream_t st) {
  const int64_t lim = int64_t(1) << 31;
  if (a.nnz * 8 < lim && a.n * 8 < lim) return launch_gb<G, true>(a, init, iters, st);
  return launch_gb<G, false>(a, init, iters, st);
}

}  // namespace

// Lanes per row: the power of two (4..64) that covers the mean row length
// with kEntries entries per lane.
int cg_group_size(int64_t n, int64_t nnz) {
  const double mean = n > 0 ? double(nnz) / double(n) : 0.0;
  int g = 4;
  while (g < 64 && g * kEntries < mean) g *= 2;
  return g;
}

// Enough workgroups for one pass over the rows (two rows per lane group), at
// most 2048: every loop kernel rebuilds its scalar from this many partials.
int cg_grid(int64_t n, int64_t nnz) {
  const int64_t lanes = ((n + 1) / 2) * cg_group_size(n, nnz);
  int64_t g = (lanes + kBlock - 1) / kBlock;
  if (g > 2048) g = 2048;
  if (g < 1) g = 1;
  return int(g);
}

// Vector kernels: at most 256 workgroups (the next kernel re-sums their
// partials in every workgroup, so few partials keep that cheap).
int cg_vec_grid(int64_t n) {
  int64_t g = (n + kBlock - 1) / kBlock;
  if (g > 256) g = 256;
  if (g < 1) g = 1;
  return int(g);
}

hipError_t launch_cg(const CgArgs& a, bool init, int iters, hipStream_t st) {
  switch (cg_group_size(a.n, a.nnz)) {
    case 4: return launch_g<4>(a, init, iters, st);
    case 8: return launch_g<8>(a, init, iters, st);
    case 16: return launch_g<16>(a, init, iters, st);
    case 32: return launch_g<32>(a, init, iters, st);
    default: return launch_g<64>(a, init, iters, st);
  }
}

}  // namespace rsm
