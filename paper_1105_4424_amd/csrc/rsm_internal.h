// rsm_internal.h -- descriptors shared by the host planner and the gfx950 kernels.
//
// The planner (api.cpp) validates a task, reduces every tiler to a
// canonical device descriptor and picks a kernel family; the launchers
// (k_*.hip) only launch.  Nothing here is part of the public C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "rsm.h"

namespace rsm {

constexpr int kMaxRank = RSM_MAX_RANK;

// ---------------------------------------------------------------------------
// Generic tiler descriptor (any affine tiler, int64 arithmetic).
// origin/paving/fitting are stored reduced into [0, s_d) so that every step
// of an incremental walk is an add plus at most one conditional subtract.
// ---------------------------------------------------------------------------
struct GTiler {
  int32_t arr_rank;
  int32_t pat_rank;
  int64_t shape[kMaxRank];
  int64_t origin[kMaxRank];              // o mod s
  int64_t pav[kMaxRank][kMaxRank];       // P mod s  [d][k]
  int64_t fit[kMaxRank][kMaxRank];       // F mod s  [d][k]
  int64_t pat_shape[kMaxRank];
};

enum TaskKind : int32_t { kCopy = 0, kSum = 1, kWsum = 2, kDot = 3 };

struct GenericArgs {
  int32_t rep_rank;
  int32_t n_in;
  int64_t rep_shape[kMaxRank];
  int64_t n_rep;   // |s_r|
  int64_t n_pat;   // |s_p| (flat pattern length walked by every tiler)
  int64_t n_q;     // output pattern elements (WSUM: coeffs are [n_q][n_pat])
  GTiler in[2];
  GTiler out;
  const void* x[2];
  void* y;
  const void* coeffs;
};

// Canonical 3-D view [B, R, C] of an axis-aligned tiler: diagonal paving
// (repetition dim d steps array dim d by p[d]), origin o, and a 1-D pattern
// of `taps` elements along axis `ax` with unit fitting, or a 2-D pattern
// along axes (1, 2) with unit fitting.  All values fit in int32.
struct Win3 {
  int32_t A[3];     // array shape
  int32_t rep[3];   // repetition shape
  int32_t o[3];     // origin as given (may be negative)
  int32_t p[3];     // paving diagonal (>= 0)
  int32_t ax;       // tap axis for 1-D patterns (1 or 2); 0 for 2-D patterns
  int32_t taps;     // 1-D: pattern length; 2-D: rows of the pattern
  int32_t taps2;    // 2-D: columns of the pattern; 1 otherwise
};

// Unsigned 32-bit division by a run-time constant via multiply-high
// (round-up method of Granlund & Montgomery, 1994): q = (hi(n*m) + n) >> s,
// exact for every n < 2^32 when d >= 1.
struct FastDiv {
  uint32_t d, m, s;
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t s = 0;
  while ((uint64_t(1) << s) < d) ++s;
  f.s = s;
  f.m = uint32_t(((uint64_t(1) << 32) * ((uint64_t(1) << s) - d)) / d + 1);
  return f;
}

__host__ __device__ inline uint32_t fdiv(uint32_t n, const FastDiv& f) {
#if defined(__HIP_DEVICE_COMPILE__)
  uint32_t hi = __umulhi(n, f.m);
#else
  uint32_t hi = uint32_t((uint64_t(n) * f.m) >> 32);
#endif
  return uint32_t((uint64_t(hi) + n) >> f.s);
}

// 1-D tap filter (FIR) over a Win3 view, identity output tiler.
struct FirArgs {
  Win3 w;
  FastDiv div_rc;     // divide by rep[2]
  FastDiv div_rr;     // divide by rep[1]
  uint32_t n_out;     // rep[0]*rep[1]*rep[2]
  const float* x;
  float* y;
  const float* c;
};

// Two chained FIR stages, the first along axis 2 and the second along axis 1.
struct FirChainArgs {
  Win3 h;             // stage 0 (taps along columns), on x
  Win3 v;             // stage 1 (taps along rows), on the stage-0 output
  FastDiv div_rc;     // divide by v.rep[2]
  FastDiv div_rr;     // divide by v.rep[1]
  uint32_t n_out;
  const float* x;
  float* y;
  const float* ch;
  const float* cv;
};

// Adjoint of an injective FIR stage (no input element read twice).
struct FirAdjArgs {
  Win3 w;
  FastDiv div_rc, div_rr;
  uint32_t n_rep;
  const float* x;      // nullable when gc is not requested
  const float* gy;
  float* gx;           // nullable
  const float* c;
  float* partial;      // [gridDim.x][taps] per-block weight-gradient partials, nullable
  float* gc;           // weight gradient (written by the last workgroup), nullable
  uint32_t* counter;   // null: partials only (reduced by a second kernel); else zero on
                       // entry, workgroups count in and the last one reduces and resets it
  int32_t accumulate;
};

// Input gradient of a 1-D tap tiler in gather form (overlapping or wrapping
// windows): one thread per input element.
struct FirGatherArgs {
  Win3 w;              // ax = 1 or 2; outer axes do not wrap
  FastDiv div_a2;      // divide by A[2]
  FastDiv div_a1;      // divide by A[1]
  FastDiv div_p[3];    // divide by max(p[d], 1)
  int32_t o_mod;       // o[ax] mod A[ax], in [0, A[ax])
  uint32_t n_arr;      // A[0] A[1] A[2]
  const float* gy;     // [rep[0], rep[1], rep[2]]
  float* gx;           // [A[0], A[1], A[2]], every element written
  const float* c;      // [taps]
  int32_t accumulate;
};

// Both gradients of a 1-D tap tiler along columns whose windows overlap or
// wrap (1 <= p[2] <= 16, taps <= 16, A[2] and rep[2] below 2^28): work items
// (array row, chunk of 256 repetitions).
struct FirOverlapArgs {
  Win3 w;              // ax = 2; outer axes do not wrap
  FastDiv div_a1;      // divide by A[1]
  FastDiv div_a2;      // divide by A[2]
  FastDiv div_p;       // divide by p[2]
  FastDiv div_chunks;  // divide by n_chunks
  FastDiv div_p0;      // divide by max(p[0], 1)
  FastDiv div_p1;      // divide by max(p[1], 1)
  int32_t o_mod;       // o[2] mod A[2]
  int32_t step_mod;    // (p[2] (256 / taps)) mod A[2]: column step between a lane's pairs
  int32_t n_chunks;    // max(ceil(A[2] / (256 p[2])), ceil(rep[2] / 256))
  uint32_t n_items;    // A[0] A[1] n_chunks
  const float* x;      // needed when partial is set
  const float* gy;
  float* gx;           // nullable; every element written
  const float* c;
  float* partial;      // [grid][taps] weight-gradient partials, nullable
  int32_t accumulate;
};

struct FirChainAdjArgs {
  Win3 h, v;
  FastDiv div_rc, div_rr;
  uint32_t n_out;
  const float* x;
  const float* gy;
  float* gx;           // nullable
  const float* ch;
  const float* cv;
  float* partial;      // [gridDim.x][h.taps + v.taps], nullable
  float* gch;          // weight gradients (written by the last workgroup), nullable
  float* gcv;
  uint32_t* counter;   // as in FirAdjArgs
  int32_t accumulate;
  // training step (launch_fir_chain_train): gy is not read but formed per
  // output as 2 wl[o] y[o] from the forward value y[o], which is stored to y
  const float* wl;
  float* y;
};

// Weighted sum whose output pattern has q > 1 elements along the tap axis
// (polyphase stage): y[.., q r + j, ..] = sum_i c[j T + i] x[.., (o + p r + i) mod A, ..]
// along axis w.ax (1 or 2) of the [B, R, C] view; the output array is the
// repetition shape with the tap axis multiplied by q.  Outer axes do not wrap.
struct PolyArgs {
  Win3 w;
  int32_t q;           // outputs per repetition
  int32_t n_chunks;    // columns kernel: items of 256 repetitions per row
  FastDiv div_chunks;  // divide by n_chunks
  FastDiv div_rc;      // divide by rep[2]
  FastDiv div_rr;      // divide by rep[1]
  uint32_t n_items;    // columns kernel: rep[0] rep[1] n_chunks; otherwise rep[0] rep[1] rep[2]
  const float* x;
  float* y;            // forward output
  const float* c;      // [q][T]
  const float* gy;     // weight gradient: output gradient
  float* partial;      // weight gradient: [grid][q T]
};

// Both gradients of a polyphase stage along columns in one pass (T <= 16,
// q <= 4, p <= 16): items (row, chunk of 256 repetitions), ownership of the
// columns whose first lift falls in the chunk.
struct PolyAdjArgs {
  Win3 w;
  int32_t q;
  int32_t n_chunks;    // max(ceil(A[2] / (256 p)), ceil(rep[2] / 256))
  int32_t o_mod;       // o[2] mod A[2]
  FastDiv div_chunks;  // divide by n_chunks
  FastDiv div_rr;      // divide by rep[1]
  FastDiv div_p;       // divide by p[2]
  uint32_t n_items;    // rep[0] rep[1] n_chunks
  const float* x;      // needed when partial is set
  const float* gy;
  float* gx;           // nullable; every element written
  const float* c;
  float* partial;      // [grid][q T] weight-gradient partials, nullable
  int32_t accumulate;
};

// Input gradient of a polyphase stage as a gather (one thread per element).
struct PolyGatherArgs {
  Win3 w;
  int32_t q;
  FastDiv div_a2, div_a1;
  FastDiv div_p[3];    // divide by max(p[d], 1)
  int32_t o_mod;       // o[ax] mod A[ax]
  uint32_t n_arr;
  const float* gy;
  float* gx;           // every element written
  const float* c;
  int32_t accumulate;
};

// Small-pattern reduction: a group of G lanes (G = 2^k >= |pattern|, G <= 64)
// per repetition, one lane per pattern element, butterfly reduction.
struct PatternReduceArgs {
  int32_t rep_rank;
  int32_t group_log2;
  int64_t rep_shape[kMaxRank];
  int64_t n_rep;
  int64_t n_pat;
  GTiler in;
  GTiler out;
  const float* x;
  float* y;
  const float* c;      // nullable (SUM)
};

// pattern_reduce in 32-bit arithmetic for ranks <= 4: every array below 2^31
// elements and every product P[d][k] r_k (reduced P) below 2^32, so the
// walk reduces each product with a multiply-high division.  The arguments
// are a fifth of PatternReduceArgs, which shortens the launch of a small task.
struct PatternReduceSmallArgs {
  uint32_t n_rep;
  int32_t rep_rank;
  int32_t group_log2;
  int32_t n_pat;
  FastDiv rep_div[4];      // by rep_shape[k]
  int32_t in_rank, pat_rank, out_rank, pad0;
  uint32_t in_s[4], in_o[4], in_p[4][4], in_f[4][4], pat_s[4];
  FastDiv in_div[4];
  uint32_t out_s[4], out_o[4], out_p[4][4];
  FastDiv out_div[4];
  const float* x;
  float* y;
  const float* c;      // nullable (SUM)
};

// Generic adjoint: gx by atomic scatter-add, weight gradient by partials.
struct GenericAdjArgs {
  int32_t rep_rank;
  int64_t rep_shape[kMaxRank];
  int64_t n_rep;
  int64_t n_pat;
  int64_t n_q;         // output pattern elements (c is [n_q][n_pat])
  GTiler in;
  GTiler out;
  const float* x;
  const float* gy;
  float* gx;
  const float* c;      // nullable (SUM)
};

struct GenericCoefGradArgs {
  int32_t rep_rank;
  int64_t rep_shape[kMaxRank];
  int64_t n_rep;
  int64_t n_pat;       // input pattern elements
  int64_t n_q;         // output pattern elements; partial rows are [n_q n_pat][gridDim.x]
  GTiler in;
  GTiler out;
  const float* x;
  const float* gy;
  float* partial;      // [n_pat][gridDim.x]
  int64_t chunk;       // repetitions per block
};

// Dense matrix product recognised from DOT tilers: C[M,N] = A . B with
// A element (m,k) at a + m*lda_m + k*lda_k and B element (k,n) at
// b + k*ldb_k + n*ldb_n (one stride of each pair is 1).
struct GemmArgs {
  int32_t M, N, K;
  int64_t a_sm, a_sk;   // strides of A along m and k
  int64_t b_sk, b_sn;   // strides of B along k and n
  int64_t c_sm;         // row stride of C (column stride 1)
  const void* a;
  const void* b;
  float* c;
};

// 2-D k x k window with stride s along rows and columns of [frames, H, W]
// (identity along frames), identity output [frames, RH, RW].
struct Filter2DProblem {
  int32_t H, W;           // input array (per frame)
  int32_t RH, RW;         // output (repetition) shape per frame
  int32_t oh, ow;         // origin reduced into [0, H), [0, W)
  int32_t k, s;           // pattern side (3, 5, 7, 9), paving stride (1, 2, 4)
  int32_t tc;             // tile class (0..2)
  int32_t tile_h, tile_w; // outputs per tile
  int32_t tiles_w;        // tiles along a row of outputs
  int32_t tiles_per_frame;
  int32_t frames;
  int64_t n_tiles;        // tiles of this problem
  const float* x;
  float* y;
  const float* c;         // k*k weights, row-major
};

// CSR sparse matrix-vector product (indirect tilers).
struct CsrArgs {
  int64_t n_rows;
  int64_t n_cols;
  int64_t nnz;
  const int32_t* row_ptr;   // n_rows + 1
  const int32_t* col_idx;   // nnz
  const void* vals;         // nnz (FP32 or FP64)
  const void* x;            // n_cols
  void* y;                  // n_rows
};

// Device-resident state of one conjugate-gradient solve (library workspace).
struct CgState {
  double rho[2];       // rho_k = <r_k, r_k> in slot k mod 2 (written by cg_spmv)
  double bnorm;        // ||b||                     (written once at start)
  int64_t k;           // iterations completed      (written by cg_xr)
  int64_t k_spmv;      // iteration of the last cg_spmv (written by cg_spmv)
  int32_t done;        // stop test fired           (written by cg_spmv)
  int32_t breakdown;   // <p, A p> <= 0 was met     (written by cg_xr)
};

struct CgArgs {
  int64_t n, nnz;
  const int32_t* row_ptr;   // n + 1
  const int32_t* col_idx;   // nnz
  const double* vals;       // nnz
  const double* b;          // n
  double* x;                // n: x0 in, iterate out
  double* r;                // n, workspace
  double* p0;               // n, workspace: directions p_k of even k
  double* p1;               // n, workspace: directions p_k of odd k (p_{-1} = 0)
  double* q;                // n, workspace
  double* part_pq;          // grid_rows, workspace
  double* part_rr;          // max(grid_rows, grid_vec), workspace
  double* part_bb;          // grid_rows, workspace
  CgState* st;              // workspace
  double* res;              // nullable, max_iter + 1
  double* alpha;            // nullable, max_iter
  double* beta;             // nullable, max_iter
  double tol;
  int64_t max_iter;
  int32_t grid_rows;        // workgroups of the sparse-product kernels (cg_init, cg_spmv)
  int32_t grid_vec;         // workgroups of the vector kernel (cg_xr)
};

// ---------------------------------------------------------------------------
// launchers (return hipError_t of the launch)
// ---------------------------------------------------------------------------
hipError_t launch_indices(const GTiler& t, int rep_rank, const int64_t* rep_shape,
                          int64_t n_rep, int64_t n_pat, int64_t* d_idx, hipStream_t st);
hipError_t launch_generic(const GenericArgs& a, int max_rank, int in_dtype, int out_dtype,
                          int kind, int elem_bytes, hipStream_t st);
hipError_t launch_pattern_reduce(const PatternReduceArgs& a, int max_rank, hipStream_t st);
// The 32-bit form of the same kernel when the task fits it (false: use
// launch_pattern_reduce).
bool pattern_reduce_small_args(const PatternReduceArgs& a, PatternReduceSmallArgs* s);
hipError_t launch_pattern_reduce_small(const PatternReduceSmallArgs& a, hipStream_t st);
hipError_t launch_fir(const FirArgs& a, bool vec4, hipStream_t st);
hipError_t launch_fir_chain(const FirChainArgs& a, bool vec4, hipStream_t st);
hipError_t launch_fir_adjoint(const FirAdjArgs& a, bool vec4, int* grid_out, hipStream_t st);
hipError_t launch_fir_gx_gather(const FirGatherArgs& a, hipStream_t st);
hipError_t launch_fir_adjoint_overlap_cols(const FirOverlapArgs& a, hipStream_t st);
int fir_overlap_cols_grid(uint32_t n_items, int p);
int fir_adjoint_grid(const FirAdjArgs& a);
hipError_t launch_fir_chain_adjoint(const FirChainAdjArgs& a, bool vec4, hipStream_t st);
int fir_chain_adjoint_grid(const FirChainAdjArgs& a, bool vec4);
hipError_t launch_reduce_partial_pair(const float* partial, int n_blocks, int n0, float* out0, int n1,
                                      float* out1, int row_stride, int accumulate, hipStream_t st);
hipError_t launch_reduce_partials(const float* partial, int n_blocks, int n_coef, int row_stride,
                                  float* out, int accumulate, hipStream_t st);
hipError_t launch_generic_adjoint(const GenericAdjArgs& a, int max_rank, hipStream_t st);
hipError_t launch_generic_coef_grad(const GenericCoefGradArgs& a, int max_rank, int n_blocks,
                                    hipStream_t st);
hipError_t launch_reduce_rows(const float* partial, int64_t n_rows, int64_t n_cols,
                              float* out, int accumulate, hipStream_t st);
hipError_t launch_zero(void* p, int64_t bytes, hipStream_t st);
bool poly_supported(const Win3& w, int q);
bool poly_gc_supported(const Win3& w, int q);
int poly_chunks(const Win3& w);
hipError_t launch_poly(const PolyArgs& a, hipStream_t st);
// Columns form with the window read as 16-byte vectors (one thread per
// repetition); x may be null when planning without an array.
bool poly_cols_vec_ok(const Win3& w, int q, const void* x);
hipError_t launch_poly_cols_vec(const PolyArgs& a, hipStream_t st);
hipError_t launch_poly_gx_gather(const PolyGatherArgs& a, hipStream_t st);
int poly_gc_grid(uint32_t n_rep);
hipError_t launch_poly_gc(const PolyArgs& a, hipStream_t st);
bool poly_adj_cols_supported(const Win3& w, int q);
int poly_adj_cols_grid(const Win3& w, int q, uint32_t n_items);   // workgroups = partial rows
hipError_t launch_poly_adj_cols(const PolyAdjArgs& a, hipStream_t st);
int64_t gemm_lds_bytes_per_operand(const GemmArgs& g, int compute);   // LDS per workgroup, one operand
int gemm_tile_side(const GemmArgs& g, int compute);                   // output tile side (128 or 256)
hipError_t launch_gemm(const GemmArgs& a, int compute, hipStream_t st);
const char* gemm_variant_name(const GemmArgs& a, int compute);
bool gemm_supported(const GemmArgs& a, int compute);
hipError_t launch_filter2d(const Filter2DProblem& p, hipStream_t st);
hipError_t launch_csr(const CsrArgs& a, int dtype, hipStream_t st);
int csr_group_size(int64_t n_rows, int64_t nnz);
// forward + loss gradient + adjoint of a fused 8-tap pair (vec4 layout only);
// same grid and partial rows as launch_fir_chain_adjoint
hipError_t launch_fir_chain_train(const FirChainAdjArgs& a, hipStream_t st);
// Training step of an injective pair with any tap counts (<= 16 per stage):
// one thread per output; partial rows [grid][h.taps + v.taps].
int fir_chain_train_generic_grid(const FirChainAdjArgs& a);
hipError_t launch_fir_chain_train_generic(const FirChainAdjArgs& a, hipStream_t st);
// dL/dy = 2 (w y) of the loss sum(w y^2), elementwise over n values
hipError_t launch_loss_grad(const float* y, const float* w, float* g, int64_t n, hipStream_t st);

// The training step behind rsm_run_chain_train.  With fixed_partial set, the
// weight-gradient partial rows go to that device buffer of fixed_bytes
// (RSM_E_UNSUPPORTED if they need more) instead of the stream's workspace, so
// the call allocates nothing.
rsm_status chain_train_step(const rsm_stage* stages, int32_t n_stages, const void* d_in, const void* d_w,
                            void* d_out, void* d_gx, void* const* d_gc, uint32_t flags, void* hip_stream,
                            float* fixed_partial, size_t fixed_bytes);
// init: r = b - A x, p = r, fresh state; then `iters` loop iterations
hipError_t launch_cg(const CgArgs& a, bool init, int iters, hipStream_t st);
int cg_grid(int64_t n, int64_t nnz);
int cg_vec_grid(int64_t n);
// d_tiles: n_tiles entries of two uint32 (problem index, tile within the
// problem); buf_floats: the LDS buffer, at least filter2d_buf_floats() of
// every problem's tile class
hipError_t launch_filter2d_persistent(const Filter2DProblem* d_probs, const void* d_tiles, int64_t n_tiles,
                                      int grid, int buf_floats, hipStream_t st);
int filter2d_persistent_grid(int buf_floats);
int filter2d_buf_floats(int k, int s, int tc);
bool filter2d_supported(int k, int s);
void filter2d_set_tiles(Filter2DProblem* p, int tc);
size_t filter2d_lds_bytes(int k, int s, int tc);

// Planner hook shared with the batch: true when (rep, in, out, task) is a
// k x k weighted window the 2-D filter kernels handle; fills everything in
// *fp except the tile class.
bool plan_filter2d(const rsm_space& rep, const rsm_tiler& in, const rsm_tiler& out,
                   const rsm_task& task, Filter2DProblem* fp);

// Device workspace owned by the library, one per (device, stream), grown on
// demand (never while the stream is being captured: RSM_E_UNSUPPORTED).
// *counter (if given) receives a 32-bit completion counter that is zero
// between kernels (kernels that use it leave it at zero).
void* workspace(size_t bytes, hipStream_t st, rsm_status* err, uint32_t** counter = nullptr);

// Weight-gradient reduction of the adjoint kernels: true = the last workgroup
// reduces in the same launch, false = a second small kernel reduces.
bool reduce_in_kernel();

// Error reporting: sets the thread-local detail string and returns s.
rsm_status fail(rsm_status s, const std::string& msg);
rsm_status hip_fail(hipError_t e, const char* what);

}  // namespace rsm
