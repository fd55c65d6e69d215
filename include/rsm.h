/*
 * rsm.h -- C-ABI of librsm: RSM repetitive tasks on one MI355X (gfx950).
 *
 * A repetitive task (MARTE Repetitive Structure Modeling; the paper relies on
 * it for its repetitive operations, Sec. 3 and Sec. 7, and on its Shaped
 * multiplicity for the repetition space, Sec. 6.1) is
 *
 *   for every r in the repetition space (shape s_r, row-major):
 *     pat_t(r)[i] = A_t[ (o_t + P_t r + F_t i) mod s_t ]      gather, per input tiler t
 *     y(r)        = task(pat_1(r), pat_2(r))                  elementary task
 *     B[ (o_b + P_b r + F_b j) mod s_b ] = y(r)[j]            scatter, output tiler
 *
 * The modulo is componentwise and floored (results in [0, s_d) also for
 * negative operands).  Arrays are dense and row-major (dimension 0 slowest).
 * P has one column per repetition dimension and F one column per pattern
 * dimension; both are stored row-major with leading dimension RSM_MAX_RANK:
 * entry (d, k) is at [d][k].
 *
 * The buffer descriptor follows the paper's DataAllocate class (Sec. 5):
 * baseAddress -> device pointer, dimAllocation -> array_shape,
 * typeAllocation -> dtype, spaceAddress -> always device global memory (HBM).
 * Port direction (Sec. 6.3) maps to const pointers for inputs.
 *
 * Conventions for every call below:
 *  - Ownership: the caller owns every buffer passed in.  The library owns only
 *    opaque handles (rsm_batch) and internal device workspaces, one per
 *    (device, stream), grown on demand (weight-gradient partial rows of the
 *    adjoints, unfused chain intermediates, transposed matrix operands, CG
 *    vectors); descriptor structs are copied at call time.  Calls on one
 *    stream share that stream's workspace (the stream orders them); calls on
 *    different streams use different workspaces and may run concurrently.
 *    Growing a workspace synchronises its stream and allocates; while the
 *    stream is being captured into a graph that is impossible, and the call
 *    returns RSM_E_UNSUPPORTED instead (make the same call once before
 *    capturing).
 *  - Streams: compute calls are asynchronous on the given hipStream_t (NULL =
 *    the null stream).  Errors detectable on the host are returned before any
 *    launch, with nothing written.  A failed HIP call returns RSM_E_HIP; the
 *    detail is in rsm_last_error().
 *  - Output elements that the output tiler does not reach are left untouched.
 *    Calls whose output tiler writes an element twice race on it; request
 *    RSM_CHECK_SINGLE_ASSIGN to have the host reject such tilers.
 *  - No C++ exception crosses this interface.
 */
#ifndef RSM_H
#define RSM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define RSM_MAX_RANK 8
#define RSM_ABI_VERSION 1

typedef enum {
  RSM_OK = 0,
  RSM_E_INVALID = 1,     /* null pointer, bad enum, inconsistent arguments     */
  RSM_E_RANK = 2,        /* a rank outside [0, RSM_MAX_RANK]                    */
  RSM_E_SHAPE = 3,       /* non-positive extent, shapes that do not agree       */
  RSM_E_OVERFLOW = 4,    /* index arithmetic would not fit in 62 bits           */
  RSM_E_OVERLAP = 5,     /* output tiler writes an element twice (when checked) */
  RSM_E_UNSUPPORTED = 6, /* valid request that no kernel of the library handles */
  RSM_E_HIP = 7,         /* a HIP runtime call failed                           */
  RSM_E_NOMEM = 8        /* device or host allocation failed                    */
} rsm_status;

typedef enum { RSM_F32 = 0, RSM_BF16 = 1, RSM_F64 = 2, RSM_I64 = 3 } rsm_dtype;

typedef enum {
  RSM_TASK_COPY = 0, /* y(r)[j] = pat(r)[j]; |in pattern| == |out pattern|, same dtype */
  RSM_TASK_SUM = 1,  /* y(r) = sum_i pat(r)[i]                                         */
  RSM_TASK_WSUM = 2, /* y(r)[j] = sum_i c[j][i] pat(r)[i]; c is [|out pattern|][|in
                        pattern|] (one row of taps per output element; with a scalar
                        output pattern simply pattern-shaped)                           */
  RSM_TASK_DOT = 3   /* y(r) = sum_i pat_1(r)[i] pat_2(r)[i]; two input tilers         */
} rsm_task_kind;

/* Flags. */
#define RSM_CHECK_SINGLE_ASSIGN 0x1u /* host check: no output element written twice   */
#define RSM_ACCUMULATE 0x2u          /* adjoint: add into gx / gc instead of overwrite */
#define RSM_NO_FUSE 0x4u             /* chains: run stages one by one                  */
#define RSM_FORCE_GENERIC 0x8u       /* use the generic gather kernel (any tiler)      */
#define RSM_PLAN_ADJOINT 0x20u       /* rsm_plan: name the adjoint's kernel family      */
#define RSM_REDUCE_IN_KERNEL 0x80u   /* adjoint: weight gradients summed by the last    */
                                     /* workgroup of the same launch (tap kernels; one  */
                                     /* launch, but slower than the default second one) */

/* Repetition space: the Shaped multiplicity of the repeated task. rank 0 = one repetition. */
typedef struct {
  int32_t rank;
  int32_t reserved;
  int64_t shape[RSM_MAX_RANK];
} rsm_space;

/* One array and the tiler that reads or writes it. */
typedef struct {
  int32_t array_rank;                              /* d_a                              */
  int32_t dtype;                                   /* rsm_dtype of the array elements  */
  int64_t array_shape[RSM_MAX_RANK];               /* s (all > 0)                      */
  int32_t pattern_rank;                            /* d_p; 0 = scalar pattern          */
  int32_t reserved;
  int64_t pattern_shape[RSM_MAX_RANK];             /* s_p (all > 0)                    */
  int64_t origin[RSM_MAX_RANK];                    /* o, any sign                      */
  int64_t paving[RSM_MAX_RANK][RSM_MAX_RANK];      /* P: [d][k], d < d_a, k < d_r      */
  int64_t fitting[RSM_MAX_RANK][RSM_MAX_RANK];     /* F: [d][k], d < d_a, k < d_p      */
} rsm_tiler;

/* Elementary task. */
typedef struct {
  int32_t kind;        /* rsm_task_kind                                                 */
  int32_t compute;     /* RSM_F32: FP32 arithmetic (F32 arrays, or BF16 arrays widened);
                          RSM_BF16: BF16 products with FP32 accumulation (DOT on BF16
                          arrays: the matrix-core path); RSM_F64: FP64 arrays             */
  const void* coeffs;  /* WSUM: device pointer, [|out pattern|][|in pattern|] row-major,
                          FP32 (FP64 if compute is RSM_F64); ignored otherwise          */
} rsm_task;

/* One stage of a chain: stage k reads array k and writes array k+1. */
typedef struct {
  rsm_space rep;
  rsm_tiler in;
  rsm_tiler out;
  rsm_task task;
} rsm_stage;

/*
 * rsm_validate -- host-only check of a task description (no device access).
 * Checks ranks, extents, dtypes, task/pattern agreement, 62-bit index range,
 * and with RSM_CHECK_SINGLE_ASSIGN that the output tiler writes each element
 * at most once (costs O(|s_r| |s_p|) host time and |s_out| bytes of memory).
 */
rsm_status rsm_validate(const rsm_space* rep, const rsm_tiler* in, int32_t n_in,
                        const rsm_tiler* out, const rsm_task* task, uint32_t flags);

/*
 * rsm_plan -- name of the kernel family the planner picks for a task
 * (e.g. "fir_cols_vec4", "filter2d_k5_s2", "pattern_reduce", "gemm_mfma_bf16_nn",
 * "generic").  With RSM_PLAN_ADJOINT in flags (n_in = 1): the family
 * rsm_run_adjoint picks for the task's input gradient ("fir_adjoint",
 * "fir_adjoint_vec4", "fir_adjoint_overlap_cols", "fir_adjoint_gather" or
 * "generic_adjoint"), decided from shapes alone (16-byte aligned buffers
 * assumed).
 * Host only.  Writes a NUL-terminated string of at most len bytes.
 */
rsm_status rsm_plan(const rsm_space* rep, const rsm_tiler* in, int32_t n_in,
                    const rsm_tiler* out, const rsm_task* task, uint32_t flags,
                    char* name, int32_t len);

/*
 * rsm_plan_ports -- where the planned kernel keeps each port's working set,
 * in the memory spaces of the paper's platform model (the MemoryMapping of
 * Sec. 5-6, which maps every flowPort to an OpenCL address space) as they
 * exist on gfx950.  One entry per port, in order: inputs 0 .. n_in - 1,
 * the output, then (WSUM only) the coefficients.  `space` is where a
 * workgroup holds the port's data while it computes; `bytes_per_workgroup`
 * is how much of it one workgroup holds there (0: the port is streamed
 * through registers element by element, nothing is staged).  Host only;
 * decided from shapes alone, like rsm_plan.  Writes min(max_ports, count)
 * entries and the count to *n_ports (RSM_E_INVALID if ports is too short).
 */
typedef enum {
  RSM_MEM_GLOBAL = 0,    /* device memory (HBM): read or written in place, per element */
  RSM_MEM_CONSTANT = 1,  /* uniform across the workgroup: scalar registers / scalar cache */
  RSM_MEM_LOCAL = 2,     /* LDS: staged once per workgroup, shared by its threads */
  RSM_MEM_PRIVATE = 3    /* per-thread registers (VGPR / AGPR) */
} rsm_mem_space;

typedef struct {
  int32_t port;                 /* 0 .. n_in - 1 inputs, n_in output, n_in + 1 coefficients */
  int32_t is_output;            /* 1 for the output port */
  int32_t space;                /* rsm_mem_space */
  int32_t reserved;
  int64_t bytes_per_workgroup;
} rsm_port_placement;

rsm_status rsm_plan_ports(const rsm_space* rep, const rsm_tiler* in, int32_t n_in,
                          const rsm_tiler* out, const rsm_task* task, uint32_t flags,
                          rsm_port_placement* ports, int32_t max_ports, int32_t* n_ports);

/*
 * Placement as a decision.  The paper's MemoryMapping model gives every
 * flowPort a DataAllocate whose spaceAddress is one of the OpenCL address
 * spaces global, constant, local, private (Sec. 5), and the port's
 * direction decides what is read-only (Sec. 6).  `spaces` is such a request
 * for one task: a HOST array of n_spaces entries, one rsm_mem_space per port
 * in port order (inputs 0 .. n_in - 1, the output, then the coefficients of
 * a WSUM task), RSM_MEM_ANY where the caller leaves the choice open; NULL =
 * no request at all.  The planner takes, among the kernel families that can
 * run the task, the first in its order of preference whose placement meets
 * every requested space.  For example the taps of a 1-D weighted sum may be
 * kept in registers with the weights in scalar registers (input private,
 * weights constant), or the window staged in LDS with the weights in LDS
 * (input, output and weights local), or everything read in place (global);
 * overlapping column windows on a common 16-byte phase, and polyphase
 * stages along columns, may also read each window straight into registers
 * with the weights in registers (input private, output global, weights
 * private);
 * a k x k window keeps its tile in LDS with its weights in constant memory,
 * or, for at most 64 pattern elements, one element per lane in registers
 * (weights in registers too); a matrix product stages both operands
 * in LDS and accumulates in registers.
 * Errors: RSM_E_INVALID for a malformed request (wrong count, unknown space,
 * the output port in constant memory: it is written); RSM_E_UNSUPPORTED when
 * no family of the library meets the request (e.g. an input array in
 * constant memory, or 81 elements of a 9 x 9 window in registers).
 *
 * rsm_plan_placed -- host only: the family that honours the request (name,
 * nullable, of at most len bytes) and its placement of every port (ports,
 * nullable, as rsm_plan_ports; *n_ports = port count).
 * rsm_run_placed -- rsm_run with the request: runs the family
 * rsm_plan_placed names.  With spaces NULL both behave as rsm_plan /
 * rsm_plan_ports and rsm_run.
 */
#define RSM_MEM_ANY (-1)

rsm_status rsm_plan_placed(const rsm_space* rep, const rsm_tiler* in, int32_t n_in,
                           const rsm_tiler* out, const rsm_task* task, uint32_t flags,
                           const int32_t* spaces, int32_t n_spaces, char* name, int32_t len,
                           rsm_port_placement* ports, int32_t max_ports, int32_t* n_ports);

rsm_status rsm_run_placed(const rsm_space* rep, const rsm_tiler* in, const void* const* d_in,
                          int32_t n_in, const rsm_tiler* out, void* d_out, const rsm_task* task,
                          const int32_t* spaces, int32_t n_spaces, uint32_t flags, void* hip_stream);

/*
 * rsm_indices -- the index table of one tiler (the index step of the
 * definition above): d_idx[r * |s_p| + i] = linear offset of e(r, i) in the
 * tiler's array, int64, r and i flat row-major.  d_idx is a device buffer of
 * |s_r| * |s_p| int64 elements.
 */
rsm_status rsm_indices(const rsm_space* rep, const rsm_tiler* t, int64_t* d_idx,
                       void* hip_stream);

/*
 * rsm_run -- one repetitive task.  d_in is a HOST array of n_in DEVICE
 * pointers (one per input tiler, in order); d_out is the output array.
 * Task/dtype combinations: COPY any dtype (bit-exact, output dtype = input
 * dtype); SUM/WSUM on F32 or BF16 arrays computed in FP32 (F64 in FP64) with
 * an F32 (F64) output; DOT on two F32 arrays (FP32), two BF16 arrays (compute
 * BF16: FP32 accumulation, F32 output) or two F64 arrays.  SUM and DOT
 * need a single-element output pattern (RSM_E_SHAPE otherwise); WSUM may
 * write an output pattern of any size (the elementary task producing a
 * pattern, as in a polyphase filter: each repetition writes q outputs, each
 * from its own row of taps).
 */
rsm_status rsm_run(const rsm_space* rep, const rsm_tiler* in, const void* const* d_in,
                   int32_t n_in, const rsm_tiler* out, void* d_out, const rsm_task* task,
                   uint32_t flags, void* hip_stream);

/*
 * Validation and planning (the host side of a call: checking the descriptors
 * against Sec. 6.1's shaped repetition space and the tiler definition above,
 * then choosing a kernel family and its launch shape) cost microseconds per
 * call, which a small task feels.  Two ways avoid repeating them:
 *
 *  - rsm_run keeps, per host thread, the last 32 descriptors it validated
 *    successfully together with their plans; a call whose descriptors
 *    (every entry below the ranks, the task's kind and compute type, whether
 *    weights are given, the flags, and whether each input starts on a
 *    16-byte boundary) equal a kept one is launched directly.
 *    rsm_plan_cache_hits() counts such calls on the calling thread.
 *
 *  - rsm_prepare validates and plans one task once and returns an opaque
 *    handle that the library owns until rsm_prepared_destroy (NULL is
 *    ignored).  rsm_run_prepared then takes only the arrays: d_in a HOST
 *    array of n_in DEVICE pointers, d_out, and for a WSUM task the DEVICE
 *    weights d_coeffs (NULL: RSM_E_INVALID; ignored for other tasks; the
 *    task's own coeffs field is ignored by rsm_prepare).  The arrays must
 *    have the shapes and dtypes the descriptors state, as for rsm_run.  The
 *    plan assumes inputs starting on 16-byte boundaries; a call with other
 *    addresses plans again for them (same results, host cost of rsm_run).
 *    flags: RSM_CHECK_SINGLE_ASSIGN (checked once, at rsm_prepare) and
 *    RSM_FORCE_GENERIC; any other flag is RSM_E_INVALID.  A handle is read
 *    only after creation: calls on different streams or threads may share it.
 *    rsm_prepared_name writes the planned family (at most len bytes).
 */
typedef struct rsm_prepared_s* rsm_prepared;

uint64_t rsm_plan_cache_hits(void);

rsm_status rsm_prepare(const rsm_space* rep, const rsm_tiler* in, int32_t n_in, const rsm_tiler* out,
                       const rsm_task* task, uint32_t flags, rsm_prepared* handle);

rsm_status rsm_prepared_name(const struct rsm_prepared_s* handle, char* name, int32_t len);

rsm_status rsm_run_prepared(const struct rsm_prepared_s* handle, const void* const* d_in, void* d_out,
                            const void* d_coeffs, void* hip_stream);

void rsm_prepared_destroy(rsm_prepared handle);

/*
 * rsm_run_chain -- n_stages single-input tasks where stage k's output array
 * is stage k+1's input array (stage k's out tiler and stage k+1's in tiler
 * describe the same array).  d_mid is a HOST array of n_stages-1 DEVICE
 * pointers for the intermediate arrays.  When the planner can fuse two
 * consecutive weighted-sum stages (1-D patterns along different axes, identity
 * output tilers) and d_mid is NULL or d_mid[k] is NULL, the intermediate is
 * never written to memory.  Otherwise the stages run one by one: into the
 * given d_mid[k] (written; elements a stage's output tiler does not cover
 * keep their contents), or, when d_mid or one of its entries is NULL, into
 * intermediate arrays in the library's workspace, zero-filled first.
 * RSM_NO_FUSE forces stage-by-stage execution.
 */
rsm_status rsm_run_chain(const rsm_stage* stages, int32_t n_stages, const void* d_in,
                         void* const* d_mid, void* d_out, uint32_t flags, void* hip_stream);

/*
 * rsm_run_adjoint -- adjoint of a SUM task (scalar output pattern) or of a
 * WSUM task with any output pattern (the task is linear in its input and in
 * its weights):
 *   gx[e_in(r,i)] = sum over (r,i,j) with e_in(r,i) hitting it of c[j][i] * gy[e_out(r,j)]
 *   gc[j][i]      = sum_r gy[e_out(r,j)] * x[e_in(r,i)]
 * (j = 0 only for a scalar output pattern; d_gc is shaped like the
 * coefficients).  A WSUM whose output pattern of q elements lies along the
 * tap axis of a 1-D window (a polyphase stage: q consecutive outputs per
 * window) takes a gather for gx and per-repetition partial sums for gc.
 * d_x: the task's input array (needed for gc only; may be NULL if d_gc is
 * NULL).  d_gy: gradient w.r.t. the output array.  d_gx (input-array shaped)
 * and d_gc (pattern-shaped, WSUM only) are FP32 device buffers, each NULL to
 * skip it.  Without RSM_ACCUMULATE they are overwritten (gx elements no
 * repetition reads become 0); with it the result is added.  The weight
 * gradient is reduced deterministically (fixed-order tree).  gx is
 * deterministic on the tap-tiler paths (with RSM_REDUCE_IN_KERNEL the
 * weight gradient is summed by the launch's last workgroup, in the same
 * order: the same bits): a plain store per element where no
 * element is read twice, and a gather over the (repetition, tap) pairs that
 * reach each element, in a fixed order, where 1-D windows overlap or wrap
 * onto each other; only the generic path for other tilers whose reads
 * overlap adds with atomics.
 */
rsm_status rsm_run_adjoint(const rsm_space* rep, const rsm_tiler* in, const void* d_x,
                           const rsm_tiler* out, const void* d_gy, const rsm_task* task,
                           void* d_gx, void* d_gc, uint32_t flags, void* hip_stream);

/*
 * rsm_run_chain_adjoint -- adjoint of a chain of SUM/WSUM stages.
 * d_in: the chain's input array; d_mid: forward intermediates (HOST array of
 * DEVICE pointers).  d_mid may be NULL (or hold a NULL entry): a fused pair
 * recomputes the intermediate on chip, and a chain run stage by stage first
 * recomputes every intermediate into the library's workspace (zero-filled,
 * as rsm_run_chain does without d_mid).  d_gy: gradient w.r.t. the last
 * output; d_gx: gradient w.r.t. d_in (nullable); d_gc: HOST array of
 * n_stages DEVICE pointers to per-stage weight gradients (array nullable,
 * entries nullable).
 */
rsm_status rsm_run_chain_adjoint(const rsm_stage* stages, int32_t n_stages, const void* d_in,
                                 const void* const* d_mid, const void* d_gy, void* d_gx,
                                 void* const* d_gc, uint32_t flags, void* hip_stream);

/*
 * rsm_run_chain_train -- one training step of a two-stage chain under the
 * loss L = sum over output elements o of w[o] * y[o]^2 (y the chain's output):
 * the forward (Sec. 3 and 6.1 repetitive tasks chained, as rsm_run_chain),
 * dL/dy = 2 (w y), and the adjoint of both stages (as rsm_run_chain_adjoint).
 * d_w: loss weights, FP32, shaped like the output array; d_out: receives y;
 * d_gx (nullable): dL/dx, input-shaped; d_gc (HOST array of 2 DEVICE
 * pointers, nullable, entries nullable): the stages' weight gradients.
 * RSM_ACCUMULATE adds into d_gx and d_gc.  Stages: FP32 SUM or WSUM tasks
 * (single-stage adjoints as rsm_run_adjoint).  A pair of weighted sums along
 * columns then rows whose windows do not overlap (at most 16 taps each, any
 * alignment and origin) runs fused in one pass over the input: d_in is read
 * once and dL/dy is formed in registers, never stored (8 taps per stage on
 * 16-byte aligned rows take a lane-pair kernel).  Every other chain
 * (overlapping windows, multi-element output patterns, other tilers; or any
 * chain with RSM_NO_FUSE / RSM_FORCE_GENERIC) runs stage by stage: the
 * forward into a workspace intermediate and d_out, dL/dy into the
 * workspace, then the adjoint of each stage in reverse.  Chains of other
 * than two stages return RSM_E_UNSUPPORTED.  Weight gradients are reduced in
 * a fixed order (deterministic).
 */
rsm_status rsm_run_chain_train(const rsm_stage* stages, int32_t n_stages, const void* d_in, const void* d_w,
                               void* d_out, void* d_gx, void* const* d_gc, uint32_t flags, void* hip_stream);

/*
 * rsm_run_chain_train_noalloc -- rsm_run_chain_train for callers that cannot
 * allocate device memory: code being captured into a graph, tight serving
 * loops, harnesses that forbid hipMalloc.  Same arguments, results (the
 * same kernels: the same bits) and errors as rsm_run_chain_train for the
 * chains it runs fused in one pass; chains that rsm_run_chain_train runs
 * stage by stage need workspace and return RSM_E_UNSUPPORTED here.  The
 * weight-gradient partial rows live in a fixed 256 KiB array of device
 * memory inside the library instead of the stream's workspace, so the call
 * never allocates (no hipMalloc, hipFree or allocating library routine); a
 * step whose partial rows would not fit returns RSM_E_UNSUPPORTED.  Every device holds its own copy of the array
 * until the process ends, and every call on a device shares that copy (it
 * keeps the last call's contents; nothing in it needs to start at zero):
 * calls that may overlap on one device -- on different streams, or from
 * different host threads without ordering -- race on it and must not be
 * made.  The first call on each device looks up the array's address there.
 */
rsm_status rsm_run_chain_train_noalloc(const rsm_stage* stages, int32_t n_stages, const void* d_in,
                                       const void* d_w, void* d_out, void* d_gx, void* const* d_gc,
                                       uint32_t flags, void* hip_stream);

/*
 * rsm_run_csr -- the repetitive task with data-dependent (indirect) tilers
 * that the paper's conjugate-gradient case study runs on the GPU (Sec. 7,
 * the sparse DGEMV): for every row r of a CSR matrix the pattern is the
 * row's stored entries, read through a contiguous tiler on d_vals and an
 * indirect tiler (fitting given by d_col_idx) on d_x; the task is DOT and the
 * output tiler is the identity on d_y:
 *     y[r] = sum over k in [row_ptr[r], row_ptr[r+1]) of vals[k] * x[col_idx[k]]
 * d_row_ptr: n_rows + 1 int32, d_col_idx: nnz int32 (device buffers);
 * d_vals (nnz), d_x (n_cols), d_y (n_rows): dtype RSM_F64 or RSM_F32.  Row
 * bounds outside [0, nnz] are clamped and column indices outside [0, n_cols)
 * contribute nothing, so malformed input cannot fault; with
 * RSM_CHECK_INDICES the host copies the index arrays and rejects them
 * (RSM_E_INVALID) instead.  Limits: n_rows, n_cols, nnz < 2^31.
 */
#define RSM_CHECK_INDICES 0x10u
#define RSM_NO_GRAPH 0x40u   /* rsm_cg_solve: launch iteration batches directly, no graph replay */
rsm_status rsm_run_csr(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t* d_row_ptr,
                       const int32_t* d_col_idx, const void* d_vals, const void* d_x, void* d_y,
                       int32_t dtype, uint32_t flags, void* hip_stream);

/*
 * rsm_cg_solve -- the conjugate-gradient loop of the paper's case study
 * (Sec. 7) on one device, FP64: every matrix-vector product is the
 * indirect-tiler task of rsm_run_csr, the inner products and vector updates
 * are element-wise repetitions, and the loop runs while the continue
 * condition ||r_k|| > tol ||b|| holds (the relative-residual rule of the
 * paper's Table 1, tol = 1e-10 there) and k < max_iter.  Recurrences
 * (Hestenes-Stiefel): r0 = b - A x0, p0 = r0; alpha = <r,r> / <p,Ap>;
 * x += alpha p; r -= alpha A p; beta = <r',r'> / <r,r>; p = r' + beta p.
 * The scalars stay on the device; the host reads a 32-byte state block after
 * every check_every iterations (so the call is BLOCKING and synchronises the
 * stream that often; iterations launched past the stop test do nothing).
 * A: n x n CSR (d_row_ptr n + 1 int32, d_col_idx nnz int32, d_vals nnz
 * FP64), symmetric positive definite.  d_b: n FP64.  d_x: n FP64, x0 on
 * entry, the last iterate on return.  d_res (max_iter + 1), d_alpha and
 * d_beta (max_iter each) are optional FP64 device buffers (NULL = skip) that
 * receive ||r_k|| and the step scalars.  info (host) receives the iteration
 * count, the final recursive residual norm, ||b||, converged and breakdown
 * (<p, A p> <= 0 met: A not positive definite; x then holds the last
 * iterate).  Inner products are reduced in a fixed order: repeated calls
 * give identical bits.  Uses the stream's library workspace (4 n + 3 * 2048
 * doubles); the captured graph is kept per device, so CG solves on one
 * device must not run concurrently.  RSM_CHECK_INDICES validates the
 * index arrays on the host first.  Each batch of check_every iterations is
 * replayed from a HIP graph that the library captures once and keeps per
 * device while the call's arguments (buffers, sizes, tol, max_iter,
 * check_every) stay the same; RSM_NO_GRAPH launches the batches directly
 * instead (the same kernels: the same bits).  The library keeps, per device,
 * one capture stream (default priority) and the last captured graph until
 * the process ends.  Limits: n, nnz < 2^31.
 */
typedef struct {
  int64_t iterations;
  double residual_norm;
  double rhs_norm;
  int32_t converged;
  int32_t breakdown;
} rsm_cg_info;

rsm_status rsm_cg_solve(int64_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col_idx,
                        const double* d_vals, const double* d_b, double* d_x, double tol,
                        int64_t max_iter, int32_t check_every, uint32_t flags, double* d_res,
                        double* d_alpha, double* d_beta, rsm_cg_info* info, void* hip_stream);

/*
 * Batched execution of many independent single-input tasks in one launch.
 * rsm_batch_create copies the descriptions, chooses a tile shape per problem
 * (timing candidates on the given stream unless the tuning cache at
 * tune_cache_path, NULL = none, already holds the choice; the cache is
 * rewritten with new choices), uploads a device descriptor table, and
 * returns an opaque handle.  Problems that the persistent kernel does not
 * handle run through rsm_run inside the same rsm_batch_run call.
 * rsm_batch_run captures one HIP graph holding the persistent launch on its
 * first call (on a private stream) and replays it on the given stream
 * afterwards; the device pointers given at create time are used every time.
 * Persistent problems: FP32 weighted-sum (WSUM) k x k windows (k in 3,5,7,9)
 * with equal row/column stride s in 1,2,4, unit fitting and an identity
 * output tiler.  Batches on one device must not run concurrently with each
 * other (each owns a private queue, but the caller's streams order replays).
 * rsm_batch_destroy frees the handle.
 */
typedef struct {
  rsm_space rep;
  rsm_tiler in;
  rsm_tiler out;
  rsm_task task;
  const void* d_in;
  void* d_out;
} rsm_problem;

typedef struct rsm_batch_s* rsm_batch;

typedef struct {
  int64_t n_problems;      /* problems in the batch                              */
  int64_t n_persistent;    /* of which handled by the persistent kernel          */
  int64_t n_tiles;         /* tiles in the persistent kernel's queue             */
  int64_t grid;            /* persistent workgroups launched                     */
  int64_t tuned_classes;   /* problem classes timed during create (cache misses) */
  int64_t cached_classes;  /* problem classes taken from the cache               */
} rsm_batch_info;

rsm_status rsm_batch_create(const rsm_problem* problems, int32_t n, const char* tune_cache_path,
                            uint32_t flags, void* hip_stream, rsm_batch* out);
rsm_status rsm_batch_run(rsm_batch b, void* hip_stream);
/* The same problems with the same tile shapes, one kernel launch per problem
 * in list order on the stream (no persistent kernel, no graph): the baseline
 * the batched launch is compared against. */
rsm_status rsm_batch_run_plain(rsm_batch b, void* hip_stream);
rsm_status rsm_batch_query(rsm_batch b, rsm_batch_info* info);
rsm_status rsm_batch_destroy(rsm_batch b); /* waits for the device, then frees */

/* Tile shape chosen for problem k of a batch (rows, cols of outputs per tile). */
rsm_status rsm_batch_tile(rsm_batch b, int32_t k, int32_t* tile_rows, int32_t* tile_cols);

/*
 * rsm_time_next_kernel -- measurement hook.  The next rsm_run_chain,
 * rsm_run_chain_adjoint or rsm_run_chain_train call made on this host thread
 * records
 * hip_event_start on its stream immediately before launching the fused
 * chain kernel and hip_event_stop immediately after it (no other launch of
 * the call lies between them), then forgets both; calls that take the
 * unfused path forget them without recording.  The events are hipEvent_t
 * handles created and owned by the caller (either may be NULL).  Passing
 * NULL, NULL disarms the hook.  Always returns RSM_OK.
 */
rsm_status rsm_time_next_kernel(void* hip_event_start, void* hip_event_stop);

/* Name of a status code; any value is accepted (unknown ones give
 * "RSM_E_UNKNOWN"), so the argument is a plain int32_t. */
const char* rsm_status_string(int32_t status);
const char* rsm_last_error(void); /* thread-local detail of the last failing call */
int32_t rsm_abi_version(void);

#ifdef __cplusplus
}
#endif

#endif /* RSM_H */
