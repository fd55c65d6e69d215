// api.cpp -- C-ABI entry points, validation and the kernel planner.
//
// Every entry point validates its descriptors on the host, reduces each
// tiler to a canonical descriptor, picks a kernel family and launches it on
// the caller's stream.  No exception leaves this file.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "rsm_internal.h"

namespace rsm {

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
static thread_local std::string g_last_error;

// Measurement hook (rsm_time_next_kernel): events recorded around the main
// kernel of the next chain call on this thread, then forgotten.
struct KernelProbe {
  hipEvent_t start = nullptr, stop = nullptr;
};
static thread_local KernelProbe g_probe;

// Takes (and disarms) the probe; every chain call does this on entry.
static KernelProbe take_probe() {
  KernelProbe p = g_probe;
  g_probe = KernelProbe{};
  return p;
}


// Launches `launch` between the probe's events (either may be absent).
template <typename F>
static hipError_t probed(const KernelProbe& p, hipStream_t st, F launch) {
  hipError_t e;
  if (p.start && (e = hipEventRecord(p.start, st)) != hipSuccess) return e;
  if ((e = launch()) != hipSuccess) return e;
  if (p.stop && (e = hipEventRecord(p.stop, st)) != hipSuccess) return e;
  return hipSuccess;
}

rsm_status fail(rsm_status s, const std::string& msg) {
  g_last_error = msg;
  return s;
}


rsm_status hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")";
  return RSM_E_HIP;
}

// ---------------------------------------------------------------------------
// workspace: one grow-only device buffer per (device, stream)
// ---------------------------------------------------------------------------
// Calls on one stream are ordered by the stream, so they may share a buffer;
// calls on different streams get different buffers and never see each
// other's partial results, intermediates or completion counter.
namespace {
struct Workspace {
  int dev = -1;
  hipStream_t stream = nullptr;
  void* ptr = nullptr;
  size_t bytes = 0;
};
std::mutex g_ws_mutex;
std::vector<Workspace> g_ws;  // one entry per (device, stream) that has used it

bool stream_capturing(hipStream_t st, rsm_status* err) {
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  const hipError_t e = hipStreamIsCapturing(st, &cs);
  if (e != hipSuccess) {
    *err = hip_fail(e, "hipStreamIsCapturing");
    return true;
  }
  return cs != hipStreamCaptureStatusNone;
}
}  // namespace

// Layout: [256 bytes: completion counter, kept at zero between kernels][data]
void* workspace(size_t bytes, hipStream_t st, rsm_status* err, uint32_t** counter) {
  *err = RSM_OK;
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    *err = hip_fail(e, "hipGetDevice");
    return nullptr;
  }
  constexpr size_t kHead = 256;
  std::lock_guard<std::mutex> lock(g_ws_mutex);
  Workspace* w = nullptr;
  for (Workspace& c : g_ws)
    if (c.dev == dev && c.stream == st) w = &c;
  if (!w) {
    g_ws.push_back(Workspace{});
    w = &g_ws.back();
    w->dev = dev;
    w->stream = st;
  }
  if (!(w->ptr && w->bytes >= bytes)) {
    // allocation is not allowed while the stream is being captured: the
    // caller runs the same call once outside capture first
    if (stream_capturing(st, err)) {
      if (*err == RSM_OK)
        *err = fail(RSM_E_UNSUPPORTED,
                    "the library workspace of this stream must grow (to " + std::to_string(bytes) +
                        " bytes), which is not possible while the stream is being captured; run the "
                        "same call once before capturing");
      return nullptr;
    }
    size_t want = bytes < (size_t(1) << 20) ? (size_t(1) << 20) : bytes;
    if (w->ptr) {
      // earlier launches on this stream may still use the old buffer
      e = hipStreamSynchronize(st);
      if (e != hipSuccess) {
        *err = hip_fail(e, "hipStreamSynchronize (workspace growth)");
        return nullptr;
      }
      (void)hipFree(w->ptr);
      w->ptr = nullptr;
      w->bytes = 0;
    }
    e = hipMalloc(&w->ptr, want + kHead);
    if (e != hipSuccess) {
      w->ptr = nullptr;
      *err = fail(RSM_E_NOMEM, std::string("workspace hipMalloc failed: ") + hipGetErrorString(e));
      return nullptr;
    }
    // zeroed on the stream itself, so the stream's next kernels see it
    e = launch_zero(w->ptr, kHead, st);
    if (e != hipSuccess) {
      *err = hip_fail(e, "zero fill (workspace counter)");
      return nullptr;
    }
    w->bytes = want;
  }
  if (counter) *counter = static_cast<uint32_t*>(w->ptr);
  return static_cast<char*>(w->ptr) + kHead;
}

// ---------------------------------------------------------------------------
// validation
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t kLimit62 = int64_t(1) << 62;

bool mul_ok(int64_t a, int64_t b, int64_t* out) {
  int64_t r;
  if (__builtin_mul_overflow(a, b, &r) || r >= kLimit62 || r <= -kLimit62) return false;
  *out = r;
  return true;
}

int64_t floor_mod(int64_t a, int64_t m) {
  int64_t q = a % m;
  return q < 0 ? q + m : q;
}

bool dtype_ok(int32_t d) { return d == RSM_F32 || d == RSM_BF16 || d == RSM_F64 || d == RSM_I64; }

int elem_size(int32_t d) {
  switch (d) {
    case RSM_F32: return 4;
    case RSM_BF16: return 2;
    case RSM_F64: return 8;
    case RSM_I64: return 8;
  }
  return 0;
}

int64_t prod(const int64_t* v, int n) {
  int64_t p = 1;
  for (int k = 0; k < n; ++k) p *= v[k];
  return p;
}

rsm_status check_space(const rsm_space* rep, int64_t* n_rep) {
  if (!rep) return fail(RSM_E_INVALID, "repetition space is NULL");
  if (rep->rank < 0 || rep->rank > RSM_MAX_RANK)
    return fail(RSM_E_RANK, "repetition rank " + std::to_string(rep->rank) + " outside [0, 8]");
  int64_t n = 1;
  for (int k = 0; k < rep->rank; ++k) {
    if (rep->shape[k] < 0)
      return fail(RSM_E_SHAPE, "negative repetition extent in dimension " + std::to_string(k));
    if (!mul_ok(n, rep->shape[k], &n))
      return fail(RSM_E_OVERFLOW, "repetition space has more than 2^62 points");
  }
  *n_rep = n;
  return RSM_OK;
}

rsm_status check_tiler(const rsm_tiler* t, const rsm_space* rep, const char* name,
                       int64_t* n_pat) {
  const std::string who(name);
  if (!t) return fail(RSM_E_INVALID, who + " tiler is NULL");
  if (t->array_rank < 0 || t->array_rank > RSM_MAX_RANK)
    return fail(RSM_E_RANK, who + ": array rank " + std::to_string(t->array_rank) + " outside [0, 8]");
  if (t->pattern_rank < 0 || t->pattern_rank > RSM_MAX_RANK)
    return fail(RSM_E_RANK, who + ": pattern rank " + std::to_string(t->pattern_rank) + " outside [0, 8]");
  if (!dtype_ok(t->dtype)) return fail(RSM_E_INVALID, who + ": unknown dtype");
  int64_t n_arr = 1;
  for (int d = 0; d < t->array_rank; ++d) {
    if (t->array_shape[d] <= 0)
      return fail(RSM_E_SHAPE, who + ": array extent " + std::to_string(d) + " is not positive");
    if (!mul_ok(n_arr, t->array_shape[d], &n_arr))
      return fail(RSM_E_OVERFLOW, who + ": array has more than 2^62 elements");
  }
  int64_t np = 1;
  for (int k = 0; k < t->pattern_rank; ++k) {
    if (t->pattern_shape[k] <= 0)
      return fail(RSM_E_SHAPE, who + ": pattern extent " + std::to_string(k) + " is not positive");
    if (!mul_ok(np, t->pattern_shape[k], &np))
      return fail(RSM_E_OVERFLOW, who + ": pattern has more than 2^62 elements");
  }
  // Reduced steps are < s_d; the walk multiplies them by indices below the
  // repetition / pattern extents and adds up to 16 such terms.
  for (int d = 0; d < t->array_rank; ++d) {
    const int64_t s = t->array_shape[d];
    int64_t tmp;
    for (int k = 0; k < rep->rank; ++k)
      if (!mul_ok(s, rep->shape[k] + 1, &tmp) || !mul_ok(tmp, 16, &tmp))
        return fail(RSM_E_OVERFLOW, who + ": paving arithmetic would exceed 62 bits");
    for (int k = 0; k < t->pattern_rank; ++k)
      if (!mul_ok(s, t->pattern_shape[k] + 1, &tmp) || !mul_ok(tmp, 16 * 64, &tmp))
        return fail(RSM_E_OVERFLOW, who + ": fitting arithmetic would exceed 62 bits");
  }
  *n_pat = np;
  return RSM_OK;
}

// e(r, i) on the host (used by the single-assignment check only)
int64_t host_offset(const rsm_tiler& t, int rep_rank, const int64_t* r, const int64_t* i) {
  int64_t lin = 0;
  for (int d = 0; d < t.array_rank; ++d) {
    const int64_t s = t.array_shape[d];
    int64_t v = floor_mod(t.origin[d], s);
    for (int k = 0; k < rep_rank; ++k) v = (v + floor_mod(t.paving[d][k], s) * r[k] % s) % s;
    for (int k = 0; k < t.pattern_rank; ++k) v = (v + floor_mod(t.fitting[d][k], s) * i[k] % s) % s;
    lin = lin * s + v;
  }
  return lin;
}

rsm_status check_single_assign(const rsm_space& rep, const rsm_tiler& out, int64_t n_rep,
                               int64_t n_pat) {
  const int64_t n_out = prod(out.array_shape, out.array_rank);
  if (n_out > (int64_t(1) << 33))
    return fail(RSM_E_UNSUPPORTED, "single-assignment check limited to 2^33 output elements");
  std::vector<uint8_t> hit(size_t(n_out), 0);
  int64_t r[RSM_MAX_RANK] = {0}, i[RSM_MAX_RANK] = {0};
  for (int64_t rf = 0; rf < n_rep; ++rf) {
    int64_t f = rf;
    for (int k = rep.rank - 1; k >= 0; --k) { r[k] = f % rep.shape[k]; f /= rep.shape[k]; }
    for (int64_t pf = 0; pf < n_pat; ++pf) {
      int64_t g = pf;
      for (int k = out.pattern_rank - 1; k >= 0; --k) { i[k] = g % out.pattern_shape[k]; g /= out.pattern_shape[k]; }
      const int64_t e = host_offset(out, rep.rank, r, i);
      if (hit[size_t(e)]) return fail(RSM_E_OVERLAP, "output tiler writes element " + std::to_string(e) + " twice");
      hit[size_t(e)] = 1;
    }
  }
  return RSM_OK;
}

struct Checked {
  int64_t n_rep = 0;
  int64_t n_pat_in[2] = {0, 0};
  int64_t n_pat_out = 0;
};

rsm_status check_task(const rsm_space* rep, const rsm_tiler* in, int32_t n_in, const rsm_tiler* out,
                      const rsm_task* task, uint32_t flags, Checked* c) {
  rsm_status s = check_space(rep, &c->n_rep);
  if (s) return s;
  if (!task) return fail(RSM_E_INVALID, "task is NULL");
  if (task->kind < RSM_TASK_COPY || task->kind > RSM_TASK_DOT)
    return fail(RSM_E_INVALID, "unknown task kind " + std::to_string(task->kind));
  if (!in) return fail(RSM_E_INVALID, "input tilers are NULL");
  const int need = task->kind == RSM_TASK_DOT ? 2 : 1;
  if (n_in != need)
    return fail(RSM_E_INVALID, "task needs " + std::to_string(need) + " input tiler(s), got " + std::to_string(n_in));
  for (int t = 0; t < n_in; ++t) {
    s = check_tiler(&in[t], rep, t ? "input 1" : "input 0", &c->n_pat_in[t]);
    if (s) return s;
  }
  s = check_tiler(out, rep, "output", &c->n_pat_out);
  if (s) return s;
  const int32_t dt = in[0].dtype;
  if (task->kind == RSM_TASK_COPY) {
    if (c->n_pat_in[0] != c->n_pat_out)
      return fail(RSM_E_SHAPE, "COPY: input and output patterns differ in size");
    if (out->dtype != dt) return fail(RSM_E_INVALID, "COPY: output dtype differs from input dtype");
  } else {
    // a weighted sum may write an output pattern (one row of taps per output
    // element); SUM and DOT produce one value per repetition
    if (c->n_pat_out != 1 && task->kind != RSM_TASK_WSUM)
      return fail(RSM_E_SHAPE, "SUM and DOT need a single-element output pattern");
    if (dt == RSM_I64) return fail(RSM_E_UNSUPPORTED, "arithmetic on int64 arrays is not supported");
    if (task->kind == RSM_TASK_DOT) {
      if (in[1].dtype != dt) return fail(RSM_E_INVALID, "DOT: the two inputs differ in dtype");
      if (c->n_pat_in[0] != c->n_pat_in[1]) return fail(RSM_E_SHAPE, "DOT: patterns differ in size");
    }
    const int32_t want_out = dt == RSM_F64 ? RSM_F64 : RSM_F32;
    if (out->dtype != want_out)
      return fail(RSM_E_INVALID, dt == RSM_F64 ? "FP64 task needs an F64 output" : "task needs an F32 output");
    if (task->compute == RSM_F64 && dt != RSM_F64)
      return fail(RSM_E_INVALID, "compute F64 needs F64 arrays");
    if (dt == RSM_F64 && task->compute != RSM_F64)
      return fail(RSM_E_INVALID, "F64 arrays need compute F64");
    if (task->compute == RSM_BF16 && (task->kind != RSM_TASK_DOT || dt != RSM_BF16))
      return fail(RSM_E_INVALID, "compute BF16 is the DOT task on BF16 arrays");
    if (task->compute != RSM_F32 && task->compute != RSM_BF16 && task->compute != RSM_F64)
      return fail(RSM_E_INVALID, "unknown compute dtype");
    if (task->kind == RSM_TASK_WSUM && !task->coeffs && c->n_rep > 0)
      return fail(RSM_E_INVALID, "WSUM needs coefficients");
  }
  if ((flags & RSM_CHECK_SINGLE_ASSIGN) && c->n_rep > 0) {
    s = check_single_assign(*rep, *out, c->n_rep, c->n_pat_out);
    if (s) return s;
  }
  return RSM_OK;
}

// ---------------------------------------------------------------------------
// canonical descriptors
// ---------------------------------------------------------------------------
GTiler to_gtiler(const rsm_tiler& t, int rep_rank) {
  GTiler g;
  std::memset(&g, 0, sizeof(g));
  g.arr_rank = t.array_rank;
  g.pat_rank = t.pattern_rank;
  for (int d = 0; d < kMaxRank; ++d) {
    g.shape[d] = d < t.array_rank ? t.array_shape[d] : 1;
    g.pat_shape[d] = d < t.pattern_rank ? t.pattern_shape[d] : 1;
  }
  for (int d = 0; d < t.array_rank; ++d) {
    const int64_t s = t.array_shape[d];
    g.origin[d] = floor_mod(t.origin[d], s);
    for (int k = 0; k < rep_rank; ++k) g.pav[d][k] = floor_mod(t.paving[d][k], s);
    for (int k = 0; k < t.pattern_rank; ++k) g.fit[d][k] = floor_mod(t.fitting[d][k], s);
  }
  return g;
}

bool is_scalar_pattern(const rsm_tiler& t) {
  for (int k = 0; k < t.pattern_rank; ++k)
    if (t.pattern_shape[k] != 1) return false;
  return true;
}

bool is_identity_out(const rsm_space& rep, const rsm_tiler& t) {
  if (t.array_rank != rep.rank) return false;
  for (int d = 0; d < rep.rank; ++d) {
    if (t.array_shape[d] != rep.shape[d] || t.origin[d] != 0) return false;
    for (int k = 0; k < rep.rank; ++k)
      if (t.paving[d][k] != (d == k ? 1 : 0)) return false;
  }
  for (int k = 0; k < t.pattern_rank; ++k)
    if (t.pattern_shape[k] != 1) return false;
  return true;
}

constexpr int64_t kI30 = int64_t(1) << 30;

// Axis-aligned view [B, R, C]; see Win3.
bool canon_win3(const rsm_space& rep, const rsm_tiler& t, Win3* w) {
  const int da = t.array_rank;
  if (da < 1 || da > 3 || rep.rank != da) return false;
  const int sh = 3 - da;
  for (int d = 0; d < 3; ++d) { w->A[d] = 1; w->rep[d] = 1; w->o[d] = 0; w->p[d] = 0; }
  int64_t total = 1;
  for (int d = 0; d < da; ++d) {
    for (int k = 0; k < da; ++k)
      if (d != k && t.paving[d][k] != 0) return false;
    if (t.paving[d][d] < 0) return false;
    if (t.array_shape[d] >= kI30 || rep.shape[d] >= kI30) return false;
    const int64_t reach = std::abs(t.origin[d]) + t.paving[d][d] * (rep.shape[d] > 0 ? rep.shape[d] : 1);
    if (reach >= kI30) return false;
    total *= t.array_shape[d];
    w->A[d + sh] = int32_t(t.array_shape[d]);
    w->rep[d + sh] = int32_t(rep.shape[d]);
    w->o[d + sh] = int32_t(t.origin[d]);
    w->p[d + sh] = int32_t(t.paving[d][d]);
  }
  if (total >= (int64_t(1) << 31)) return false;
  int64_t rtotal = int64_t(w->rep[0]) * w->rep[1] * w->rep[2];
  if (rtotal >= (int64_t(1) << 31)) return false;
  if (t.pattern_rank == 1) {
    int axis = -1;
    for (int d = 0; d < da; ++d) {
      if (t.fitting[d][0] == 0) continue;
      if (t.fitting[d][0] != 1 || axis >= 0) return false;
      axis = d + sh;
    }
    if (axis < 1) return false;
    if (t.pattern_shape[0] >= kI30) return false;
    w->ax = axis;
    w->taps = int32_t(t.pattern_shape[0]);
    w->taps2 = 1;
    return true;
  }
  if (t.pattern_rank == 2) {
    if (da < 2) return false;
    for (int d = 0; d < da; ++d)
      for (int k = 0; k < 2; ++k) {
        const int64_t want = (d + sh == 1 + k) ? 1 : 0;
        if (t.fitting[d][k] != want) return false;
      }
    if (t.pattern_shape[0] >= 4096 || t.pattern_shape[1] >= 4096) return false;
    w->ax = 0;
    w->taps = int32_t(t.pattern_shape[0]);
    w->taps2 = int32_t(t.pattern_shape[1]);
    return true;
  }
  return false;
}

// Non-tap axes must not wrap: o >= 0 and o + p (rep - 1) < A.
bool outer_axes_inside(const Win3& w, int skip_axis) {
  for (int d = 0; d < 3; ++d) {
    if (d == skip_axis) continue;
    if (w.o[d] < 0) return false;
    if (int64_t(w.o[d]) + int64_t(w.p[d]) * (w.rep[d] - 1) >= w.A[d]) return false;
  }
  return true;
}

// Each array element read by at most one repetition (1-D pattern).
bool fir_injective(const Win3& w) {
  for (int d = 0; d < 3; ++d) {
    if (d == w.ax) continue;
    if (w.rep[d] > 1 && w.p[d] < 1) return false;
  }
  return w.p[w.ax] >= w.taps && int64_t(w.p[w.ax]) * w.rep[w.ax] <= w.A[w.ax];
}

// Every array element read exactly once.
bool fir_exact_cover(const Win3& w) {
  for (int d = 0; d < 3; ++d) {
    if (d == w.ax) continue;
    if (w.rep[d] != w.A[d] || (w.A[d] > 1 && w.p[d] != 1)) return false;
  }
  return w.p[w.ax] == w.taps && int64_t(w.p[w.ax]) * w.rep[w.ax] == w.A[w.ax];
}

bool fir_vec4(const Win3& w, const void* x) {
  if (w.ax != 2) return false;
  if (w.taps % 4 || w.p[2] % 4 || floor_mod(w.o[2], 4) || w.A[2] % 4) return false;
  return x == nullptr || (reinterpret_cast<uintptr_t>(x) & 15) == 0;
}

enum class Fam { Empty, Generic, PatternReduce, Fir, Filter2D, Gemm, Poly };

struct Plan {
  bool ok = true;   // false: no family meets the requested placement
  Fam fam = Fam::Generic;
  std::string name = "generic";
  Win3 win{};
  int poly_q = 0;
  bool poly_vec = false;   // columns: window read as 16-byte vectors into registers
  bool vec4 = false;
  GemmArgs gemm{};
  Filter2DProblem f2d{};
  int max_rank = 1;
};

int max_rank_of(const rsm_space& rep, const rsm_tiler* in, int n_in, const rsm_tiler& out) {
  int m = rep.rank;
  for (int t = 0; t < n_in; ++t) {
    m = std::max(m, in[t].array_rank);
    m = std::max(m, in[t].pattern_rank);
  }
  m = std::max(m, out.array_rank);
  m = std::max(m, out.pattern_rank);
  return std::max(m, 1);
}

// A DOT task whose tilers form C[m,n] = sum_k A(m,k) B(k,n).
bool match_gemm(const rsm_space& rep, const rsm_tiler* in, const rsm_tiler& out, GemmArgs* g) {
  if (rep.rank != 2 || !is_identity_out(rep, out)) return false;
  const rsm_tiler& A = in[0];
  const rsm_tiler& B = in[1];
  if (A.array_rank != 2 || B.array_rank != 2 || A.pattern_rank != 1 || B.pattern_rank != 1) return false;
  const int64_t M = rep.shape[0], N = rep.shape[1], K = A.pattern_shape[0];
  if (B.pattern_shape[0] != K) return false;
  for (int d = 0; d < 2; ++d)
    if (A.origin[d] != 0 || B.origin[d] != 0) return false;
  if (M >= kI30 || N >= kI30 || K >= kI30) return false;
  // A: rep dim 0 walks one array axis with step 1, the pattern walks the other with step 1.
  if (A.paving[0][0] == 1 && A.paving[0][1] == 0 && A.paving[1][0] == 0 && A.paving[1][1] == 0 &&
      A.fitting[0][0] == 0 && A.fitting[1][0] == 1 && A.array_shape[0] == M && A.array_shape[1] == K) {
    g->a_sm = K; g->a_sk = 1;
  } else if (A.paving[1][0] == 1 && A.paving[1][1] == 0 && A.paving[0][0] == 0 && A.paving[0][1] == 0 &&
             A.fitting[1][0] == 0 && A.fitting[0][0] == 1 && A.array_shape[0] == K && A.array_shape[1] == M) {
    g->a_sm = 1; g->a_sk = M;
  } else {
    return false;
  }
  if (B.paving[1][1] == 1 && B.paving[1][0] == 0 && B.paving[0][0] == 0 && B.paving[0][1] == 0 &&
      B.fitting[0][0] == 1 && B.fitting[1][0] == 0 && B.array_shape[0] == K && B.array_shape[1] == N) {
    g->b_sk = N; g->b_sn = 1;
  } else if (B.paving[0][1] == 1 && B.paving[0][0] == 0 && B.paving[1][0] == 0 && B.paving[1][1] == 0 &&
             B.fitting[1][0] == 1 && B.fitting[0][0] == 0 && B.array_shape[0] == N && B.array_shape[1] == K) {
    g->b_sk = 1; g->b_sn = K;
  } else {
    return false;
  }
  // a single row (column) is k-contiguous whatever the storage order says
  if (M == 1) { g->a_sk = 1; g->a_sm = K; }
  if (N == 1) { g->b_sk = 1; g->b_sn = K; }
  g->M = int32_t(M); g->N = int32_t(N); g->K = int32_t(K);
  g->c_sm = N;
  return true;
}

// A weighted sum whose output pattern has q > 1 elements laid along the tap
// axis of a 1-D window tiler (a polyphase stage): the output array is the
// repetition shape with the tap axis q times longer, origin 0, paving
// diagonal (q on the tap axis, 1 elsewhere), pattern [q] with unit fitting
// on that axis.
bool match_poly(const rsm_space& rep, const rsm_tiler& in, const rsm_tiler& out, Win3* w, int* q) {
  if (!canon_win3(rep, in, w) || w->ax < 1 || !outer_axes_inside(*w, w->ax)) return false;
  const int da = rep.rank;
  if (out.array_rank != da || out.pattern_rank != 1) return false;
  const int64_t qv = out.pattern_shape[0];
  if (qv < 2 || qv > 64) return false;
  const int d_ax = w->ax - (3 - da);
  for (int d = 0; d < da; ++d) {
    if (out.origin[d] != 0) return false;
    if (out.array_shape[d] != rep.shape[d] * (d == d_ax ? qv : 1)) return false;
    if (out.fitting[d][0] != (d == d_ax ? 1 : 0)) return false;
    for (int k = 0; k < da; ++k)
      if (out.paving[d][k] != (d == k ? (d == d_ax ? qv : 1) : 0)) return false;
  }
  if (int64_t(w->rep[0]) * w->rep[1] * w->rep[2] * qv >= (int64_t(1) << 31)) return false;
  *q = int(qv);
  return poly_supported(*w, *q);
}

// Where a planned family keeps each port's data while a workgroup computes
// (the address spaces of the paper's MemoryMapping, Sec. 5-6: global =
// device memory read or written in place, constant = uniform across the
// workgroup in scalar registers, local = LDS, private = VGPR/AGPR), and how
// many bytes of it one workgroup holds there.  Ports: inputs, the output,
// then the coefficients of a weighted sum.
struct Placement {
  int count = 0;
  int space[4] = {RSM_MEM_GLOBAL, RSM_MEM_GLOBAL, RSM_MEM_GLOBAL, RSM_MEM_GLOBAL};
  int64_t bytes[4] = {0, 0, 0, 0};
};

Placement placement_of(const Plan& p, const rsm_tiler* in, int n_in, const rsm_task& task) {
  constexpr int kThreadsPerWg = 256;
  Placement pl;
  const bool coeffs = task.kind == RSM_TASK_WSUM;
  pl.count = n_in + 1 + (coeffs ? 1 : 0);
  const int out = n_in, cf = n_in + 1;
  auto set = [&](int k, int space, int64_t bytes) {
    pl.space[k] = space;
    pl.bytes[k] = bytes;
  };
  const int64_t in_es = elem_size(in[0].dtype);
  switch (p.fam) {
    case Fam::Empty:
    case Fam::Generic:
      break;   // every element read and written in place, weights read per term
    case Fam::PatternReduce:
      // one pattern element per lane, reduced across the lane group
      set(0, RSM_MEM_PRIVATE, kThreadsPerWg * in_es);
      if (coeffs) set(cf, RSM_MEM_PRIVATE, kThreadsPerWg * 4);
      break;
    case Fam::Fir:
      // each thread holds the taps of its window; the taps' weights are
      // uniform across the workgroup
      set(0, RSM_MEM_PRIVATE, int64_t(kThreadsPerWg) * p.win.taps * in_es);
      if (coeffs) set(cf, RSM_MEM_CONSTANT, int64_t(p.win.taps) * 4);
      break;
    case Fam::Poly:
      if (p.poly_vec) {
        // each thread holds its window (16 floats) and the shifted weights
        // of its q outputs in registers; outputs stored in place
        set(0, RSM_MEM_PRIVATE, int64_t(kThreadsPerWg) * 16 * in_es);
        if (coeffs) set(cf, RSM_MEM_PRIVATE, int64_t(kThreadsPerWg) * 16 * p.poly_q * 4);
        break;
      }
      if (p.win.ax == 2) {
        // a chunk's input segment, its outputs and the q x T weights in LDS
        set(0, RSM_MEM_LOCAL, (int64_t(p.win.p[2]) * 255 + p.win.taps) * in_es);
        set(out, RSM_MEM_LOCAL, int64_t(p.poly_q) * 256 * 4);
      } else {
        // each thread holds its window in registers, lanes along columns
        set(0, RSM_MEM_PRIVATE, int64_t(kThreadsPerWg) * p.win.taps * in_es);
      }
      if (coeffs) set(cf, RSM_MEM_LOCAL, int64_t(p.poly_q) * p.win.taps * 4);
      break;
    case Fam::Filter2D: {
      // the tile's input region (halo included) in LDS; the k x k weights,
      // uniform and read-only, through the scalar unit
      set(0, RSM_MEM_LOCAL, int64_t(filter2d_lds_bytes(p.f2d.k, p.f2d.s, 1)));
      if (coeffs) set(cf, RSM_MEM_CONSTANT, int64_t(p.f2d.k) * p.f2d.k * 4);
      break;
    }
    case Fam::Gemm: {
      // double-buffered k-tiles of both operands in LDS; the output tile in
      // accumulator registers for the whole k loop
      const int compute = in[0].dtype == RSM_BF16 ? RSM_BF16 : RSM_F32;
      const int64_t lds = gemm_lds_bytes_per_operand(p.gemm, compute);
      const int64_t side = gemm_tile_side(p.gemm, compute);
      set(0, RSM_MEM_LOCAL, lds);
      if (n_in > 1) set(1, RSM_MEM_LOCAL, lds);
      set(out, RSM_MEM_PRIVATE, side * side * 4);
      break;
    }
  }
  return pl;
}

// A requested space per port (RSM_MEM_ANY: no request) met by a placement.
bool meets(const Placement& pl, const int32_t* req) {
  if (!req) return true;
  for (int k = 0; k < pl.count; ++k)
    if (req[k] != RSM_MEM_ANY && req[k] != pl.space[k]) return false;
  return true;
}

// The kernel family for a task: the first candidate, in order of preference,
// whose port placement meets the request `req` (one space per port, or NULL
// for none).  plan.ok is false when no candidate meets it.
Plan make_plan(const rsm_space& rep, const rsm_tiler* in, int n_in, const rsm_tiler& out,
               const rsm_task& task, uint32_t flags, const void* const* d_in, int64_t n_rep,
               int64_t n_pat, const int32_t* req = nullptr) {
  std::vector<Plan> cands;
  Plan base;
  base.max_rank = max_rank_of(rep, in, n_in, out);
  if (n_rep == 0) {
    base.fam = Fam::Empty;
    base.name = "empty";
    return base;   // nothing runs: any placement is met
  }
  const Plan generic = base;   // fam Generic, name "generic"
  const bool f32 = in[0].dtype == RSM_F32 && task.compute == RSM_F32;
  if (!(flags & RSM_FORCE_GENERIC)) {
    if (task.kind == RSM_TASK_DOT) {
      GemmArgs g{};
      const bool bf = in[0].dtype == RSM_BF16 && (task.compute == RSM_BF16 || task.compute == RSM_F32);
      if ((bf || f32) && match_gemm(rep, in, out, &g)) {
        const int compute = bf ? RSM_BF16 : RSM_F32;
        // operands read in place (k-contiguous) must start on a 16-byte boundary
        bool aligned = true;
        if (d_in) {
          if (g.a_sk == 1 && (reinterpret_cast<uintptr_t>(d_in[0]) & 15)) aligned = false;
          if (g.b_sk == 1 && (reinterpret_cast<uintptr_t>(d_in[1]) & 15)) aligned = false;
        }
        if (aligned && gemm_supported(g, compute)) {
          Plan p = base;
          p.fam = Fam::Gemm;
          p.gemm = g;   // operand pointers are set per call (a plan holds none)
          p.name = gemm_variant_name(g, compute);
          cands.push_back(p);
        }
      }
    } else if (task.kind != RSM_TASK_COPY && f32) {
      // SUM / WSUM on FP32
      Win3 w{};
      int q = 0;
      if (task.kind == RSM_TASK_WSUM && match_poly(rep, in[0], out, &w, &q)) {
        Plan p = base;
        p.fam = Fam::Poly;
        p.win = w;
        p.poly_q = q;
        p.name = w.ax == 2 ? "polyphase_cols" : "polyphase_rows";
        // along columns, windows on a common 16-byte phase read straight
        // into registers (13 taps every 8, 3 outputs, 30 x 1080 x 1920:
        // 102-105 us staged in LDS, 72-73 us in registers)
        if (w.ax == 2 && poly_cols_vec_ok(w, q, d_in ? d_in[0] : nullptr)) {
          Plan v = p;
          v.poly_vec = true;
          v.name = "polyphase_cols_vec";
          cands.push_back(v);
        }
        cands.push_back(p);
      }
      if (task.kind == RSM_TASK_WSUM && is_identity_out(rep, out) && canon_win3(rep, in[0], &w) && w.ax >= 1 &&
          outer_axes_inside(w, w.ax)) {
        Plan p = base;
        p.fam = Fam::Fir;
        p.win = w;
        p.vec4 = fir_vec4(w, d_in ? d_in[0] : nullptr);
        p.name = w.ax == 2 ? (p.vec4 ? "fir_cols_vec4" : "fir_cols") : "fir_rows";
        // the same taps with the window staged in LDS (columns) or the
        // weights in LDS (rows): the polyphase kernels with one output
        Plan l = base;
        const bool lds = poly_supported(w, 1);
        if (lds) {
          l.fam = Fam::Poly;
          l.win = w;
          l.poly_q = 1;
          l.name = w.ax == 2 ? "fir_cols_lds" : "fir_rows_lds_weights";
        }
        // Along columns, windows that overlap or leave gaps (taps != step)
        // make each lane's taps a strided read that neighbouring lanes
        // repeat or skip; row segments staged in LDS read every line once
        // (30 x 1080 x 1920: 13 taps every 8, 116 -> 73 us; 6 every 8,
        // 102 -> 47 us).  Exact covers stay in registers (8 every 8 off the
        // 16-byte grid: 43 us against 64 us staged).
        if (lds && w.ax == 2 && !p.vec4 && w.taps != w.p[2]) {
          // windows on a common 16-byte phase: read straight into registers
          // as 16-byte vectors (13 taps every 8: 74 us staged, 55 us)
          if (poly_cols_vec_ok(w, 1, d_in ? d_in[0] : nullptr)) {
            Plan v = l;
            v.poly_vec = true;
            v.name = "fir_cols_window_vec";
            cands.push_back(v);
          }
          cands.push_back(l);
          cands.push_back(p);
        } else {
          cands.push_back(p);
          if (lds) cands.push_back(l);
        }
      }
      Filter2DProblem fp{};
      if (plan_filter2d(rep, in[0], out, task, &fp)) {
        Plan p = base;
        p.fam = Fam::Filter2D;
        p.f2d = fp;
        p.name = "filter2d_k" + std::to_string(fp.k) + "_s" + std::to_string(fp.s);
        cands.push_back(p);
      }
      if (n_pat <= 64 && is_scalar_pattern(out)) {
        Plan p = base;
        p.fam = Fam::PatternReduce;
        p.name = "pattern_reduce";
        cands.push_back(p);
      }
    }
  }
  cands.push_back(generic);
  for (const Plan& c : cands)
    if (meets(placement_of(c, in, n_in, task), req)) return c;
  Plan none = generic;
  none.ok = false;
  return none;
}

// Launch arguments of the polyphase kernels (pointers left to the caller).
// forward = true: the forward kernels' item layout (row chunks along columns);
// false: one item per repetition (weight-gradient kernel).
PolyArgs poly_args(const Win3& w, int q, int64_t n_rep, bool forward) {
  PolyArgs a{};
  a.w = w;
  a.q = q;
  a.div_rc = make_fastdiv(uint32_t(w.rep[2]));
  a.div_rr = make_fastdiv(uint32_t(w.rep[1]));
  a.n_chunks = poly_chunks(w);
  a.div_chunks = make_fastdiv(uint32_t(a.n_chunks));
  if (forward && w.ax == 2)
    a.n_items = uint32_t(int64_t(w.rep[0]) * w.rep[1] * a.n_chunks);
  else
    a.n_items = uint32_t(n_rep);
  return a;
}

// ---------------------------------------------------------------------------
// execution of one planned task
// ---------------------------------------------------------------------------
// Runs a task by a plan made for these descriptors (make_plan; the launch
// arguments that depend on the arrays' addresses are filled in here).
rsm_status exec_planned(Plan p, const rsm_space& rep, const rsm_tiler* in, const void* const* d_in, int n_in,
                        const rsm_tiler& out, void* d_out, const rsm_task& task, const Checked& c,
                        hipStream_t st) {
  hipError_t e = hipSuccess;
  switch (p.fam) {
    case Fam::Empty:
      return RSM_OK;
    case Fam::Gemm: {
      // the plan is made once per descriptor: the operands are this call's
      p.gemm.a = d_in[0];
      p.gemm.b = d_in[1];
      p.gemm.c = static_cast<float*>(d_out);
      const int compute = in[0].dtype == RSM_BF16 ? RSM_BF16 : RSM_F32;
      e = launch_gemm(p.gemm, compute, st);
      if (e != hipSuccess) return fail(RSM_E_HIP, g_last_error);  // detail set by launch_gemm
      return RSM_OK;
    }
    case Fam::Fir: {
      FirArgs a{};
      a.w = p.win;
      a.div_rc = make_fastdiv(uint32_t(p.win.rep[2]));
      a.div_rr = make_fastdiv(uint32_t(p.win.rep[1]));
      a.n_out = uint32_t(c.n_rep);
      a.x = static_cast<const float*>(d_in[0]);
      a.y = static_cast<float*>(d_out);
      a.c = static_cast<const float*>(task.coeffs);
      e = launch_fir(a, p.vec4, st);
      if (e != hipSuccess) return hip_fail(e, "fir launch");
      return RSM_OK;
    }
    case Fam::Poly: {
      PolyArgs a = poly_args(p.win, p.poly_q, c.n_rep, true);
      a.x = static_cast<const float*>(d_in[0]);
      a.y = static_cast<float*>(d_out);
      a.c = static_cast<const float*>(task.coeffs);
      e = p.poly_vec ? launch_poly_cols_vec(a, st) : launch_poly(a, st);
      if (e != hipSuccess) return hip_fail(e, "polyphase launch");
      return RSM_OK;
    }
    case Fam::Filter2D: {
      Filter2DProblem fp = p.f2d;
      fp.x = static_cast<const float*>(d_in[0]);
      fp.y = static_cast<float*>(d_out);
      fp.c = static_cast<const float*>(task.coeffs);
      filter2d_set_tiles(&fp, 1);
      e = launch_filter2d(fp, st);
      if (e != hipSuccess) return hip_fail(e, "filter2d launch");
      return RSM_OK;
    }
    case Fam::PatternReduce: {
      PatternReduceArgs a{};
      a.rep_rank = rep.rank;
      for (int k = 0; k < kMaxRank; ++k) a.rep_shape[k] = k < rep.rank ? rep.shape[k] : 1;
      a.n_rep = c.n_rep;
      a.n_pat = c.n_pat_in[0];
      int g = 0;
      while ((int64_t(1) << g) < a.n_pat) ++g;
      a.group_log2 = g;
      a.in = to_gtiler(in[0], rep.rank);
      a.out = to_gtiler(out, rep.rank);
      a.x = static_cast<const float*>(d_in[0]);
      a.y = static_cast<float*>(d_out);
      a.c = task.kind == RSM_TASK_WSUM ? static_cast<const float*>(task.coeffs) : nullptr;
      PatternReduceSmallArgs sa;
      e = pattern_reduce_small_args(a, &sa) ? launch_pattern_reduce_small(sa, st)
                                            : launch_pattern_reduce(a, p.max_rank, st);
      if (e != hipSuccess) return hip_fail(e, "pattern_reduce launch");
      return RSM_OK;
    }
    case Fam::Generic: {
      GenericArgs a;
      std::memset(&a, 0, sizeof(a));
      a.rep_rank = rep.rank;
      a.n_in = n_in;
      for (int k = 0; k < kMaxRank; ++k) a.rep_shape[k] = k < rep.rank ? rep.shape[k] : 1;
      a.n_rep = c.n_rep;
      a.n_pat = c.n_pat_in[0];
      a.n_q = c.n_pat_out;
      for (int t = 0; t < n_in; ++t) {
        a.in[t] = to_gtiler(in[t], rep.rank);
        a.x[t] = d_in[t];
      }
      a.out = to_gtiler(out, rep.rank);
      a.y = d_out;
      a.coeffs = task.coeffs;
      e = launch_generic(a, p.max_rank, in[0].dtype, out.dtype, task.kind, elem_size(in[0].dtype), st);
      if (e != hipSuccess) return hip_fail(e, "generic launch");
      return RSM_OK;
    }
  }
  return fail(RSM_E_UNSUPPORTED, "no kernel family");
}

rsm_status exec_run(const rsm_space& rep, const rsm_tiler* in, const void* const* d_in, int n_in,
                    const rsm_tiler& out, void* d_out, const rsm_task& task, uint32_t flags,
                    const Checked& c, hipStream_t st, const int32_t* req = nullptr) {
  const Plan p = make_plan(rep, in, n_in, out, task, flags, d_in, c.n_rep, c.n_pat_in[0], req);
  if (!p.ok) return fail(RSM_E_UNSUPPORTED, "no kernel of this library keeps the ports where requested");
  return exec_planned(p, rep, in, d_in, n_in, out, d_out, task, c, st);
}

// ---------------------------------------------------------------------------
// plans cached by descriptor
// ---------------------------------------------------------------------------
// Validation and planning read only the entries of the descriptors below
// their ranks, the task's kind and compute type, whether weights are given,
// the flags, and (for the families that read in place with 16-byte loads)
// whether each input starts on a 16-byte boundary.  The key lists exactly
// those; equal keys give the same validation result and the same plan.
bool descriptor_key(const rsm_space* rep, const rsm_tiler* in, int n_in, const rsm_tiler* out,
                    const rsm_task* task, uint32_t flags, const void* const* d_in,
                    std::vector<int64_t>* key) {
  if (!rep || !in || !out || !task || n_in < 1 || n_in > 2) return false;
  if (rep->rank < 0 || rep->rank > RSM_MAX_RANK) return false;
  key->clear();
  key->push_back(rep->rank);
  for (int k = 0; k < rep->rank; ++k) key->push_back(rep->shape[k]);
  key->push_back(n_in);
  for (int t = 0; t <= n_in; ++t) {
    const rsm_tiler& x = t < n_in ? in[t] : *out;
    if (x.array_rank < 0 || x.array_rank > RSM_MAX_RANK || x.pattern_rank < 0 || x.pattern_rank > RSM_MAX_RANK)
      return false;
    key->push_back(x.array_rank);
    key->push_back(x.pattern_rank);
    key->push_back(x.dtype);
    for (int k = 0; k < x.pattern_rank; ++k) key->push_back(x.pattern_shape[k]);
    for (int d = 0; d < x.array_rank; ++d) {
      key->push_back(x.array_shape[d]);
      key->push_back(x.origin[d]);
      for (int k = 0; k < rep->rank; ++k) key->push_back(x.paving[d][k]);
      for (int k = 0; k < x.pattern_rank; ++k) key->push_back(x.fitting[d][k]);
    }
  }
  int64_t align = 0;
  for (int t = 0; t < n_in; ++t)
    if (d_in && (reinterpret_cast<uintptr_t>(d_in[t]) & 15)) align |= int64_t(1) << t;
  key->push_back(task->kind);
  key->push_back(task->compute);
  key->push_back(task->coeffs != nullptr);
  key->push_back(flags);
  key->push_back(align);
  return true;
}

uint64_t key_hash(const std::vector<int64_t>& key) {
  uint64_t h = 1469598103934665603ull;   // FNV-1a over the 64-bit words
  for (int64_t v : key) {
    h ^= uint64_t(v);
    h *= 1099511628211ull;
  }
  return h;
}

struct CachedPlan {
  uint64_t hash = 0;
  std::vector<int64_t> key;
  Checked c;
  Plan plan;
};

constexpr int kPlanCache = 32;
thread_local CachedPlan g_plan_cache[kPlanCache];
thread_local int g_plan_cache_next = 0;
thread_local int g_plan_cache_used = 0;
thread_local uint64_t g_plan_cache_hits = 0;

const CachedPlan* plan_cache_find(const std::vector<int64_t>& key, uint64_t h) {
  for (int k = 0; k < g_plan_cache_used; ++k)
    if (g_plan_cache[k].hash == h && g_plan_cache[k].key == key) return &g_plan_cache[k];
  return nullptr;
}

void plan_cache_put(const std::vector<int64_t>& key, uint64_t h, const Checked& c, const Plan& p) {
  CachedPlan& e = g_plan_cache[g_plan_cache_next];
  g_plan_cache_next = (g_plan_cache_next + 1) % kPlanCache;
  if (g_plan_cache_used < kPlanCache) ++g_plan_cache_used;
  e.hash = h;
  e.key = key;
  e.c = c;
  e.plan = p;
}

// A placement request: one rsm_mem_space (or RSM_MEM_ANY) per port, in port
// order (inputs, output, coefficients); NULL = no request.  An output port is
// written, so it cannot sit in constant memory, which is read-only while a
// kernel runs (port direction, Sec. 6).
rsm_status check_spaces(const int32_t* spaces, int32_t n_spaces, int count, int n_in) {
  if (!spaces) return RSM_OK;
  if (n_spaces != count)
    return fail(RSM_E_INVALID, "placement request needs one space per port (" + std::to_string(count) + "), got " +
                                   std::to_string(n_spaces));
  for (int k = 0; k < count; ++k) {
    if (spaces[k] < RSM_MEM_ANY || spaces[k] > RSM_MEM_PRIVATE)
      return fail(RSM_E_INVALID, "unknown memory space " + std::to_string(spaces[k]) + " for port " +
                                     std::to_string(k));
    if (k == n_in && spaces[k] == RSM_MEM_CONSTANT)
      return fail(RSM_E_INVALID, "the output port is written: it cannot be placed in constant memory");
  }
  return RSM_OK;
}

bool ptrs_ok(const void* const* d, int n) {
  if (!d) return false;
  for (int k = 0; k < n; ++k)
    if (!d[k]) return false;
  return true;
}

// ---------------------------------------------------------------------------
// adjoint
// ---------------------------------------------------------------------------
rsm_status check_adjoint(const rsm_space* rep, const rsm_tiler* in, const rsm_tiler* out,
                         const rsm_task* task, Checked* c) {
  rsm_status s = check_task(rep, in, 1, out, task, 0, c);
  if (s) return s;
  if (task->kind != RSM_TASK_SUM && task->kind != RSM_TASK_WSUM)
    return fail(RSM_E_UNSUPPORTED, "adjoint is defined here for SUM and WSUM tasks");
  if (in->dtype != RSM_F32 || task->compute != RSM_F32)
    return fail(RSM_E_UNSUPPORTED, "adjoint supports FP32 arrays and FP32 compute");
  return RSM_OK;
}

struct AdjPlan {
  bool poly = false;     // weighted sum with q outputs per repetition along the tap axis
  int q = 1;
  bool fir = false;
  bool vec4 = false;
  bool exact = false;
  bool gather = false;   // windows overlap or wrap: input gradient as a gather
  bool overlap_cols = false;   // ... along columns, steps <= 16: one fused kernel
  Win3 w{};
};

// Chunks of 256 repetitions per row for the fused column kernel: enough to
// own every column (256 p columns each) and to hold every repetition.
int64_t overlap_chunks(const Win3& w) {
  const int64_t own = (int64_t(w.A[2]) + 256 * int64_t(w.p[2]) - 1) / (256 * int64_t(w.p[2]));
  const int64_t reps = (int64_t(w.rep[2]) + 255) / 256;
  return std::max<int64_t>(std::max(own, reps), 1);
}

int64_t overlap_items(const Win3& w) { return int64_t(w.A[0]) * w.A[1] * overlap_chunks(w); }

// Input gradient of a 1-D tap tiler as a gather over input elements: the tap
// axis steps forward (or has one repetition) and no two repetitions share an
// index along the other axes.
bool fir_gather_ok(const Win3& w) {
  for (int d = 0; d < 3; ++d) {
    if (d == w.ax) continue;
    if (w.rep[d] > 1 && w.p[d] < 1) return false;
  }
  return w.p[w.ax] >= 1 || w.rep[w.ax] == 1;
}

AdjPlan plan_adjoint(const rsm_space& rep, const rsm_tiler& in, const rsm_tiler& out,
                     const rsm_task& task, uint32_t flags, const void* x, const void* gx) {
  AdjPlan a;
  if (flags & RSM_FORCE_GENERIC) return a;
  Win3 w{};
  int q = 0;
  if (task.kind == RSM_TASK_WSUM && match_poly(rep, in, out, &w, &q) && fir_gather_ok(w)) {
    a.poly = true;
    a.q = q;
    a.w = w;
    return a;
  }
  if (task.kind == RSM_TASK_WSUM && is_identity_out(rep, out) && canon_win3(rep, in, &w) &&
      w.ax >= 1 && w.taps <= 16 && outer_axes_inside(w, w.ax)) {
    if (fir_injective(w)) {
      a.fir = true;
      a.w = w;
      a.exact = fir_exact_cover(w);
      a.vec4 = fir_vec4(w, x) && fir_vec4(w, gx);
    } else if (fir_gather_ok(w)) {
      // the weight gradient keeps the per-repetition kernel (it reads x only)
      a.fir = true;
      a.gather = true;
      a.w = w;
      a.vec4 = fir_vec4(w, x);
      a.overlap_cols = w.ax == 2 && w.p[2] >= 1 && w.p[2] <= 16 && w.A[2] < (1 << 28) &&
                       w.rep[2] < (1 << 28) && overlap_items(w) < (int64_t(1) << 31);
    }
  }
  return a;
}

// Workspace bytes the adjoint of one stage needs.
size_t adjoint_ws_bytes(const AdjPlan& ap, int64_t n_rep, int64_t n_pat, int64_t n_q, bool want_gc) {
  if (!want_gc) return 0;
  if (ap.poly && poly_adj_cols_supported(ap.w, ap.q)) {
    const Win3& w = ap.w;
    const int64_t chunks = std::max<int64_t>(
        std::max<int64_t>((int64_t(w.A[2]) + 256 * int64_t(w.p[2]) - 1) / (256 * int64_t(w.p[2])),
                          (int64_t(w.rep[2]) + 255) / 256),
        1);
    return size_t(poly_adj_cols_grid(w, ap.q, uint32_t(int64_t(w.rep[0]) * w.rep[1] * chunks))) * size_t(ap.q) *
           size_t(w.taps) * sizeof(float);
  }
  if (ap.poly && poly_gc_supported(ap.w, ap.q))
    return size_t(poly_gc_grid(uint32_t(n_rep))) * size_t(ap.q) * size_t(ap.w.taps) * sizeof(float);
  if (ap.overlap_cols)
    return size_t(fir_overlap_cols_grid(uint32_t(overlap_items(ap.w)), ap.w.p[2])) * size_t(ap.w.taps) *
           sizeof(float);
  if (ap.fir) {
    FirAdjArgs tmp{};
    tmp.n_rep = uint32_t(n_rep);
    return size_t(fir_adjoint_grid(tmp)) * size_t(ap.w.taps) * sizeof(float);
  }
  const int64_t nblk = std::min<int64_t>(std::max<int64_t>((n_rep + 4095) / 4096, 1), 1024);
  return size_t(nblk) * size_t(n_pat) * size_t(n_q) * sizeof(float);
}

rsm_status exec_adjoint(const rsm_space& rep, const rsm_tiler& in, const void* d_x,
                        const rsm_tiler& out, const void* d_gy, const rsm_task& task, void* d_gx,
                        void* d_gc, uint32_t flags, const Checked& c, void* ws, uint32_t* counter,
                        hipStream_t st) {
  const int accumulate = (flags & RSM_ACCUMULATE) ? 1 : 0;
  hipError_t e;
  const AdjPlan ap = plan_adjoint(rep, in, out, task, flags, d_x, d_gx);
  if (c.n_rep == 0) {
    // nothing reads the input: the gradients are zero
    if (!accumulate) {
      if (d_gx && (e = launch_zero(d_gx, prod(in.array_shape, in.array_rank) * 4, st)) != hipSuccess)
        return hip_fail(e, "zero gx");
      if (d_gc && (e = launch_zero(d_gc, c.n_pat_in[0] * c.n_pat_out * 4, st)) != hipSuccess)
        return hip_fail(e, "zero gc");
    }
    return RSM_OK;
  }
  const int64_t n_arr = prod(in.array_shape, in.array_rank);
  if (ap.poly && poly_adj_cols_supported(ap.w, ap.q)) {
    // both gradients in one pass over row chunks; the kernel visits the rows
    // the repetitions read, so rows no repetition reads are cleared first
    const Win3& w = ap.w;
    const bool all_rows = w.rep[0] == w.A[0] && w.rep[1] == w.A[1] && w.o[0] == 0 && w.o[1] == 0 &&
                          (w.A[0] == 1 || w.p[0] == 1) && (w.A[1] == 1 || w.p[1] == 1);
    if (d_gx && !accumulate && !all_rows && (e = launch_zero(d_gx, n_arr * 4, st)) != hipSuccess)
      return hip_fail(e, "zero gx");
    PolyAdjArgs o{};
    o.w = w;
    o.q = ap.q;
    o.n_chunks = int32_t(std::max<int64_t>(
        std::max<int64_t>((int64_t(w.A[2]) + 256 * int64_t(w.p[2]) - 1) / (256 * int64_t(w.p[2])),
                          (int64_t(w.rep[2]) + 255) / 256),
        1));
    o.o_mod = int32_t(floor_mod(w.o[2], w.A[2]));
    o.div_chunks = make_fastdiv(uint32_t(o.n_chunks));
    o.div_rr = make_fastdiv(uint32_t(w.rep[1]));
    o.div_p = make_fastdiv(uint32_t(w.p[2]));
    o.n_items = uint32_t(int64_t(w.rep[0]) * w.rep[1] * o.n_chunks);
    o.x = static_cast<const float*>(d_x);
    o.gy = static_cast<const float*>(d_gy);
    o.gx = static_cast<float*>(d_gx);
    o.c = static_cast<const float*>(task.coeffs);
    o.partial = d_gc ? static_cast<float*>(ws) : nullptr;
    o.accumulate = accumulate;
    if ((e = launch_poly_adj_cols(o, st)) != hipSuccess) return hip_fail(e, "polyphase adjoint");
    const int nc = ap.q * w.taps;
    if (d_gc && (e = launch_reduce_partials(o.partial, poly_adj_cols_grid(w, ap.q, o.n_items), nc, nc,
                                            static_cast<float*>(d_gc), accumulate, st)) != hipSuccess)
      return hip_fail(e, "weight-gradient reduction");
    return RSM_OK;
  }
  if (ap.poly) {
    const Win3& w = ap.w;
    if (d_gx) {
      PolyGatherArgs g{};
      g.w = w;
      g.q = ap.q;
      g.div_a2 = make_fastdiv(uint32_t(w.A[2]));
      g.div_a1 = make_fastdiv(uint32_t(w.A[1]));
      for (int d = 0; d < 3; ++d) g.div_p[d] = make_fastdiv(uint32_t(std::max(w.p[d], 1)));
      g.o_mod = int32_t(floor_mod(w.o[w.ax], w.A[w.ax]));
      g.n_arr = uint32_t(n_arr);
      g.gy = static_cast<const float*>(d_gy);
      g.gx = static_cast<float*>(d_gx);
      g.c = static_cast<const float*>(task.coeffs);
      g.accumulate = accumulate;
      if ((e = launch_poly_gx_gather(g, st)) != hipSuccess) return hip_fail(e, "polyphase gather adjoint");
    }
    if (d_gc && poly_gc_supported(w, ap.q)) {
      PolyArgs a = poly_args(w, ap.q, c.n_rep, false);
      a.x = static_cast<const float*>(d_x);
      a.gy = static_cast<const float*>(d_gy);
      a.partial = static_cast<float*>(ws);
      const int nc = ap.q * w.taps;
      if ((e = launch_poly_gc(a, st)) != hipSuccess) return hip_fail(e, "polyphase weight gradient");
      if ((e = launch_reduce_partials(a.partial, poly_gc_grid(a.n_items), nc, nc, static_cast<float*>(d_gc),
                                      accumulate, st)) != hipSuccess)
        return hip_fail(e, "weight-gradient reduction");
      return RSM_OK;
    }
    if (!d_gc) return RSM_OK;
    d_gx = nullptr;   // the generic weight-gradient path below, input gradient done
  }
  if (ap.overlap_cols) {
    const Win3& w = ap.w;
    FirOverlapArgs o{};
    o.w = w;
    o.div_a1 = make_fastdiv(uint32_t(w.A[1]));
    o.div_a2 = make_fastdiv(uint32_t(w.A[2]));
    o.div_p = make_fastdiv(uint32_t(w.p[2]));
    o.n_chunks = int32_t(overlap_chunks(w));
    o.div_chunks = make_fastdiv(uint32_t(o.n_chunks));
    o.div_p0 = make_fastdiv(uint32_t(std::max(w.p[0], 1)));
    o.div_p1 = make_fastdiv(uint32_t(std::max(w.p[1], 1)));
    o.o_mod = int32_t(floor_mod(w.o[2], w.A[2]));
    o.step_mod = int32_t((int64_t(w.p[2]) * (256 / w.taps)) % w.A[2]);
    o.n_items = uint32_t(overlap_items(w));
    o.x = static_cast<const float*>(d_x);
    o.gy = static_cast<const float*>(d_gy);
    o.gx = static_cast<float*>(d_gx);
    o.c = static_cast<const float*>(task.coeffs);
    o.partial = d_gc ? static_cast<float*>(ws) : nullptr;
    o.accumulate = accumulate;
    if ((e = launch_fir_adjoint_overlap_cols(o, st)) != hipSuccess) return hip_fail(e, "fir overlap adjoint");
    if (d_gc &&
        (e = launch_reduce_partials(o.partial, fir_overlap_cols_grid(o.n_items, w.p[2]), w.taps, w.taps,
                                    static_cast<float*>(d_gc), accumulate, st)) != hipSuccess)
      return hip_fail(e, "weight-gradient reduction");
    return RSM_OK;
  }
  if (ap.gather && d_gx) {
    FirGatherArgs g{};
    g.w = ap.w;
    g.div_a2 = make_fastdiv(uint32_t(ap.w.A[2]));
    g.div_a1 = make_fastdiv(uint32_t(ap.w.A[1]));
    for (int d = 0; d < 3; ++d) g.div_p[d] = make_fastdiv(uint32_t(std::max(ap.w.p[d], 1)));
    g.o_mod = int32_t(floor_mod(ap.w.o[ap.w.ax], ap.w.A[ap.w.ax]));
    g.n_arr = uint32_t(n_arr);
    g.gy = static_cast<const float*>(d_gy);
    g.gx = static_cast<float*>(d_gx);
    g.c = static_cast<const float*>(task.coeffs);
    g.accumulate = accumulate;
    if ((e = launch_fir_gx_gather(g, st)) != hipSuccess) return hip_fail(e, "fir gather adjoint");
    if (!d_gc) return RSM_OK;
    d_gx = nullptr;   // the per-repetition kernel below forms the weight gradient only
  }
  if (ap.fir) {
    if (d_gx && !accumulate && !ap.exact) {
      if ((e = launch_zero(d_gx, n_arr * 4, st)) != hipSuccess) return hip_fail(e, "zero gx");
    }
    FirAdjArgs a{};
    a.w = ap.w;
    a.div_rc = make_fastdiv(uint32_t(ap.w.rep[2]));
    a.div_rr = make_fastdiv(uint32_t(ap.w.rep[1]));
    a.n_rep = uint32_t(c.n_rep);
    a.x = d_gc ? static_cast<const float*>(d_x) : nullptr;
    a.gy = static_cast<const float*>(d_gy);
    a.gx = static_cast<float*>(d_gx);
    a.c = static_cast<const float*>(task.coeffs);
    a.partial = d_gc ? static_cast<float*>(ws) : nullptr;
    a.gc = static_cast<float*>(d_gc);
    a.counter = (flags & RSM_REDUCE_IN_KERNEL) ? counter : nullptr;
    a.accumulate = accumulate;
    int grid = 0;
    if ((e = launch_fir_adjoint(a, ap.vec4, &grid, st)) != hipSuccess) return hip_fail(e, "fir adjoint");
    if (d_gc && !a.counter &&
        (e = launch_reduce_partials(a.partial, grid, ap.w.taps, ap.w.taps, static_cast<float*>(d_gc),
                                    accumulate, st)) != hipSuccess)
      return hip_fail(e, "weight-gradient reduction");
    return RSM_OK;
  }
  // generic path
  const int mr = max_rank_of(rep, &in, 1, out);
  if (d_gx) {
    if (!accumulate && (e = launch_zero(d_gx, n_arr * 4, st)) != hipSuccess) return hip_fail(e, "zero gx");
    GenericAdjArgs a;
    std::memset(&a, 0, sizeof(a));
    a.rep_rank = rep.rank;
    for (int k = 0; k < kMaxRank; ++k) a.rep_shape[k] = k < rep.rank ? rep.shape[k] : 1;
    a.n_rep = c.n_rep;
    a.n_pat = c.n_pat_in[0];
    a.n_q = c.n_pat_out;
    a.in = to_gtiler(in, rep.rank);
    a.out = to_gtiler(out, rep.rank);
    a.gy = static_cast<const float*>(d_gy);
    a.gx = static_cast<float*>(d_gx);
    a.c = task.kind == RSM_TASK_WSUM ? static_cast<const float*>(task.coeffs) : nullptr;
    if ((e = launch_generic_adjoint(a, mr, st)) != hipSuccess) return hip_fail(e, "generic adjoint");
  }
  if (d_gc) {
    GenericCoefGradArgs a;
    std::memset(&a, 0, sizeof(a));
    a.rep_rank = rep.rank;
    for (int k = 0; k < kMaxRank; ++k) a.rep_shape[k] = k < rep.rank ? rep.shape[k] : 1;
    a.n_rep = c.n_rep;
    a.n_pat = c.n_pat_in[0];
    a.n_q = c.n_pat_out;
    a.in = to_gtiler(in, rep.rank);
    a.out = to_gtiler(out, rep.rank);
    a.x = static_cast<const float*>(d_x);
    a.gy = static_cast<const float*>(d_gy);
    a.partial = static_cast<float*>(ws);
    const int64_t nblk = std::min<int64_t>(std::max<int64_t>((c.n_rep + 4095) / 4096, 1), 1024);
    a.chunk = (c.n_rep + nblk - 1) / nblk;
    if ((e = launch_generic_coef_grad(a, mr, int(nblk), st)) != hipSuccess)
      return hip_fail(e, "generic weight gradient");
    if ((e = launch_reduce_rows(a.partial, a.n_q * a.n_pat, nblk, static_cast<float*>(d_gc), accumulate, st)) !=
        hipSuccess)
      return hip_fail(e, "weight-gradient reduction");
  }
  return RSM_OK;
}

// ---------------------------------------------------------------------------
// chains
// ---------------------------------------------------------------------------
rsm_status check_chain(const rsm_stage* stages, int32_t n, std::vector<Checked>* cs) {
  if (!stages || n < 1) return fail(RSM_E_INVALID, "chain needs at least one stage");
  cs->resize(size_t(n));
  for (int k = 0; k < n; ++k) {
    const rsm_stage& s = stages[k];
    if (s.task.kind == RSM_TASK_DOT) return fail(RSM_E_INVALID, "chain stages take one input");
    rsm_status r = check_task(&s.rep, &s.in, 1, &s.out, &s.task, 0, &(*cs)[size_t(k)]);
    if (r) return fail(r, "stage " + std::to_string(k) + ": " + g_last_error);
    if (k > 0) {
      const rsm_tiler& a = stages[k - 1].out;
      const rsm_tiler& b = s.in;
      bool same = a.array_rank == b.array_rank && a.dtype == b.dtype;
      for (int d = 0; same && d < a.array_rank; ++d) same = a.array_shape[d] == b.array_shape[d];
      if (!same)
        return fail(RSM_E_SHAPE, "stage " + std::to_string(k) + " input array differs from stage " +
                                     std::to_string(k - 1) + " output array");
    }
  }
  return RSM_OK;
}

// Two FP32 weighted-sum stages, columns then rows, identity outputs.
bool chain_fusable(const rsm_stage* st, int n, const void* x, Win3* h, Win3* v, bool* vec4) {
  if (n != 2) return false;
  for (int k = 0; k < 2; ++k) {
    if (st[k].task.kind != RSM_TASK_WSUM || st[k].task.compute != RSM_F32 || st[k].in.dtype != RSM_F32)
      return false;
    if (!is_identity_out(st[k].rep, st[k].out)) return false;
  }
  if (!canon_win3(st[0].rep, st[0].in, h) || !canon_win3(st[1].rep, st[1].in, v)) return false;
  if (h->ax != 2 || v->ax != 1) return false;
  if (!outer_axes_inside(*h, 2) || !outer_axes_inside(*v, 1)) return false;
  // stage 1 reads the stage-0 output array [h.rep]
  for (int d = 0; d < 3; ++d)
    if (v->A[d] != h->rep[d]) return false;
  *vec4 = fir_vec4(*h, x);
  return true;
}

}  // namespace

bool plan_filter2d(const rsm_space& rep, const rsm_tiler& in, const rsm_tiler& out,
                   const rsm_task& task, Filter2DProblem* fp) {
  if (task.kind != RSM_TASK_WSUM || in.dtype != RSM_F32 || task.compute != RSM_F32) return false;
  if (!is_identity_out(rep, out)) return false;
  Win3 w{};
  if (!canon_win3(rep, in, &w) || w.ax != 0) return false;
  if (w.taps != w.taps2 || w.p[1] != w.p[2] || !filter2d_supported(w.taps, w.p[1])) return false;
  // identity along frames
  if (w.o[0] != 0 || w.rep[0] != w.A[0] || (w.A[0] > 1 && w.p[0] != 1)) return false;
  // each frame is addressed as one buffer of 32-bit byte offsets
  if (int64_t(w.A[1]) * w.A[2] * 4 >= (int64_t(1) << 31)) return false;
  *fp = Filter2DProblem{};
  fp->H = w.A[1];
  fp->W = w.A[2];
  fp->RH = w.rep[1];
  fp->RW = w.rep[2];
  fp->oh = int32_t(floor_mod(w.o[1], w.A[1]));
  fp->ow = int32_t(floor_mod(w.o[2], w.A[2]));
  fp->k = w.taps;
  fp->s = w.p[1];
  fp->frames = w.A[0];
  return true;
}

// CSR arguments shared by the sparse entry points.
rsm_status check_csr_sizes(int64_t n_rows, int64_t n_cols, int64_t nnz) {
  if (n_rows < 0 || n_cols < 0 || nnz < 0) return fail(RSM_E_SHAPE, "negative CSR size");
  const int64_t lim = int64_t(1) << 31;
  if (n_rows >= lim || n_cols >= lim || nnz >= lim) return fail(RSM_E_UNSUPPORTED, "CSR sizes limited to 2^31");
  return RSM_OK;
}

// Copies the index arrays to the host and checks them (blocking).
rsm_status check_csr_indices(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t* d_row_ptr,
                             const int32_t* d_col_idx, hipStream_t st) {
  std::vector<int32_t> rp(static_cast<size_t>(n_rows + 1)), ci(static_cast<size_t>(nnz));
  hipError_t e;
  if ((e = hipMemcpyAsync(rp.data(), d_row_ptr, rp.size() * 4, hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (nnz && (e = hipMemcpyAsync(ci.data(), d_col_idx, ci.size() * 4, hipMemcpyDeviceToHost, st)) != hipSuccess) ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return hip_fail(e, "index copy for checking");
  if (rp[0] != 0 || rp[size_t(n_rows)] != nnz) return fail(RSM_E_INVALID, "row_ptr must start at 0 and end at nnz");
  for (int64_t r = 0; r < n_rows; ++r)
    if (rp[size_t(r + 1)] < rp[size_t(r)]) return fail(RSM_E_INVALID, "row_ptr decreases at row " + std::to_string(r));
  for (int64_t k = 0; k < nnz; ++k)
    if (ci[size_t(k)] < 0 || ci[size_t(k)] >= n_cols)
      return fail(RSM_E_INVALID, "column index out of range at entry " + std::to_string(k));
  return RSM_OK;
}

}  // namespace rsm

// ===========================================================================
// C-ABI
// ===========================================================================
using namespace rsm;

#define RSM_GUARD_BEGIN try {
#define RSM_GUARD_END                                                   \
  }                                                                     \
  catch (const std::bad_alloc&) {                                       \
    return fail(RSM_E_NOMEM, "host allocation failed");                 \
  }                                                                     \
  catch (...) {                                                         \
    return fail(RSM_E_INVALID, "internal error (exception)");           \
  }

extern "C" {

rsm_status rsm_time_next_kernel(void* hip_event_start, void* hip_event_stop) {
  g_probe.start = static_cast<hipEvent_t>(hip_event_start);
  g_probe.stop = static_cast<hipEvent_t>(hip_event_stop);
  return RSM_OK;
}

int32_t rsm_abi_version(void) { return RSM_ABI_VERSION; }

const char* rsm_status_string(int32_t status) {
  switch (status) {
    case RSM_OK: return "RSM_OK";
    case RSM_E_INVALID: return "RSM_E_INVALID";
    case RSM_E_RANK: return "RSM_E_RANK";
    case RSM_E_SHAPE: return "RSM_E_SHAPE";
    case RSM_E_OVERFLOW: return "RSM_E_OVERFLOW";
    case RSM_E_OVERLAP: return "RSM_E_OVERLAP";
    case RSM_E_UNSUPPORTED: return "RSM_E_UNSUPPORTED";
    case RSM_E_HIP: return "RSM_E_HIP";
    case RSM_E_NOMEM: return "RSM_E_NOMEM";
  }
  return "RSM_E_UNKNOWN";
}

const char* rsm_last_error(void) { return g_last_error.c_str(); }

rsm_status rsm_validate(const rsm_space* rep, const rsm_tiler* in, int32_t n_in,
                        const rsm_tiler* out, const rsm_task* task, uint32_t flags) {
  RSM_GUARD_BEGIN
  Checked c;
  return check_task(rep, in, n_in, out, task, flags, &c);
  RSM_GUARD_END
}

rsm_status rsm_plan(const rsm_space* rep, const rsm_tiler* in, int32_t n_in, const rsm_tiler* out,
                    const rsm_task* task, uint32_t flags, char* name, int32_t len) {
  RSM_GUARD_BEGIN
  Checked c;
  if (flags & RSM_PLAN_ADJOINT) {
    if (n_in != 1) return fail(RSM_E_INVALID, "the adjoint takes one input tiler");
    rsm_status s = check_adjoint(rep, in, out, task, &c);
    if (s) return s;
    if (!name || len <= 0) return fail(RSM_E_INVALID, "name buffer is NULL");
    const AdjPlan ap = plan_adjoint(*rep, *in, *out, *task, flags, nullptr, nullptr);
    const char* fam = ap.poly           ? (poly_adj_cols_supported(ap.w, ap.q) ? "polyphase_adjoint_cols"
                                           : poly_gc_supported(ap.w, ap.q)     ? "polyphase_adjoint_gather"
                                                                               : "polyphase_adjoint_gather_generic_gc")
                      : ap.overlap_cols ? "fir_adjoint_overlap_cols"
                      : ap.gather ? "fir_adjoint_gather"
                      : ap.fir  ? (ap.vec4 ? "fir_adjoint_vec4" : "fir_adjoint")
                                : "generic_adjoint";
    std::snprintf(name, size_t(len), "%s", fam);
    return RSM_OK;
  }
  rsm_status s = check_task(rep, in, n_in, out, task, flags & ~RSM_CHECK_SINGLE_ASSIGN, &c);
  if (s) return s;
  if (!name || len <= 0) return fail(RSM_E_INVALID, "name buffer is NULL");
  const Plan p = make_plan(*rep, in, n_in, *out, *task, flags, nullptr, c.n_rep, c.n_pat_in[0]);
  std::snprintf(name, size_t(len), "%s", p.name.c_str());
  return RSM_OK;
  RSM_GUARD_END
}

rsm_status rsm_plan_ports(const rsm_space* rep, const rsm_tiler* in, int32_t n_in, const rsm_tiler* out,
                          const rsm_task* task, uint32_t flags, rsm_port_placement* ports, int32_t max_ports,
                          int32_t* n_ports) {
  return rsm_plan_placed(rep, in, n_in, out, task, flags, nullptr, 0, nullptr, 0, ports, max_ports, n_ports);
}

rsm_status rsm_plan_placed(const rsm_space* rep, const rsm_tiler* in, int32_t n_in, const rsm_tiler* out,
                           const rsm_task* task, uint32_t flags, const int32_t* spaces, int32_t n_spaces,
                           char* name, int32_t len, rsm_port_placement* ports, int32_t max_ports,
                           int32_t* n_ports) {
  RSM_GUARD_BEGIN
  Checked c;
  rsm_status s = check_task(rep, in, n_in, out, task, flags & ~RSM_CHECK_SINGLE_ASSIGN, &c);
  if (s) return s;
  const int count = n_in + 1 + (task->kind == RSM_TASK_WSUM ? 1 : 0);
  if ((s = check_spaces(spaces, n_spaces, count, n_in)) != RSM_OK) return s;
  const Plan p = make_plan(*rep, in, n_in, *out, *task, flags, nullptr, c.n_rep, c.n_pat_in[0], spaces);
  if (!p.ok) return fail(RSM_E_UNSUPPORTED, "no kernel of this library keeps the ports where requested");
  if (name && len > 0) std::snprintf(name, size_t(len), "%s", p.name.c_str());
  if (n_ports) *n_ports = count;
  if (ports) {
    if (max_ports < count) return fail(RSM_E_INVALID, "ports array too short");
    const Placement pl = placement_of(p, in, n_in, *task);
    for (int k = 0; k < count; ++k) {
      ports[k] = rsm_port_placement{};
      ports[k].port = k;
      ports[k].is_output = k == n_in ? 1 : 0;
      ports[k].space = pl.space[k];
      ports[k].bytes_per_workgroup = pl.bytes[k];
    }
  } else if (!name && !n_ports) {
    return fail(RSM_E_INVALID, "nothing to return: name, ports and n_ports are all NULL");
  }
  return RSM_OK;
  RSM_GUARD_END
}

rsm_status rsm_run_placed(const rsm_space* rep, const rsm_tiler* in, const void* const* d_in, int32_t n_in,
                          const rsm_tiler* out, void* d_out, const rsm_task* task, const int32_t* spaces,
                          int32_t n_spaces, uint32_t flags, void* hip_stream) {
  RSM_GUARD_BEGIN
  Checked c;
  rsm_status s = check_task(rep, in, n_in, out, task, flags, &c);
  if (s) return s;
  const int count = n_in + 1 + (task->kind == RSM_TASK_WSUM ? 1 : 0);
  if ((s = check_spaces(spaces, n_spaces, count, n_in)) != RSM_OK) return s;
  if (c.n_rep > 0 && (!ptrs_ok(d_in, n_in) || !d_out)) return fail(RSM_E_INVALID, "NULL device pointer");
  return exec_run(*rep, in, d_in, n_in, *out, d_out, *task, flags, c, static_cast<hipStream_t>(hip_stream),
                  spaces);
  RSM_GUARD_END
}

rsm_status rsm_indices(const rsm_space* rep, const rsm_tiler* t, int64_t* d_idx, void* hip_stream) {
  RSM_GUARD_BEGIN
  int64_t n_rep = 0, n_pat = 0;
  rsm_status s = check_space(rep, &n_rep);
  if (s) return s;
  s = check_tiler(t, rep, "tiler", &n_pat);
  if (s) return s;
  if (n_rep == 0) return RSM_OK;
  if (!d_idx) return fail(RSM_E_INVALID, "index buffer is NULL");
  int64_t total;
  if (!mul_ok(n_rep, n_pat, &total)) return fail(RSM_E_OVERFLOW, "index table has more than 2^62 entries");
  const GTiler g = to_gtiler(*t, rep->rank);
  hipError_t e = launch_indices(g, rep->rank, rep->shape, n_rep, n_pat, d_idx,
                                static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return hip_fail(e, "index launch");
  return RSM_OK;
  RSM_GUARD_END
}

rsm_status rsm_run(const rsm_space* rep, const rsm_tiler* in, const void* const* d_in, int32_t n_in,
                   const rsm_tiler* out, void* d_out, const rsm_task* task, uint32_t flags,
                   void* hip_stream) {
  RSM_GUARD_BEGIN
  const hipStream_t st = static_cast<hipStream_t>(hip_stream);
  // a descriptor seen before on this thread skips validation and planning
  thread_local std::vector<int64_t> key;
  const bool keyed = descriptor_key(rep, in, n_in, out, task, flags, d_in, &key);
  const uint64_t h = keyed ? key_hash(key) : 0;
  if (keyed) {
    if (const CachedPlan* e = plan_cache_find(key, h)) {
      ++g_plan_cache_hits;
      if (e->c.n_rep == 0) return RSM_OK;
      if (!ptrs_ok(d_in, n_in) || !d_out) return fail(RSM_E_INVALID, "NULL device pointer");
      return exec_planned(e->plan, *rep, in, d_in, n_in, *out, d_out, *task, e->c, st);
    }
  }
  Checked c;
  rsm_status s = check_task(rep, in, n_in, out, task, flags, &c);
  if (s) return s;
  if (c.n_rep == 0) {
    if (keyed) plan_cache_put(key, h, c, Plan{});
    return RSM_OK;
  }
  if (!ptrs_ok(d_in, n_in) || !d_out) return fail(RSM_E_INVALID, "NULL device pointer");
  const Plan p = make_plan(*rep, in, n_in, *out, *task, flags, d_in, c.n_rep, c.n_pat_in[0]);
  if (keyed) plan_cache_put(key, h, c, p);
  return exec_planned(p, *rep, in, d_in, n_in, *out, d_out, *task, c, st);
  RSM_GUARD_END
}

uint64_t rsm_plan_cache_hits(void) { return g_plan_cache_hits; }

}  // extern "C"

// A task validated and planned once.  The plan assumes inputs that start on
// 16-byte boundaries; a call with other addresses plans again for them.
struct rsm_prepared_s {
  rsm_space rep;
  rsm_tiler in[2];
  int32_t n_in;
  rsm_tiler out;
  rsm_task task;
  uint32_t flags;
  rsm::Checked c;
  rsm::Plan plan;
};

extern "C" {

rsm_status rsm_prepare(const rsm_space* rep, const rsm_tiler* in, int32_t n_in, const rsm_tiler* out,
                       const rsm_task* task, uint32_t flags, rsm_prepared* handle) {
  RSM_GUARD_BEGIN
  if (!handle) return fail(RSM_E_INVALID, "handle pointer is NULL");
  *handle = nullptr;
  if (!task) return fail(RSM_E_INVALID, "task is NULL");
  if (flags & ~uint32_t(RSM_CHECK_SINGLE_ASSIGN | RSM_FORCE_GENERIC))
    return fail(RSM_E_INVALID, "rsm_prepare takes RSM_CHECK_SINGLE_ASSIGN and RSM_FORCE_GENERIC only");
  // the weights are given per call: validate as if they were
  rsm_task tk = *task;
  tk.coeffs = tk.kind == RSM_TASK_WSUM ? static_cast<const void*>(task) : nullptr;
  Checked c;
  rsm_status s = check_task(rep, in, n_in, out, &tk, flags, &c);
  if (s) return s;
  rsm_prepared_s* p = new (std::nothrow) rsm_prepared_s();
  if (!p) return fail(RSM_E_NOMEM, "prepared task");
  p->rep = *rep;
  for (int t = 0; t < n_in; ++t) p->in[t] = in[t];
  p->n_in = n_in;
  p->out = *out;
  p->task = *task;
  p->task.coeffs = nullptr;
  p->flags = flags & RSM_FORCE_GENERIC;
  p->c = c;
  p->plan = make_plan(*rep, in, n_in, *out, tk, flags, nullptr, c.n_rep, c.n_pat_in[0]);
  *handle = p;
  return RSM_OK;
  RSM_GUARD_END
}

rsm_status rsm_prepared_name(const rsm_prepared_s* handle, char* name, int32_t len) {
  RSM_GUARD_BEGIN
  if (!handle) return fail(RSM_E_INVALID, "handle is NULL");
  if (!name || len <= 0) return fail(RSM_E_INVALID, "name buffer is NULL");
  std::snprintf(name, size_t(len), "%s", handle->plan.name.c_str());
  return RSM_OK;
  RSM_GUARD_END
}

rsm_status rsm_run_prepared(const rsm_prepared_s* h, const void* const* d_in, void* d_out,
                            const void* d_coeffs, void* hip_stream) {
  RSM_GUARD_BEGIN
  if (!h) return fail(RSM_E_INVALID, "handle is NULL");
  if (h->c.n_rep == 0) return RSM_OK;
  if (!ptrs_ok(d_in, h->n_in) || !d_out) return fail(RSM_E_INVALID, "NULL device pointer");
  rsm_task tk = h->task;
  if (tk.kind == RSM_TASK_WSUM) {
    if (!d_coeffs) return fail(RSM_E_INVALID, "WSUM needs coefficients");
    tk.coeffs = d_coeffs;
  }
  const hipStream_t st = static_cast<hipStream_t>(hip_stream);
  bool aligned = true;
  for (int t = 0; t < h->n_in; ++t) aligned = aligned && !(reinterpret_cast<uintptr_t>(d_in[t]) & 15);
  if (aligned) return exec_planned(h->plan, h->rep, h->in, d_in, h->n_in, h->out, d_out, tk, h->c, st);
  return exec_run(h->rep, h->in, d_in, h->n_in, h->out, d_out, tk, h->flags, h->c, st);
  RSM_GUARD_END
}

void rsm_prepared_destroy(rsm_prepared_s* handle) { delete handle; }

namespace rsm {
namespace {

// Both stages' weight gradients from a fused pair's partial rows
// [grid][taps0 + taps1] in one launch; a null output skips its columns.
hipError_t reduce_chain_partials(const float* partial, int grid, int taps0, float* g0, int taps1, float* g1,
                                 int row_stride, int accumulate, hipStream_t st) {
  if (g0 && g1) return launch_reduce_partial_pair(partial, grid, taps0, g0, taps1, g1, row_stride, accumulate, st);
  if (g0) return launch_reduce_partial_pair(partial, grid, taps0, g0, 0, nullptr, row_stride, accumulate, st);
  if (g1)
    return launch_reduce_partial_pair(partial + taps0, grid, 0, nullptr, taps1, g1, row_stride, accumulate, st);
  return hipSuccess;
}

// Bytes of workspace for the intermediate arrays of a chain (outputs of
// stages 0 .. n - 2), each rounded to 256 bytes; offs[k] = offset of the
// array of stage k.
size_t chain_mid_bytes(const rsm_stage* stages, int n, std::vector<size_t>* offs) {
  size_t total = 0;
  offs->assign(size_t(n > 1 ? n - 1 : 0), 0);
  for (int k = 0; k + 1 < n; ++k) {
    (*offs)[size_t(k)] = total;
    const rsm_tiler& o = stages[k].out;
    total += (size_t(prod(o.array_shape, o.array_rank)) * elem_size(o.dtype) + 255) & ~size_t(255);
  }
  return total;
}

// Runs stages 0 .. n - 2 of a chain into the intermediate arrays mids[k]
// (zero-filled first: elements a stage's output tiler does not cover read
// as zero in the next stage).  Chain stages are SUM / WSUM tasks, whose
// forward kernels take no workspace, so mids may live in the workspace.
rsm_status chain_forward_mids(const rsm_stage* stages, int n, const void* d_in, void* const* mids,
                              const std::vector<Checked>& cs, uint32_t flags, hipStream_t st) {
  for (int k = 0; k + 1 < n; ++k) {
    const rsm_stage& sg = stages[k];
    const int64_t bytes = prod(sg.out.array_shape, sg.out.array_rank) * int64_t(elem_size(sg.out.dtype));
    hipError_t e = launch_zero(mids[k], bytes, st);
    if (e != hipSuccess) return hip_fail(e, "zero intermediate");
    const void* src = k == 0 ? d_in : mids[k - 1];
    rsm_status s = exec_run(sg.rep, &sg.in, &src, 1, sg.out, mids[k], sg.task, flags & RSM_FORCE_GENERIC,
                            cs[size_t(k)], st);
    if (s) return s;
  }
  return RSM_OK;
}

// Workspace of the stage-by-stage chain adjoint: two intermediate-gradient
// buffers (alternating between stages) and the weight-gradient partial rows.
struct StagedLayout {
  size_t max_mid = 0, max_part = 0;
  std::vector<AdjPlan> aps;
  size_t bytes() const { return 2 * max_mid + max_part; }
};

StagedLayout staged_layout(const rsm_stage* stages, int n, const void* d_in, const void* const* d_mid,
                           void* const* d_gc, uint32_t flags, const std::vector<Checked>& cs) {
  StagedLayout l;
  l.aps.resize(size_t(n));
  for (int k = 0; k < n; ++k) {
    const rsm_stage& sg = stages[k];
    // a recomputed intermediate lives in the workspace, 256-byte aligned:
    // planned as aligned (no pointer)
    const void* xk = k == 0 ? d_in : (d_mid ? d_mid[k - 1] : nullptr);
    l.aps[size_t(k)] = plan_adjoint(sg.rep, sg.in, sg.out, sg.task, flags, xk, nullptr);
    l.max_part = std::max(l.max_part, adjoint_ws_bytes(l.aps[size_t(k)], cs[size_t(k)].n_rep,
                                                       cs[size_t(k)].n_pat_in[0], cs[size_t(k)].n_pat_out,
                                                       d_gc && d_gc[k]));
    if (k > 0) l.max_mid = std::max(l.max_mid, size_t(prod(sg.in.array_shape, sg.in.array_rank)) * 4);
  }
  l.max_mid = (l.max_mid + 255) & ~size_t(255);
  l.max_part = (l.max_part + 255) & ~size_t(255);
  return l;
}

// The chain's adjoint stage by stage, in reverse, from the forward
// intermediates fwd_mid; ws holds the layout's buffers.
rsm_status staged_adjoint(const rsm_stage* stages, int n, const void* d_in, const std::vector<void*>& fwd_mid,
                          const void* d_gy, void* d_gx, void* const* d_gc, uint32_t flags,
                          const std::vector<Checked>& cs, const StagedLayout& lay, char* ws, uint32_t* counter,
                          hipStream_t st) {
  const int accumulate = (flags & RSM_ACCUMULATE) ? 1 : 0;
  char* gbuf[2] = {ws, ws + lay.max_mid};
  void* part = ws + 2 * lay.max_mid;
  const void* g = d_gy;
  rsm_status s = RSM_OK;
  for (int k = n - 1; k >= 0; --k) {
    const rsm_stage& sg = stages[k];
    const void* xk = k == 0 ? d_in : fwd_mid[size_t(k - 1)];
    void* gxk = k == 0 ? d_gx : gbuf[k & 1];
    void* gck = d_gc ? d_gc[k] : nullptr;
    // intermediate gradients are overwritten; the caller's buffers follow the flags
    uint32_t fk = flags & (RSM_FORCE_GENERIC | RSM_REDUCE_IN_KERNEL);
    if (accumulate) fk |= RSM_ACCUMULATE;
    if (k > 0 && accumulate) {
      // accumulate applies to the caller's gc, not to the intermediate gradient
      if (gck) {
        s = exec_adjoint(sg.rep, sg.in, xk, sg.out, g, sg.task, nullptr, gck, fk, cs[size_t(k)], part,
                         counter, st);
        if (s) return s;
      }
      s = exec_adjoint(sg.rep, sg.in, xk, sg.out, g, sg.task, gxk, nullptr, fk & ~RSM_ACCUMULATE,
                       cs[size_t(k)], part, counter, st);
    } else {
      s = exec_adjoint(sg.rep, sg.in, xk, sg.out, g, sg.task, gxk, gck, fk, cs[size_t(k)], part,
                       counter, st);
    }
    if (s) return s;
    g = gxk;
    if (!g && k > 0) return fail(RSM_E_INVALID, "internal: missing intermediate gradient");
  }
  return RSM_OK;
}

// Training step of any two-stage chain of SUM / WSUM stages, stage by
// stage: the forward into the workspace intermediate and d_out, dL/dy =
// 2 (w y) into the workspace, then the staged adjoint.  Workspace layout:
// [adjoint buffers | forward intermediate | dL/dy].
rsm_status train_staged(const rsm_stage* stages, const void* d_in, const void* d_w, void* d_out, void* d_gx,
                        void* const* d_gc, uint32_t flags, const std::vector<Checked>& cs, hipStream_t st) {
  std::vector<size_t> mid_offs;
  const size_t mid_bytes = (chain_mid_bytes(stages, 2, &mid_offs) + 255) & ~size_t(255);
  const int64_t n_out = prod(stages[1].out.array_shape, stages[1].out.array_rank);
  const StagedLayout lay = staged_layout(stages, 2, d_in, nullptr, d_gc, flags, cs);
  rsm_status s = RSM_OK;
  uint32_t* counter = nullptr;
  char* ws = static_cast<char*>(workspace(lay.bytes() + mid_bytes + size_t(n_out) * 4 + 256, st, &s, &counter));
  if (s) return s;
  std::vector<void*> fwd_mid(1, ws + lay.bytes() + mid_offs[0]);
  float* g = reinterpret_cast<float*>(ws + lay.bytes() + mid_bytes);
  if ((s = chain_forward_mids(stages, 2, d_in, fwd_mid.data(), cs, flags, st)) != RSM_OK) return s;
  const void* src = fwd_mid[0];
  if ((s = exec_run(stages[1].rep, &stages[1].in, &src, 1, stages[1].out, d_out, stages[1].task,
                    flags & RSM_FORCE_GENERIC, cs[1], st)) != RSM_OK)
    return s;
  hipError_t e = launch_loss_grad(static_cast<const float*>(d_out), static_cast<const float*>(d_w), g, n_out, st);
  if (e != hipSuccess) return hip_fail(e, "loss gradient");
  return staged_adjoint(stages, 2, d_in, fwd_mid, g, d_gx, d_gc, flags, cs, lay, ws, counter, st);
}

}  // namespace
}  // namespace rsm

rsm_status rsm_run_chain(const rsm_stage* stages, int32_t n_stages, const void* d_in,
                         void* const* d_mid, void* d_out, uint32_t flags, void* hip_stream) {
  const KernelProbe probe = take_probe();
  RSM_GUARD_BEGIN
  std::vector<Checked> cs;
  rsm_status s = check_chain(stages, n_stages, &cs);
  if (s) return s;
  if (!d_in || !d_out) return fail(RSM_E_INVALID, "NULL device pointer");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const bool no_mid = !d_mid || !d_mid[0];
  Win3 h{}, v{};
  bool vec4 = false;
  if (!(flags & RSM_NO_FUSE) && !(flags & RSM_FORCE_GENERIC) && no_mid &&
      chain_fusable(stages, n_stages, d_in, &h, &v, &vec4)) {
    if (cs[1].n_rep == 0) return RSM_OK;
    FirChainArgs a{};
    a.h = h;
    a.v = v;
    a.div_rc = make_fastdiv(uint32_t(v.rep[2]));
    a.div_rr = make_fastdiv(uint32_t(v.rep[1]));
    a.n_out = uint32_t(cs[1].n_rep);
    a.x = static_cast<const float*>(d_in);
    a.y = static_cast<float*>(d_out);
    a.ch = static_cast<const float*>(stages[0].task.coeffs);
    a.cv = static_cast<const float*>(stages[1].task.coeffs);
    hipError_t e = probed(probe, st, [&] { return launch_fir_chain(a, vec4, st); });
    if (e != hipSuccess) return hip_fail(e, "fused chain launch");
    return RSM_OK;
  }
  std::vector<void*> mids(d_mid ? d_mid : nullptr, d_mid ? d_mid + (n_stages - 1) : nullptr);
  if (n_stages > 1 && (!d_mid || !ptrs_ok(const_cast<const void* const*>(d_mid), n_stages - 1))) {
    // no intermediate buffers given: the library's workspace holds them
    // (zero-filled first, as in chain_forward_mids)
    std::vector<size_t> offs;
    const size_t bytes = chain_mid_bytes(stages, n_stages, &offs);
    char* ws = static_cast<char*>(workspace(bytes, st, &s, nullptr));
    if (s) return s;
    mids.resize(size_t(n_stages - 1));
    for (int k = 0; k + 1 < n_stages; ++k) {
      mids[size_t(k)] = ws + offs[size_t(k)];
      const rsm_tiler& o = stages[k].out;
      hipError_t e = launch_zero(mids[size_t(k)], prod(o.array_shape, o.array_rank) * elem_size(o.dtype), st);
      if (e != hipSuccess) return hip_fail(e, "zero intermediate");
    }
  }
  for (int k = 0; k < n_stages; ++k) {
    const void* src = k == 0 ? d_in : mids[size_t(k - 1)];
    void* dst = k == n_stages - 1 ? d_out : mids[size_t(k)];
    const rsm_stage& sg = stages[k];
    s = exec_run(sg.rep, &sg.in, &src, 1, sg.out, dst, sg.task, flags, cs[size_t(k)], st);
    if (s) return s;
  }
  return RSM_OK;
  RSM_GUARD_END
}

rsm_status rsm_run_adjoint(const rsm_space* rep, const rsm_tiler* in, const void* d_x,
                           const rsm_tiler* out, const void* d_gy, const rsm_task* task, void* d_gx,
                           void* d_gc, uint32_t flags, void* hip_stream) {
  RSM_GUARD_BEGIN
  Checked c;
  rsm_status s = check_adjoint(rep, in, out, task, &c);
  if (s) return s;
  if (!d_gx && !d_gc) return RSM_OK;
  if (d_gc && task->kind != RSM_TASK_WSUM) return fail(RSM_E_INVALID, "weight gradient needs a WSUM task");
  if (c.n_rep > 0 && (!d_gy || (d_gc && !d_x))) return fail(RSM_E_INVALID, "NULL device pointer");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const AdjPlan ap = plan_adjoint(*rep, *in, *out, *task, flags, d_x, d_gx);
  const size_t wsb = adjoint_ws_bytes(ap, c.n_rep, c.n_pat_in[0], c.n_pat_out, d_gc != nullptr);
  void* ws = nullptr;
  uint32_t* counter = nullptr;
  if (wsb) {
    ws = workspace(wsb, st, &s, &counter);
    if (s) return s;
  }
  return exec_adjoint(*rep, *in, d_x, *out, d_gy, *task, d_gx, d_gc, flags, c, ws, counter, st);
  RSM_GUARD_END
}

rsm_status rsm_run_chain_adjoint(const rsm_stage* stages, int32_t n_stages, const void* d_in,
                                 const void* const* d_mid, const void* d_gy, void* d_gx,
                                 void* const* d_gc, uint32_t flags, void* hip_stream) {
  const KernelProbe probe = take_probe();
  RSM_GUARD_BEGIN
  std::vector<Checked> cs;
  rsm_status s = check_chain(stages, n_stages, &cs);
  if (s) return s;
  for (int k = 0; k < n_stages; ++k) {
    Checked tmp;
    s = check_adjoint(&stages[k].rep, &stages[k].in, &stages[k].out, &stages[k].task, &tmp);
    if (s) return fail(s, "stage " + std::to_string(k) + ": " + g_last_error);
    if (d_gc && d_gc[k] && stages[k].task.kind != RSM_TASK_WSUM)
      return fail(RSM_E_INVALID, "weight gradient needs a WSUM stage");
  }
  if (!d_in || !d_gy) return fail(RSM_E_INVALID, "NULL device pointer");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int accumulate = (flags & RSM_ACCUMULATE) ? 1 : 0;
  const bool no_mid = !d_mid || !d_mid[0];
  Win3 h{}, v{};
  bool vec4 = false;
  hipError_t e;
  if (!(flags & RSM_NO_FUSE) && !(flags & RSM_FORCE_GENERIC) && no_mid &&
      chain_fusable(stages, n_stages, d_in, &h, &v, &vec4) && h.taps <= 16 && v.taps <= 16 &&
      fir_injective(h) && fir_injective(v) && cs[1].n_rep > 0) {
    vec4 = vec4 && fir_vec4(h, d_gx);
    float* gch = d_gc ? static_cast<float*>(d_gc[0]) : nullptr;
    float* gcv = d_gc ? static_cast<float*>(d_gc[1]) : nullptr;
    if (d_gx && !accumulate && !(fir_exact_cover(h) && fir_exact_cover(v))) {
      if ((e = launch_zero(d_gx, int64_t(h.A[0]) * h.A[1] * h.A[2] * 4, st)) != hipSuccess)
        return hip_fail(e, "zero gx");
    }
    FirChainAdjArgs a{};
    a.h = h;
    a.v = v;
    a.div_rc = make_fastdiv(uint32_t(v.rep[2]));
    a.div_rr = make_fastdiv(uint32_t(v.rep[1]));
    a.n_out = uint32_t(cs[1].n_rep);
    a.x = static_cast<const float*>(d_in);
    a.gy = static_cast<const float*>(d_gy);
    a.gx = static_cast<float*>(d_gx);
    a.ch = static_cast<const float*>(stages[0].task.coeffs);
    a.cv = static_cast<const float*>(stages[1].task.coeffs);
    a.accumulate = accumulate;
    a.gch = gch;
    a.gcv = gcv;
    const int grid = fir_chain_adjoint_grid(a, vec4);
    const int nc = h.taps + v.taps;
    if (gch || gcv) {
      a.partial = static_cast<float*>(workspace(size_t(grid) * nc * sizeof(float), st, &s, &a.counter));
      if (s) return s;
      if (!(flags & RSM_REDUCE_IN_KERNEL)) a.counter = nullptr;
    }
    if ((e = probed(probe, st, [&] { return launch_fir_chain_adjoint(a, vec4, st); })) != hipSuccess)
      return hip_fail(e, "fused chain adjoint");
    if (a.partial && !a.counter &&
        (e = reduce_chain_partials(a.partial, grid, h.taps, gch, v.taps, gcv, nc, accumulate, st)) !=
            hipSuccess)
      return hip_fail(e, "weight-gradient reduction");
    return RSM_OK;
  }
  // stage by stage, in reverse; intermediate gradients live in the workspace,
  // and so do the forward intermediates when the caller gives none (they are
  // recomputed first)
  const bool have_mid = n_stages == 1 || (d_mid && ptrs_ok(d_mid, n_stages - 1));
  std::vector<size_t> mid_offs;
  const size_t fwd_bytes = have_mid ? 0 : chain_mid_bytes(stages, n_stages, &mid_offs);
  std::vector<void*> fwd_mid(size_t(n_stages > 1 ? n_stages - 1 : 0), nullptr);
  if (have_mid)
    for (int k = 0; k + 1 < n_stages; ++k) fwd_mid[size_t(k)] = const_cast<void*>(d_mid[k]);
  const StagedLayout lay = staged_layout(stages, n_stages, d_in, have_mid ? d_mid : nullptr, d_gc, flags, cs);
  uint32_t* counter = nullptr;
  char* ws = static_cast<char*>(workspace(lay.bytes() + fwd_bytes + 256, st, &s, &counter));
  if (s) return s;
  if (!have_mid) {
    for (int k = 0; k + 1 < n_stages; ++k) fwd_mid[size_t(k)] = ws + lay.bytes() + mid_offs[size_t(k)];
    if ((s = chain_forward_mids(stages, n_stages, d_in, fwd_mid.data(), cs, flags, st)) != RSM_OK) return s;
  }
  return staged_adjoint(stages, n_stages, d_in, fwd_mid, d_gy, d_gx, d_gc, flags, cs, lay, ws, counter, st);
  RSM_GUARD_END
}

rsm_status rsm_run_chain_train(const rsm_stage* stages, int32_t n_stages, const void* d_in, const void* d_w,
                               void* d_out, void* d_gx, void* const* d_gc, uint32_t flags, void* hip_stream) {
  return rsm::chain_train_step(stages, n_stages, d_in, d_w, d_out, d_gx, d_gc, flags, hip_stream, nullptr, 0);
}

}  // extern "C"

namespace rsm {

rsm_status chain_train_step(const rsm_stage* stages, int32_t n_stages, const void* d_in, const void* d_w,
                            void* d_out, void* d_gx, void* const* d_gc, uint32_t flags, void* hip_stream,
                            float* fixed_partial, size_t fixed_bytes) {
  const KernelProbe probe = take_probe();
  RSM_GUARD_BEGIN
  std::vector<Checked> cs;
  rsm_status s = check_chain(stages, n_stages, &cs);
  if (s) return s;
  for (int k = 0; k < n_stages; ++k) {
    Checked tmp;
    s = check_adjoint(&stages[k].rep, &stages[k].in, &stages[k].out, &stages[k].task, &tmp);
    if (s) return fail(s, "stage " + std::to_string(k) + ": " + g_last_error);
    if (d_gc && d_gc[k] && stages[k].task.kind != RSM_TASK_WSUM)
      return fail(RSM_E_INVALID, "weight gradient needs a WSUM stage");
  }
  if (!d_in || !d_w || !d_out) return fail(RSM_E_INVALID, "NULL device pointer");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const int accumulate = (flags & RSM_ACCUMULATE) ? 1 : 0;
  if (n_stages != 2) return fail(RSM_E_UNSUPPORTED, "the training step takes a chain of two stages");
  Win3 h{}, v{};
  bool vec4 = false;
  const bool fusable = !(flags & (RSM_NO_FUSE | RSM_FORCE_GENERIC)) &&
                       chain_fusable(stages, n_stages, d_in, &h, &v, &vec4) && fir_injective(h) &&
                       fir_injective(v) && h.taps <= 16 && v.taps <= 16;
  const bool pair8 = fusable && h.taps == 8 && v.taps == 8 && vec4 && fir_vec4(h, d_gx);
  if (!fusable) {
    // any other pair of stages: forward stage by stage, dL/dy = 2 w y, then
    // the stage-by-stage adjoint, through the library's workspace
    if (fixed_partial)
      return fail(RSM_E_UNSUPPORTED,
                  "without allocation the training step takes only chains it runs in one pass (two "
                  "weighted sums along columns then rows, windows that do not overlap, at most 16 taps "
                  "each); this chain runs stage by stage through the library's workspace");
    return train_staged(stages, d_in, d_w, d_out, d_gx, d_gc, flags, cs, st);
  }
  if (cs[1].n_rep == 0) return RSM_OK;
  hipError_t e;
  if (d_gx && !accumulate && !(fir_exact_cover(h) && fir_exact_cover(v))) {
    if ((e = launch_zero(d_gx, int64_t(h.A[0]) * h.A[1] * h.A[2] * 4, st)) != hipSuccess)
      return hip_fail(e, "zero gx");
  }
  FirChainAdjArgs a{};
  a.h = h;
  a.v = v;
  a.div_rc = make_fastdiv(uint32_t(v.rep[2]));
  a.div_rr = make_fastdiv(uint32_t(v.rep[1]));
  a.n_out = uint32_t(cs[1].n_rep);
  a.x = static_cast<const float*>(d_in);
  a.gx = static_cast<float*>(d_gx);
  a.ch = static_cast<const float*>(stages[0].task.coeffs);
  a.cv = static_cast<const float*>(stages[1].task.coeffs);
  a.accumulate = accumulate;
  a.wl = static_cast<const float*>(d_w);
  a.y = static_cast<float*>(d_out);
  float* gch = d_gc ? static_cast<float*>(d_gc[0]) : nullptr;
  float* gcv = d_gc ? static_cast<float*>(d_gc[1]) : nullptr;
  // 8-tap lane-pair kernel: partial rows of 8 + 8 (the horizontal taps split
  // over the two lanes); other pairs: one thread per output, rows of t0 + t1
  const int grid = pair8 ? fir_chain_adjoint_grid(a, true) : fir_chain_train_generic_grid(a);
  const int nc = h.taps + v.taps;
  if (gch || gcv) {
    const size_t need = size_t(grid) * nc * sizeof(float);
    if (fixed_partial) {
      // the caller's fixed buffer (no allocation on this path)
      if (need > fixed_bytes)
        return fail(RSM_E_UNSUPPORTED, "weight-gradient partial rows need " + std::to_string(need) +
                                           " bytes, more than the fixed scratch buffer's " +
                                           std::to_string(fixed_bytes));
      a.partial = fixed_partial;
    } else {
      a.partial = static_cast<float*>(workspace(need, st, &s, nullptr));
      if (s) return s;
    }
  }
  if ((e = probed(probe, st, [&] {
         return pair8 ? launch_fir_chain_train(a, st) : launch_fir_chain_train_generic(a, st);
       })) != hipSuccess)
    return hip_fail(e, "fused training step");
  if ((gch || gcv) && (e = reduce_chain_partials(a.partial, grid, h.taps, gch, v.taps, gcv, nc, accumulate,
                                                 st)) != hipSuccess)
    return hip_fail(e, "weight-gradient reduction");
  return RSM_OK;
  RSM_GUARD_END
}

}  // namespace rsm

extern "C" {

rsm_status rsm_run_csr(int64_t n_rows, int64_t n_cols, int64_t nnz, const int32_t* d_row_ptr,
                       const int32_t* d_col_idx, const void* d_vals, const void* d_x, void* d_y,
                       int32_t dtype, uint32_t flags, void* hip_stream) {
  RSM_GUARD_BEGIN
  rsm_status s = check_csr_sizes(n_rows, n_cols, nnz);
  if (s != RSM_OK) return s;
  if (dtype != RSM_F64 && dtype != RSM_F32) return fail(RSM_E_INVALID, "CSR dtype must be F64 or F32");
  if (n_rows == 0) return RSM_OK;
  if (!d_row_ptr || !d_y || (nnz > 0 && (!d_col_idx || !d_vals)) || (n_cols > 0 && !d_x))
    return fail(RSM_E_INVALID, "NULL device pointer");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if ((flags & RSM_CHECK_INDICES) &&
      (s = check_csr_indices(n_rows, n_cols, nnz, d_row_ptr, d_col_idx, st)) != RSM_OK)
    return s;
  CsrArgs a{n_rows, n_cols, nnz, d_row_ptr, d_col_idx, d_vals, d_x, d_y};
  hipError_t e;
  if ((e = launch_csr(a, dtype, st)) != hipSuccess) return hip_fail(e, "csr launch");
  return RSM_OK;
  RSM_GUARD_END
}

namespace rsm {
namespace {

// One captured batch of CG iterations per device, replayed while the launch
// arguments stay the same (a solver called again on the same buffers, as in
// a time-stepping loop).  Captured on a library stream (capture is not
// allowed on the null stream) and replayed on the caller's.  The graph holds
// kernel launches only.
struct CgGraph {
  unsigned char key[sizeof(CgArgs)];
  int iters = 0;
  bool valid = false;
  hipGraphExec_t exec = nullptr;
  hipStream_t cap = nullptr;
};
CgGraph g_cg_graph[64];
std::mutex g_cg_mutex;

hipError_t cg_graph_launch(const CgArgs& a, int iters, hipStream_t st) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= 64) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_cg_mutex);
  CgGraph& g = g_cg_graph[dev];
  if (!(g.valid && g.iters == iters && std::memcmp(g.key, &a, sizeof(CgArgs)) == 0)) {
    if (g.exec) {
      (void)hipGraphExecDestroy(g.exec);
      g.exec = nullptr;
    }
    g.valid = false;
    if (!g.cap && (e = hipStreamCreateWithFlags(&g.cap, hipStreamNonBlocking)) != hipSuccess) return e;
    if ((e = hipStreamBeginCapture(g.cap, hipStreamCaptureModeThreadLocal)) != hipSuccess) return e;
    const hipError_t le = launch_cg(a, false, iters, g.cap);
    hipGraph_t graph = nullptr;
    e = hipStreamEndCapture(g.cap, &graph);
    if (le != hipSuccess || e != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      return le != hipSuccess ? le : e;
    }
    e = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) {
      g.exec = nullptr;
      return e;
    }
    std::memcpy(g.key, &a, sizeof(CgArgs));
    g.iters = iters;
    g.valid = true;
  }
  return hipGraphLaunch(g.exec, st);
}

}  // namespace
}  // namespace rsm

rsm_status rsm_cg_solve(int64_t n, int64_t nnz, const int32_t* d_row_ptr, const int32_t* d_col_idx,
                        const double* d_vals, const double* d_b, double* d_x, double tol, int64_t max_iter,
                        int32_t check_every, uint32_t flags, double* d_res, double* d_alpha, double* d_beta,
                        rsm_cg_info* info, void* hip_stream) {
  RSM_GUARD_BEGIN
  if (!info) return fail(RSM_E_INVALID, "NULL info");
  *info = rsm_cg_info{};
  rsm_status s = check_csr_sizes(n, n, nnz);
  if (s != RSM_OK) return s;
  if (!(tol >= 0.0)) return fail(RSM_E_INVALID, "tol must be >= 0");
  if (max_iter < 0) return fail(RSM_E_INVALID, "max_iter must be >= 0");
  if (check_every < 1) return fail(RSM_E_INVALID, "check_every must be >= 1");
  if (n == 0) {
    info->converged = 1;
    return RSM_OK;
  }
  if (!d_row_ptr || !d_b || !d_x || (nnz > 0 && (!d_col_idx || !d_vals)))
    return fail(RSM_E_INVALID, "NULL device pointer");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if ((flags & RSM_CHECK_INDICES) && (s = check_csr_indices(n, n, nnz, d_row_ptr, d_col_idx, st)) != RSM_OK)
    return s;
  const int grid_rows = cg_grid(n, nnz), grid_vec = cg_vec_grid(n);
  const size_t vec = (size_t(n) * sizeof(double) + 255) & ~size_t(255);
  const size_t part = (size_t(std::max(grid_rows, grid_vec)) * sizeof(double) + 255) & ~size_t(255);
  char* ws = static_cast<char*>(workspace(4 * vec + 3 * part + 256, st, &s, nullptr));
  if (s != RSM_OK) return s;
  CgArgs a{};
  a.n = n;
  a.nnz = nnz;
  a.row_ptr = d_row_ptr;
  a.col_idx = d_col_idx;
  a.vals = d_vals;
  a.b = d_b;
  a.x = d_x;
  a.r = reinterpret_cast<double*>(ws);
  a.p0 = reinterpret_cast<double*>(ws + vec);
  a.p1 = reinterpret_cast<double*>(ws + 2 * vec);
  a.q = reinterpret_cast<double*>(ws + 3 * vec);
  a.part_pq = reinterpret_cast<double*>(ws + 4 * vec);
  a.part_rr = reinterpret_cast<double*>(ws + 4 * vec + part);
  a.part_bb = reinterpret_cast<double*>(ws + 4 * vec + 2 * part);
  a.st = reinterpret_cast<CgState*>(ws + 4 * vec + 3 * part);
  a.res = d_res;
  a.alpha = d_alpha;
  a.beta = d_beta;
  a.tol = tol;
  a.max_iter = max_iter;
  a.grid_rows = grid_rows;
  a.grid_vec = grid_vec;
  hipError_t e = launch_cg(a, true, 0, st);
  if (e != hipSuccess) return hip_fail(e, "cg start launch");
  // Launch batches of check_every iterations and read the state after each;
  // the stop test fires by iteration max_iter at the latest, so the loop
  // ends after at most max_iter / check_every + 2 batches.
  CgState h{};
  for (int64_t launched = 0;; launched += check_every) {
    e = (flags & RSM_NO_GRAPH) ? launch_cg(a, false, check_every, st) : cg_graph_launch(a, check_every, st);
    if (e != hipSuccess) return hip_fail(e, "cg loop launch");
    if ((e = hipMemcpyAsync(&h, a.st, sizeof(h), hipMemcpyDeviceToHost, st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return hip_fail(e, "cg state read");
    if (h.done || h.breakdown) break;
    if (launched > max_iter + 2 * int64_t(check_every))
      return fail(RSM_E_HIP, "cg loop did not reach its stop test");
  }
  const double rho = h.rho[h.k & 1];
  info->iterations = h.k;
  info->residual_norm = std::sqrt(rho);
  info->rhs_norm = h.bnorm;
  info->breakdown = h.breakdown;
  info->converged = !h.breakdown && !(std::sqrt(rho) > tol * h.bnorm);
  return RSM_OK;
  RSM_GUARD_END
}

}  // extern "C"
