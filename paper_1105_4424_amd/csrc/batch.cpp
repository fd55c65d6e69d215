// batch.cpp -- many independent repetitive tasks behind one handle.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "rsm_internal.h"

struct rsm_batch_s {
  std::vector<rsm_problem> problems;
  std::vector<int32_t> tile_rows, tile_cols;
  rsm_batch_info info{};
};

using namespace rsm;

extern "C" {

rsm_status rsm_batch_create(const rsm_problem* problems, int32_t n, const char* /*tune_cache_path*/,
                            uint32_t flags, void* /*hip_stream*/, rsm_batch* out) {
  try {
    if (!out) return fail(RSM_E_INVALID, "output handle pointer is NULL");
    *out = nullptr;
    if (n < 0 || (n > 0 && !problems)) return fail(RSM_E_INVALID, "bad problem list");
    for (int k = 0; k < n; ++k) {
      const rsm_problem& p = problems[k];
      rsm_status s = rsm_validate(&p.rep, &p.in, 1, &p.out, &p.task, flags & RSM_CHECK_SINGLE_ASSIGN);
      if (s) return fail(s, "problem " + std::to_string(k) + ": " + rsm_last_error());
      if (p.task.kind == RSM_TASK_DOT) return fail(RSM_E_INVALID, "batched problems take one input");
    }
    rsm_batch_s* b = new rsm_batch_s;
    b->problems.assign(problems, problems + n);
    b->tile_rows.assign(size_t(n), 0);
    b->tile_cols.assign(size_t(n), 0);
    b->info.n_problems = n;
    *out = b;
    return RSM_OK;
  } catch (const std::bad_alloc&) {
    return fail(RSM_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(RSM_E_INVALID, "internal error (exception)");
  }
}

rsm_status rsm_batch_run(rsm_batch b, void* hip_stream) {
  if (!b) return fail(RSM_E_INVALID, "batch handle is NULL");
  for (size_t k = 0; k < b->problems.size(); ++k) {
    const rsm_problem& p = b->problems[k];
    const void* src = p.d_in;
    rsm_status s = rsm_run(&p.rep, &p.in, &src, 1, &p.out, p.d_out, &p.task, 0, hip_stream);
    if (s) return s;
  }
  return RSM_OK;
}

rsm_status rsm_batch_query(rsm_batch b, rsm_batch_info* info) {
  if (!b || !info) return fail(RSM_E_INVALID, "NULL argument");
  *info = b->info;
  return RSM_OK;
}

rsm_status rsm_batch_tile(rsm_batch b, int32_t k, int32_t* tile_rows, int32_t* tile_cols) {
  if (!b || !tile_rows || !tile_cols) return fail(RSM_E_INVALID, "NULL argument");
  if (k < 0 || size_t(k) >= b->problems.size()) return fail(RSM_E_INVALID, "problem index out of range");
  *tile_rows = b->tile_rows[size_t(k)];
  *tile_cols = b->tile_cols[size_t(k)];
  return RSM_OK;
}

rsm_status rsm_batch_destroy(rsm_batch b) {
  delete b;
  return RSM_OK;
}

}  // extern "C"
