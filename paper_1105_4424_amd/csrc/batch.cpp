// batch.cpp -- many independent repetitive tasks behind one handle.
//
// Problems that are k x k weighted windows (the 2-D filter family) go to one
// persistent kernel: the host orders them by decreasing estimated cost
// (max of HBM time and FP32 ALU time), lays their tiles out in that order,
// and uploads the descriptor table and the (problem, tile) table once.  The persistent kernel walks the (problem, tile) table round-robin.
// The first rsm_batch_run captures the persistent launch into a HIP
// graph on a private stream; every call replays the graph on the caller's
// stream.  Remaining problems run through rsm_run in the same call.
//
// Tile shapes come from an autotuner: problems are grouped into classes
// (window side, stride, output-size bucket); for each class missing from the
// tuning cache every tile class is timed with HIP events over that class's
// own problems (plain launches, best of 3), and the fastest is kept.  The
// cache is a small JSON object keyed by class, stamped with the device
// architecture and the kernel revision; a file that does not parse or carries
// another stamp is ignored and rewritten.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <map>
#include <new>
#include <sstream>
#include <string>
#include <vector>

#include "rsm_internal.h"

namespace {

constexpr const char* kKernelRevision = "filter2d-r11";
constexpr double kHbmBytesPerS = 8.0e12;
constexpr double kFp32FmaPerS = 39.3e12;   // unpacked FP32 FMA issue rate of the chip

std::string arch_name() {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  const size_t colon = a.find(':');
  return colon == std::string::npos ? a : a.substr(0, colon);
}

std::string class_key(const rsm::Filter2DProblem& p) {
  const int64_t outs = int64_t(p.RH) * p.RW * p.frames;
  const int bucket = outs < (int64_t(1) << 12) ? 0 : outs < (int64_t(1) << 16) ? 1 : 2;
  return "k" + std::to_string(p.k) + "_s" + std::to_string(p.s) + "_b" + std::to_string(bucket);
}

double est_cost(const rsm::Filter2DProblem& p) {
  const double outs = double(p.RH) * p.RW * p.frames;
  const double bytes = 4.0 * (double(p.H) * p.W * p.frames + outs);
  const double fmas = outs * p.k * p.k;
  return std::max(bytes / kHbmBytesPerS, fmas / kFp32FmaPerS);
}

// {"revision": "...", "arch": "...", "choices": {"k3_s1_b2": 1, ...}}
bool load_cache(const std::string& path, const std::string& arch, std::map<std::string, int>* out) {
  std::ifstream f(path);
  if (!f) return false;
  std::stringstream ss;
  ss << f.rdbuf();
  const std::string t = ss.str();
  auto field = [&](const std::string& name) -> std::string {
    const std::string key = "\"" + name + "\"";
    size_t i = t.find(key);
    if (i == std::string::npos) return "";
    i = t.find('"', t.find(':', i + key.size()) + 1);
    if (i == std::string::npos) return "";
    const size_t j = t.find('"', i + 1);
    return j == std::string::npos ? "" : t.substr(i + 1, j - i - 1);
  };
  if (field("revision") != kKernelRevision || field("arch") != arch) return false;
  size_t i = t.find("\"choices\"");
  if (i == std::string::npos) return false;
  i = t.find('{', i);
  const size_t end = t.find('}', i);
  if (i == std::string::npos || end == std::string::npos) return false;
  std::map<std::string, int> m;
  size_t pos = i + 1;
  while (true) {
    const size_t a = t.find('"', pos);
    if (a == std::string::npos || a > end) break;
    const size_t b = t.find('"', a + 1);
    const size_t c = t.find(':', b);
    if (b == std::string::npos || c == std::string::npos || c > end) return false;
    char* e = nullptr;
    const long v = std::strtol(t.c_str() + c + 1, &e, 10);
    if (e == t.c_str() + c + 1 || v < 0 || v > 2) return false;
    m[t.substr(a + 1, b - a - 1)] = int(v);
    pos = size_t(e - t.c_str());
  }
  *out = m;
  return true;
}

void save_cache(const std::string& path, const std::string& arch, const std::map<std::string, int>& m) {
  const std::string tmp = path + ".tmp";
  {
    std::ofstream f(tmp);
    if (!f) return;
    f << "{\"revision\": \"" << kKernelRevision << "\", \"arch\": \"" << arch << "\", \"choices\": {";
    bool first = true;
    for (const auto& kv : m) {
      f << (first ? "" : ", ") << "\"" << kv.first << "\": " << kv.second;
      first = false;
    }
    f << "}}\n";
  }
  std::rename(tmp.c_str(), path.c_str());
}

}  // namespace

struct rsm_batch_s {
  std::vector<rsm_problem> problems;
  std::vector<int> persistent;                 // problem indices, in queue order
  std::vector<int> others;                     // problem indices run through rsm_run
  std::vector<rsm::Filter2DProblem> fp;        // per problem (valid for persistent ones)
  rsm::Filter2DProblem* d_probs = nullptr;
  uint32_t* d_tiles = nullptr;                 // [n_tiles][2]: problem (table row), tile
  int64_t n_tiles = 0;
  int grid = 0;
  int buf_floats = 4;   // LDS of the persistent kernel (floats)
  int device = 0;
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  rsm_batch_info info{};

  ~rsm_batch_s() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (d_probs) (void)hipFree(d_probs);
    if (d_tiles) (void)hipFree(d_tiles);
  }
};

using namespace rsm;

namespace {

// Times tile class tc over the given problems (plain launches), best of 3, in ms.
// Times tile class tc for one class of problems the way the batch runs them:
// a table of these problems' tiles walked by the persistent kernel (three
// back-to-back launches after a warm-up, so the figure is GPU time).  In the
// batch a class shares the chip with every other class, so what counts is
// its cost in a full machine, not the latency of its few tiles alone: the
// table repeats the class's tiles until it holds at least four resident
// grids' worth, and the time is divided by the repeat count.  (Timed alone
// and unrepeated, small classes favoured their smallest tiles, whose extra
// halo the whole batch then paid.)
rsm_status time_class(rsm_batch_s* b, const std::vector<int>& idx, int tc, hipStream_t st, float* ms) {
  std::vector<Filter2DProblem> probs;
  std::vector<uint32_t> tiles;
  for (int k : idx) {
    Filter2DProblem p = b->fp[size_t(k)];
    filter2d_set_tiles(&p, tc);
    for (int64_t t = 0; t < p.n_tiles; ++t) {
      tiles.push_back(uint32_t(probs.size()));
      tiles.push_back(uint32_t(t));
    }
    probs.push_back(p);
  }
  const int64_t class_tiles = int64_t(tiles.size() / 2);
  *ms = 0.0f;
  if (class_tiles == 0) return RSM_OK;
  const int64_t fill = 4 * int64_t(filter2d_persistent_grid(filter2d_buf_floats(probs[0].k, probs[0].s, tc)));
  const int64_t reps = std::max<int64_t>(1, (fill + class_tiles - 1) / class_tiles);
  const std::vector<uint32_t> once = tiles;
  for (int64_t r = 1; r < reps; ++r) tiles.insert(tiles.end(), once.begin(), once.end());
  const int64_t n_tiles = int64_t(tiles.size() / 2);
  void *d_probs = nullptr, *d_tiles = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e;
  rsm_status s = RSM_OK;
  if ((e = hipMalloc(&d_probs, sizeof(Filter2DProblem) * probs.size())) != hipSuccess ||
      (e = hipMalloc(&d_tiles, sizeof(uint32_t) * tiles.size())) != hipSuccess) {
    s = fail(RSM_E_NOMEM, std::string("autotuner tables: ") + hipGetErrorString(e));
  } else if ((e = hipMemcpy(d_probs, probs.data(), sizeof(Filter2DProblem) * probs.size(),
                            hipMemcpyHostToDevice)) != hipSuccess ||
             (e = hipMemcpy(d_tiles, tiles.data(), sizeof(uint32_t) * tiles.size(), hipMemcpyHostToDevice)) !=
                 hipSuccess ||
             (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
    s = hip_fail(e, "autotuner setup");
  } else {
    const int bf = filter2d_buf_floats(probs[0].k, probs[0].s, tc);
    const int grid = int(std::min<int64_t>(filter2d_persistent_grid(bf), n_tiles));
    auto launch = [&] {
      return launch_filter2d_persistent(static_cast<const Filter2DProblem*>(d_probs), d_tiles, n_tiles, grid, bf,
                                        st);
    };
    if ((e = launch()) != hipSuccess || (e = hipEventRecord(e0, st)) != hipSuccess ||
        (e = launch()) != hipSuccess || (e = launch()) != hipSuccess || (e = launch()) != hipSuccess ||
        (e = hipEventRecord(e1, st)) != hipSuccess || (e = hipEventSynchronize(e1)) != hipSuccess) {
      s = hip_fail(e, "autotuner launch");
    } else {
      float t = 0.0f;
      (void)hipEventElapsedTime(&t, e0, e1);
      *ms = t / 3.0f / float(reps);
    }
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  // the launches above must be done before the tables go away
  (void)hipStreamSynchronize(st);
  if (d_probs) (void)hipFree(d_probs);
  if (d_tiles) (void)hipFree(d_tiles);
  return s;
}

// Tile order: problems grouped by code path (k, s, tile class), groups in
// decreasing order of their total estimated cost, problems inside a group in
// decreasing cost.  The persistent kernel inlines one code path per group
// and all of them together exceed the instruction cache that two CUs share;
// since the workgroups in flight at any moment work on a window of
// consecutive tiles, grouping keeps that window on one or two code paths.
rsm_status build_queue(rsm_batch_s* b) {
  auto path = [&](int i) {
    const Filter2DProblem& f = b->fp[size_t(i)];
    return (int64_t(f.k) << 16) | (int64_t(f.s) << 8) | int64_t(f.tc);
  };
  std::map<int64_t, double> group_cost;
  for (int i : b->persistent) group_cost[path(i)] += est_cost(b->fp[size_t(i)]);
  std::stable_sort(b->persistent.begin(), b->persistent.end(), [&](int x, int y) {
    const int64_t px = path(x), py = path(y);
    if (px != py) {
      const double cx = group_cost[px], cy = group_cost[py];
      return cx != cy ? cx > cy : px < py;
    }
    return est_cost(b->fp[size_t(x)]) > est_cost(b->fp[size_t(y)]);
  });
  const size_t n = b->persistent.size();
  std::vector<Filter2DProblem> table(n);
  int64_t total = 0;
  for (size_t i = 0; i < n; ++i) {
    table[i] = b->fp[size_t(b->persistent[i])];
    total += table[i].n_tiles;
  }
  b->n_tiles = total;
  if (b->n_tiles >= (int64_t(1) << 31)) return fail(RSM_E_UNSUPPORTED, "batch has more than 2^31 tiles");
  // XCD-aware layout.  Workgroup b runs table entries b, b + grid, ... and
  // the hardware deals workgroups round-robin to the 8 XCDs, so with grid a
  // multiple of 8 entry p runs on XCD p mod 8, and each XCD has its own L2.
  // Each problem's tiles (row-major over the tile grid) are cut into 8
  // contiguous bands, band x going to XCD x (remainder tiles to the XCDs
  // with the fewest tiles so far), and entry 8 j + x holds the j-th tile of
  // XCD x: spatial neighbours, which share halo rows and cache lines, share
  // an L2, and every XCD gets an eighth of every problem in the same order.
  constexpr int kXcd = 8;
  std::vector<std::vector<uint32_t>> band(kXcd);
  std::vector<int64_t> len(kXcd, 0);
  for (size_t i = 0; i < n; ++i) {
    const int64_t nt = table[i].n_tiles, q = nt / kXcd;
    int rem = int(nt % kXcd);
    std::vector<int> order(kXcd);
    for (int x = 0; x < kXcd; ++x) order[size_t(x)] = x;
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) { return len[size_t(a)] < len[size_t(c)]; });
    std::vector<int64_t> size(kXcd, q);
    for (int r = 0; r < rem; ++r) size[size_t(order[size_t(r)])] += 1;
    int64_t k = 0;
    for (int x = 0; x < kXcd; ++x)
      for (int64_t c = 0; c < size[size_t(x)]; ++c, ++k) {
        band[size_t(x)].push_back(uint32_t(i));
        band[size_t(x)].push_back(uint32_t(k));
        len[size_t(x)] += 1;
      }
  }
  std::vector<uint32_t> tiles;
  tiles.reserve(size_t(2 * std::max<int64_t>(total, 1)));
  const int64_t longest = *std::max_element(len.begin(), len.end());
  for (int64_t j = 0; j < longest; ++j)
    for (int x = 0; x < kXcd; ++x)
      if (j < len[size_t(x)]) {
        tiles.push_back(band[size_t(x)][size_t(2 * j)]);
        tiles.push_back(band[size_t(x)][size_t(2 * j + 1)]);
      }
  if (tiles.empty()) tiles.assign(2, 0u);
  hipError_t e;
  if ((e = hipMalloc(&b->d_probs, sizeof(Filter2DProblem) * std::max<size_t>(n, 1))) != hipSuccess ||
      (e = hipMalloc(&b->d_tiles, sizeof(uint32_t) * tiles.size())) != hipSuccess)
    return fail(RSM_E_NOMEM, std::string("batch tables: ") + hipGetErrorString(e));
  if ((e = hipMemcpy(b->d_probs, table.data(), sizeof(Filter2DProblem) * n, hipMemcpyHostToDevice)) !=
          hipSuccess ||
      (e = hipMemcpy(b->d_tiles, tiles.data(), sizeof(uint32_t) * tiles.size(), hipMemcpyHostToDevice)) !=
          hipSuccess)
    return hip_fail(e, "batch table upload");
  b->buf_floats = 4;
  for (const Filter2DProblem& f : table) b->buf_floats = std::max(b->buf_floats, filter2d_buf_floats(f.k, f.s, f.tc));
  const int g = filter2d_persistent_grid(b->buf_floats);
  b->grid = int(std::max<int64_t>(1, std::min<int64_t>(g, b->n_tiles)));
  if ((e = hipStreamCreateWithFlags(&b->cap_stream, hipStreamNonBlocking)) != hipSuccess)
    return hip_fail(e, "hipStreamCreateWithFlags");
  return RSM_OK;
}

}  // namespace

extern "C" {

rsm_status rsm_batch_create(const rsm_problem* problems, int32_t n, const char* tune_cache_path,
                            uint32_t flags, void* hip_stream, rsm_batch* out) {
  rsm_batch_s* b = nullptr;
  try {
    if (!out) return fail(RSM_E_INVALID, "output handle pointer is NULL");
    *out = nullptr;
    if (n < 0 || (n > 0 && !problems)) return fail(RSM_E_INVALID, "bad problem list");
    for (int k = 0; k < n; ++k) {
      const rsm_problem& p = problems[k];
      if (p.task.kind == RSM_TASK_DOT) return fail(RSM_E_INVALID, "batched problems take one input");
      rsm_status s = rsm_validate(&p.rep, &p.in, 1, &p.out, &p.task, flags & RSM_CHECK_SINGLE_ASSIGN);
      if (s) return fail(s, "problem " + std::to_string(k) + ": " + rsm_last_error());
      if (!p.d_in || !p.d_out) return fail(RSM_E_INVALID, "problem " + std::to_string(k) + ": NULL buffer");
    }
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    b = new rsm_batch_s;
    (void)hipGetDevice(&b->device);
    b->problems.assign(problems, problems + n);
    b->fp.resize(size_t(n));
    for (int k = 0; k < n; ++k) {
      const rsm_problem& p = problems[k];
      Filter2DProblem f{};
      int64_t n_rep = 1;
      for (int d = 0; d < p.rep.rank; ++d) n_rep *= p.rep.shape[d];
      if (n_rep > 0 && !(flags & RSM_FORCE_GENERIC) && plan_filter2d(p.rep, p.in, p.out, p.task, &f)) {
        f.x = static_cast<const float*>(p.d_in);
        f.y = static_cast<float*>(p.d_out);
        f.c = static_cast<const float*>(p.task.coeffs);
        filter2d_set_tiles(&f, 1);
        b->fp[size_t(k)] = f;
        b->persistent.push_back(k);
      } else {
        b->others.push_back(k);
      }
    }
    // ---- autotune tile classes ----
    const std::string arch = arch_name();
    std::map<std::string, int> cache;
    const std::string path = tune_cache_path ? tune_cache_path : "";
    if (!path.empty()) load_cache(path, arch, &cache);
    std::map<std::string, std::vector<int>> classes;
    for (int k : b->persistent) classes[class_key(b->fp[size_t(k)])].push_back(k);
    bool changed = false;
    for (const auto& kv : classes) {
      auto it = cache.find(kv.first);
      int choice;
      if (it != cache.end()) {
        choice = it->second;
        b->info.cached_classes += 1;
      } else {
        float best = 1e30f;
        choice = 1;
        for (int tc = 0; tc < 3; ++tc) {
          float ms = 0.0f;
          rsm_status s = time_class(b, kv.second, tc, st, &ms);
          if (s) {
            delete b;
            return s;
          }
          if (ms < best) {
            best = ms;
            choice = tc;
          }
        }
        cache[kv.first] = choice;
        changed = true;
        b->info.tuned_classes += 1;
      }
      for (int k : kv.second) filter2d_set_tiles(&b->fp[size_t(k)], choice);
    }
    if (changed && !path.empty()) save_cache(path, arch, cache);
    if (!b->persistent.empty()) {
      rsm_status s = build_queue(b);
      if (s) {
        delete b;
        return s;
      }
    }
    b->info.n_problems = n;
    b->info.n_persistent = int64_t(b->persistent.size());
    b->info.n_tiles = b->n_tiles;
    b->info.grid = b->grid;
    *out = b;
    return RSM_OK;
  } catch (const std::bad_alloc&) {
    delete b;
    return fail(RSM_E_NOMEM, "host allocation failed");
  } catch (...) {
    delete b;
    return fail(RSM_E_INVALID, "internal error (exception)");
  }
}

rsm_status rsm_batch_run(rsm_batch b, void* hip_stream) {
  if (!b) return fail(RSM_E_INVALID, "batch handle is NULL");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  hipError_t e;
  if (!b->persistent.empty()) {
    if (!b->exec) {
      if ((e = hipStreamBeginCapture(b->cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
        return hip_fail(e, "hipStreamBeginCapture");
      e = launch_filter2d_persistent(b->d_probs, b->d_tiles, b->n_tiles, b->grid, b->buf_floats, b->cap_stream);
      hipGraph_t g = nullptr;
      const hipError_t e2 = hipStreamEndCapture(b->cap_stream, &g);
      if (e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(e, "persistent launch during capture");
      }
      if (e2 != hipSuccess) return hip_fail(e2, "hipStreamEndCapture");
      b->graph = g;
      if ((e = hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0)) != hipSuccess) {
        b->exec = nullptr;
        return hip_fail(e, "hipGraphInstantiate");
      }
    }
    if ((e = hipGraphLaunch(b->exec, st)) != hipSuccess) return hip_fail(e, "hipGraphLaunch");
  }
  for (int k : b->others) {
    const rsm_problem& p = b->problems[size_t(k)];
    const void* src = p.d_in;
    rsm_status s = rsm_run(&p.rep, &p.in, &src, 1, &p.out, p.d_out, &p.task, 0, hip_stream);
    if (s) return s;
  }
  return RSM_OK;
}

rsm_status rsm_batch_run_plain(rsm_batch b, void* hip_stream) {
  if (!b) return fail(RSM_E_INVALID, "batch handle is NULL");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  for (int k : b->persistent) {
    hipError_t e = launch_filter2d(b->fp[size_t(k)], st);
    if (e != hipSuccess) return hip_fail(e, "filter2d launch");
  }
  for (int k : b->others) {
    const rsm_problem& p = b->problems[size_t(k)];
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
  const bool pers = std::find(b->persistent.begin(), b->persistent.end(), k) != b->persistent.end();
  *tile_rows = pers ? b->fp[size_t(k)].tile_h : 0;
  *tile_cols = pers ? b->fp[size_t(k)].tile_w : 0;
  return RSM_OK;
}

rsm_status rsm_batch_destroy(rsm_batch b) {
  if (!b) return RSM_OK;
  // a replay may still be running on some stream: wait before freeing its tables
  (void)hipDeviceSynchronize();
  delete b;
  return RSM_OK;
}

}  // extern "C"
