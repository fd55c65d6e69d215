"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle (plain C) is built with gcc and both sanitizers and driven
  through every function on small inputs, including the multi-output
  weighted sum, the CSR product and the CG loop.
* The library's host code (validation, planner, placement requests, error
  paths of the compute entry points) is built with hipcc, the sanitizers on
  the host side only (device code is compiled as usual and never launched),
  and driven by a seeded fuzzer: random tilers with ranks up to 9, zero,
  negative and huge extents, extreme origins / pavings / fittings, unknown
  task kinds and dtypes, wrong input counts, NULL pointers and random
  placement requests.  Every call must return a status without a sanitizer
  report; calls with a valid description and NULL buffers must refuse
  before any launch (there is no GPU here).
"""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1105_4424_amd", "csrc")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"

ORACLE_DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
typedef struct {
  int32_t arr_rank, pat_rank;
  int64_t shape[8], origin[8], paving[64], fitting[64], pat_shape[8];
} or_tiler;
int oracle_indices(int32_t, const int64_t*, const or_tiler*, int64_t*);
int oracle_run(int32_t, const int64_t*, int32_t, const or_tiler*, const double* const*, const or_tiler*,
               double*, int64_t*, double*, int32_t, const double*);
int oracle_run_sample(int32_t, const int64_t*, int32_t, const or_tiler*, const double* const*, int64_t,
                      int32_t, const double*, int64_t, const int64_t*, double*, double*);
int oracle_adjoint(int32_t, const int64_t*, const or_tiler*, const double*, const or_tiler*, const double*,
                   const double*, double*, double*, double*, double*);
int oracle_run_csr(int64_t, const int32_t*, const int32_t*, const double*, const double*, double*, double*);
int64_t oracle_cg(int64_t, const int32_t*, const int32_t*, const double*, const double*, double*, double,
                  int64_t, double*, double*, double*);

static or_tiler tap1(int64_t n, int64_t o, int64_t p, int64_t taps) {
  or_tiler t; memset(&t, 0, sizeof t);
  t.arr_rank = 1; t.pat_rank = 1; t.shape[0] = n; t.origin[0] = o; t.paving[0] = p; t.fitting[0] = 1;
  t.pat_shape[0] = taps;
  return t;
}
int main(void) {
  /* 1-D windows of 13 taps every 8 over 70 elements, wrapping; 3 outputs per window */
  const int64_t reps[1] = {9};
  or_tiler in = tap1(70, -6, 8, 13);
  or_tiler out1; memset(&out1, 0, sizeof out1);
  out1.arr_rank = 1; out1.shape[0] = 9; out1.paving[0] = 1;
  or_tiler out3 = tap1(27, 0, 3, 3);
  double x[70], c[39], y[27], ya[27], g[27], gx[70], gxa[70], gc[39], gca[39];
  int64_t hits[27], idx[9 * 13];
  for (int i = 0; i < 70; ++i) x[i] = (i * 37 % 11) - 5.0;
  for (int i = 0; i < 39; ++i) c[i] = 0.1 * (i % 7) - 0.3;
  for (int i = 0; i < 27; ++i) g[i] = 0.05 * (i % 5) - 0.1;
  const double* xs[1] = {x};
  if (oracle_indices(1, reps, &in, idx)) return 1;
  for (int kind = 0; kind < 3; ++kind) {          /* COPY needs a 13-element output: skipped */
    if (kind == 0) continue;
    memset(hits, 0, sizeof hits);
    if (oracle_run(1, reps, 1, &in, xs, &out1, y, hits, ya, kind, c)) return 2;
  }
  memset(hits, 0, sizeof hits);
  if (oracle_run(1, reps, 1, &in, xs, &out3, y, hits, ya, 2, c)) return 3;       /* q = 3 */
  if (oracle_run(1, reps, 1, &in, xs, &out3, y, hits, ya, 1, c) == 0) return 4;  /* SUM refuses q = 3 */
  int64_t pick[3] = {0, 4, 8};
  if (oracle_run_sample(1, reps, 1, &in, xs, 3, 2, c, 3, pick, y, ya)) return 5;
  memset(gx, 0, sizeof gx); memset(gxa, 0, sizeof gxa); memset(gc, 0, sizeof gc); memset(gca, 0, sizeof gca);
  if (oracle_adjoint(1, reps, &in, x, &out3, g, c, gx, gxa, gc, gca)) return 6;
  if (oracle_adjoint(1, reps, &in, x, &out1, g, NULL, gx, gxa, NULL, NULL)) return 7;
  /* DOT of two 1-D patterns */
  or_tiler two[2] = {tap1(70, -6, 8, 13), tap1(70, 3, 7, 13)};
  const double* xx[2] = {x, x};
  memset(hits, 0, sizeof hits);
  if (oracle_run(1, reps, 2, two, xx, &out1, y, hits, ya, 3, NULL)) return 8;
  /* CSR: a 6 x 6 SPD tridiagonal matrix, product and CG */
  int32_t rp[7], ci[16];
  double va[16], b[6], xv[6], yv[6], yva[6], res[7], al[6], be[6];
  int k = 0;
  for (int r = 0; r < 6; ++r) {
    rp[r] = k;
    for (int cc = r - 1; cc <= r + 1; ++cc)
      if (cc >= 0 && cc < 6) { ci[k] = cc; va[k] = cc == r ? 4.0 : -1.0; ++k; }
  }
  rp[6] = k;
  for (int i = 0; i < 6; ++i) { b[i] = i - 2.5; xv[i] = 0.0; }
  if (oracle_run_csr(6, rp, ci, va, b, yv, yva)) return 9;
  if (oracle_cg(6, rp, ci, va, b, xv, 1e-10, 6, res, al, be) < 0) return 10;
  printf("oracle ok\n");
  return 0;
}
"""

PLANNER_DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <string.h>
#include "rsm.h"

static uint64_t st = 0x9e3779b97f4a7c15ull;
static uint64_t rnd(void) { st ^= st << 13; st ^= st >> 7; st ^= st << 17; return st; }
static int64_t pick(const int64_t* v, int n) { return v[rnd() % (uint64_t)n]; }
static const int64_t ext[] = {1, 1, 2, 3, 4, 7, 8, 16, 33, 64, 0, -1, -5, 1ll << 20, 1ll << 31, 1ll << 40, 1ll << 62};
static const int64_t stp[] = {0, 1, 1, 2, -1, 3, 8, -7, 1ll << 20, -(1ll << 31), 1ll << 62};

static void rand_tiler(rsm_tiler* t, int rep_rank) {
  memset(t, 0, sizeof *t);
  t->array_rank = (int32_t)(rnd() % 10) - (rnd() % 16 == 0 ? 1 : 0);
  t->dtype = (int32_t)(rnd() % 6) - (rnd() % 8 == 0 ? 1 : 0);
  t->pattern_rank = (int32_t)(rnd() % 4) - (rnd() % 16 == 0 ? 1 : 0);
  for (int d = 0; d < RSM_MAX_RANK; ++d) {
    t->array_shape[d] = pick(ext, rnd() % 4 ? 9 : 17);
    t->pattern_shape[d] = pick(ext, rnd() % 4 ? 6 : 17);
    t->origin[d] = pick(stp, 11);
    for (int k = 0; k < RSM_MAX_RANK; ++k) {
      t->paving[d][k] = (k == d && rnd() % 2) ? 1 : pick(stp, rnd() % 4 ? 6 : 11);
      t->fitting[d][k] = pick(stp, rnd() % 4 ? 6 : 11);
    }
  }
  (void)rep_rank;
}

int main(void) {
  char name[64];
  rsm_port_placement ports[8];
  int32_t n_ports = 0;
  long statuses[16] = {0};
  for (int it = 0; it < 20000; ++it) {
    rsm_space rep;
    memset(&rep, 0, sizeof rep);
    rep.rank = (int32_t)(rnd() % 5) - (rnd() % 32 == 0 ? 1 : 0);
    for (int d = 0; d < RSM_MAX_RANK; ++d) rep.shape[d] = pick(ext, rnd() % 4 ? 8 : 17);
    rsm_tiler in[2], out;
    rand_tiler(&in[0], rep.rank);
    rand_tiler(&in[1], rep.rank);
    rand_tiler(&out, rep.rank);
    rsm_task task;
    memset(&task, 0, sizeof task);
    task.kind = (int32_t)(rnd() % 5) - (rnd() % 16 == 0 ? 1 : 0);
    task.compute = (int32_t)(rnd() % 4);
    task.coeffs = (rnd() % 2) ? (const void*)0x1000 : NULL;   /* never dereferenced on the host */
    const int32_t n_in = (int32_t)(rnd() % 4);
    const uint32_t flags = (uint32_t)(rnd() % 256) & ~(uint32_t)RSM_CHECK_SINGLE_ASSIGN;
    int s = rsm_validate(&rep, in, n_in, &out, &task, flags);
    statuses[s & 15]++;
    s = rsm_plan(&rep, in, n_in, &out, &task, flags, name, (int32_t)(rnd() % 70));
    statuses[s & 15]++;
    s = rsm_plan_ports(&rep, in, n_in, &out, &task, 0, ports, (int32_t)(rnd() % 9), &n_ports);
    statuses[s & 15]++;
    int32_t spaces[6];
    for (int k = 0; k < 6; ++k) spaces[k] = (int32_t)(rnd() % 6) - 2;
    s = rsm_plan_placed(&rep, in, n_in, &out, &task, 0, (rnd() % 3) ? spaces : NULL, (int32_t)(rnd() % 6),
                        (rnd() % 2) ? name : NULL, 64, (rnd() % 2) ? ports : NULL, 8, &n_ports);
    statuses[s & 15]++;
    /* host-detectable errors of the compute entry points: NULL buffers */
    const void* dptr[2] = {NULL, NULL};
    s = rsm_run(&rep, in, dptr, n_in, &out, NULL, &task, flags, NULL);
    statuses[s & 15]++;
    s = rsm_run_placed(&rep, in, dptr, n_in, &out, NULL, &task, spaces, (int32_t)(rnd() % 6), 0, NULL);
    statuses[s & 15]++;
    rsm_prepared ph = NULL;
    s = rsm_prepare(&rep, in, n_in, &out, &task, flags & (rnd() % 2 ? 0xffu : 0x8u), (rnd() % 16) ? &ph : NULL);
    statuses[s & 15]++;
    if (ph) {
      s = rsm_prepared_name(ph, (rnd() % 2) ? name : NULL, (int32_t)(rnd() % 70));
      statuses[s & 15]++;
      s = rsm_run_prepared(ph, dptr, NULL, NULL, NULL);
      statuses[s & 15]++;
    }
    rsm_prepared_destroy(ph);
    s = rsm_run_adjoint(&rep, &in[0], NULL, &out, NULL, &task, NULL, NULL, flags, NULL);
    statuses[s & 15]++;
    rsm_stage stg[2];
    stg[0].rep = rep; stg[0].in = in[0]; stg[0].out = out; stg[0].task = task;
    stg[1] = stg[0];
    s = rsm_run_chain(stg, (int32_t)(rnd() % 3), NULL, NULL, NULL, flags, NULL);
    statuses[s & 15]++;
    s = rsm_run_chain_train(stg, 2, NULL, NULL, NULL, NULL, NULL, 0, NULL);
    statuses[s & 15]++;
    (void)rsm_last_error();
  }
  /* small valid tilers with the single-assignment check (host O(|s_r| |s_p|)) */
  for (int it = 0; it < 2000; ++it) {
    rsm_space rep;
    memset(&rep, 0, sizeof rep);
    rep.rank = 1 + (int32_t)(rnd() % 3);
    for (int d = 0; d < rep.rank; ++d) rep.shape[d] = 1 + (int64_t)(rnd() % 6);
    rsm_tiler in, out;
    memset(&in, 0, sizeof in);
    memset(&out, 0, sizeof out);
    in.array_rank = out.array_rank = rep.rank;
    in.dtype = out.dtype = RSM_F32;
    in.pattern_rank = 1;
    in.pattern_shape[0] = 1 + (int64_t)(rnd() % 5);
    for (int d = 0; d < rep.rank; ++d) {
      in.array_shape[d] = 1 + (int64_t)(rnd() % 9);
      out.array_shape[d] = 1 + (int64_t)(rnd() % 9);
      in.origin[d] = (int64_t)(rnd() % 21) - 10;
      out.origin[d] = (int64_t)(rnd() % 21) - 10;
      in.fitting[d][0] = (int64_t)(rnd() % 5) - 2;
      for (int k = 0; k < rep.rank; ++k) {
        in.paving[d][k] = (int64_t)(rnd() % 7) - 3;
        out.paving[d][k] = (int64_t)(rnd() % 5) - 2;
      }
    }
    rsm_task task;
    memset(&task, 0, sizeof task);
    task.kind = RSM_TASK_SUM;
    task.compute = RSM_F32;
    int s = rsm_validate(&rep, &in, 1, &out, &task, RSM_CHECK_SINGLE_ASSIGN);
    statuses[s & 15]++;
  }
  for (int s = -2; s < 12; ++s) (void)rsm_status_string(s);
  for (int s = 0; s < 9; ++s) printf("%s %ld\n", rsm_status_string(s), statuses[s]);
  return 0;
}
"""

SOURCES = ["api.cpp", "batch.cpp", "k_generic.hip", "k_window.hip", "k_gemm.hip", "k_filter2d.hip", "k_sparse.hip",
           "k_cg.hip", "k_fir_gather.hip", "k_polyphase.hip", "noalloc.hip"]
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]


def _env():
    env = dict(os.environ)
    # the environment is passed on as it is; a library preloaded ahead of the
    # ASan runtime is tolerated instead of refused
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:halt_on_error=1:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    return env


def test_oracle_under_asan_and_ubsan(tmp_path):
    drv = tmp_path / "drv.c"
    drv.write_text(ORACLE_DRIVER)
    exe = tmp_path / "oracle_san"
    subprocess.check_call(["gcc", "-std=c99", "-O1", "-g", "-fsanitize=address,undefined",
                           "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                           os.path.join(ROOT, "oracle", "rsm_oracle.c"), str(drv), "-lm", "-o", str(exe)])
    env = _env()
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1"
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "oracle ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr


@pytest.mark.slow
def test_planner_under_asan_and_ubsan(tmp_path):
    drv = tmp_path / "drv.cpp"
    drv.write_text(PLANNER_DRIVER)
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-I" + os.path.join(ROOT, "include"),
              "-I" + CSRC, "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-w"] + HOST_SAN

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run([HIPCC] + common + ["-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    srcs = [os.path.join(CSRC, s) for s in SOURCES] + [str(drv)]
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(compile_one, srcs))
    exe = str(tmp_path / "planner_san")
    r = subprocess.run([HIPCC, "--offload-arch=gfx950"] + HOST_SAN + objs + ["-o", exe], capture_output=True,
                       text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    r = subprocess.run([exe], capture_output=True, text=True, env=_env(), timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    counts = dict(line.split() for line in r.stdout.strip().splitlines())
    # the fuzzer reaches success and every host-side refusal
    assert int(counts["RSM_OK"]) > 0
    for st in ("RSM_E_INVALID", "RSM_E_RANK", "RSM_E_SHAPE", "RSM_E_OVERFLOW", "RSM_E_UNSUPPORTED"):
        assert int(counts[st]) > 0, (st, counts)
