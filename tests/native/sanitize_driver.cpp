// Driver for the host-sanitizer build of libqw: the library's host code is
// compiled with AddressSanitizer and UndefinedBehaviorSanitizer (device code
// unchanged) and this program, linked with both runtimes, calls it through
// the C ABI of qw.h. Any report of either sanitizer ends the run with a
// non-zero status (halt_on_error for UBSan is set by the test).
//
//   sanitize_driver host     no device needed: argument validation of every
//                            entry point, the error paths of plan and server
//                            creation, Taylor coefficients, error strings.
//   sanitize_driver device   a short real run on the current device: plans
//                            of d = 1, 2, 3 in both precisions, state, jump,
//                            fused jump + reductions, steps, batched calls,
//                            autotuning with a schedule cache file, and a
//                            server on three streams with cancellation,
//                            timed waits and graph capture, then teardown.
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include <unistd.h>

#include <vector>

#include "qw.h"

static int g_fail = 0;

#define EXPECT(cond)                                                              \
  do {                                                                            \
    if (!(cond)) {                                                                \
      fprintf(stderr, "%s:%d: expectation failed: %s (last error: %s)\n", __FILE__, \
              __LINE__, #cond, qw_last_error());                                  \
      ++g_fail;                                                                   \
    }                                                                             \
  } while (0)

#define EXPECT_STATUS(call, want) EXPECT((call) == (want))

static void host_checks() {
  const int64_t N3[3] = {16, 16, 16};
  const int64_t bad[3] = {16, 12, 16};
  qw_plan_t p = nullptr;
  EXPECT_STATUS(qw_plan(nullptr, 3, N3, 0.1, QW_C64, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_plan(&p, 0, N3, 0.1, QW_C64, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_plan(&p, 4, N3, 0.1, QW_C64, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_plan(&p, 3, nullptr, 0.1, QW_C64, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_plan(&p, 3, N3, NAN, QW_C64, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_plan(&p, 3, N3, -0.1, QW_C64, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_plan(&p, 3, N3, 1.5, QW_C64, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_plan(&p, 3, N3, 0.1, (qw_dtype)7, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_plan(&p, 3, bad, 0.1, QW_C64, nullptr), QW_ERR_UNSUPPORTED);
  EXPECT(p == nullptr);
  EXPECT(strlen(qw_last_error()) > 0);
  EXPECT(strlen(qw_version()) > 0);

  // Every plan-level call rejects a NULL plan before touching a device.
  double origin[3] = {0, 0, 0}, k0[3] = {0.1, 0.1, 0.1}, c[8];
  qw_obs obs;
  qw_drift drift;
  float ms[8];
  int n = 0, a = 0, b = 0, cc = 0, d = 0;
  double best = 0;
  int64_t xmin[3], len[3], io[3] = {0, 0, 0};
  void* f = (void*)0x1000;  // never dereferenced: the plan check comes first
  EXPECT_STATUS(qw_destroy(nullptr), QW_OK);
  EXPECT_STATUS(qw_step(nullptr, f, 1, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_step_noalloc(nullptr, f, 1, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_step_batched(nullptr, 2, f, c, 1, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_evolve_fft(nullptr, f, f, 1, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_evolve_fft_real(nullptr, f, f, 0.5, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_evolve_fft_batched(nullptr, 2, f, f, c, nullptr, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_transform(nullptr, f, f, 1, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_bcc_transform(nullptr, f, f, 1, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_bcc_step(nullptr, f, 1, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_bcc_observables(nullptr, f, origin, &obs, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_bcc_evolve_fft(nullptr, f, f, 1.0, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_kspace_drift(nullptr, f, &drift, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_observables(nullptr, f, origin, nullptr, &obs, nullptr), QW_ERR_INVALID);
  qw_obs two[2];
  double nw[6];
  EXPECT_STATUS(qw_newton_wigner(nullptr, f, origin, two, nw, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_marginals(nullptr, f, io, c, 8, xmin, len, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_evolve_fft_observables(nullptr, f, f, 1, origin, &obs, nullptr), QW_ERR_INVALID);
  double raw[QW_OBS_RAW_DOUBLES] = {0};
  EXPECT_STATUS(qw_evolve_fft_observables_async(nullptr, f, f, 1, origin, raw, nullptr),
                QW_ERR_INVALID);
  EXPECT_STATUS(qw_obs_from_raw(nullptr, raw, origin, &obs), QW_ERR_INVALID);
  EXPECT_STATUS(qw_prepare_state(nullptr, f, k0, 2.0, origin, 1, 0, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_evolve_fft_timed(nullptr, f, f, 1, nullptr, ms, &n), QW_ERR_INVALID);
  EXPECT_STATUS(qw_set_schedule(nullptr, 0, 4, 128, 1), QW_ERR_INVALID);
  EXPECT_STATUS(qw_get_schedule(nullptr, &a, &b, &cc, &d), QW_ERR_INVALID);
  EXPECT_STATUS(qw_autotune(nullptr, nullptr, &best), QW_ERR_INVALID);
  EXPECT_STATUS(qw_evolve_dispersive(nullptr, f, k0, 2.0, origin, 1, 0, 2, 1.0, nullptr),
                QW_ERR_INVALID);
  EXPECT_STATUS(qw_set_step_kernel(2, 0, 0), QW_ERR_INVALID);
  EXPECT_STATUS(qw_set_step_kernel(0, 0, 0), QW_OK);
  EXPECT_STATUS(qw_set_fft_kernel(2), QW_ERR_INVALID);
  EXPECT_STATUS(qw_set_fft_kernel(1), QW_OK);

  // Host-only arithmetic: the Taylor coefficients of omega (Prop. 1).
  for (int dim = 1; dim <= 3; ++dim)
    for (int order = 0; order <= 2; ++order) {
      double coef[16];
      for (double& x : coef) x = -1.0;
      EXPECT_STATUS(qw_dispersion_taylor(dim, 0.3, k0, order, coef), QW_OK);
      EXPECT(coef[0] > 0.0 && coef[0] < M_PI);
    }
  EXPECT_STATUS(qw_dispersion_taylor(3, 0.3, k0, 3, c), QW_ERR_UNSUPPORTED);
  EXPECT_STATUS(qw_dispersion_taylor(3, 0.3, nullptr, 1, c), QW_ERR_INVALID);
  EXPECT_STATUS(qw_dispersion_taylor(0, 0.3, k0, 1, c), QW_ERR_INVALID);

  // Server calls on a NULL server.
  qw_result res;
  qw_server_info info;
  int64_t tk = 0;
  int done = 0;
  qw_request rq;
  memset(&rq, 0, sizeof rq);
  EXPECT_STATUS(qw_server_create(nullptr, 1 << 20, 4, 1), QW_ERR_INVALID);
  EXPECT_STATUS(qw_server_submit(nullptr, &rq, &tk), QW_ERR_INVALID);
  EXPECT_STATUS(qw_server_poll(nullptr, 1, &res, &done), QW_ERR_INVALID);
  EXPECT_STATUS(qw_server_wait(nullptr, 1, &res), QW_ERR_INVALID);
  EXPECT_STATUS(qw_server_wait_for(nullptr, 1, 0.0, &res, &done), QW_ERR_INVALID);
  EXPECT_STATUS(qw_server_cancel(nullptr, 1, &done), QW_ERR_INVALID);
  EXPECT_STATUS(qw_server_hold(nullptr, 1), QW_ERR_INVALID);
  EXPECT_STATUS(qw_server_stats(nullptr, &info), QW_ERR_INVALID);
  EXPECT_STATUS(qw_server_configure(nullptr, 1, 1, 4), QW_ERR_INVALID);
  EXPECT_STATUS(qw_server_destroy(nullptr), QW_OK);
}

// Host checks that need a device to get past plan creation.
static void plan_arg_checks(qw_plan_t p, void* field) {
  double origin[3] = {8, 8, 8}, k0[3] = {0.1, 0.1, 0.1}, m2[2] = {0.1, 0.2};
  qw_obs obs;
  EXPECT_STATUS(qw_step(p, nullptr, 1, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_step(p, field, -1, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_step_batched(p, -1, field, m2, 1, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_step_batched(p, 0, field, m2, 1, nullptr), QW_OK);  // nothing to do
  EXPECT_STATUS(qw_evolve_fft(p, field, nullptr, 1, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_evolve_fft_real(p, field, field, NAN, nullptr), QW_ERR_UNSUPPORTED);
  EXPECT_STATUS(qw_evolve_fft(p, field, field, (int64_t(1) << 53) + 1, nullptr), QW_ERR_UNSUPPORTED);
  EXPECT_STATUS(qw_evolve_fft_observables(p, field, field, 1, nullptr, &obs, nullptr),
                QW_ERR_INVALID);
  EXPECT_STATUS(qw_evolve_fft_observables_async(p, field, field, 1, origin, nullptr, nullptr),
                QW_ERR_INVALID);
  EXPECT_STATUS(qw_obs_from_raw(p, nullptr, origin, &obs), QW_ERR_INVALID);
  EXPECT_STATUS(qw_transform(p, field, field, 0, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_prepare_state(p, field, k0, -1.0, origin, 1, 0, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_prepare_state(p, field, k0, 2.0, origin, 0, 0, nullptr), QW_ERR_INVALID);
  EXPECT_STATUS(qw_set_schedule(p, 0, 5, 128, 1), QW_ERR_INVALID);
  EXPECT_STATUS(qw_set_schedule(p, 0, 4, 100, 1), QW_ERR_INVALID);
  EXPECT_STATUS(qw_set_schedule(p, -1, 4, 128, 1), QW_ERR_INVALID);
}

static bool near(double a, double b, double tol) { return fabs(a - b) <= tol; }

static void other_plans();
static void server_run();

static void device_run() {
  const char* cache = "sanitize_tune_cache.txt";
  unlink(cache);
  setenv("QW_TUNE_CACHE", cache, 1);
  hipStream_t st = nullptr;
  EXPECT(hipStreamCreate(&st) == hipSuccess);
  const qw_dtype dts[2] = {QW_C64, QW_C128};
  for (int di = 0; di < 2; ++di) {
    const qw_dtype dt = dts[di];
    const double tol = dt == QW_C64 ? 1e-4 : 1e-10;
    for (int dim = 1; dim <= 3; ++dim) {
      const int64_t n = dim == 1 ? 8192 : (dim == 2 ? 64 : 16);  // 1D: the four-step split
      int64_t N[3] = {n, n, n};
      qw_plan_t p = nullptr;
      EXPECT_STATUS(qw_plan(&p, dim, N, 0.2, dt, st), QW_OK);
      if (!p) continue;
      const int s = dim == 1 ? 2 : 4;
      int64_t V = 1;
      for (int i = 0; i < dim; ++i) V *= n;
      const size_t bytes = (size_t)s * V * (dt == QW_C64 ? 8 : 16);
      void *x = nullptr, *y = nullptr, *z = nullptr;
      EXPECT(hipMalloc(&x, 2 * bytes) == hipSuccess);
      EXPECT(hipMalloc(&y, 2 * bytes) == hipSuccess);
      EXPECT(hipMalloc(&z, bytes) == hipSuccess);
      double k0[3] = {0.2, -0.1, 0.1}, ctr[3] = {n / 2.0, n / 2.0, n / 2.0};
      plan_arg_checks(p, x);
      EXPECT_STATUS(qw_prepare_state(p, x, k0, 3.0, ctr, 0.6, 0.8, st), QW_OK);
      qw_obs o0, o1, o2;
      EXPECT_STATUS(qw_observables(p, x, ctr, x, &o0, st), QW_OK);
      EXPECT(near(o0.norm2, 1.0, tol));
      EXPECT_STATUS(qw_evolve_fft(p, x, y, 1000, st), QW_OK);
      EXPECT_STATUS(qw_evolve_fft_observables(p, x, z, 1000, ctr, &o1, st), QW_OK);
      EXPECT_STATUS(qw_evolve_fft_observables(p, x, nullptr, 1000, ctr, &o2, st), QW_OK);
      EXPECT(near(o1.norm2, 1.0, tol) && near(o1.mean[0], o2.mean[0], 1e-9));
      {
        // pageable record (the copy then completes within the call); pinned
        // host memory allocated here trips the sanitizer runtime's device
        // allocator when the HIP runtime unloads at exit
        double raw[QW_OBS_RAW_DOUBLES];
        qw_obs o3;
        EXPECT_STATUS(qw_evolve_fft_observables_async(p, x, z, 1000, ctr, raw, st), QW_OK);
        EXPECT(hipStreamSynchronize(st) == hipSuccess);
        EXPECT_STATUS(qw_obs_from_raw(p, raw, ctr, &o3), QW_OK);
        EXPECT(o3.norm2 == o1.norm2 && o3.mean[0] == o1.mean[0] && o3.second[0] == o1.second[0]);
      }
      EXPECT_STATUS(qw_evolve_fft_real(p, x, z, 10.5, st), QW_OK);
      int64_t ts[3] = {1000, -3, 1000};
      qw_obs so[3];
      EXPECT_STATUS(qw_evolve_fft_series(p, x, 3, ts, ctr, so, st), QW_OK);
      EXPECT(near(so[0].norm2, 1.0, tol) && near(so[0].mean[0], o1.mean[0], 1e-3) &&
             so[0].mean[0] == so[2].mean[0]);
      EXPECT_STATUS(qw_step(p, y, 3, st), QW_OK);
      EXPECT_STATUS(qw_step_noalloc(p, y, 2, st), QW_OK);
      EXPECT_STATUS(qw_transform(p, y, z, 1, st), QW_OK);
      EXPECT_STATUS(qw_transform(p, z, z, -1, st), QW_OK);
      double m2[2] = {0.1, 0.3};
      EXPECT(hipMemcpyAsync((char*)x + bytes, x, bytes, hipMemcpyDeviceToDevice, st) == hipSuccess);
      EXPECT_STATUS(qw_step_batched(p, 2, x, m2, 2, st), QW_OK);
      int64_t t2[2] = {7, -7};
      EXPECT_STATUS(qw_evolve_fft_batched(p, 2, x, y, m2, t2, st), QW_OK);
      qw_drift dr;
      EXPECT_STATUS(qw_kspace_drift(p, y, &dr, st), QW_OK);
      qw_obs sec[2];
      double nw[6];
      EXPECT_STATUS(qw_newton_wigner(p, y, ctr, sec, nw, st),
                    dim == 1 ? QW_ERR_UNSUPPORTED : QW_OK);  // 1D above 4096 sites
      float ms[8];
      int np = 0;
      EXPECT_STATUS(qw_evolve_fft_timed(p, x, y, 5, st, ms, &np), QW_OK);
      EXPECT(np >= 1 && np <= 8);
      double best = 0.0, best2 = 0.0;
      EXPECT_STATUS(qw_autotune(p, st, &best), QW_OK);
      EXPECT_STATUS(qw_autotune(p, st, &best2), QW_OK);  // from the cache file
      EXPECT(near(best, best2, 1e-5));
      EXPECT(hipStreamSynchronize(st) == hipSuccess);
      EXPECT(hipFree(x) == hipSuccess && hipFree(y) == hipSuccess && hipFree(z) == hipSuccess);
      EXPECT_STATUS(qw_destroy(p), QW_OK);
    }
  }
  unsetenv("QW_TUNE_CACHE");
  unlink(cache);
  EXPECT(hipStreamDestroy(st) == hipSuccess);
  other_plans();
  server_run();
}

// Weyl and cubic-supercell plans.
static void other_plans() {
  hipStream_t st = nullptr;
  EXPECT(hipStreamCreate(&st) == hipSuccess);
  {
    int64_t N[3] = {16, 16, 16};
    qw_plan_t w = nullptr;
    EXPECT_STATUS(qw_plan_weyl(&w, 3, N, QW_C64, st), QW_OK);
    qw_plan_t p = nullptr;
    EXPECT_STATUS(qw_plan(&p, 3, N, 0.1, QW_C64, st), QW_OK);
    void* f = nullptr;
    EXPECT(hipMalloc(&f, 2 * 4 * 4096 * 8) == hipSuccess);
    EXPECT(hipMemsetAsync(f, 0, 2 * 4 * 4096 * 8, st) == hipSuccess);
    double origin[3] = {0, 0, 0};
    qw_obs o;
    if (w) {
      EXPECT_STATUS(qw_step(w, f, 2, st), QW_OK);
      EXPECT_STATUS(qw_evolve_fft(w, f, f, 9, st), QW_OK);
    }
    if (p) {
      EXPECT_STATUS(qw_bcc_step(p, f, 2, st), QW_OK);
      EXPECT_STATUS(qw_bcc_transform(p, f, f, 1, st), QW_OK);
      EXPECT_STATUS(qw_bcc_evolve_fft(p, f, f, 3.0, st), QW_OK);
      EXPECT_STATUS(qw_bcc_observables(p, f, origin, &o, st), QW_OK);
    }
    EXPECT(hipStreamSynchronize(st) == hipSuccess);
    EXPECT(hipFree(f) == hipSuccess);
    qw_destroy(w);
    qw_destroy(p);
  }

  EXPECT(hipStreamDestroy(st) == hipSuccess);
}

// Server: three streams, graphs on, a burst with cancellations and timed waits.
static void server_run() {
  qw_server_t srv = nullptr;
  EXPECT_STATUS(qw_server_create(&srv, (size_t)256 << 20, 8, 3), QW_OK);
  if (srv) {
    EXPECT_STATUS(qw_server_configure(srv, 1, 1, 8), QW_OK);
    std::vector<int64_t> tks;
    EXPECT_STATUS(qw_server_hold(srv, 1), QW_OK);
    for (int i = 0; i < 96; ++i) {
      qw_request r;
      memset(&r, 0, sizeof r);
      r.dim = 1 + i % 3;
      const int64_t n = r.dim == 1 ? (i % 2 ? 1024 : 8192) : (r.dim == 2 ? 32 : 16);
      for (int a = 0; a < 3; ++a) r.N[a] = a < r.dim ? n : 1;
      r.m = 0.05 * (i % 5);
      r.dtype = i % 4 == 3 ? QW_C128 : QW_C64;
      for (int a = 0; a < r.dim; ++a) {
        r.k0[a] = 0.1 * (a + 1);
        r.center[a] = n / 2;
      }
      r.sigma = 2.0;
      r.c_plus = 1.0;
      r.c_minus = 0.5;
      r.t = 1 + 37 * i;
      int64_t tk = -1;
      EXPECT_STATUS(qw_server_submit(srv, &r, &tk), QW_OK);
      tks.push_back(tk);
      if (i == 40) EXPECT_STATUS(qw_server_hold(srv, 0), QW_OK);
    }
    int cancelled = 0, c = 0;
    for (size_t i = 60; i < tks.size(); i += 7) {
      EXPECT_STATUS(qw_server_cancel(srv, tks[i], &c), QW_OK);
      cancelled += c;
    }
    int ok = 0, cc = 0;
    for (size_t i = 0; i < tks.size(); ++i) {
      qw_result res;
      int done = 0;
      if (i % 2) {
        EXPECT_STATUS(qw_server_wait_for(srv, tks[i], 120.0, &res, &done), QW_OK);
        EXPECT(done == 1);
      } else {
        EXPECT_STATUS(qw_server_wait(srv, tks[i], &res), QW_OK);
      }
      if (res.status == QW_OK) {
        ++ok;
        if (!(fabs(res.obs.norm2 - 1.0) < 1e-4))
          fprintf(stderr, "request %zu: batch of %d, norm2 %.9f\n", i, res.batch_size,
                  res.obs.norm2);
        EXPECT(fabs(res.obs.norm2 - 1.0) < 1e-4);
      } else {
        EXPECT(res.status == QW_ERR_CANCELLED);
        ++cc;
      }
    }
    EXPECT(cc == cancelled && ok + cc == (int)tks.size());
    qw_server_info info;
    EXPECT_STATUS(qw_server_stats(srv, &info), QW_OK);
    EXPECT(info.completed == (int64_t)tks.size() && info.cancelled == cancelled);
    // a second pass of the same shapes replays captured graphs
    std::vector<int64_t> again;
    for (int i = 0; i < 24; ++i) {
      qw_request r;
      memset(&r, 0, sizeof r);
      r.dim = 3;
      r.N[0] = r.N[1] = r.N[2] = 16;
      r.m = 0.1;
      r.dtype = QW_C64;
      r.k0[0] = 0.1;
      r.center[0] = r.center[1] = r.center[2] = 8;
      r.sigma = 2.0;
      r.c_plus = 1.0;
      r.t = i;
      int64_t tk = -1;
      EXPECT_STATUS(qw_server_submit(srv, &r, &tk), QW_OK);
      again.push_back(tk);
    }
    for (int64_t tk : again) {
      qw_result res;
      EXPECT_STATUS(qw_server_wait(srv, tk, &res), QW_OK);
      EXPECT(res.status == QW_OK);
    }
    // destroy with requests still queued
    EXPECT_STATUS(qw_server_hold(srv, 1), QW_OK);
    for (int i = 0; i < 5; ++i) {
      qw_request r;
      memset(&r, 0, sizeof r);
      r.dim = 2;
      r.N[0] = r.N[1] = 32;
      r.N[2] = 1;
      r.m = 0.1;
      r.k0[0] = 0.1;
      r.center[0] = r.center[1] = 16;
      r.sigma = 2.0;
      r.c_plus = 1.0;
      r.t = i;
      int64_t tk = -1;
      EXPECT_STATUS(qw_server_submit(srv, &r, &tk), QW_OK);
    }
    EXPECT_STATUS(qw_server_destroy(srv), QW_OK);
  }
}

int main(int argc, char** argv) {
  const bool device = argc > 1 && strcmp(argv[1], "device") == 0;
  const bool server = argc > 1 && strcmp(argv[1], "server") == 0;
  host_checks();
  printf("host checks done (%d failures)\n", g_fail);
  fflush(stdout);
  if (device) {
    device_run();
    printf("device run done (%d failures)\n", g_fail);
  }
  if (server) {
    server_run();
    printf("server run done (%d failures)\n", g_fail);
  }
  printf(g_fail ? "FAILED\n" : "OK\n");
  return g_fail ? 1 : 0;
}
