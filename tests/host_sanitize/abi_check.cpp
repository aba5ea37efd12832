// Exercises the C ABI of libresolvent from a host program built with AddressSanitizer and UndefinedBehaviorSanitizer
// on the host code (the runtime and this driver; the device kernels are not instrumented).  The host part (argument
// checking, error strings, the FIR design) runs without a GPU; with --gpu every entry point also runs once on
// small operators of each kind and precision.  Exit status 0 when every call returned what it should.
#include <hip/hip_runtime.h>

#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <vector>

#include <sanitizer/lsan_interface.h>

#include "resolvent.h"

namespace {

int g_failures = 0;

void expect(const char* what, int got, int want) {
  if (got != want) {
    std::printf("FAIL %s: status %d (%s), expected %d; last error: %s\n", what, got, resolvent_strerror(got), want,
                resolvent_last_error());
    ++g_failures;
  }
}

void check_host_part() {
  for (int s = -1; s <= 9; ++s)
    if (resolvent_strerror(s) == nullptr) {
      std::printf("FAIL strerror(%d) is NULL\n", s);
      ++g_failures;
    }
  // FIR design (host only): a band-pass response, and malformed requests
  const double nu[4] = {-1.0, -0.5, 0.5, 1.0}, gain[4] = {0.0, 1.0, 1.0, 0.0};
  std::vector<double> taps(2 * 65, 0.0);
  expect("fir_design order 64", resolvent_fir_design(64, 4, nu, gain, taps.data()), RES_OK);
  for (double t : taps)
    if (!std::isfinite(t)) {
      std::printf("FAIL fir_design: non-finite tap\n");
      ++g_failures;
      break;
    }
  expect("fir_design odd order", resolvent_fir_design(63, 4, nu, gain, taps.data()), RES_EINVAL);
  expect("fir_design one breakpoint", resolvent_fir_design(64, 1, nu, gain, taps.data()), RES_EINVAL);
  expect("fir_design NULL taps", resolvent_fir_design(64, 4, nu, gain, nullptr), RES_EINVAL);
  const double bad_nu[4] = {-1.0, 0.5, -0.5, 1.0};
  expect("fir_design unordered breakpoints", resolvent_fir_design(64, 4, bad_nu, gain, taps.data()), RES_EINVAL);
  // grid of an array of frequencies (host only)
  {
    std::vector<double> w(256);
    for (int j = 0; j < 256; ++j) w[j] = -3.0 + j * (6.0 / 255.0);
    resolvent_grid g;
    int64_t P = 0;
    expect("grid_from_omegas", resolvent_grid_from_omegas(w.data(), 256, 0.001, 256, &g, &P), RES_OK);
    if (P % 256 != 0 || g.n_omega != 256 || std::fabs(std::fabs(g.domega) * P * 0.001 - 2.0 * M_PI) > 1e-12) {
      std::printf("FAIL grid_from_omegas: P %lld, domega %.17g\n", (long long)P, g.domega);
      ++g_failures;
    }
    expect("grid_from_omegas one frequency", resolvent_grid_from_omegas(w.data(), 1, 0.001, 1, &g, &P), RES_EGRID);
    expect("grid_from_omegas NULL out", resolvent_grid_from_omegas(w.data(), 256, 0.001, 1, nullptr, &P),
           RES_EINVAL);
    w[100] += 1e-3;
    expect("grid_from_omegas non-uniform", resolvent_grid_from_omegas(w.data(), 256, 0.001, 1, &g, nullptr),
           RES_EGRID);
  }
  // descriptors rejected before any device work
  resolvent_op* op = nullptr;
  expect("op_create NULL desc", resolvent_op_create(nullptr, nullptr, &op), RES_EINVAL);
  resolvent_op_desc d;
  std::memset(&d, 0, sizeof(d));
  d.kind = RES_OP_TRIDIAG;
  d.precision = RES_FP64;
  d.h = 0.0;
  expect("op_create NULL out", resolvent_op_create(&d, nullptr, nullptr), RES_EINVAL);
  expect("op_create h = 0", resolvent_op_create(&d, nullptr, &op), RES_EINVAL);
  d.h = 0.01;
  d.precision = 7;
  expect("op_create bad precision", resolvent_op_create(&d, nullptr, &op), RES_EINVAL);
  resolvent_grid g{0.0, 1.0, 4};
  resolvent_run r{RES_PERIODIC, 0, 1, 1};
  expect("apply NULL op", resolvent_apply(nullptr, &g, &r, 1, nullptr, nullptr, nullptr), RES_EINVAL);
  expect("backward NULL op",
         resolvent_apply_backward(nullptr, &g, &r, 1, nullptr, nullptr, nullptr, nullptr, 0, nullptr), RES_EINVAL);
  if (resolvent_last_error() == nullptr) {
    std::printf("FAIL last_error is NULL\n");
    ++g_failures;
  }
}

struct Dev {
  void* p = nullptr;
  explicit Dev(size_t bytes) {
    if (hipMalloc(&p, bytes) != hipSuccess) p = nullptr;
  }
  ~Dev() {
    if (p) (void)hipFree(p);
  }
};

void fill_random(void* dst, size_t count, bool fp64, unsigned seed) {
  std::mt19937_64 rng(seed);
  std::normal_distribution<double> n01;
  if (fp64) {
    std::vector<double> h(2 * count);
    for (auto& x : h) x = n01(rng);
    (void)hipMemcpy(dst, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice);
  } else {
    std::vector<float> h(2 * count);
    for (auto& x : h) x = (float)n01(rng);
    (void)hipMemcpy(dst, h.data(), h.size() * sizeof(float), hipMemcpyHostToDevice);
  }
}

// Direct, adjoint, modes, Arnoldi and reverse-mode calls on one operator (periodic method).
void exercise_runs(resolvent_op* op, const char* name, int64_t N, int fp64, int64_t P, double h, bool mu) {
  std::printf("runs: %s\n", name);
  const int nw = 4, k = 2;
  const size_t es = fp64 ? 16 : 8, count = (size_t)nw * k * N;
  Dev f(count * es), u(count * es), z(count * es), V(count * es), U(count * es), fg(count * es),
      mg((size_t)N * sizeof(double));
  fill_random(f.p, count, fp64, 1);
  fill_random(z.p, count, fp64, 2);
  const double dw = 2.0 * M_PI / ((double)P * h);
  resolvent_grid g{-1.0, dw, nw};
  resolvent_run per{RES_PERIODIC, 0, 2, 1};
  resolvent_run tr{RES_TRANSIENT, 3 * P, 1, 1};
  char what[160];
  std::snprintf(what, sizeof(what), "%s apply periodic", name);
  expect(what, resolvent_apply(op, &g, &per, k, f.p, u.p, nullptr), RES_OK);
  std::snprintf(what, sizeof(what), "%s apply transient", name);
  expect(what, resolvent_apply(op, &g, &tr, k, f.p, u.p, nullptr), RES_OK);
  std::snprintf(what, sizeof(what), "%s adjoint apply", name);
  expect(what, resolvent_adjoint_apply(op, &g, &per, k, z.p, u.p, nullptr), RES_OK);
  resolvent_grid bad{-1.0, dw * 1.001, nw};
  std::snprintf(what, sizeof(what), "%s apply, incommensurate grid", name);
  expect(what, resolvent_apply(op, &bad, &per, k, f.p, u.p, nullptr), RES_EGRID);
  std::vector<double> gains((size_t)nw * k), hist((size_t)3 * nw * k * 2), khist((size_t)2 * nw * k);
  std::snprintf(what, sizeof(what), "%s modes", name);
  expect(what, resolvent_modes(op, &g, &per, k, 3, f.p, gains.data(), V.p, U.p, hist.data(), nullptr), RES_OK);
  std::snprintf(what, sizeof(what), "%s krylov", name);
  expect(what, resolvent_krylov(op, &g, &per, k, 2, f.p, gains.data(), V.p, U.p, khist.data(), nullptr), RES_OK);
  std::snprintf(what, sizeof(what), "%s backward", name);
  expect(what,
         resolvent_apply_backward(op, &g, &per, k, f.p, z.p, fg.p, mu ? (double*)mg.p : nullptr, 16, nullptr),
         RES_OK);
  std::snprintf(what, sizeof(what), "%s backward, forcing only", name);
  expect(what, resolvent_apply_backward(op, &g, &per, k, f.p, z.p, fg.p, nullptr, 0, nullptr), RES_OK);
  size_t wsb = 0;
  std::snprintf(what, sizeof(what), "%s workspace size", name);
  expect(what, resolvent_workspace_size(op, &g, &per, k, &wsb), RES_OK);
  if (wsb == 0 || wsb > RESOLVENT_NOALLOC_SCRATCH_BYTES) {
    std::printf("FAIL %s: %zu bytes\n", what, wsb);
    ++g_failures;
  }
  std::snprintf(what, sizeof(what), "%s noalloc apply", name);
  expect(what, resolvent_apply_noalloc(op, &g, &per, k, f.p, u.p, nullptr), RES_OK);
  std::snprintf(what, sizeof(what), "%s check", name);
  expect(what, resolvent_op_check(op, nullptr), RES_OK);
}

void check_gpu_part() {
  // 1-D advection-diffusion-reaction, N = 200, dx = 0.1: nu u'' - U u' - 0.1 u
  const int64_t N = 200;
  std::vector<double> lo(2 * N, 0.0), di(2 * N, 0.0), up(2 * N, 0.0);
  for (int64_t i = 0; i < N; ++i) {
    lo[2 * i] = 105.0;
    di[2 * i] = -200.1;
    di[2 * i + 1] = 0.3;
    up[2 * i] = 95.0;
  }
  const double h = 0.002;
  for (int prec : {RES_FP64, RES_MIXED}) {
    resolvent_op_desc d;
    std::memset(&d, 0, sizeof(d));
    d.kind = RES_OP_TRIDIAG;
    d.precision = prec;
    d.h = h;
    d.ninst = 1;
    d.lower = lo.data();
    d.diag = di.data();
    d.upper = up.data();
    d.nx = N;
    d.probe = 1;
    d.probe_tol = 1e-6;
    d.probe_tmax = 100.0;
    d.probe_seed = 7;
    resolvent_op* op = nullptr;
    expect("op_create tridiagonal", resolvent_op_create(&d, nullptr, &op), RES_OK);
    if (!op) continue;
    if (resolvent_op_size(op) != N) {
      std::printf("FAIL op_size\n");
      ++g_failures;
    }
    const int fp64 = prec == RES_FP64;
    exercise_runs(op, fp64 ? "tridiagonal fp64" : "tridiagonal mixed", N, fp64, 500, h, true);
    int32_t plan[4], m = 0;
    double us = 0;
    expect("get_plan", resolvent_op_get_plan(op, plan), RES_OK);
    expect("set_plan", resolvent_op_set_plan(op, plan), RES_OK);
    expect("set_step_power 2", resolvent_op_set_step_power(op, 2), RES_OK);
    expect("get_step_power", resolvent_op_get_step_power(op, &m), RES_OK);
    expect("set_step_power 3", resolvent_op_set_step_power(op, 3), RES_EINVAL);
    expect("tune", resolvent_op_tune(op, 2, 64, plan, &us, nullptr), RES_OK);
    double ms = 0;
    int64_t launches = 0;
    expect("set_timing", resolvent_op_set_timing(op, 1), RES_OK);
    std::vector<double> w(N, 1.0), b(N, 0.5);
    expect("set_weights", resolvent_op_set_weights(op, b.data(), w.data(), w.data(), w.data()), RES_OK);
    exercise_runs(op, fp64 ? "weighted fp64" : "weighted mixed", N, fp64, 500, h, true);
    expect("get_timing", resolvent_op_get_timing(op, RES_TIMING_STEPPER, &ms, &launches), RES_OK);
    expect("clear weights", resolvent_op_set_weights(op, nullptr, nullptr, nullptr, nullptr), RES_OK);
    expect("set_diagonal", resolvent_op_set_diagonal(op, di.data(), 0, nullptr), RES_OK);
    expect("set_backward_rows", resolvent_op_set_backward_rows(op, 1), RES_OK);
    expect("set_graphs", resolvent_op_set_graphs(op, 1), RES_OK);
    // signal runs, FIR and the TRM iteration
    const int64_t ns = 64;
    const size_t es = fp64 ? 16 : 8;
    Dev sf((size_t)ns * N * es), sy((size_t)ns * N * es), taps(65 * 16);
    fill_random(sf.p, (size_t)ns * N, fp64, 3);
    expect("signal_run C2", resolvent_signal_run(op, 1, ns, 1, 2, 0, sf.p, sy.p, nullptr), RES_OK);
    expect("signal_run adjoint C1", resolvent_signal_run(op, 1, ns, 1, 1, 1, sf.p, sy.p, nullptr), RES_OK);
    expect("signal_run aliased", resolvent_signal_run(op, 1, ns, 1, 2, 0, sf.p, sf.p, nullptr), RES_EINVAL);
    const double nu[2] = {-1.0, 1.0}, gn[2] = {1.0, 1.0};
    std::vector<double> ht(2 * 17);
    expect("fir_design order 16", resolvent_fir_design(16, 2, nu, gn, ht.data()), RES_OK);
    (void)hipMemcpy(taps.p, ht.data(), ht.size() * sizeof(double), hipMemcpyHostToDevice);
    expect("fir_apply", resolvent_fir_apply(fp64, ns, N, 16, (const double*)taps.p, sf.p, sy.p, nullptr), RES_OK);
    const double om[3] = {-2.0, 0.0, 2.0};
    std::vector<double> tg(3 * 2), ta(3 * 2);
    expect("trm_modes", resolvent_trm_modes(op, 1, ns, 1, 2, sf.p, 3, om, 2, 16, 1, 8, 4, 1.0, tg.data(), ta.data(),
                                            nullptr, nullptr, nullptr, nullptr),
           RES_OK);
    expect("check", resolvent_op_check(op, nullptr), RES_OK);
    resolvent_op_destroy(op);
  }
  // 2-D five-point and 3-D three-component grids
  for (int three : {0, 1}) {
    const int64_t nx = three ? 12 : 24, ny = three ? 8 : 10, nz = three ? 6 : 1, lines = ny * nz;
    const int64_t nodes = nx * ny * nz, ncomp = three ? 3 : 1;
    std::vector<double> c(lines, 25.0), df(nodes, three ? -150.5 : -100.5), cpl(lines * 9, 0.0);
    for (int64_t l = 0; l < lines; ++l) cpl[l * 9 + 1] = 0.1;
    for (int prec : {RES_FP64, RES_MIXED}) {
      resolvent_op_desc d;
      std::memset(&d, 0, sizeof(d));
      d.kind = three ? RES_OP_ADR3D3C : RES_OP_ADR2D;
      d.precision = prec;
      d.h = 0.005;
      d.ninst = 1;
      d.nx = nx;
      d.ny = ny;
      d.nz = nz;
      d.cxm = d.cxp = d.cym = d.cyp = c.data();
      d.czm = d.czp = c.data();
      d.dfield = df.data();
      d.coupling = three ? cpl.data() : nullptr;
      resolvent_op* op = nullptr;
      expect(three ? "op_create 3-D" : "op_create 2-D", resolvent_op_create(&d, nullptr, &op), RES_OK);
      if (!op) continue;
      char name[64];
      std::snprintf(name, sizeof(name), "%s %s", three ? "3-D" : "2-D", prec == RES_FP64 ? "fp64" : "mixed");
      exercise_runs(op, name, nodes * ncomp, prec == RES_FP64, 200, 0.005, true);
      expect("grid set_step_power", resolvent_op_set_step_power(op, 2), RES_ENOTSUP);
      expect("grid set_diagonal", resolvent_op_set_diagonal(op, df.data(), 0, nullptr), RES_OK);
      resolvent_op_destroy(op);
    }
  }
}

}  // namespace

int main(int argc, char** argv) {
  std::setvbuf(stdout, nullptr, _IONBF, 0);  // the leak check at exit ends the process without flushing
  const bool gpu = argc > 1 && std::strcmp(argv[1], "--gpu") == 0;
  check_host_part();
  if (gpu) check_gpu_part();
  std::printf("%s: %d failure(s)\n", gpu ? "host and GPU parts" : "host part", g_failures);
  // Leak check now (it ends the process with an error report if the program leaked), then leave without the
  // runtimes' teardown: after a GPU part, the HIP runtime's unload at exit trips an internal consistency check of
  // the sanitizer's device-allocation hooks, after everything above has run.
  __lsan_do_leak_check();
  std::_Exit(g_failures == 0 ? 0 : 1);
}
