// Internals of the host runtime shared by its translation units (internal): runtime.cpp (set-up, workspace, the
// handle's C ABI), runs.cpp (run scheduling), iterations.cpp (the block power and Arnoldi iterations), backward.cpp
// (the reverse mode) and trm_host.cpp (the transient-response method's host side).  It holds the operator handle,
// its workspace types, run plans and the declarations of the helpers the files share.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/resolvent.h"
#include "kernels.h"
#include "runtime_internal.h"

using namespace res;
typedef std::complex<double> cd;

namespace rt {

// Message of the last error on this thread, for resolvent_last_error.
extern thread_local std::string g_last_error;

inline int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                                   \
  do {                                                                                                  \
    hipError_t e_ = (expr);                                                                             \
    if (e_ != hipSuccess) return fail(RES_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

inline double env_double(const char* name, double dflt) {
  const char* v = std::getenv(name);
  return v ? std::atof(v) : dflt;
}
inline long env_long(const char* name, long dflt) {
  const char* v = std::getenv(name);
  return v ? std::atol(v) : dflt;
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

// Banded matrix: m[i][d + r] = M_{i, i + d}, |d| <= r.
struct Band {
  int64_t n = 0;
  int r = 0;
  std::vector<cd> m;
  Band() {}
  Band(int64_t n_, int r_) : n(n_), r(r_), m((size_t)n_ * (2 * r_ + 1), cd(0, 0)) {}
  cd& at(int64_t i, int d) { return m[(size_t)i * (2 * r + 1) + (d + r)]; }
  cd get(int64_t i, int d) const {
    if (d < -r || d > r) return cd(0, 0);
    return m[(size_t)i * (2 * r + 1) + (d + r)];
  }
};

Band band_mul(const Band& A, const Band& B);

// Workspace carved from a caller-independent fixed device array (the no-allocation apply): named slots are handed
// out front to back, 256-byte aligned, and the run's buffer sizes follow `ArenaSizes` instead of the free device
// memory.
struct ArenaSizes {
  int horner_chunk = 1;        // frequencies per FP64 pre-filter block
  int64_t snap_rows = 0;       // snapshot rows buffered between projection flushes
  bool table = false;          // whole forcing period as one table (else tiles)
  int64_t tile_rows = 0;       // kernel steps per forcing tile
  int64_t max_nsplit = 1;      // split-K limit of the projection (its FP64 partials live in the arena too)
  size_t total = 0;            // bytes of all slots, alignment included
};
struct Arena {
  char* base = nullptr;
  size_t cap = 0, used = 0;
  std::map<std::string, std::pair<void*, size_t>> slots;
  ArenaSizes sz;
};

}  // namespace rt

using namespace rt;

// The operator handle: its stencils, stepper plan, workspace and caches.
struct resolvent_op {
  int kind = 0, prec = 0;
  double h = 0;
  int64_t N = 0;  // unknowns per column
  int ninst = 1;
  std::vector<int64_t> off;
  int64_t* d_off = nullptr;
  // 1-D three-point operator
  std::vector<cd> zl, zd, zu;  // Z = h L (instance boundaries zeroed)
  void* d_tri[2] = {nullptr, nullptr};   // FP64 [N][3] of Z (0) and Z^H (1)
  void* d_band[2] = {nullptr, nullptr};  // working precision [N][9] of P(Z), P(Z^H)
  Band hband[2];                          // host FP64 P(Z), P(Z^H)
  void* d_band64[2] = {nullptr, nullptr}; // FP64 copies (multi-step forcing combination)
  int step_power = 4;                     // RK4 steps per kernel step of the 1-D march (1, 2 or 4)
  bool plan_default = true;               // the stepper plan is the default one (follows the step power)
  void* d_bandm[2] = {nullptr, nullptr};  // working precision [N][8m+1] of P(Z)^m, P(Z^H)^m (m = step_power > 1)
  std::vector<Seg1D> segs;               // workgroup regions of one column
  std::vector<Seg1D> segs_k;             // regions of all k columns of the current run (upload source)
  int step_cfg = -1;                     // stepper kernel configuration
  int64_t step_block = 0;                // steps per launch when regions carry halos (0: unlimited)
  int64_t step_chunk = 0;                // owned unknowns per workgroup (0: whole column in one workgroup)
  int cur_state = 0;                     // which of the two state buffers holds the current state
  bool step_persist = false;             // one cooperative launch per march, neighbour exchange in-kernel
  bool coop_refused = false;             // the device refused a cooperative launch: relaunch at every exchange
  void* xch = nullptr;                   // uncached exchange rows of the persistent stepper
  size_t xch_bytes = 0;
  // 2-D / 3-D structured-grid operator: host coefficients of Z = h L (FP64) and device copies of Z and Z^H
  int ncomp = 1;
  int64_t nx = 0, ny = 1, nz = 1;
  std::vector<double> gx[6];             // cxm, cxp, cym, cyp, czm, czp per x-line (times h)
  std::vector<double> gd;                // diagonal per node (times h)
  std::vector<double> gK;                // coupling per x-line [3][3] (times h), 3-component operators
  std::vector<void*> gbufs;              // device allocations of the grid coefficients
  GridOpDev g64[2], gw[2];               // FP64 and working-precision coefficient sets of Z (0) and Z^H (1)
  // opt-in timing: event pairs per kernel class
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> tev[4];
  const void* march_band = nullptr;      // step stencil used by march_1d (L or L^H)
  const GridOpDev* march_grid = nullptr; // coefficient set used by march_grid (L or L^H)
  // workspace and caches
  std::map<std::string, DevBuf> ws;
  std::map<int64_t, void*> btab;
  std::map<int64_t, void*> btab64;        // FP64 phase tables of the mixed-precision operator (reverse mode)
  int* d_flag = nullptr;
  double decay_time = -1;
  // graph capture: set while the caller's stream (or the library's own capture) records; nothing may then
  // allocate, copy from the host or synchronise
  bool capturing = false;
  bool use_graphs = false;               // resolvent_modes replays its middle iterations from a captured graph
  hipStream_t cap_stream = nullptr;      // private stream for that capture (default priority)
  hipStream_t side_stream = nullptr;     // forcing-table synthesis beside the march (default priority)
  std::vector<hipEvent_t> side_ev;       // chunk events of that synthesis
  int plan_version = 0;                  // bumped by every stepper plan change
  int segs_dev_k = -1, segs_dev_version = -1;  // what the device copy of the regions describes
  // diagonal B, C and metrics W_f, W_y (resolvent_op_set_weights): rows of d_wsc, each [N] FP64
  bool weighted = false;
  void* d_wsc = nullptr;
  bool rev_rows64 = false;               // reverse mode of a mixed-precision operator keeps FP64 rows
  int scale_role = 0;                    // 0: apply/adjoint_apply (y = C R B f), 1: gains and modes (Euclidean R~)
  // host sources of the TRM driver's asynchronous uploads, kept in the handle so that they outlive the copies
  std::vector<double> trm_om, trm_D;
  std::vector<cd> trm_E;
  cd trm_one = cd(1.0, 0.0);
  int device = 0;                        // the device the handle was created on
  Arena* arena = nullptr;                 // set while a no-allocation call runs: the workspace comes from it
  hipStream_t arena_stream = nullptr;     // that call's stream
  bool fp64() const { return prec == RES_FP64; }
  size_t wsize() const { return fp64() ? 16 : 8; }  // bytes per complex in working precision
};

namespace rt {

// Opt-in timing of one launch (or launch group) of kernel class `kind`.
struct TimedLaunch {
  resolvent_op* op;
  int kind;
  hipStream_t st;
  hipEvent_t a = nullptr, b = nullptr;
  TimedLaunch(resolvent_op* o, int k, hipStream_t s) : op(o), kind(k), st(s) {
    if (!op->timing || op->capturing || op->arena) return;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
      a = b = nullptr;
      return;
    }
    (void)hipEventRecord(a, st);
  }
  ~TimedLaunch() {
    if (!a) return;
    (void)hipEventRecord(b, st);
    op->tev[kind].push_back({a, b});
  }
};

#define RES_TRY(expr)          \
  do {                         \
    int rc_ = (expr);          \
    if (rc_ != RES_OK) return rc_; \
  } while (0)

struct Plan {
  double w0, dw;
  int nw;
  int64_t P;
  int method;
  int64_t S;                               // total steps
  int64_t forced_end;                      // forcing active for s < forced_end
  int64_t pfirst, pstride, pcount;         // projected steps pfirst + m*pstride, m < pcount
  double scale;                            // projection normalisation
};

struct ForceSpec {
  const void* frc = nullptr;   // forcing rows or null (unforced)
  int64_t row0 = 0, period = 0;
  cd phi = cd(1, 0);
};

struct SnapSpec {
  void* snap = nullptr;        // snapshot rows or null
  int64_t ld = 0, first = 0, stride = 1, count = 0, row0 = 0;
};

// Rows of the diagonal scalings (resolvent_op_set_weights): input and output scales of a run by role and
// direction, and the mode transforms.
enum { kWscB = 0, kWscC, kWscCWy, kWscBInvWf, kWscBInvSqrtWf, kWscCSqrtWy, kWscInvSqrtWf, kWscInvSqrtWy, kWscSqrtWf,
       kWscRows };

// Gains and modes of the Euclidean R~ while in scope (no-op without weights).
struct ModesRole {
  resolvent_op* op;
  ModesRole(resolvent_op* o) : op(o) { op->scale_role = 1; }
  ~ModesRole() { op->scale_role = 0; }
};

// Marks the handle as capturing while the caller's stream records a graph.
struct CaptureScope {
  resolvent_op* op;
  bool prev;
  CaptureScope(resolvent_op* o, hipStream_t st) : op(o), prev(o->capturing) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs == hipStreamCaptureStatusActive) op->capturing = true;
  }
  ~CaptureScope() { op->capturing = prev; }
};

// ---- runtime.cpp: the handle's set-up, workspace and small batched linear algebra ----
// Named workspace slot of at least `bytes` (grown on demand; carved from the arena in a no-allocation call).
int ws_get(resolvent_op* op, const std::string& name, size_t bytes, void** out);
// hipMalloc + synchronous copy of host data (set-up only).
int upload(void** dst, const void* src, size_t bytes);
// Uncached exchange areas that are no longer used (kept allocated until the process ends).
std::vector<void*>& retired_exchange_areas();
bool is_grid(const resolvent_op* op);
// Split-K factor of the per-frequency reductions for the longest instance, and that length.
int nsplit_for(int64_t maxlen);
int64_t max_instance_len(const resolvent_op* op);
// CholeskyQR2 of the [nw][k][N] FP64 blocks X in place (X <- Q); rtot receives R = R2 R1.
int cholqr2(resolvent_op* op, int nw, int k, double* X, void* rtot, double* norm_hist, hipStream_t st);
// V <- W_f^{-1/2} V, U <- W_y^{-1/2} U (modes of the Euclidean R~ back to the problem's metrics).
int modes_to_problem(resolvent_op* op, int nw, int k, void* V, void* U, hipStream_t st);

// ---- runs.cpp: run scheduling ----
int make_plan(const resolvent_op* op, const resolvent_grid* g, const resolvent_run* r, Plan* pl);
// RK4 steps per kernel step of a run (the operator's step power where the schedule allows it).
int run_power(const resolvent_op* op, const Plan& pl);
int phase_table(resolvent_op* op, int64_t P, void** out);
int phase_table64(resolvent_op* op, int64_t P, void** out);
// G_j = h Q_j(Z) F_j (FP64 Horner passes; m-step combination for m > 1).
int prefilter(resolvent_op* op, const Plan& pl, int k, const void* in, int in_fp64, void* G, int sigma, int M,
              hipStream_t st, int out_fp64 = -1);
// Forcing rows sum_j e^{i sigma w_j t_s} G_j (phase GEMM mode 0).
int synth_rows(int fp64, int nw, int64_t P, double w0h, int sigma, const void* btab, const void* G, int64_t ncols,
               int64_t s0, int64_t stride, int64_t M, void* out, hipStream_t st);
// acc_j += scale sum_m e^{-i sigma w_j t_m} rows_m (phase GEMM mode 1, FP64 accumulation).
int project_rows(resolvent_op* op, int fp64, int nw, int64_t P, double w0h, int sigma, void* btab, const void* rows,
                 int64_t ld, int64_t ncols, int64_t s0, int64_t stride, int64_t count, double scale, double* acc,
                 hipStream_t st);
int march_1d(resolvent_op* op, int k, int64_t n, const ForceSpec& fs, const SnapSpec& ss, const void* dsegs,
             int64_t nseg, hipStream_t st, int mstep = 1);
int march_grid(resolvent_op* op, int k, int64_t n, const ForceSpec& fs, const SnapSpec& ss, hipStream_t st);
// Device copy of the stepper regions of all k columns.
int upload_regions(resolvent_op* op, int k, void** dsegs, int64_t* nseg, hipStream_t st);
// One run of any operator kind into the FP64 accumulator acc (sigma = +1 direct, -1 adjoint).
int run_any(resolvent_op* op, const Plan& pl, int k, const void* in, int in_fp64, double* acc, int sigma,
            hipStream_t st);
// resolvent_apply / resolvent_adjoint_apply after the argument checks.
int apply_common(resolvent_op* op, const resolvent_grid* g, const resolvent_run* r, int k, const void* in, void* out,
                 int sigma, hipStream_t st);
int zero_device(void* p, size_t bytes, hipStream_t st);

}  // namespace rt
