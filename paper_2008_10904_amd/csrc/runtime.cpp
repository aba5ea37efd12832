// Host runtime of the resolvent library: the C ABI of include/resolvent.h, operator set-up (RK4 step stencils
// of L and L^H), run scheduling (synthesis table or tiles, stepper launches, projection flushes), the block
// power iteration driver and the decay probe.  All device work is stream-ordered on the caller's stream.
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

namespace {

thread_local std::string g_last_error;

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

#define HIP_TRY(expr)                                                                                   \
  do {                                                                                                  \
    hipError_t e_ = (expr);                                                                             \
    if (e_ != hipSuccess) return fail(RES_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

double env_double(const char* name, double dflt) {
  const char* v = std::getenv(name);
  return v ? std::atof(v) : dflt;
}
long env_long(const char* name, long dflt) {
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

Band band_mul(const Band& A, const Band& B) {
  Band C(A.n, A.r + B.r);
  for (int64_t i = 0; i < A.n; ++i)
    for (int e = -A.r; e <= A.r; ++e) {
      const int64_t k = i + e;
      if (k < 0 || k >= A.n) continue;
      const cd a = A.get(i, e);
      if (a == cd(0, 0)) continue;
      for (int f = -B.r; f <= B.r; ++f) {
        const int64_t jcol = k + f;
        if (jcol < 0 || jcol >= A.n) continue;
        C.at(i, e + f) += a * B.get(k, f);
      }
    }
  return C;
}

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

}  // namespace

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

namespace {

// Uncached exchange areas that are no longer used; kept allocated until the process ends.
std::vector<void*>& retired_exchange_areas() {
  static std::vector<void*> v;
  return v;
}

int ws_get(resolvent_op* op, const std::string& name, size_t bytes, void** out) {
  if (op->arena) {
    Arena& a = *op->arena;
    auto it = a.slots.find(name);
    if (it != a.slots.end() && it->second.second >= bytes) {
      *out = it->second.first;
      return RES_OK;
    }
    const size_t off = (a.used + 255) & ~(size_t)255;
    if (off + bytes > a.cap)
      return fail(RES_EINVAL, "no-allocation scratch exhausted at '" + name + "' (" + std::to_string(off + bytes) +
                              " of " + std::to_string(a.cap) + " bytes)");
    a.slots[name] = {a.base + off, bytes};
    a.used = off + bytes;
    *out = a.base + off;
    return RES_OK;
  }
  DevBuf& b = op->ws[name];
  if (b.bytes < bytes) {
    if (op->capturing)
      return fail(RES_EINVAL, "workspace '" + name + "' must grow during graph capture: make one uncaptured call "
                              "with the same sizes first");
    if (b.p) HIP_TRY(hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
    if (hipMalloc(&b.p, bytes) != hipSuccess) {
      b.p = nullptr;
      (void)hipGetLastError();
      return fail(RES_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes for " + name + " failed");
    }
    b.bytes = bytes;
  }
  *out = b.p;
  return RES_OK;
}

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

int upload(void** dst, const void* src, size_t bytes) {
  HIP_TRY(hipMalloc(dst, bytes));
  HIP_TRY(hipMemcpy(*dst, src, bytes, hipMemcpyHostToDevice));
  return RES_OK;
}

// P(Z) = I + Z + Z^2/2 + Z^3/6 + Z^4/24 of a tridiagonal Z, as a radius-4 band.
Band rk4_step_band(const std::vector<cd>& zl, const std::vector<cd>& zd, const std::vector<cd>& zu) {
  const int64_t n = (int64_t)zd.size();
  Band Z(n, 1);
  for (int64_t i = 0; i < n; ++i) {
    Z.at(i, -1) = zl[i];
    Z.at(i, 0) = zd[i];
    Z.at(i, 1) = zu[i];
  }
  Band Z2 = band_mul(Z, Z), Z3 = band_mul(Z2, Z), Z4 = band_mul(Z3, Z);
  Band P(n, kBandRadius);
  for (int64_t i = 0; i < n; ++i) {
    P.at(i, 0) += 1.0;
    for (int d = -1; d <= 1; ++d) P.at(i, d) += Z.get(i, d);
    for (int d = -2; d <= 2; ++d) P.at(i, d) += Z2.get(i, d) / 2.0;
    for (int d = -3; d <= 3; ++d) P.at(i, d) += Z3.get(i, d) / 6.0;
    for (int d = -4; d <= 4; ++d) P.at(i, d) += Z4.get(i, d) / 24.0;
  }
  return P;
}

// Working-precision bands of P(Z)^m and P(Z^H)^m for m = op->step_power > 1 (FP64 products of the host bands,
// rounded once).
int build_power_bands(resolvent_op* op) {
  for (int s = 0; s < 2; ++s) {
    if (op->d_bandm[s]) HIP_TRY(hipFree(op->d_bandm[s]));
    op->d_bandm[s] = nullptr;
    if (op->step_power <= 1) continue;
    Band Pm = op->hband[s];
    for (int q = 1; q < op->step_power; q *= 2) Pm = band_mul(Pm, Pm);
    if (op->fp64()) {
      RES_TRY(upload(&op->d_bandm[s], Pm.m.data(), Pm.m.size() * sizeof(cd)));
    } else {
      std::vector<std::complex<float>> pf(Pm.m.size());
      for (size_t i = 0; i < Pm.m.size(); ++i)
        pf[i] = std::complex<float>((float)Pm.m[i].real(), (float)Pm.m[i].imag());
      RES_TRY(upload(&op->d_bandm[s], pf.data(), pf.size() * sizeof(std::complex<float>)));
    }
  }
  return RES_OK;
}

int build_1d_stencils(resolvent_op* op) {
  const int64_t n = op->N;
  // adjoint tridiagonal: (Z^H)_{i,i-1} = conj(Z_{i-1,i}), (Z^H)_{i,i+1} = conj(Z_{i+1,i})
  std::vector<cd> al(n), ad(n), au(n);
  for (int64_t i = 0; i < n; ++i) {
    ad[i] = std::conj(op->zd[i]);
    al[i] = i > 0 ? std::conj(op->zu[i - 1]) : cd(0, 0);
    au[i] = i + 1 < n ? std::conj(op->zl[i + 1]) : cd(0, 0);
  }
  const std::vector<cd>* L3[2][3] = {{&op->zl, &op->zd, &op->zu}, {&al, &ad, &au}};
  for (int s = 0; s < 2; ++s) {
    std::vector<cd> tri((size_t)n * 3);
    for (int64_t i = 0; i < n; ++i) {
      tri[3 * i + 0] = (*L3[s][0])[i];
      tri[3 * i + 1] = (*L3[s][1])[i];
      tri[3 * i + 2] = (*L3[s][2])[i];
    }
    if (op->d_tri[s]) HIP_TRY(hipFree(op->d_tri[s]));
    op->d_tri[s] = nullptr;
    RES_TRY(upload(&op->d_tri[s], tri.data(), tri.size() * sizeof(cd)));
    Band P = rk4_step_band(*L3[s][0], *L3[s][1], *L3[s][2]);
    if (op->d_band[s]) HIP_TRY(hipFree(op->d_band[s]));
    op->d_band[s] = nullptr;
    if (op->d_band64[s]) HIP_TRY(hipFree(op->d_band64[s]));
    op->d_band64[s] = nullptr;
    RES_TRY(upload(&op->d_band64[s], P.m.data(), P.m.size() * sizeof(cd)));
    if (op->fp64()) {
      RES_TRY(upload(&op->d_band[s], P.m.data(), P.m.size() * sizeof(cd)));
    } else {
      std::vector<std::complex<float>> pf(P.m.size());
      for (size_t i = 0; i < P.m.size(); ++i) pf[i] = std::complex<float>((float)P.m[i].real(), (float)P.m[i].imag());
      RES_TRY(upload(&op->d_band[s], pf.data(), pf.size() * sizeof(std::complex<float>)));
    }
    op->hband[s] = std::move(P);
  }
  return build_power_bands(op);
}

bool is_grid(const resolvent_op* op) { return op->kind == RES_OP_ADR2D || op->kind == RES_OP_ADR3D3C; }

// Device coefficient sets of Z and Z^H (real coefficients, so Z^H = Z^T): x-neighbour coefficients swap (they are
// constant along x), y/z-neighbour coefficients move to the neighbouring line, the coupling matrix transposes.
int build_grid_coefficients(resolvent_op* op) {
  for (void* b : op->gbufs) (void)hipFree(b);
  op->gbufs.clear();
  const int64_t nl = op->ny * op->nz, nn = nl * op->nx;
  std::vector<double> tx[6];
  for (int a = 0; a < 6; ++a) tx[a].assign(nl, 0.0);
  std::vector<double> tK(op->gK.size(), 0.0);
  for (int64_t l = 0; l < nl; ++l) {
    const int64_t iy = l % op->ny, iz = l / op->ny;
    tx[0][l] = op->gx[1][l];
    tx[1][l] = op->gx[0][l];
    tx[2][l] = iy > 0 ? op->gx[3][l - 1] : 0.0;             // cym' = cyp of the line below
    tx[3][l] = iy + 1 < op->ny ? op->gx[2][l + 1] : 0.0;    // cyp' = cym of the line above
    tx[4][l] = iz > 0 ? op->gx[5][l - op->ny] : 0.0;
    tx[5][l] = iz + 1 < op->nz ? op->gx[4][l + op->ny] : 0.0;
    if (!op->gK.empty())
      for (int c = 0; c < 3; ++c)
        for (int cp = 0; cp < 3; ++cp) tK[l * 9 + c * 3 + cp] = op->gK[l * 9 + cp * 3 + c];
  }
  auto up = [&](const std::vector<double>& v, bool f64, const void** dst) -> int {
    *dst = nullptr;
    if (v.empty()) return RES_OK;
    void* d = nullptr;
    if (f64) {
      RES_TRY(upload(&d, v.data(), v.size() * sizeof(double)));
    } else {
      std::vector<float> f(v.begin(), v.end());
      RES_TRY(upload(&d, f.data(), f.size() * sizeof(float)));
    }
    op->gbufs.push_back(d);
    *dst = d;
    return RES_OK;
  };
  for (int s = 0; s < 2; ++s) {
    const std::vector<double>* X = s == 0 ? op->gx : tx;
    const std::vector<double>& K = s == 0 ? op->gK : tK;
    for (int pass = 0; pass < 2; ++pass) {
      const bool f64 = pass == 0;
      if (!f64 && op->fp64()) {
        op->gw[s] = op->g64[s];
        continue;
      }
      GridOpDev& g = f64 ? op->g64[s] : op->gw[s];
      g.ncomp = op->ncomp;
      g.nx = op->nx;
      g.ny = op->ny;
      g.nz = op->nz;
      RES_TRY(up(X[0], f64, &g.cxm));
      RES_TRY(up(X[1], f64, &g.cxp));
      RES_TRY(up(X[2], f64, &g.cym));
      RES_TRY(up(X[3], f64, &g.cyp));
      RES_TRY(up(X[4], f64, &g.czm));
      RES_TRY(up(X[5], f64, &g.czp));
      RES_TRY(up(op->gd, f64, &g.d));
      RES_TRY(up(K, f64, &g.K));
      g.kmask = 0;
      for (size_t i = 0; i < K.size(); ++i)
        if (K[i] != 0.0) g.kmask |= 1 << (int)(i % 9);
      g.kv = K.empty() || g.kmask == 0 ? 0 : (g.kmask & ~0x006) == 0 ? 1 : (g.kmask & ~0x048) == 0 ? 2 : 3;
      g.lc = nullptr;
      if (!f64 && op->ncomp == 3) {  // packed line coefficients of the one-launch FP32 step
        std::vector<double> pk((size_t)nl * 8, 0.0);
        for (int64_t l = 0; l < nl; ++l) {
          for (int a = 0; a < 6; ++a) pk[l * 8 + a] = X[a][l];
          if (g.kv == 1 || g.kv == 2) {
            pk[l * 8 + 6] = K[l * 9 + (g.kv == 1 ? 1 : 3)];
            pk[l * 8 + 7] = K[l * 9 + (g.kv == 1 ? 2 : 6)];
          }
        }
        RES_TRY(up(pk, false, &g.lc));
      }
    }
  }
  (void)nn;
  return RES_OK;
}

// Workgroup regions of one column.  chunk == 0: the whole column in one workgroup (no halo, any number of
// steps per launch).  Otherwise owned chunks of `chunk` unknowns with a halo of 4 * block unknowns on each side
// (the step stencil's radius times the steps per launch), clipped to the column.
void plan_1d_regions(resolvent_op* op, int64_t chunk, int64_t block, std::vector<Seg1D>* out) {
  out->clear();
  const int64_t n = op->N;
  if (chunk <= 0 || chunk >= n) {
    out->push_back(Seg1D{0, 0, 0, (int32_t)n, (int32_t)n, -1, -1});
    return;
  }
  const int64_t halo = (int64_t)kBandRadius * block;
  for (int64_t o0 = 0; o0 < n; o0 += chunk) {
    const int64_t o1 = std::min(n, o0 + chunk);
    const int64_t r0 = std::max<int64_t>(0, o0 - halo), r1 = std::min(n, o1 + halo);
    const int32_t i = (int32_t)out->size();
    out->push_back(Seg1D{0, (int32_t)(o0 - r0), r0, (int32_t)(r1 - r0), (int32_t)(o1 - o0), i - 1, -1});
  }
  out->front().left = -1;
  for (size_t i = 0; i + 1 < out->size(); ++i) (*out)[i].right = (int32_t)(i + 1);
}

int smallest_cfg(int64_t len) {
  static const int order[] = {0, 1, 2, 3, 4, 6};  // one default per capacity 64 .. 2048
  for (int c : order)
    if (step1d_capacity(c) >= len) return c;
  return -1;
}

// Default stepper plan: a column of up to 256 unknowns in one workgroup; longer columns in owned chunks of 128
// with a halo of 64 (16 steps per block), marched by one persistent cooperative launch with in-kernel neighbour
// exchange when the grid is co-resident, else by relaunches every 16 steps.
// RESOLVENT_STEP1D="cfg,chunk,block[,persist]" overrides it.
// Apply a stepper plan: regions of one column, the kernel configuration (raised to the smallest that holds the
// longest region when needed) and whether the march runs as one persistent launch.
int apply_plan(resolvent_op* op, int cfg, int64_t chunk, int64_t block, int persist) {
  if (cfg < 0 || cfg >= kStep1DConfigs) return fail(RES_EINVAL, "stepper configuration out of range");
  if (chunk < 0 || block < 0) return fail(RES_EINVAL, "negative chunk or block");
  if (chunk > 0 && chunk < op->N && block < 1) return fail(RES_EINVAL, "a chunked plan needs block >= 1");
  std::vector<Seg1D> regs;
  plan_1d_regions(op, chunk, block, &regs);
  int64_t maxlen = 0;
  for (auto& r : regs) maxlen = std::max<int64_t>(maxlen, r.ndof);
  if (step1d_capacity(cfg) < maxlen) {
    const int c = smallest_cfg(maxlen);
    if (c < 0) return fail(RES_ENOTSUP, "stepper region of " + std::to_string(maxlen) + " unknowns is too long");
    cfg = c;
  }
  op->segs = regs;
  ++op->plan_version;
  op->step_cfg = cfg;
  op->step_chunk = (chunk > 0 && chunk < op->N) ? chunk : 0;
  op->step_block = op->step_chunk ? block : 0;
  // persistent exchange needs the halo inside the immediate neighbours and blocks made of whole prefetch rounds
  op->step_persist = persist && op->step_chunk > 0 && (int64_t)kBandRadius * block <= chunk &&
                     block % step1d_prefetch(cfg) == 0;
  return RES_OK;
}

// Default stepper plan: a column of up to 256 unknowns in one workgroup; longer columns in owned chunks with halos,
// marched by one persistent cooperative launch with in-kernel neighbour exchange when the grid is co-resident,
// else by relaunches at every exchange.  The chunking follows the step power (the fastest measured plans on a
// GL column of 2,000 unknowns): 4 steps per kernel step: chunks of 256, exchange every 32 steps, 512 threads;
// 2: chunks of 256, every 32 steps, 512 threads; 1: chunks of 128, every 16 steps, 256 threads.
// RESOLVENT_STEP1D="cfg,chunk,block[,persist]" overrides it; resolvent_op_tune searches for a faster one.
int plan_1d_default(resolvent_op* op) {
  int cfg;
  int64_t chunk = 0, block = 0;
  int persist = 1;
  if (op->N <= 256) {
    cfg = smallest_cfg(op->N);
  } else if (op->step_power == 4) {
    block = 32;
    chunk = 256;
    cfg = 10;  // 512 threads x 1 unknown, prefetch 4
  } else if (op->step_power == 2) {
    block = 32;
    chunk = 256;
    cfg = 13;  // 512 threads x 1 unknown, prefetch 8
  } else {
    block = 16;
    chunk = 128;
    cfg = 12;  // 256 threads x 1 unknown, prefetch 8
  }
  if (const char* e = std::getenv("RESOLVENT_STEP1D")) {
    int c = -1, pe = 1;
    long ch = 0, bl = 0;
    const int got = std::sscanf(e, "%d,%ld,%ld,%d", &c, &ch, &bl, &pe);
    if (got >= 3 && c >= 0 && c < kStep1DConfigs) {
      cfg = c;
      chunk = ch;
      block = bl;
      persist = got >= 4 ? pe : 1;
    }
  }
  RES_TRY(apply_plan(op, cfg, chunk, block, persist));
  op->plan_default = true;
  return RES_OK;
}

int phase_table(resolvent_op* op, int64_t P, void** out) {
  auto it = op->btab.find(P);
  if (it != op->btab.end()) {
    *out = it->second;
    return RES_OK;
  }
  if (op->arena) {  // built on the device, stream-ordered, into the arena (no host staging buffer to keep alive)
    RES_TRY(ws_get(op, "phase_table", (size_t)P * op->wsize(), out));
    launch_phase_table(*out, op->fp64(), P, op->arena_stream);
    HIP_TRY(hipGetLastError());
    return RES_OK;
  }
  if (op->capturing) return fail(RES_EINVAL, "phase table must be built by an uncaptured call first");
  void* d = nullptr;
  if (op->fp64()) {
    std::vector<cd> t((size_t)P);
    for (int64_t m = 0; m < P; ++m) t[m] = std::polar(1.0, 2.0 * M_PI * (double)m / (double)P);
    RES_TRY(upload(&d, t.data(), t.size() * sizeof(cd)));
  } else {
    std::vector<std::complex<float>> t((size_t)P);
    for (int64_t m = 0; m < P; ++m) {
      const cd z = std::polar(1.0, 2.0 * M_PI * (double)m / (double)P);
      t[m] = std::complex<float>((float)z.real(), (float)z.imag());
    }
    RES_TRY(upload(&d, t.data(), t.size() * sizeof(std::complex<float>)));
  }
  op->btab[P] = d;
  *out = d;
  return RES_OK;
}

// FP64 table e^{2 pi i m / P} whatever the working precision (the reverse mode always runs in FP64).
int phase_table64(resolvent_op* op, int64_t P, void** out) {
  if (op->fp64()) return phase_table(op, P, out);
  auto it = op->btab64.find(P);
  if (it != op->btab64.end()) {
    *out = it->second;
    return RES_OK;
  }
  if (op->capturing) return fail(RES_EINVAL, "phase table must be built by an uncaptured call first");
  std::vector<cd> t((size_t)P);
  for (int64_t m = 0; m < P; ++m) t[m] = std::polar(1.0, 2.0 * M_PI * (double)m / (double)P);
  void* d = nullptr;
  RES_TRY(upload(&d, t.data(), t.size() * sizeof(cd)));
  op->btab64[P] = d;
  *out = d;
  return RES_OK;
}

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

int make_plan(const resolvent_op* op, const resolvent_grid* g, const resolvent_run* r, Plan* pl) {
  if (!g || !r) return fail(RES_EINVAL, "grid and run must not be NULL");
  if (g->n_omega < 1) return fail(RES_EINVAL, "n_omega must be >= 1");
  if (!(std::fabs(g->domega) > 0)) return fail(RES_EGRID, "domega must be nonzero");
  const double Pd = 2.0 * M_PI / (std::fabs(g->domega) * op->h);
  const int64_t P = (int64_t)std::llround(Pd);
  if (P < 1 || std::fabs(std::fabs(g->domega) * (double)P * op->h - 2.0 * M_PI) > 1e-9 * 2.0 * M_PI)
    return fail(RES_EGRID, "|domega| * P * h != 2 pi for integer P (P ~ " + std::to_string(Pd) + ")");
  if (g->n_omega > P) return fail(RES_EGRID, "more frequencies than steps per period (aliasing)");
  pl->w0 = g->omega0;
  pl->dw = g->domega;
  pl->nw = g->n_omega;
  pl->P = P;
  pl->method = r->method;
  if (r->method == RES_TRANSIENT) {
    if (r->tail < 0) return fail(RES_EINVAL, "tail must be >= 0");
    pl->S = P + r->tail;
    pl->forced_end = P;
    pl->pfirst = 0;
    pl->pstride = 1;
    pl->pcount = pl->S;
    pl->scale = 1.0 / (double)P;
  } else if (r->method == RES_PERIODIC) {
    if (r->periods < 1) return fail(RES_EINVAL, "periods must be >= 1");
    const int64_t D = r->stride < 1 ? 1 : r->stride;
    if (P % D != 0 || P / D < g->n_omega)
      return fail(RES_EGRID, "projection stride must divide P and leave at least n_omega samples per period");
    pl->S = (int64_t)r->periods * P;
    pl->forced_end = pl->S;
    pl->pfirst = (int64_t)(r->periods - 1) * P;
    pl->pstride = D;
    pl->pcount = P / D;
    pl->scale = (double)D / (double)P;
  } else {
    return fail(RES_EINVAL, "unknown method");
  }
  return RES_OK;
}

int nsplit_for(int64_t maxlen) {
  int64_t s = (maxlen + 2047) / 2048;
  if (s < 1) s = 1;
  if (s > 1024) s = 1024;
  return (int)s;
}

int64_t max_instance_len(const resolvent_op* op) {
  int64_t m = 0;
  for (int i = 0; i < op->ninst; ++i) m = std::max(m, op->off[i + 1] - op->off[i]);
  return m;
}

// Flush `rows` buffered snapshot rows (the first being projected sample m_first) into acc.
void trace_norm(const char* what, const void* p, int64_t count, int fp64, hipStream_t st);

// acc[j][n] += scale * sum_m e^{-i sigma w_j t_m} rows[m][n] for m < count, t_m = (s0 + m*stride) h,
// w_j = w0 + j dw, dw = 2 pi / (P h); rows have leading dimension ld; the GEMM runs in FP64 if fp64 != 0.
int project_rows(resolvent_op* op, int fp64, int nw, int64_t P, double w0h, int sigma, void* btab, const void* rows,
                 int64_t ld, int64_t ncols, int64_t s0, int64_t stride, int64_t count, double scale, double* acc,
                 hipStream_t st) {
  if (count <= 0) return RES_OK;
  PhaseGemmArgs a{};
  a.mode = 1;
  a.M = nw;
  a.Ncols = ncols;
  a.K = count;
  a.btab = btab;
  a.P = P;
  a.sigma = sigma;
  a.w0h = w0h;
  a.s0 = s0;
  a.stride = stride;
  a.bmat = rows;
  a.ldb = ld;
  a.out = acc;
  a.scale = scale;
  // split K so that the grid has enough workgroups
  const int64_t tiles = ((nw + 63) / 64) * ((ncols + 63) / 64);
  int64_t nsplit = 1;
  if (tiles < 1024) nsplit = std::min<int64_t>((1024 + tiles - 1) / tiles, (count + 63) / 64);
  if (nsplit < 1) nsplit = 1;
  if (op->arena) nsplit = std::min<int64_t>(nsplit, op->arena->sz.max_nsplit);
  const int64_t kps = ((count + nsplit - 1) / nsplit + 15) / 16 * 16;
  nsplit = (count + kps - 1) / kps;
  a.k_per_split = kps;
  if (nsplit > 1) {
    void* part = nullptr;
    RES_TRY(ws_get(op, "proj_partial", (size_t)nsplit * nw * ncols * sizeof(cd), &part));
    a.partial = part;
    if (launch_phase_gemm(a, fp64, st)) return fail(RES_EINVAL, "projection GEMM launch");
    launch_reduce_partials(part, acc, (int64_t)nw * ncols, (int)nsplit, scale, st);
  } else {
    a.partial = nullptr;
    if (launch_phase_gemm(a, fp64, st)) return fail(RES_EINVAL, "projection GEMM launch");
  }
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

// out[r][n] = sum_j e^{i sigma w_j t_r} G[j][n] for r < M, t_r = (s0 + r*stride) hs with w0h = w0 hs and a
// table of period P (dw hs = 2 pi / P); G is [nw][ncols].
int synth_rows(int fp64, int nw, int64_t P, double w0h, int sigma, const void* btab, const void* G, int64_t ncols,
               int64_t s0, int64_t stride, int64_t M, void* out, hipStream_t st) {
  if (M <= 0) return RES_OK;
  PhaseGemmArgs a{};
  a.mode = 0;
  a.M = M;
  a.Ncols = ncols;
  a.K = nw;
  a.btab = btab;
  a.P = P;
  a.sigma = sigma;
  a.w0h = w0h;
  a.s0 = s0;
  a.stride = stride;
  a.bmat = G;
  a.ldb = ncols;
  a.out = out;
  a.k_per_split = nw;
  if (launch_phase_gemm(a, fp64, st)) return fail(RES_EINVAL, "synthesis GEMM launch");
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

int flush_projection(resolvent_op* op, const Plan& pl, int k, int sigma, void* btab, const void* snap,
                     int64_t snap_ld, int64_t m_first, int64_t rows, double* acc, hipStream_t st) {
  if (rows <= 0) return RES_OK;
  trace_norm("snapshots", snap, rows * snap_ld, op->fp64(), st);
  TimedLaunch tl(op, RES_TIMING_PROJECTION, st);
  return project_rows(op, op->fp64(), pl.nw, pl.P, pl.w0 * op->h, sigma, btab, snap, snap_ld, (int64_t)k * op->N,
                      pl.pfirst + m_first * pl.pstride, pl.pstride, rows, pl.scale, acc, st);
}

// Opt-in diagnostics (RESOLVENT_TRACE=1): synchronise and print the 2-norm of a device complex array.
void trace_norm(const char* what, const void* p, int64_t count, int fp64, hipStream_t st) {
  static const bool on = env_long("RESOLVENT_TRACE", 0) != 0;
  if (!on || p == nullptr) return;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone) return;
  (void)hipStreamSynchronize(st);
  double s = 0;
  if (fp64) {
    std::vector<cd> h(count);
    (void)hipMemcpy(h.data(), p, count * sizeof(cd), hipMemcpyDeviceToHost);
    for (auto& z : h) s += std::norm(z);
  } else {
    std::vector<std::complex<float>> h(count);
    (void)hipMemcpy(h.data(), p, count * sizeof(std::complex<float>), hipMemcpyDeviceToHost);
    for (auto& z : h) s += std::norm(std::complex<double>(z.real(), z.imag()));
  }
  std::fprintf(stderr, "[resolvent trace] %-28s count=%lld norm=%.6e err=%s\n", what, (long long)count,
               std::sqrt(s), hipGetErrorString(hipGetLastError()));
}

int zero_device(void* p, size_t bytes, hipStream_t st) {
  if (launch_zero(p, bytes, st)) return fail(RES_EINVAL, "zero fill of a size that is not a multiple of 4 bytes");
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

struct ForceSpec {
  const void* frc = nullptr;   // forcing rows or null (unforced)
  int64_t row0 = 0, period = 0;
  cd phi = cd(1, 0);
};
struct SnapSpec {
  void* snap = nullptr;        // snapshot rows or null
  int64_t ld = 0, first = 0, stride = 1, count = 0, row0 = 0;
};

// March n kernel steps of mstep RK4 steps each (op->march_band holds P(Z)^mstep; forcing rows and snapshot
// positions count kernel steps) for all k columns from the current state buffer.  With halo regions the march is
// cut into launches of op->step_block RK4 steps, the state ping-ponging between two buffers; otherwise one launch.
int march_1d(resolvent_op* op, int k, int64_t n, const ForceSpec& fs, const SnapSpec& ss, const void* dsegs,
             int64_t nseg, hipStream_t st, int mstep = 1) {
  const int64_t ncols = (int64_t)k * op->N;
  void* sb[2];
  RES_TRY(ws_get(op, "state0", (size_t)ncols * op->wsize(), &sb[0]));
  RES_TRY(ws_get(op, "state1", (size_t)ncols * op->wsize(), &sb[1]));
  const bool halo = op->step_block > 0;
  if (op->step_block % mstep != 0) return fail(RES_EINVAL, "exchange interval not a multiple of the step power");
  const int64_t kblock = op->step_block / mstep;  // kernel steps between exchanges
  bool persist = op->step_persist && kblock % step1d_prefetch(op->step_cfg) == 0 && !op->coop_refused;
  void* xbuf = nullptr;
  if (persist) {
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (step1d_coresident(op->fp64(), op->step_cfg, dev, mstep) < nseg) persist = false;
  }
  if (persist) {
    // Exchange rows in uncached device memory: every access of the persistent stepper's neighbour exchange then
    // goes to the device-coherent level, across XCDs, without L2 write-back/invalidate fences.  Uncached memory
    // is never freed once a kernel has used it (an outgrown area is retired, not released); it is reclaimed when
    // the process ends.  Every slot starts empty for each launch.
    const size_t need = (size_t)4 * ncols * op->wsize();  // [2 buffers][2 directions][ncols]
    if (op->arena && op->xch_bytes < need) persist = false;  // no allocation: relaunch at every exchange instead
  }
  if (persist) {
    const size_t need = (size_t)4 * ncols * op->wsize();
    if (op->xch_bytes < need) {
      if (op->capturing) return fail(RES_EINVAL, "exchange area must be allocated by an uncaptured call first");
      void* p = nullptr;
      HIP_TRY(hipExtMallocWithFlags(&p, need, hipDeviceMallocUncached));
      if (op->xch) retired_exchange_areas().push_back(op->xch);
      op->xch = p;
      op->xch_bytes = need;
    }
    xbuf = op->xch;
    launch_fill_empty(xbuf, op->fp64(), 4 * ncols, st);
  }
  const int64_t blk = (halo && !persist) ? kblock : n;
  for (int64_t b0 = 0; b0 < n; b0 += blk) {
    const int64_t nb = std::min(blk, n - b0);
    Step1DArgs a{};
    a.fp64 = op->fp64();
    a.cfg = op->step_cfg;
    a.mstep = mstep;
    a.segs = (const Seg1D*)dsegs;
    a.nseg = nseg;
    a.band = op->march_band;
    a.state_in = sb[op->cur_state];
    a.state_out = (halo && !persist) ? sb[1 - op->cur_state] : sb[op->cur_state];
    a.N = op->N;
    a.row_len = ncols;
    a.n_steps = nb;
    a.frc = fs.frc;
    a.frc_row0 = fs.row0 + b0;
    a.frc_period = fs.period;
    a.phi_re = fs.phi.real();
    a.phi_im = fs.phi.imag();
    if (ss.snap != nullptr && ss.count > 0) {
      // samples m with first + m*stride in [b0, b0 + nb)
      const int64_t mlo = b0 <= ss.first ? 0 : (b0 - ss.first + ss.stride - 1) / ss.stride;
      const int64_t last = b0 + nb - 1;
      const int64_t mhi = last < ss.first ? 0 : std::min(ss.count, (last - ss.first) / ss.stride + 1);
      if (mhi > mlo) {
        a.snap = ss.snap;
        a.snap_ld = ss.ld;
        a.snap_first = ss.first + mlo * ss.stride - b0;
        a.snap_stride = ss.stride;
        a.snap_count = mhi - mlo;
        a.snap_row0 = ss.row0 + mlo;
      }
    }
    a.persist = persist ? 1 : 0;
    a.xbuf = xbuf;
    a.block = persist ? kblock : nb;
    a.spin_ns = 2000000000ull;
    a.err = op->d_flag;
    int rc;
    if (persist && env_long("RESOLVENT_REFUSE_COOPERATIVE", 0) != 0) {
      rc = -2;  // the refusal a device can give, forced from the host (tests of the fallback below)
    } else {
      TimedLaunch tl(op, RES_TIMING_STEPPER, st);
      rc = launch_step1d(a, st);
    }
    if (rc) {
      (void)hipGetLastError();  // report the failed launch once, not again from the next call's error check
      if (persist && rc == -2 && !op->capturing) {
        // The device refused the cooperative launch (its co-residency resources may be held by another process):
        // nothing ran, so march with a relaunch at every exchange instead, for the rest of the handle's life.
        op->coop_refused = true;
        return march_1d(op, k, n, fs, ss, dsegs, nseg, st, mstep);
      }
      return fail(RES_EHIP, "stepper launch failed (" + std::to_string(rc) + ")");
    }
    if (halo && !persist) op->cur_state = 1 - op->cur_state;
  }
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

// March n steps of all k columns of a grid operator (Z or Z^H chosen by op->march_grid), the state ping-ponging
// between state0 and state1: 2-D one-component operators take one fused launch per step, and so do 3-D
// three-component operators with an FP32 state (the four stages pipelined along z); FP64 3-D states take two
// launches of two Horner stages each (the second writes the new state).
int march_grid(resolvent_op* op, int k, int64_t n, const ForceSpec& fs, const SnapSpec& ss, hipStream_t st) {
  const int64_t ncols = (int64_t)k * op->N;
  const size_t ws = op->wsize();
  const GridOpDev& g = *op->march_grid;
  const bool fused = g.ncomp == 1 && g.nz == 1;
  const bool fused3 = g.ncomp == 3 && !op->fp64();  // one launch per step (FP32 state); FP64 takes two passes
  void* sb[2];
  void* v2 = nullptr;
  RES_TRY(ws_get(op, "state0", (size_t)ncols * ws, &sb[0]));
  RES_TRY(ws_get(op, "state1", (size_t)ncols * ws, &sb[1]));
  if (!fused && !fused3) RES_TRY(ws_get(op, "gv1", (size_t)ncols * ws, &v2));
  TimedLaunch tl(op, RES_TIMING_STEPPER, st);
  int64_t next = (ss.snap != nullptr && ss.count > 0) ? ss.first : -1, m = 0;
  for (int64_t t = 0; t < n; ++t) {
    const void* frow = nullptr;
    if (fs.frc != nullptr) {
      int64_t row = fs.row0 + t;
      if (fs.period > 0) row %= fs.period;
      frow = (const char*)fs.frc + (size_t)row * ncols * ws;
    }
    void* srow = nullptr;
    if (t == next) {
      srow = (char*)ss.snap + (size_t)(ss.row0 + m) * ss.ld * ws;
      ++m;
      next = m < ss.count ? next + ss.stride : -1;
    }
    void* uin = sb[op->cur_state];
    void* uout = sb[1 - op->cur_state];
    if (fused) {
      if (launch_grid_step2d(g, op->fp64(), k, uin, uout, frow, fs.phi.real(), fs.phi.imag(), srow, st))
        return fail(RES_EINVAL, "2-D step launch");
    } else if (fused3) {
      if (launch_grid_step3d(g, k, uin, uout, frow, fs.phi.real(), fs.phi.imag(), srow, st))
        return fail(RES_EINVAL, "3-D step launch");
    } else if (launch_grid_pair3d(g, op->fp64(), k, uin, nullptr, v2, 0, nullptr, 0, 0, nullptr, st) ||
               launch_grid_pair3d(g, op->fp64(), k, uin, v2, uout, 1, frow, fs.phi.real(), fs.phi.imag(), srow,
                                  st)) {
      return fail(RES_EINVAL, "3-D step launch");
    }
    op->cur_state = 1 - op->cur_state;
  }
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

// Device copy of the regions of all k columns; uploaded again only when k or the plan changed.
int upload_regions(resolvent_op* op, int k, void** dsegs, int64_t* nseg, hipStream_t st) {
  if (is_grid(op)) {
    *dsegs = nullptr;
    *nseg = 0;
    return RES_OK;
  }
  if (!op->arena && op->segs_dev_k == k && op->segs_dev_version == op->plan_version) {
    *nseg = (int64_t)k * (int64_t)op->segs.size();
    return ws_get(op, "segs", (size_t)*nseg * sizeof(Seg1D), dsegs);
  }
  if (op->capturing) return fail(RES_EINVAL, "stepper regions must be uploaded by an uncaptured call first");
  std::vector<Seg1D>& segs = op->segs_k;  // kept in the handle: the upload is asynchronous
  segs.clear();
  const int32_t g = (int32_t)op->segs.size();
  for (int c = 0; c < k; ++c)
    for (auto sg : op->segs) {
      sg.col = c;
      if (sg.left >= 0) sg.left += c * g;
      if (sg.right >= 0) sg.right += c * g;
      segs.push_back(sg);
    }
  RES_TRY(ws_get(op, "segs", segs.size() * sizeof(Seg1D), dsegs));
  HIP_TRY(hipMemcpyAsync(*dsegs, segs.data(), segs.size() * sizeof(Seg1D), hipMemcpyHostToDevice, st));
  *nseg = (int64_t)segs.size();
  if (!op->arena) {  // the arena's slot is not the handle's cached copy
    op->segs_dev_k = k;
    op->segs_dev_version = op->plan_version;
  }
  return RES_OK;
}

// RK4 steps per kernel step for this run: the operator's step power when every step the run must see (period
// and forcing boundaries, projected samples, exchange interval) falls on a multiple of it, else 1.
int run_power(const resolvent_op* op, const Plan& pl) {
  const int64_t m = op->step_power;
  if (m <= 1 || is_grid(op)) return 1;
  if (pl.forced_end != pl.S || pl.P % m || pl.S % m || pl.pfirst % m || pl.pstride % m || op->step_block % m)
    return 1;
  return (int)m;
}

// G_j = h Q_j(Z) F_j by three Horner passes in FP64 (and, when M > 1, the combined forcing of M steps,
// sum_{r<M} e^{i sigma w_j r h} P^(M-1-r) G_j, by M - 1 Horner passes of P(Z)), written in the working precision.
// Each frequency's pre-filter is independent, so the FP64 work blocks hold a group of frequencies at a time, as
// many as fit in RESOLVENT_HORNER_BUDGET_GB (default 8 GiB): the 3-D workload's [96][3][12.6M] blocks would take
// 58 GB each.  G is written in FP64 if out_fp64 > 0, FP32 if out_fp64 == 0, the working precision if it is < 0.
int prefilter(resolvent_op* op, const Plan& pl, int k, const void* in, int in_fp64, void* G, int sigma, int M,
              hipStream_t st, int out_fp64 = -1) {
  const int64_t N = op->N;
  const int64_t ncols = (int64_t)k * N;
  const int nw = pl.nw;
  const int s = sigma > 0 ? 0 : 1;
  const int nbuf = M > 2 ? 3 : 2;
  const double budget = env_double("RESOLVENT_HORNER_BUDGET_GB", 8.0) * 1073741824.0;
  const double per_freq = (double)nbuf * (double)ncols * sizeof(cd);
  const int chunk = op->arena ? std::min(nw, op->arena->sz.horner_chunk)
                              : (int)std::max<int64_t>(1, std::min<int64_t>(nw, (int64_t)(budget / per_freq)));
  void *y1, *y2, *y3 = nullptr;
  RES_TRY(ws_get(op, "horner_a", (size_t)chunk * ncols * sizeof(cd), &y1));
  RES_TRY(ws_get(op, "horner_b", (size_t)chunk * ncols * sizeof(cd), &y2));
  if (M > 2) RES_TRY(ws_get(op, "horner_c", (size_t)chunk * ncols * sizeof(cd), &y3));
  const double sw0h = sigma * pl.w0 * op->h, sdwh = sigma * pl.dw * op->h;
  const size_t in_es = in_fp64 ? sizeof(cd) : sizeof(std::complex<float>);
  const int o64 = out_fp64 < 0 ? op->fp64() : (out_fp64 > 0 ? 1 : 0);
  const size_t out_es = o64 ? sizeof(cd) : sizeof(std::complex<float>);
  for (int j0 = 0; j0 < nw; j0 += chunk) {
    const int nc = std::min(chunk, nw - j0);
    const void* inc = (const char*)in + (size_t)j0 * ncols * in_es;
    void* Gc = (char*)G + (size_t)j0 * ncols * out_es;
    if (is_grid(op)) {
      const GridOpDev& g = op->g64[s];
      if (launch_grid_horner(g, nullptr, inc, in_fp64, y1, 1, k, nc, sw0h, sdwh, op->h, 0, st, j0) ||
          launch_grid_horner(g, (const cx<double>*)y1, inc, in_fp64, y2, 1, k, nc, sw0h, sdwh, op->h, 1, st, j0) ||
          launch_grid_horner(g, (const cx<double>*)y2, inc, in_fp64, Gc, o64, k, nc, sw0h, sdwh, op->h, 2, st, j0))
        return fail(RES_EINVAL, "n_omega * k too large for the forcing pre-filter grid");
      continue;
    }
    const cx<double>* tri = (const cx<double>*)op->d_tri[s];
    launch_tri_horner(tri, nullptr, inc, in_fp64, y1, 1, N, k, nc, sw0h, sdwh, op->h, 0, st, j0);
    launch_tri_horner(tri, (const cx<double>*)y1, inc, in_fp64, y2, 1, N, k, nc, sw0h, sdwh, op->h, 1, st, j0);
    if (M == 1) {
      launch_tri_horner(tri, (const cx<double>*)y2, inc, in_fp64, Gc, o64, N, k, nc, sw0h, sdwh, op->h, 2, st, j0);
      continue;
    }
    // G in FP64, then G^(M) = sum_{r<M} e^{i sw_j r h} P^(M-1-r) G by M-1 Horner passes of P (the last one writes
    // the working precision)
    launch_tri_horner(tri, (const cx<double>*)y2, inc, in_fp64, y1, 1, N, k, nc, sw0h, sdwh, op->h, 2, st, j0);
    const cx<double>* band = (const cx<double>*)op->d_band64[s];
    const cx<double>* x = (const cx<double>*)y1;
    for (int i = 1; i < M; ++i) {
      const bool last = i == M - 1;
      void* out = last ? Gc : (i & 1 ? y2 : y3);
      launch_band_horner(band, x, (const cx<double>*)y1, out, last ? o64 : 1, N, k, nc, sw0h, sdwh, i, st, j0);
      x = (const cx<double>*)out;
    }
  }
  return RES_OK;
}

// One time-marched run: acc[j][c][:] = R_d(sigma w_j)-run of in[j][c][:], with L (sigma = +1) or L^H (sigma = -1).
// `in` is [nw][k][N] complex of dtype in_fp64; acc is FP64 [nw][k][N] and is overwritten.
int run_1d(resolvent_op* op, const Plan& pl, int k, const void* in, int in_fp64, double* acc, int sigma,
           hipStream_t st) {
  const int64_t N = op->N;
  const int64_t ncols = (int64_t)k * N;
  const int nw = pl.nw;
  const int s = sigma > 0 ? 0 : 1;
  const size_t ws = op->wsize();
  const int M = run_power(op, pl);  // RK4 steps per kernel step; forcing rows and samples count kernel steps
  void *G, *btab;
  RES_TRY(ws_get(op, "G", (size_t)nw * ncols * ws, &G));
  RES_TRY(phase_table(op, pl.P, &btab));
  RES_TRY(prefilter(op, pl, k, in, in_fp64, G, sigma, M, st));
  if (is_grid(op)) op->march_grid = &op->gw[s];
  HIP_TRY(hipGetLastError());
  trace_norm("run input", in, (int64_t)nw * ncols, in_fp64, st);
  trace_norm("G = hQ(Z) F", G, (int64_t)nw * ncols, op->fp64(), st);
  void* st0;
  RES_TRY(ws_get(op, "state0", (size_t)ncols * ws, &st0));
  RES_TRY(ws_get(op, "state1", (size_t)ncols * ws, &st0));
  RES_TRY(ws_get(op, "state0", (size_t)ncols * ws, &st0));
  op->cur_state = 0;
  RES_TRY(zero_device(st0, (size_t)ncols * ws, st));
  RES_TRY(zero_device(acc, (size_t)nw * ncols * sizeof(cd), st));
  op->march_band = M > 1 ? op->d_bandm[s] : op->d_band[s];

  // Snapshot rows (ncols values and one scratch slot each), buffered for the projection GEMM.  Each flush reads
  // and writes the FP64 accumulator once, so longer flushes amortise that traffic: the default buffer is 8 GiB,
  // at most a tenth of the free device memory (plus the buffer this handle already holds) and at least 64 rows;
  // RESOLVENT_SNAP_BUDGET_GB overrides it.  It is taken before the forcing table, whose budget sees what is left.
  const int64_t snap_ld = ncols + 1;
  double snap_budget;
  if (op->arena) {
    snap_budget = (double)op->arena->sz.snap_rows * (double)snap_ld * (double)ws;
  } else if (std::getenv("RESOLVENT_SNAP_BUDGET_GB")) {
    snap_budget = env_double("RESOLVENT_SNAP_BUDGET_GB", 2.0) * 1073741824.0;
  } else {
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    const auto held = op->ws.find("snapshots");
    const double held_b = held != op->ws.end() ? (double)held->second.bytes : 0.0;
    snap_budget = std::min(8.0 * 1073741824.0, 0.1 * ((double)free_b + held_b));
    if (op->capturing && held_b > 0) snap_budget = held_b;  // a captured run reuses the buffer it was sized with
  }
  int64_t snap_cap = std::max<int64_t>(64, (int64_t)(snap_budget / ((double)snap_ld * ws)));
  snap_cap = std::min<int64_t>(snap_cap, pl.pcount);
  void* snap = nullptr;
  RES_TRY(ws_get(op, "snapshots", (size_t)snap_cap * snap_ld * ws, &snap));

  // Forcing rows: the whole first period as one table when it fits in device memory (it is then synthesised
  // once per run and reused by every period), else tiles synthesised as the march goes.  The default budget
  // is the free device memory (plus the table this handle already holds) minus a reserve for the rest of the
  // run; RESOLVENT_TABLE_BUDGET_GB overrides it.
  double table_budget;
  if (op->arena) {
    table_budget = op->arena->sz.table ? 1e300 : -1.0;
  } else if (std::getenv("RESOLVENT_TABLE_BUDGET_GB")) {
    table_budget = env_double("RESOLVENT_TABLE_BUDGET_GB", 0.0) * 1073741824.0;
  } else {
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    const auto held = op->ws.find("forcing");
    const double reserve = 6.0 * 1073741824.0;
    table_budget = (double)free_b + (held != op->ws.end() ? (double)held->second.bytes : 0.0) - reserve;
  }
  const int64_t table_rows = std::min<int64_t>(pl.P, pl.forced_end) / M;  // one row per kernel step
  bool table_mode = (double)table_rows * (double)ncols * (double)ws <= table_budget;
  int64_t tile_rows = 0;
  void* frc = nullptr;
  PhaseGemmArgs syn{};
  syn.mode = 0;
  syn.Ncols = ncols;
  syn.K = nw;
  syn.btab = btab;
  syn.P = pl.P;
  syn.sigma = sigma;
  syn.w0h = pl.w0 * op->h;
  syn.stride = M;
  syn.bmat = G;
  syn.ldb = ncols;
  syn.k_per_split = nw;
  if (table_mode && ws_get(op, "forcing", (size_t)table_rows * ncols * ws, &frc) != RES_OK) {
    g_last_error.clear();
    table_mode = false;  // the allocation failed after all: fall back to tiles
  }
  // In table mode the first period's march overlaps the table's synthesis: rows are synthesised in chunks, the
  // first on the caller's stream and the others on the handle's side stream, which starts once the caller's
  // earlier work is done (a previous run may still read the table buffer); the march of the first period waits
  // for each chunk's event before it reaches the chunk's rows.  A row is synthesised in about half the time the
  // 1-D march takes to consume it, so the chunks double in size from 1,024 rows: only the first one is not
  // hidden.  Rows are independent, so every row gets the same value as from one GEMM over the whole table (chunk
  // bounds are whole 64-row tiles).  Off under graph capture and in the no-allocation entry point, for grid
  // operators, whose step kernels occupy every CU, and for marches whose workgroups take more than half the CUs:
  // there the synthesis slows the march by more than it saves (the 64-instance batch in FP64: 2.84 s per iteration
  // overlapped, 2.62 s not).  RESOLVENT_SYNTH_OVERLAP=0 turns it off.
  std::vector<int64_t> ov_bound;  // chunk c holds table rows [ov_bound[c], ov_bound[c + 1])
  int nov = 0;
  int cus = 0;
  if (table_mode && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, op->device) != hipSuccess)
    cus = 0;
  const bool cus_free = 2 * (int64_t)k * (int64_t)op->segs.size() <= (int64_t)cus;
  if (table_mode && !op->capturing && !op->arena && !is_grid(op) && cus_free &&
      env_long("RESOLVENT_SYNTH_OVERLAP", 1) != 0 && table_rows >= 4096) {
    ov_bound.push_back(0);
    for (int64_t len = 1024; ov_bound.back() < table_rows; len *= 2)
      ov_bound.push_back(std::min(table_rows, ov_bound.back() + len));
    nov = (int)ov_bound.size() - 1;
  }
  if (table_mode && nov > 0) {
    if (!op->side_stream) HIP_TRY(hipStreamCreateWithFlags(&op->side_stream, hipStreamNonBlocking));
    while ((int)op->side_ev.size() < nov) {
      hipEvent_t ev;
      HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
      op->side_ev.push_back(ev);
    }
    auto chunk = [&](int c, hipStream_t sc) -> int {
      const int64_t r0 = ov_bound[c];
      syn.M = ov_bound[c + 1] - r0;
      syn.s0 = r0 * M;
      syn.out = (char*)frc + (size_t)r0 * ncols * ws;
      TimedLaunch tl(op, RES_TIMING_SYNTHESIS, sc);
      if (launch_phase_gemm(syn, op->fp64(), sc)) return fail(RES_EINVAL, "synthesis GEMM launch");
      HIP_TRY(hipGetLastError());
      return RES_OK;
    };
    RES_TRY(chunk(0, st));
    HIP_TRY(hipEventRecord(op->side_ev[0], st));
    HIP_TRY(hipStreamWaitEvent(op->side_stream, op->side_ev[0], 0));
    for (int c = 1; c < nov; ++c) {
      RES_TRY(chunk(c, op->side_stream));
      HIP_TRY(hipEventRecord(op->side_ev[c], op->side_stream));
    }
  } else if (table_mode) {
    syn.M = table_rows;
    syn.s0 = 0;
    syn.out = frc;
    TimedLaunch tl(op, RES_TIMING_SYNTHESIS, st);
    if (launch_phase_gemm(syn, op->fp64(), st)) return fail(RES_EINVAL, "synthesis GEMM launch");
    HIP_TRY(hipGetLastError());
    trace_norm("forcing table", frc, table_rows * ncols, op->fp64(), st);
  } else {
    // Each tile's synthesis GEMM reads the whole [nw][k N] block G once, so longer tiles amortise that read over
    // more rows (one row per kernel step; on the 3-D workload G is 29 GB against 302 MB per row).  Default: the
    // rows of 2 GiB, at least 64, or up to 256 when a third of the free device memory (plus the tile this handle
    // already holds) has room for them; RESOLVENT_TILE_BUDGET_GB overrides.
    const double row_b = (double)ncols * (double)ws;
    const double budget = env_double("RESOLVENT_TILE_BUDGET_GB", 2.0) * 1073741824.0;
    tile_rows = std::max<int64_t>(64, (int64_t)(budget / row_b));
    if (op->arena) {
      tile_rows = op->arena->sz.tile_rows;
    } else if (!std::getenv("RESOLVENT_TILE_BUDGET_GB")) {
      size_t free_b = 0, total_b = 0;
      HIP_TRY(hipMemGetInfo(&free_b, &total_b));
      const auto held = op->ws.find("forcing");
      const double held_b = held != op->ws.end() ? (double)held->second.bytes : 0.0;
      if (op->capturing && held_b > 0) {
        tile_rows = std::max<int64_t>(1, (int64_t)(held_b / row_b) - 16);  // a captured run reuses its tile
      } else {
        const double room = ((double)free_b + held_b - 6.0 * 1073741824.0) / 3.0;
        tile_rows = std::max<int64_t>(tile_rows, std::min<int64_t>(256, (int64_t)(room / row_b) - 16));
      }
    }
    RES_TRY(ws_get(op, "forcing", (size_t)(tile_rows + 16) * ncols * ws, &frc));  // + prefetch padding rows
  }

  void* dsegs;
  int64_t nseg;
  RES_TRY(upload_regions(op, k, &dsegs, &nseg, st));

  int64_t buffered = 0, buf_m0 = 0;  // rows in the snapshot buffer and the sample index of the first
  int64_t s0 = 0;
  int ov_waited = 1;  // synthesis chunks below this one are ordered before the caller's stream's next work
  // however the run ends, the caller's stream waits for every chunk (the next run rewrites the table)
  struct OverlapJoin {
    resolvent_op* op;
    hipStream_t st;
    const int& nov;
    int& waited;
    ~OverlapJoin() {
      for (; waited < nov; ++waited) (void)hipStreamWaitEvent(st, op->side_ev[waited], 0);
    }
  } ov_join{op, st, nov, ov_waited};
  auto first_m_at_or_after = [&](int64_t t) -> int64_t {
    if (t <= pl.pfirst) return 0;
    return std::min(pl.pcount, (t - pl.pfirst + pl.pstride - 1) / pl.pstride);
  };
  while (s0 < pl.S) {
    // chunk end: period boundary (table mode), tile size (tile mode), forcing switch-off, snapshot capacity
    int64_t e = pl.S;
    if (table_mode) e = std::min(e, (s0 / pl.P + 1) * pl.P);
    else e = std::min(e, s0 + tile_rows * M);
    if (nov > 0 && s0 < pl.P && s0 < pl.forced_end) {  // first period: up to the end of the synthesised chunk
      int c = 0;
      while (ov_bound[c + 1] * M <= s0) ++c;
      for (; ov_waited <= c && ov_waited < nov; ++ov_waited)
        HIP_TRY(hipStreamWaitEvent(st, op->side_ev[ov_waited], 0));
      e = std::min(e, ov_bound[c + 1] * M);
    }
    if (s0 < pl.forced_end) e = std::min(e, pl.forced_end);
    int64_t ma = first_m_at_or_after(s0), mb = first_m_at_or_after(e);
    if (mb - ma > snap_cap - buffered) {
      mb = ma + (snap_cap - buffered);
      e = pl.pfirst + (mb - 1) * pl.pstride + 1;  // stop right after the last sample that fits
      e = (e + M - 1) / M * M;                     // (on a kernel step: the next sample is pstride >= M away)
    }
    ForceSpec fs;
    if (s0 < pl.forced_end) {
      if (table_mode) {
        fs.frc = frc;
        fs.row0 = (s0 % pl.P) / M;
        fs.period = table_rows;
        // table rows hold period-0 phases; period q adds e^{i sigma w0 q P h}
        fs.phi = std::polar(1.0, sigma * pl.w0 * op->h * (double)pl.P * (double)(s0 / pl.P));
      } else {
        syn.M = (e - s0) / M;
        syn.s0 = s0;
        syn.out = frc;
        TimedLaunch tl(op, RES_TIMING_SYNTHESIS, st);
        if (launch_phase_gemm(syn, op->fp64(), st)) return fail(RES_EINVAL, "synthesis GEMM launch");
        fs.frc = frc;
        fs.row0 = 0;
        fs.period = 0;
      }
    }
    SnapSpec ss;
    if (mb > ma) {
      ss.snap = snap;
      ss.ld = snap_ld;
      ss.first = (pl.pfirst + ma * pl.pstride - s0) / M;
      ss.stride = pl.pstride / M;
      ss.count = mb - ma;
      ss.row0 = buffered;
      if (buffered == 0) buf_m0 = ma;
      buffered += mb - ma;
    }
    if (is_grid(op)) RES_TRY(march_grid(op, k, e - s0, fs, ss, st));
    else RES_TRY(march_1d(op, k, (e - s0) / M, fs, ss, dsegs, nseg, st, M));
    if (buffered == snap_cap || (buffered > 0 && (e >= pl.S || mb >= pl.pcount))) {
      RES_TRY(flush_projection(op, pl, k, sigma, btab, snap, snap_ld, buf_m0, buffered, acc, st));
      buffered = 0;
    }
    s0 = e;
  }
  if (buffered > 0) RES_TRY(flush_projection(op, pl, k, sigma, btab, snap, snap_ld, buf_m0, buffered, acc, st));
  return RES_OK;
}

// Rows of the diagonal scalings (resolvent_op_set_weights): input and output scales of a run by role and
// direction, and the mode transforms.
enum { kWscB = 0, kWscC, kWscCWy, kWscBInvWf, kWscBInvSqrtWf, kWscCSqrtWy, kWscInvSqrtWf, kWscInvSqrtWy, kWscSqrtWf,
       kWscRows };

int run_any(resolvent_op* op, const Plan& pl, int k, const void* in, int in_fp64, double* acc, int sigma,
            hipStream_t st) {
  if (!op->weighted) return run_1d(op, pl, k, in, in_fp64, acc, sigma, st);  // the march dispatches on the kind
  // y = C R B f and R_y^dagger y = W_f^{-1} B R^H C W_y y (apply role); R~ = W_y^{1/2} C R B W_f^{-1/2} and R~^H
  // (gains and modes)
  int rin, rout;
  if (op->scale_role == 0) {
    rin = sigma > 0 ? kWscB : kWscCWy;
    rout = sigma > 0 ? kWscC : kWscBInvWf;
  } else {
    rin = sigma > 0 ? kWscBInvSqrtWf : kWscCSqrtWy;
    rout = sigma > 0 ? kWscCSqrtWy : kWscBInvSqrtWf;
  }
  const double* w = (const double*)op->d_wsc;
  const int64_t blocks = (int64_t)pl.nw * k;
  void* tmp;
  RES_TRY(ws_get(op, "wsc_in", (size_t)blocks * op->N * sizeof(cd), &tmp));
  launch_node_scale(in, in_fp64, tmp, 1, w + (size_t)rin * op->N, blocks, op->N, st);
  RES_TRY(run_1d(op, pl, k, tmp, 1, acc, sigma, st));
  launch_node_scale(acc, 1, acc, 1, w + (size_t)rout * op->N, blocks, op->N, st);
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

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

int apply_common(resolvent_op* op, const resolvent_grid* g, const resolvent_run* r, int k, const void* in, void* out,
                 int sigma, hipStream_t st) {
  if (!op || !in || !out) return fail(RES_EINVAL, "NULL argument");
  CaptureScope cap(op, st);
  if (k < 1) return fail(RES_EINVAL, "k must be >= 1");
  Plan pl;
  RES_TRY(make_plan(op, g, r, &pl));
  const int64_t count = (int64_t)pl.nw * k * op->N;
  double* acc;
  if (op->fp64()) {
    acc = (double*)out;
  } else {
    void* p;
    RES_TRY(ws_get(op, "acc_io", (size_t)count * sizeof(cd), &p));
    acc = (double*)p;
  }
  RES_TRY(run_any(op, pl, k, in, op->fp64(), acc, sigma, st));
  if (!op->fp64()) launch_convert(acc, 1, out, 0, count, 1.0, st);
  launch_finite(acc, 1, count, op->d_flag, st);
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

// CholeskyQR2 of X [nw][k][N] (FP64, in place): X <- Q; rtot receives R.  norm_hist (may be null) gets the
// column-norm estimator from the first Gram.
int cholqr2(resolvent_op* op, int nw, int k, double* X, void* rtot, double* norm_hist, hipStream_t st) {
  const int nsplit = nsplit_for(max_instance_len(op));
  const int km = gram_km(k);
  const size_t np = (size_t)km * (km + 1) / 2;
  void *part, *r1, *r1i, *r2i;
  const size_t mats = (size_t)nw * op->ninst * 64 * sizeof(cd);
  RES_TRY(ws_get(op, "gram_part", (size_t)nw * op->ninst * nsplit * np * sizeof(cd), &part));
  RES_TRY(ws_get(op, "qr_r1", mats, &r1));
  RES_TRY(ws_get(op, "qr_r1i", mats, &r1i));
  RES_TRY(ws_get(op, "qr_r2i", mats, &r2i));
  TimedLaunch tl(op, RES_TIMING_QR, st);
  launch_gram(X, 1, op->N, k, op->d_off, op->ninst, nw, nsplit, part, op->d_flag, st);
  launch_chol(part, nsplit, k, nw, op->ninst, r1, r1i, nullptr, nullptr, norm_hist, op->d_flag, st);
  launch_rmul(X, 1, X, 1, op->N, k, op->d_off, op->ninst, nw, nsplit, r1i, st);
  launch_gram(X, 1, op->N, k, op->d_off, op->ninst, nw, nsplit, part, op->d_flag, st);
  launch_chol(part, nsplit, k, nw, op->ninst, nullptr, r2i, r1, rtot, nullptr, op->d_flag, st);
  launch_rmul(X, 1, X, 1, op->N, k, op->d_off, op->ninst, nw, nsplit, r2i, st);
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

uint64_t splitmix64(uint64_t& x) {
  uint64_t z = (x += 0x9E3779B97F4A7C15ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Decay probe: march a random initial condition without forcing until its norm falls below tol (stable),
// diverges (RES_ESTEP) or tmax passes (RES_EUNSTABLE).
int decay_probe(resolvent_op* op, const resolvent_op_desc* d, hipStream_t st) {
  const int64_t N = op->N;
  const size_t ws = op->wsize();
  void *sb0, *sb1;
  RES_TRY(ws_get(op, "state0", (size_t)N * ws, &sb0));
  RES_TRY(ws_get(op, "state1", (size_t)N * ws, &sb1));
  op->cur_state = 0;
  uint64_t sx = d->probe_seed;
  std::vector<cd> u0(N);
  for (int64_t i = 0; i < N; ++i) {
    const double a = (double)(splitmix64(sx) >> 11) * 0x1.0p-53 * 2.0 - 1.0;
    const double b = (double)(splitmix64(sx) >> 11) * 0x1.0p-53 * 2.0 - 1.0;
    u0[i] = cd(a, b);
  }
  if (op->fp64()) {
    HIP_TRY(hipMemcpy(sb0, u0.data(), N * sizeof(cd), hipMemcpyHostToDevice));
  } else {
    std::vector<std::complex<float>> f(N);
    for (int64_t i = 0; i < N; ++i) f[i] = std::complex<float>((float)u0[i].real(), (float)u0[i].imag());
    HIP_TRY(hipMemcpy(sb0, f.data(), N * sizeof(std::complex<float>), hipMemcpyHostToDevice));
  }
  double n0 = 0;
  for (auto& z : u0) n0 += std::norm(z);
  n0 = std::sqrt(n0);
  void *dsegs, *part;
  int64_t nseg;
  RES_TRY(upload_regions(op, 1, &dsegs, &nseg, st));
  const int nsplit = nsplit_for(max_instance_len(op));
  RES_TRY(ws_get(op, "probe_part", (size_t)op->ninst * nsplit * sizeof(cd), &part));
  const double tol = d->probe_tol > 0 ? d->probe_tol : 1e-9;
  const double tmax = d->probe_tmax > 0 ? d->probe_tmax : 2000.0;
  const int64_t chunk = std::max<int64_t>(1, (int64_t)std::ceil(tmax / 50.0 / op->h));
  std::vector<cd> hpart((size_t)op->ninst * nsplit);
  op->march_band = op->d_band[0];
  int64_t steps = 0;
  op->march_grid = &op->gw[0];
  while (true) {
    if (is_grid(op)) RES_TRY(march_grid(op, 1, chunk, ForceSpec(), SnapSpec(), st));
    else RES_TRY(march_1d(op, 1, chunk, ForceSpec(), SnapSpec(), dsegs, nseg, st));
    steps += chunk;
    void* cur;
    RES_TRY(ws_get(op, op->cur_state ? "state1" : "state0", (size_t)N * ws, &cur));
    launch_gram(cur, op->fp64(), N, 1, op->d_off, op->ninst, 1, nsplit, part, op->d_flag, st);
    HIP_TRY(hipMemcpyAsync(hpart.data(), part, hpart.size() * sizeof(cd), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    double nn = 0;
    for (auto& z : hpart) nn += z.real();
    const double nrm = std::sqrt(std::max(nn, 0.0));
    const double t = steps * op->h;
    if (!std::isfinite(nrm) || nrm > 1e30 * n0) {
      int zero = 0;
      HIP_TRY(hipMemcpy(op->d_flag, &zero, sizeof(int), hipMemcpyHostToDevice));
      return fail(RES_ESTEP, "decay probe diverged after " + std::to_string(steps) +
                                 " steps: the RK4 step h is outside the stability region of L");
    }
    if (nrm <= tol * n0) {
      op->decay_time = t;
      return RES_OK;
    }
    if (t >= tmax)
      return fail(RES_EUNSTABLE, "decay probe: norm ratio " + std::to_string(nrm / n0) + " after t = " +
                                     std::to_string(t) + " (operator not stable, or decay slower than probe_tmax)");
  }
}

// ---------------------------------------------------------------------------------------------------------
// Stepper autotuner (1-D operators): candidate plans are owned-chunk sizes x steps-between-exchanges x kernel
// configurations whose capacity holds the region (chunk + two halos of 4*block) without leaving more than half
// of the threads idle, plus the single-region plans when a column fits one workgroup.  Each candidate marches
// `steps` forced steps of k columns three times on the caller's stream; the faster of the last two (timed with
// HIP events) is its time, and the fastest plan is kept.
struct PlanCand {
  int cfg;
  int64_t chunk, block;
  int persist;
};

std::vector<PlanCand> plan_candidates(const resolvent_op* op) {
  std::vector<PlanCand> c;
  const int64_t n = op->N;
  for (int cfg = 0; cfg < kStep1DConfigs; ++cfg) {
    const int64_t cap = step1d_capacity(cfg);
    if (cap >= n && cap < 2 * n) c.push_back({cfg, 0, 0, 1});
  }
  static const int64_t chunks[] = {64, 96, 128, 160, 192, 256, 384, 512, 768, 1024, 1536};
  static const int64_t blocks[] = {4, 8, 12, 16, 24, 32, 48, 64};
  for (int64_t chunk : chunks) {
    if (chunk >= n) continue;
    for (int64_t block : blocks) {
      if ((int64_t)kBandRadius * block > chunk) continue;
      const int64_t region = chunk + 2 * (int64_t)kBandRadius * block;
      for (int cfg = 0; cfg < kStep1DConfigs; ++cfg) {
        const int64_t cap = step1d_capacity(cfg);
        if (cap < region || cap >= 2 * region) continue;
        c.push_back({cfg, chunk, block, block % step1d_prefetch(cfg) == 0 ? 1 : 0});
      }
    }
  }
  return c;
}

int tune_1d(resolvent_op* op, int k, int64_t steps, PlanCand* best, double* best_us, hipStream_t st) {
  const int64_t ncols = (int64_t)k * op->N;
  const size_t ws = op->wsize();
  const int M = op->step_power;  // plans are timed in the operator's multi-step form
  const int64_t ksteps = steps / M;
  steps = ksteps * M;
  void *frc, *s0, *s1;
  RES_TRY(ws_get(op, "forcing", (size_t)(ksteps + 16) * ncols * ws, &frc));
  RES_TRY(zero_device(frc, (size_t)(ksteps + 16) * ncols * ws, st));
  RES_TRY(ws_get(op, "state0", (size_t)ncols * ws, &s0));
  RES_TRY(ws_get(op, "state1", (size_t)ncols * ws, &s1));
  RES_TRY(zero_device(s0, (size_t)ncols * ws, st));
  RES_TRY(zero_device(s1, (size_t)ncols * ws, st));
  op->march_band = M > 1 ? op->d_bandm[0] : op->d_band[0];
  ForceSpec fs;
  fs.frc = frc;
  fs.row0 = 0;
  fs.period = 0;
  const bool timing = op->timing;
  op->timing = false;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  double best_ms = -1;
  int rc = RES_OK;
  // a candidate whose launch the device refuses (a persistent grid that cannot be co-resident beside other work)
  // is skipped; the plan in effect before the search comes back if none runs
  const PlanCand before{op->step_cfg, op->step_chunk, op->step_block, op->step_persist ? 1 : 0};
  for (const PlanCand& c : plan_candidates(op)) {
    if (c.block % M != 0) continue;
    if (apply_plan(op, c.cfg, c.chunk, c.block, c.persist) != RES_OK) {
      g_last_error.clear();
      continue;
    }
    void* dsegs;
    int64_t nseg;
    if ((rc = upload_regions(op, k, &dsegs, &nseg, st)) != RES_OK) break;
    if ((rc = march_1d(op, k, ksteps, fs, SnapSpec(), dsegs, nseg, st, M)) != RES_OK) {  // warm-up
      if (rc != RES_EHIP || g_last_error.compare(0, 21, "stepper launch failed") != 0) break;
      g_last_error.clear();
      rc = RES_OK;
      continue;
    }
    double ms = -1;
    for (int rep = 0; rep < 2 && rc == RES_OK; ++rep) {  // the faster of two timed marches
      if (hipEventRecord(e0, st) != hipSuccess) { rc = fail(RES_EHIP, "event record"); break; }
      if ((rc = march_1d(op, k, ksteps, fs, SnapSpec(), dsegs, nseg, st, M)) != RES_OK) break;
      if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        rc = fail(RES_EHIP, "event timing");
        break;
      }
      float t = 0;
      (void)hipEventElapsedTime(&t, e0, e1);
      if (ms < 0 || t < ms) ms = t;
    }
    if (rc != RES_OK) break;
    if (best_ms < 0 || ms < best_ms) {
      best_ms = ms;
      *best = {op->step_cfg, op->step_chunk, op->step_block, op->step_persist ? 1 : 0};
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  op->timing = timing;
  if (rc != RES_OK || best_ms < 0) {
    const std::string err = g_last_error;
    (void)apply_plan(op, before.cfg, before.chunk, before.block, before.persist);
    g_last_error = err;
    if (rc != RES_OK) return rc;
    return fail(RES_ENOTSUP, "no stepper plan fits this operator");
  }
  *best_us = best_ms * 1e3 / (double)steps;
  return apply_plan(op, best->cfg, best->chunk, best->block, best->persist);
}

// ---------------------------------------------------------------------------------------------------------
// Reverse mode: gradient of a real objective of u_hat = resolvent_apply(f_hat) with respect to f_hat and to a real
// perturbation of L's diagonal, by the exact discrete adjoint of the classical four-stage march (see adjoint.hip).
//
// The forward trajectory is marched once in stage form (FP64, raw forcing sampled at the stage times t_s,
// t_s + h/2, t_s + h, synthesised on the half-step grid) keeping the state every C steps; the segments are then
// visited in reverse: the states of the segment are recomputed from its checkpoint, and each step runs three
// stage recomputations and four reverse stages.  The adjoint state lambda_s = dJ/du_s receives the projection's
// seed scale * sum_j e^{+i w_j t_s} g_j at the sampled steps.  The forcing gradient uses the single-step form
// u_{s+1} = P(Z) u_s + sum_j e^{i w_j t_s} h Q_j(Z) F_j:  F_grad_j = (h Q_j(Z))^H sum_{forced s} e^{-i w_j t_s}
// lambda_{s+1}, i.e. a Fourier projection of the lambda rows followed by the forcing pre-filter of Z^H at the
// negated frequencies ((h Q_w(Z))^H = h Q_{-w}(Z^H)).
AdjOpDev adj_op(const resolvent_op* op, int s) {
  AdjOpDev a{};
  if (is_grid(op)) {
    a.kind = 1;
    a.ncomp = op->ncomp;
    a.nsite = op->nx * op->ny * op->nz;
    a.g = op->g64[s];
  } else {
    a.kind = 0;
    a.ncomp = 1;
    a.nsite = op->N;
    a.tri = op->d_tri[s];
  }
  return a;
}

// One chunk of kc columns.  F: raw forcing rows [nw][kc][N] in the row precision (null without mu_grad); G: the
// scaled seed in the row precision; f_out: forcing gradient [nw][kc][N] in the working precision, or null; mu_grad
// (FP64 [nsite]) receives += this chunk's contribution.  Every row buffer holds the row precision: FP64 (r64), or
// FP32 with FP64 arithmetic in the kernels and FP64 accumulation of both gradients.
int backward_chunk(resolvent_op* op, const Plan& pl, int k, int r64, const void* F, const void* G, void* f_out,
                   double* mu_grad, int64_t C, hipStream_t st) {
  const int64_t N = op->N, ncols = (int64_t)k * N, S = pl.S;
  const int nw = pl.nw;
  const size_t rowb = (size_t)ncols * (r64 ? sizeof(cd) : sizeof(std::complex<float>));
  const double h = op->h;
  const int64_t ncp = (S + C - 1) / C;
  const AdjOpDev fwd = adj_op(op, 0), rev = adj_op(op, 1);
  const int64_t nsite = fwd.nsite;
  const bool need_states = mu_grad != nullptr;

  void *frow, *cps, *seg, *u, *acc, *y2, *y3, *y4, *ka, *kb, *ub, *lrows, *carry, *inj, *facc = nullptr;
  void *btab_half = nullptr, *btab;
  frow = cps = seg = nullptr;
  if (need_states) {
    RES_TRY(ws_get(op, "bw_frow", (size_t)(2 * C + 1) * rowb, &frow));
    RES_TRY(ws_get(op, "bw_ckpt", (size_t)ncp * rowb, &cps));
    RES_TRY(ws_get(op, "bw_seg", (size_t)C * rowb, &seg));
  }
  RES_TRY(ws_get(op, "bw_u", rowb, &u));
  RES_TRY(ws_get(op, "bw_acc", rowb, &acc));
  RES_TRY(ws_get(op, "bw_y2", rowb, &y2));
  RES_TRY(ws_get(op, "bw_y3", rowb, &y3));
  RES_TRY(ws_get(op, "bw_y4", rowb, &y4));
  RES_TRY(ws_get(op, "bw_ka", rowb, &ka));
  RES_TRY(ws_get(op, "bw_kb", rowb, &kb));
  RES_TRY(ws_get(op, "bw_ub", rowb, &ub));
  RES_TRY(ws_get(op, "bw_carry", rowb, &carry));
  RES_TRY(ws_get(op, "bw_inj", (size_t)C * rowb, &inj));
  if (f_out) {
    RES_TRY(ws_get(op, "bw_facc", (size_t)nw * ncols * sizeof(cd), &facc));
    RES_TRY(zero_device(facc, (size_t)nw * ncols * sizeof(cd), st));
  }
  if (r64) {
    if (need_states) RES_TRY(phase_table64(op, 2 * pl.P, &btab_half));
    RES_TRY(phase_table64(op, pl.P, &btab));
  } else {
    if (need_states) RES_TRY(phase_table(op, 2 * pl.P, &btab_half));
    RES_TRY(phase_table(op, pl.P, &btab));
  }
  auto row = [&](void* base, int64_t r) { return (void*)((char*)base + (size_t)r * rowb); };
  // raw forcing of steps [sa, sb) for the segment recomputation: half-step samples 2 sa .. 2 sb.  The GEMM works
  // on 64-row tiles, so the 2 C + 1 samples of a whole segment would take a third tile for a single row: with
  // `shared`, the last sample is the first one (row 0) of the segment synthesised just before (the next one in
  // time: segments are visited in reverse) and is copied instead.
  auto synth_segment = [&](int64_t sa, int64_t sb, bool shared) -> int {
    if (sa >= pl.forced_end) return RES_OK;
    const int64_t len = sb - sa;
    int64_t n = 2 * len + 1;
    if (shared) {
      HIP_TRY(hipMemcpyAsync(row(frow, 2 * len), row(frow, 0), rowb, hipMemcpyDeviceToDevice, st));
      --n;
    }
    return synth_rows(r64, nw, 2 * pl.P, pl.w0 * h * 0.5, +1, btab_half, F, ncols, 2 * sa, 1, n, frow, st);
  };
  auto frc = [&](int64_t s, int64_t r, int half) -> const void* {
    return s < pl.forced_end ? row(frow, 2 * r + half) : nullptr;
  };
  auto first_m_at_or_after = [&](int64_t t) -> int64_t {
    if (t <= pl.pfirst) return 0;
    return std::min(pl.pcount, (t - pl.pfirst + pl.pstride - 1) / pl.pstride);
  };

  // 2-D one-component grids take the four forward stages of a step in one LDS-tiled launch (launch_fwd_step2d);
  // other operators one launch per stage.  The fused step cannot update the state in place, so the checkpoint
  // march ping-pongs between u and a second row.
  const bool fused = fwd.kind == 1 && fwd.ncomp == 1 && fwd.g.nz == 1;
  // Mixed-precision three-component grids with FP32 rows march the checkpoint states, and the adjoint recursion
  // when no mu gradient is asked for, with the forward march's fused one-launch step (launch_grid_step3d, FP32
  // arithmetic): u' = P(Z) u + G_s and lambda_s = P(Z^H) lambda_{s+1} + seed_s, since P(Z)^H = P(Z^H).  Both
  // need only the states; the stage values of the recomputed segments and the reverse stages of the mu gradient
  // keep the stage kernels.
  const bool fused3 = fwd.kind == 1 && fwd.ncomp == 3 && !r64 && !op->fp64();
  void* u2 = nullptr;
  // per-column mu rows of the reverse steps (one row per column, or per grid row of the stage launches), summed at
  // the end: the columns of a node run in different threads, and the sum stays deterministic
  double* mu_cols = nullptr;
  const int mu_rows = fused ? k : rev_stage_rows(k);
  if (fused || fused3) RES_TRY(ws_get(op, "bw_u2", rowb, &u2));
  if (mu_grad) {
    void* p;
    RES_TRY(ws_get(op, "bw_mu_cols", (size_t)mu_rows * nsite * sizeof(double), &p));
    mu_cols = (double*)p;
    RES_TRY(zero_device(mu_cols, (size_t)mu_rows * nsite * sizeof(double), st));
  }

  // 1. forward march with checkpoints.  It only needs the states, so it steps u' = P(Z) u + sum_j e^{i w_j t_s} G_j
  // with the pre-filtered forcing G_j = h Q_j(Z) F_j (FP64 Horner passes, stored in the row precision): one
  // synthesised row per step instead of two half-step rows, read once per step instead of at every stage.
  void* Gpre = nullptr;
  if (need_states && pl.forced_end > 0) {
    RES_TRY(ws_get(op, "bw_Gpre", (size_t)nw * rowb, &Gpre));
    RES_TRY(prefilter(op, pl, k, F, r64, Gpre, +1, 1, st, r64));
  }
  RES_TRY(zero_device(u, rowb, st));
  void* ucur = u;
  for (int64_t c = 0; c < (need_states ? ncp : 0); ++c) {
    const int64_t sa = c * C, sb = std::min(S, sa + C);
    HIP_TRY(hipMemcpyAsync(row(cps, c), ucur, rowb, hipMemcpyDeviceToDevice, st));
    if (c == ncp - 1) break;  // the state after the last step is not needed
    const int64_t nf = std::min(sb, pl.forced_end) - sa;
    if (nf > 0) RES_TRY(synth_rows(r64, nw, pl.P, pl.w0 * h, +1, btab, Gpre, ncols, sa, 1, nf, frow, st));
    for (int64_t s = sa; s < sb; ++s) {
      const void* g = s < pl.forced_end ? row(frow, s - sa) : nullptr;
      if (fused) {
        void* unext = ucur == u ? u2 : u;
        if (launch_fwd_step2d(fwd, k, ucur, unext, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, h, st, g,
                              r64))
          return fail(RES_EINVAL, "fused forward step launch");
        ucur = unext;
        continue;
      }
      if (fused3) {
        void* unext = ucur == u ? u2 : u;
        if (launch_grid_step3d(op->gw[0], k, ucur, unext, g, 1.0, 0.0, nullptr, st))
          return fail(RES_EINVAL, "3-D step launch");
        ucur = unext;
        continue;
      }
      launch_fwd_stage(fwd, k, 1, u, nullptr, u, y2, acc, nullptr, h, st, nullptr, r64);
      launch_fwd_stage(fwd, k, 2, u, nullptr, y2, y3, acc, nullptr, h, st, nullptr, r64);
      launch_fwd_stage(fwd, k, 3, u, nullptr, y3, y2, acc, nullptr, h, st, nullptr, r64);
      launch_fwd_stage(fwd, k, 4, u, u, y2, nullptr, acc, nullptr, h, st, g, r64);
    }
  }
  HIP_TRY(hipGetLastError());

  // 2. reverse sweep over the segments.  The segment's forward recomputation keeps the three stage inputs of every
  // step but its last when they fit in half of the free device memory, so the reverse steps do not march them
  // again (the values are the same: the stages of a step depend only on its state and forcing).
  void* stg = nullptr;
  {
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    const auto held = op->ws.find("bw_stages");
    const double avail = (double)free_b + (held != op->ws.end() ? (double)held->second.bytes : 0.0);
    const size_t need = (size_t)3 * C * rowb;
    if (need_states && (double)need <= 0.5 * avail && ws_get(op, "bw_stages", need, &stg) != RES_OK) {
      g_last_error.clear();
      stg = nullptr;
    }
  }
  // The lambda rows of G consecutive segments are kept together, so that the forcing gradient's projection runs on
  // up to 256 rows at a time (64-row projections spend most of their time reading and writing the accumulator).
  // G shrinks to what a quarter of the device memory left after the stage rows holds.
  int64_t G_seg = std::max<int64_t>(1, std::min<int64_t>(ncp, 256 / C));
  if (G_seg > 1) {
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    const auto held = op->ws.find("bw_lrows");
    const double avail = (double)free_b + (held != op->ws.end() ? (double)held->second.bytes : 0.0);
    G_seg = std::max<int64_t>(1, std::min<int64_t>(G_seg, (int64_t)(0.25 * avail / ((double)C * rowb))));
  }
  RES_TRY(ws_get(op, "bw_lrows", (size_t)(G_seg * C) * rowb, &lrows));
  auto srow = [&](int64_t r, int i) { return row(stg, 3 * r + i); };
  RES_TRY(zero_device(carry, rowb, st));  // lambda_S = 0: u_S is not sampled
  for (int64_t c = ncp - 1; c >= 0; --c) {
    const int64_t sa = c * C, sb = std::min(S, sa + C), len = sb - sa;
    if (need_states) {
      RES_TRY(synth_segment(sa, sb, c + 1 < ncp && sb < pl.forced_end));
      // states u_sa .. u_{sb-1}
      HIP_TRY(hipMemcpyAsync(row(seg, 0), row(cps, c), rowb, hipMemcpyDeviceToDevice, st));
    }
    for (int64_t s = sa; need_states && s + 1 < sb; ++s) {
      const int64_t r = s - sa;
      void* us = row(seg, r);
      void* a2 = stg ? srow(r, 0) : y2;
      void* a3 = stg ? srow(r, 1) : y3;
      void* a4 = stg ? srow(r, 2) : y2;
      if (fused) {
        if (launch_fwd_step2d(fwd, k, us, row(seg, r + 1), stg ? a2 : nullptr, stg ? a3 : nullptr,
                              stg ? a4 : nullptr, frc(s, r, 0), frc(s, r, 1), frc(s, r, 2), h, st, nullptr, r64))
          return fail(RES_EINVAL, "fused forward step launch");
        continue;
      }
      launch_fwd_stage(fwd, k, 1, us, nullptr, us, a2, acc, frc(s, r, 0), h, st, nullptr, r64);
      launch_fwd_stage(fwd, k, 2, us, nullptr, a2, a3, acc, frc(s, r, 1), h, st, nullptr, r64);
      launch_fwd_stage(fwd, k, 3, us, nullptr, a3, a4, acc, frc(s, r, 1), h, st, nullptr, r64);
      launch_fwd_stage(fwd, k, 4, us, row(seg, r + 1), a4, nullptr, acc, frc(s, r, 2), h, st, nullptr, r64);
    }
    // projection seeds of the sampled steps in [sa, sb)
    const int64_t ma = first_m_at_or_after(sa), mb = first_m_at_or_after(sb);
    if (mb > ma)
      RES_TRY(synth_rows(r64, nw, pl.P, pl.w0 * h, +1, btab, G, ncols, pl.pfirst + ma * pl.pstride, pl.pstride,
                         mb - ma, inj, st));
    // lambda rows: lseg[r] = lambda_{sa + r + 1}, segment c at row (c - cg) C of its group's rows
    const int64_t cg = c / G_seg * G_seg;
    void* lseg = row(lrows, (c - cg) * C);
    HIP_TRY(hipMemcpyAsync(row(lseg, len - 1), carry, rowb, hipMemcpyDeviceToDevice, st));
    for (int64_t s = sb - 1; s >= sa; --s) {
      const int64_t r = s - sa;
      void* us = need_states ? row(seg, r) : nullptr;
      const void *s2 = y2, *s3 = y3, *s4 = y4;  // stage inputs of step s
      if (!need_states) {
        s2 = s3 = s4 = nullptr;
      } else if (stg && s + 1 < sb) {
        s2 = srow(r, 0);
        s3 = srow(r, 1);
        s4 = srow(r, 2);
      } else if (fused) {
        if (launch_fwd_step2d(fwd, k, us, nullptr, y2, y3, y4, frc(s, r, 0), frc(s, r, 1), nullptr, h, st, nullptr,
                              r64))
          return fail(RES_EINVAL, "fused forward step launch");
      } else {
        launch_fwd_stage(fwd, k, 1, us, nullptr, us, y2, nullptr, frc(s, r, 0), h, st, nullptr, r64);
        launch_fwd_stage(fwd, k, 2, us, nullptr, y2, y3, nullptr, frc(s, r, 1), h, st, nullptr, r64);
        launch_fwd_stage(fwd, k, 3, us, nullptr, y3, y4, nullptr, frc(s, r, 1), h, st, nullptr, r64);
      }
      const void* lp = row(lseg, r);
      const void* seed = nullptr;
      if (s >= pl.pfirst && (s - pl.pfirst) % pl.pstride == 0) {
        const int64_t m = (s - pl.pfirst) / pl.pstride;
        if (m < pl.pcount) seed = row(inj, m - ma);
      }
      if (fused) {
        if (launch_rev_step2d(rev, k, lp, r > 0 ? row(lseg, r - 1) : carry, s2, s3, s4, us, mu_cols, seed, h, st,
                              r64))
          return fail(RES_EINVAL, "fused reverse step launch");
        continue;
      }
      if (fused3 && !need_states) {
        if (launch_grid_step3d(op->gw[1], k, lp, r > 0 ? row(lseg, r - 1) : carry, seed, 1.0, 0.0, nullptr, st))
          return fail(RES_EINVAL, "3-D step launch");
        continue;
      }
      // Kb_3 in ka, Kb_2 in kb, Kb_1 in ub; stage 1 combines the three into lambda
      launch_rev_stage(rev, k, 4, lp, nullptr, nullptr, s4, ka, nullptr, nullptr, mu_cols, nullptr, h, st, r64);
      launch_rev_stage(rev, k, 3, lp, nullptr, ka, s3, kb, nullptr, nullptr, mu_cols, nullptr, h, st, r64);
      launch_rev_stage(rev, k, 2, lp, nullptr, kb, s2, ub, nullptr, nullptr, mu_cols, nullptr, h, st, r64);
      launch_rev_stage(rev, k, 1, lp, r > 0 ? row(lseg, r - 1) : carry, ub, us, nullptr, ka, kb, mu_cols, seed, h,
                       st, r64);
    }
    HIP_TRY(hipGetLastError());
    // forcing gradient: Fourier sums of lambda_{s+1} over the forced steps of the group, once its first segment
    // is done
    if (c == cg) {
      const int64_t ga = cg * C, gb = std::min(S, (cg + G_seg) * C);
      const int64_t nf = std::min(gb, pl.forced_end) - ga;
      if (f_out && nf > 0)
        RES_TRY(project_rows(op, r64, nw, pl.P, pl.w0 * h, +1, btab, lrows, ncols, ncols, ga, 1, nf, 1.0,
                             (double*)facc, st));
    }
  }
  if (mu_cols) launch_sum_columns(mu_cols, mu_rows, nsite, mu_grad, st);
  // 3. F_grad_j = h Q_{-w_j}(Z^H) facc_j (FP64 Horner passes, written in the working precision)
  if (f_out) {
    RES_TRY(prefilter(op, pl, k, facc, 1, f_out, -1, 1, st, op->fp64()));
    launch_finite(facc, 1, (int64_t)nw * ncols, op->d_flag, st);
  }
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

// Frees the handle's workspace (the forward drivers' state, forcing, snapshot and accumulator blocks and the reverse
// mode's own rows), so that the reverse mode can size its rows to the device memory; every driver sizes its
// workspace again on its next call.  Kept: the device copy of the stepper regions and the weighted reverse mode's
// scaled inputs (in use).
int release_workspace(resolvent_op* op) {
  if (op->capturing || op->arena) return RES_OK;
  HIP_TRY(hipDeviceSynchronize());
  for (auto& kv : op->ws) {
    const std::string& name = kv.first;
    if (name.compare(0, 6, "bw_wsc") == 0 || name == "segs") continue;
    if (kv.second.p) HIP_TRY(hipFree(kv.second.p));
    kv.second.p = nullptr;
    kv.second.bytes = 0;
  }
  return RES_OK;
}

// Copies columns [c0, c0 + kc) of a [nw][k][N] block (precision in_fp64) into a [nw][kc][N] block (precision
// out_fp64), times scale.
void gather_columns(const void* x, int in_fp64, int64_t k, int64_t c0, int64_t kc, int64_t N, int nw, void* y,
                    int out_fp64, double scale, hipStream_t st) {
  const size_t ies = in_fp64 ? sizeof(cd) : sizeof(std::complex<float>);
  const size_t oes = out_fp64 ? sizeof(cd) : sizeof(std::complex<float>);
  if (kc == k) {
    launch_convert(x, in_fp64, y, out_fp64, (int64_t)nw * k * N, scale, st);
    return;
  }
  for (int j = 0; j < nw; ++j)
    launch_convert((const char*)x + (size_t)((int64_t)j * k + c0) * N * ies, in_fp64,
                   (char*)y + (size_t)((int64_t)j * kc) * N * oes, out_fp64, kc * N, scale, st);
}

int backward(resolvent_op* op, const Plan& pl, int k, const void* f_hat, const void* g_hat, void* f_grad,
             double* mu_grad, int64_t C, hipStream_t st) {
  const int64_t N = op->N, S = pl.S;
  const int nw = pl.nw;
  const int r64 = op->fp64() || op->rev_rows64;
  const size_t res = r64 ? sizeof(cd) : sizeof(std::complex<float>);
  if (C <= 0) C = std::max<int64_t>(1, (int64_t)std::ceil(std::sqrt((double)S)));
  C = std::min<int64_t>(C, S);
  const int64_t ncp = (S + C - 1) / C;
  // The adjoint recursion for lambda is linear and does not involve the forward trajectory: only the mu gradient
  // needs the states and stage values, so without it the forcing, the forward march, its checkpoints and the
  // segment recomputation are skipped (the forcing gradient then costs one adjoint march).
  const bool need_states = mu_grad != nullptr;
  const bool f_direct = (op->fp64() ? 1 : 0) == r64;  // the caller's forcing is already in the row precision

  // Columns evolve independently under the march and the mu gradient is a sum over columns, so the columns are
  // processed in chunks of kc when the rows of all k do not fit: the bytes a chunk holds (the stage rows and the
  // extra lambda rows are sized later from what is left) against the free device memory, after the handle's
  // workspace is released when all k columns do not fit beside it.
  const double horner_budget = env_double("RESOLVENT_HORNER_BUDGET_GB", 8.0) * 1073741824.0;
  auto need = [&](int64_t kc) {
    const double row = (double)kc * N * res, blk = nw * row;
    double b = blk + (double)(2 * C + 12) * row;  // seed, lambda rows, injections, work rows
    if (f_grad) b += (double)nw * kc * N * sizeof(cd) + std::min(horner_budget, 2.0 * nw * kc * N * sizeof(cd));
    if (need_states) {
      b += blk + (kc < k || !f_direct ? blk : 0.0) + (double)(ncp + 3 * C + 1) * row;
      b += std::min(horner_budget, 2.0 * nw * kc * N * sizeof(cd)) + (double)(k + 1) * adj_op(op, 0).nsite * 8.0;
    }
    return b;
  };
  auto available = [&](double* out) -> int {
    size_t free_b = 0, total_b = 0;
    HIP_TRY(hipMemGetInfo(&free_b, &total_b));
    *out = 0.92 * (double)free_b - 2.0 * 1073741824.0;
    return RES_OK;
  };
  int64_t kc = k;
  const long forced = env_long("RESOLVENT_BACKWARD_COLUMNS", 0);
  if (forced > 0) {
    kc = std::min<int64_t>(k, forced);
  } else {
    double avail = 0;
    RES_TRY(available(&avail));
    if (need(k) > avail) {
      RES_TRY(release_workspace(op));
      RES_TRY(available(&avail));
    }
    while (kc > 1 && need(kc) > avail) --kc;
  }

  if (mu_grad) RES_TRY(zero_device(mu_grad, (size_t)adj_op(op, 0).nsite * sizeof(double), st));
  for (int64_t c0 = 0; c0 < k; c0 += kc) {
    const int64_t kcc = std::min<int64_t>(kc, k - c0);
    const size_t blk = (size_t)nw * kcc * N * res;
    void* G;
    RES_TRY(ws_get(op, "bw_G", blk, &G));
    gather_columns(g_hat, op->fp64(), k, c0, kcc, N, nw, G, r64, pl.scale, st);
    const void* F = nullptr;
    if (need_states) {
      if (kcc == k && f_direct) {
        F = f_hat;
      } else {
        void* p;
        RES_TRY(ws_get(op, "bw_F", blk, &p));
        gather_columns(f_hat, op->fp64(), k, c0, kcc, N, nw, p, r64, 1.0, st);
        F = p;
      }
    }
    // the chunk's forcing gradient goes straight to f_grad when the chunk is every column, else into the seed
    // block (no longer read by then) and is scattered from there
    void* fo = f_grad ? (kcc == k ? f_grad : G) : nullptr;
    RES_TRY(backward_chunk(op, pl, (int)kcc, r64, F, G, fo, mu_grad, C, st));
    if (f_grad && kcc < k) {
      const size_t es = op->wsize();
      for (int j = 0; j < nw; ++j)
        HIP_TRY(hipMemcpyAsync((char*)f_grad + (size_t)((int64_t)j * k + c0) * N * es,
                               (const char*)G + (size_t)((int64_t)j * kcc) * N * es, (size_t)kcc * N * es,
                               hipMemcpyDeviceToDevice, st));
    }
  }
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

// Force and response modes of the Euclidean R~ back to the problem's metrics: V <- W_f^{-1/2} V, U <- W_y^{-1/2} U
// (outputs in working precision, in place).
int modes_to_problem(resolvent_op* op, int nw, int k, void* V, void* U, hipStream_t st) {
  const double* w = (const double*)op->d_wsc;
  const int fp = op->fp64();
  if (V) launch_node_scale(V, fp, V, fp, w + (size_t)kWscInvSqrtWf * op->N, (int64_t)nw * k, op->N, st);
  if (U) launch_node_scale(U, fp, U, fp, w + (size_t)kWscInvSqrtWy * op->N, (int64_t)nw * k, op->N, st);
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

// ---- transient-response method with time-domain hand-off (Sec. 2.2, App. B, App. C) ----------------------------

// March from rest forced by the sampled signal `in` ([n][k][N], working precision; sample i at step i * every),
// writing the state at the sample times to `out` (same layout).  adjoint = 0: du/dt = L u + f.  adjoint = 1:
// -dz/dt = L^H z + g backward in time from z(T) = 0, T = (n - 1) every h, which is the forward march of L^H in
// reversed time (the samples are read and written in reversed order).  The forcing rows come from the stage-forcing
// pre-filter, in tiles of whole sample intervals.  When the samples are a multiple of the operator's step power m
// apart (and the plan's exchange interval allows it), the march takes m RK4 steps per kernel step with the band
// P(Z)^m, its forcing rows combined from the per-step rows by m - 1 Horner passes of P(Z); else one step at a time.
// The same for a grid operator: the signal at the half steps of each tile first (FP64), then the three pre-filter
// passes with the grid stencil, then the grid march (one RK4 step per launch or launch pair).
int signal_run_grid(resolvent_op* op, int k, int64_t n, int every, int scheme, int adjoint, const void* in,
                    void* out, hipStream_t st) {
  const int64_t ncols = (int64_t)k * op->N;
  const size_t ws = op->wsize();
  const int s = adjoint ? 1 : 0;
  const int64_t S = (n - 1) * (int64_t)every;
  const double tile_budget = env_double("RESOLVENT_TILE_BUDGET_GB", 2.0) * 1073741824.0;
  const double per_step = (double)ncols * (4.0 * sizeof(cd) + (double)ws) + (double)(ncols + 1) * ws / every;
  int64_t tile = std::min<int64_t>((int64_t)(tile_budget / per_step), 4096) / every * every;
  if (tile < every) tile = every;
  if (tile > S) tile = S;
  if (tile > 65535) return fail(RES_EINVAL, "sample interval too long for the grid pre-filter");
  void *H, *x2, *x1, *frc, *snap, *st0;
  RES_TRY(ws_get(op, "sig_half", (size_t)(2 * tile + 1) * ncols * sizeof(cd), &H));
  RES_TRY(ws_get(op, "sig_x2", (size_t)tile * ncols * sizeof(cd), &x2));
  RES_TRY(ws_get(op, "sig_x1", (size_t)tile * ncols * sizeof(cd), &x1));
  RES_TRY(ws_get(op, "forcing", (size_t)tile * ncols * ws, &frc));
  RES_TRY(ws_get(op, "sig_snap", (size_t)(tile / every) * (ncols + 1) * ws, &snap));
  RES_TRY(ws_get(op, "state0", (size_t)ncols * ws, &st0));
  RES_TRY(ws_get(op, "state1", (size_t)ncols * ws, &st0));
  RES_TRY(ws_get(op, "state0", (size_t)ncols * ws, &st0));
  op->cur_state = 0;
  RES_TRY(zero_device(st0, (size_t)ncols * ws, st));
  op->march_grid = &op->gw[s];
  for (int64_t s0 = 0; s0 < S; s0 += tile) {
    const int64_t rows = std::min(tile, S - s0);
    {
      TimedLaunch tl(op, RES_TIMING_SYNTHESIS, st);
      launch_signal_half_rows(in, n, every, scheme, adjoint, op->fp64(), H, s0, 2 * rows + 1, ncols, st);
      for (int pass = 0; pass < 3; ++pass)
        if (launch_grid_signal_pass(op->g64[s], H, pass == 1 ? x2 : x1, pass == 0 ? x2 : x1, frc,
                                    pass == 2 ? op->fp64() : 1, k, rows, op->h, pass, st))
          return fail(RES_EINVAL, "grid pre-filter launch");
    }
    ForceSpec fs;
    fs.frc = frc;
    SnapSpec ss;
    ss.snap = snap;
    ss.ld = ncols + 1;
    ss.first = 0;
    ss.stride = every;
    ss.count = rows / every;
    RES_TRY(march_grid(op, k, rows, fs, ss, st));
    const int64_t i0 = s0 / every;
    launch_copy_rows(snap, ncols + 1, out, adjoint ? n - 1 - i0 : i0, adjoint ? -1 : 1, rows / every, ncols,
                     op->fp64(), st);
  }
  void* cur;
  RES_TRY(ws_get(op, op->cur_state ? "state1" : "state0", (size_t)ncols * ws, &cur));
  launch_copy_rows(cur, ncols, out, adjoint ? 0 : n - 1, 1, 1, ncols, op->fp64(), st);
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

int signal_run(resolvent_op* op, int k, int64_t n, int every, int scheme, int adjoint, const void* in, void* out,
               hipStream_t st) {
  if (is_grid(op)) return signal_run_grid(op, k, n, every, scheme, adjoint, in, out, st);
  const int64_t N = op->N, ncols = (int64_t)k * N;
  const size_t ws = op->wsize();
  const int s = adjoint ? 1 : 0;
  const int64_t S = (n - 1) * (int64_t)every;
  const int M = (op->step_power > 1 && every % op->step_power == 0 && op->step_block % op->step_power == 0)
                    ? op->step_power : 1;
  const double tile_budget = env_double("RESOLVENT_TILE_BUDGET_GB", 2.0) * 1073741824.0;
  const double per_step = (double)ncols * (2.0 * sizeof(cd) + (double)ws) + (double)(ncols + 1) * ws / every;
  int64_t tile = (int64_t)(tile_budget / per_step) / every * every;
  if (tile < every) tile = every;
  if (tile > S) tile = S;
  void *x2, *x1, *frc, *snap, *st0;
  RES_TRY(ws_get(op, "sig_x2", (size_t)tile * ncols * sizeof(cd), &x2));
  RES_TRY(ws_get(op, "sig_x1", (size_t)tile * ncols * sizeof(cd), &x1));
  RES_TRY(ws_get(op, "forcing", (size_t)(tile / M + 16) * ncols * ws, &frc));  // + the stepper's prefetch rows
  RES_TRY(ws_get(op, "sig_snap", (size_t)(tile / every) * (ncols + 1) * ws, &snap));
  RES_TRY(ws_get(op, "state0", (size_t)ncols * ws, &st0));
  RES_TRY(ws_get(op, "state1", (size_t)ncols * ws, &st0));
  RES_TRY(ws_get(op, "state0", (size_t)ncols * ws, &st0));
  op->cur_state = 0;
  RES_TRY(zero_device(st0, (size_t)ncols * ws, st));
  op->march_band = M > 1 ? op->d_bandm[s] : op->d_band[s];
  void* dsegs;
  int64_t nseg;
  RES_TRY(upload_regions(op, k, &dsegs, &nseg, st));
  const cx<double>* tri = (const cx<double>*)op->d_tri[s];
  const cx<double>* band64 = (const cx<double>*)op->d_band64[s];
  for (int64_t s0 = 0; s0 < S; s0 += tile) {
    const int64_t rows = std::min(tile, S - s0);
    {
      TimedLaunch tl(op, RES_TIMING_SYNTHESIS, st);
      // passes 0 and 1 write x2 and x1; pass 2 writes the per-step rows: the forcing table itself for M = 1, else
      // FP64 rows into x2 (free again), combined below into one row per kernel step
      for (int pass = 0; pass < 3; ++pass)
        launch_signal_prefilter(in, n, every, scheme, adjoint, tri, pass == 1 ? x2 : x1, pass == 0 ? x2 : x1,
                                M > 1 ? x2 : frc, op->fp64(), M > 1 ? 1 : op->fp64(), s0, rows, N, ncols, op->h,
                                pass, st);
      if (M > 1) {
        const int64_t krows = rows / M;
        cx<double>* ya = (cx<double>*)x1;            // x1 holds rows >= 2 * krows FP64 rows: two Horner buffers
        cx<double>* yb = ya + (size_t)krows * ncols;
        const void* prev = x2;
        int64_t pstride = M;
        for (int i = 1; i < M; ++i) {
          const bool last = i == M - 1;
          void* out = last ? frc : (void*)((i & 1) ? ya : yb);
          launch_row_horner(band64, prev, pstride, x2, M, i, out, last ? op->fp64() : 1, krows, N, ncols, st);
          prev = out;
          pstride = 1;
        }
      }
    }
    ForceSpec fs;
    fs.frc = frc;
    SnapSpec ss;
    ss.snap = snap;
    ss.ld = ncols + 1;
    ss.first = 0;
    ss.stride = every / M;
    ss.count = rows / every;
    RES_TRY(march_1d(op, k, rows / M, fs, ss, dsegs, nseg, st, M));
    const int64_t i0 = s0 / every;  // sample index of the tile's first snapshot (the state before its first step)
    launch_copy_rows(snap, ncols + 1, out, adjoint ? n - 1 - i0 : i0, adjoint ? -1 : 1, rows / every, ncols,
                     op->fp64(), st);
  }
  void* cur;
  RES_TRY(ws_get(op, op->cur_state ? "state1" : "state0", (size_t)ncols * ws, &cur));
  launch_copy_rows(cur, ncols, out, adjoint ? 0 : n - 1, 1, 1, ncols, op->fp64(), st);
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

// A signal run with the diagonal B, C and metrics around it (the node scalings of run_any, by role and direction):
// observed runs C R B f and W_f^{-1} B R^H C W_y y, or the Euclidean R~ and R~^H of the gains and modes.
int signal_run_any(resolvent_op* op, int k, int64_t n, int every, int scheme, int adjoint, const void* in, void* out,
                   hipStream_t st) {
  if (!op->weighted) return signal_run(op, k, n, every, scheme, adjoint, in, out, st);
  int rin, rout;
  if (op->scale_role == 0) {
    rin = adjoint ? kWscCWy : kWscB;
    rout = adjoint ? kWscBInvWf : kWscC;
  } else {
    rin = adjoint ? kWscCSqrtWy : kWscBInvSqrtWf;
    rout = adjoint ? kWscBInvSqrtWf : kWscCSqrtWy;
  }
  const double* w = (const double*)op->d_wsc;
  const int64_t blocks = n * k;
  const int fp = op->fp64();
  void* tmp;
  RES_TRY(ws_get(op, "sig_wsc_in", (size_t)blocks * op->N * op->wsize(), &tmp));
  launch_node_scale(in, fp, tmp, fp, w + (size_t)rin * op->N, blocks, op->N, st);
  RES_TRY(signal_run(op, k, n, every, scheme, adjoint, tmp, out, st));
  launch_node_scale(out, fp, out, fp, w + (size_t)rout * op->N, blocks, op->N, st);
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

int signal_args(const resolvent_op* op, int k, int64_t n, int every, int scheme) {
  if (k < 1 || n < 2 || every < 1) return fail(RES_EINVAL, "need k >= 1, at least two samples and every >= 1");
  if (scheme < 0 || scheme > 2) return fail(RES_EINVAL, "interpolation scheme must be 0 (C0), 1 (C1) or 2 (C2)");
  return RES_OK;
}

// Linear-phase FIR design by frequency sampling with a Hamming window (App. B).  The desired amplitude response,
// linear between the breakpoints (nu non-decreasing in [-1, 1], frequency over Nyquist; held at the end values
// outside them), is sampled on M uniform frequencies nu_q = -1 + 2q/M and transformed back with an n/2-sample
// delay:  b_m = w_m (1/M) sum_q D(nu_q) e^{i pi nu_q (m - n/2)},  w_m = 0.54 - 0.46 cos(2 pi m / n).
// M = 2 max(512, 2^ceil(log2 n)).  The phases are index-exact: e^{i pi nu_q r} = (-1)^r e^{2 pi i q r / M}.
// The desired response sampled on the design grid (and M); shared by the host design and the device one.
int fir_response_samples(int order, int npts, const double* nu, const double* gain, std::vector<double>* Dout) {
  if (order < 2 || order % 2 || order > fir_max_order())
    return fail(RES_EINVAL, "FIR order must be even, >= 2 and <= " + std::to_string(fir_max_order()));
  if (npts < 2 || !nu || !gain) return fail(RES_EINVAL, "need at least two breakpoints");
  for (int i = 0; i < npts; ++i) {
    if (!std::isfinite(nu[i]) || !std::isfinite(gain[i]) || gain[i] < 0 || nu[i] < -1.0 || nu[i] > 1.0 ||
        (i > 0 && nu[i] < nu[i - 1]))
      return fail(RES_EINVAL, "breakpoints must be finite, non-decreasing in [-1, 1] with gains >= 0");
  }
  int64_t p2 = 1;
  while (p2 < order) p2 <<= 1;
  const int64_t M = 2 * std::max<int64_t>(512, p2);
  std::vector<double>& D = *Dout;
  D.assign((size_t)M, 0.0);
  for (int64_t q = 0; q < M; ++q) {
    const double x = -1.0 + 2.0 * (double)q / (double)M;
    double v;
    if (x <= nu[0]) {
      v = gain[0];
    } else if (x >= nu[npts - 1]) {
      v = gain[npts - 1];
    } else {
      int i = 0;
      while (i + 1 < npts - 1 && x > nu[i + 1]) ++i;
      const double w = nu[i + 1] - nu[i];
      v = w > 0 ? gain[i] + (gain[i + 1] - gain[i]) * (x - nu[i]) / w : gain[i + 1];
    }
    D[q] = v;
  }
  return RES_OK;
}

std::vector<cd> unit_circle(int64_t M) {
  std::vector<cd> E((size_t)M);
  for (int64_t p = 0; p < M; ++p) E[p] = std::polar(1.0, 2.0 * M_PI * (double)p / (double)M);
  return E;
}

int fir_design_host(int order, int npts, const double* nu, const double* gain, std::vector<cd>* taps) {
  std::vector<double> D;
  RES_TRY(fir_response_samples(order, npts, nu, gain, &D));
  const int64_t M = (int64_t)D.size();
  const std::vector<cd> E = unit_circle(M);
  taps->assign((size_t)order + 1, cd(0, 0));
  for (int m = 0; m <= order; ++m) {
    const int64_t r = m - order / 2;
    cd acc(0, 0);
    for (int64_t q = 0; q < M; ++q) acc += D[q] * E[(size_t)((((q * r) % M) + M) % M)];
    if (r & 1) acc = -acc;
    const double wm = 0.54 - 0.46 * std::cos(2.0 * M_PI * (double)m / (double)order);
    (*taps)[m] = acc * (wm / (double)M);
  }
  return RES_OK;
}

// Breakpoints of the flattening response (Sec. 2.2): D_j = 1/||W(w_j)|| at the analysis frequencies (largest 1),
// falling linearly to zero `margin` (rad per time unit) outside them and zero beyond, raised to 1/passes.
int flattening_breakpoints(const std::vector<double>& om, const std::vector<double>& wnorm, double dt, double margin,
                           int passes, std::vector<double>* nu, std::vector<double>* gain) {
  const size_t nw = om.size();
  std::vector<std::pair<double, double>> pts;
  double dmax = 0;
  for (size_t j = 0; j < nw; ++j) {
    if (!(wnorm[j] > 0) || !std::isfinite(wnorm[j])) return fail(RES_ENONFINITE, "zero or non-finite spectrum");
    dmax = std::max(dmax, 1.0 / wnorm[j]);
  }
  for (size_t j = 0; j < nw; ++j) pts.emplace_back(om[j] * dt / M_PI, (1.0 / wnorm[j]) / dmax);
  std::stable_sort(pts.begin(), pts.end(), [](const std::pair<double, double>& a, const std::pair<double, double>& b) {
    return a.first < b.first;
  });
  const double dm = margin * dt / M_PI;
  const double lo = std::max(-1.0, pts.front().first - dm), hi = std::min(1.0, pts.back().first + dm);
  nu->clear();
  gain->clear();
  if (lo > -1.0) nu->push_back(-1.0), gain->push_back(0.0);
  nu->push_back(lo), gain->push_back(0.0);
  for (auto& p : pts) nu->push_back(p.first), gain->push_back(std::pow(p.second, 1.0 / passes));
  nu->push_back(hi), gain->push_back(0.0);
  if (hi < 1.0) nu->push_back(1.0), gain->push_back(0.0);
  return RES_OK;
}

// The power iteration with time-domain hand-off (Sec. 2.2 with App. A): each iteration runs the direct march of
// the current forcing F, the adjoint march forced by its response Y, takes the spectra of F, Y and W at the
// analysis frequencies (gains ||Y(w_j)|| / ||F(w_j)||, amplitudes ||F(w_j)||), flattens W by `passes` passes of
// an FIR filter designed for (1/||W(w_j)||)^(1/passes) and hands it back, tapered and normalised, as the next F.
// passes = 0 hands W back unfiltered.
int trm_modes(resolvent_op* op, int k, int64_t n, int every, int scheme, const void* f0, int nw, const double* omegas,
              int iters, int order, int passes, int64_t pad, int64_t ramp, double margin, double* gains,
              double* amps, void* f_out, void* V, void* U, hipStream_t st) {
  const int64_t ncols = (int64_t)k * op->N, count = n * ncols;
  const size_t ws = op->wsize();
  const double dt = (double)every * op->h;
  void *F, *Y, *W, *Tm, *hat, *nrm, *taps, *omd, *part, *dpart, *dD = nullptr, *dE = nullptr;
  RES_TRY(ws_get(op, "trm_F", (size_t)count * ws, &F));
  RES_TRY(ws_get(op, "trm_Y", (size_t)count * ws, &Y));
  RES_TRY(ws_get(op, "trm_W", (size_t)count * ws, &W));
  RES_TRY(ws_get(op, "trm_T", (size_t)count * ws, &Tm));
  RES_TRY(ws_get(op, "trm_hat", (size_t)nw * ncols * sizeof(cd), &hat));
  RES_TRY(ws_get(op, "trm_norms", (size_t)3 * nw * sizeof(double), &nrm));
  RES_TRY(ws_get(op, "trm_taps", (size_t)(std::max(order, 0) + 1) * sizeof(cd), &taps));
  RES_TRY(ws_get(op, "trm_omegas", (size_t)nw * sizeof(double), &omd));
  RES_TRY(ws_get(op, "trm_part", (size_t)(normalise_parts() + 1) * sizeof(double), &part));
  RES_TRY(ws_get(op, "trm_dft_part", (size_t)series_dft_part_elems(n, ncols, nw) * sizeof(cd), &dpart));
  std::vector<cd>& Etab = op->trm_E;
  std::vector<double>& Dq = op->trm_D;
  if (passes > 0) {  // the design grid: the response samples (host, per iteration) and the unit circle (once)
    int64_t p2 = 1;
    while (p2 < order) p2 <<= 1;
    const int64_t M = 2 * std::max<int64_t>(512, p2);
    RES_TRY(ws_get(op, "trm_design_D", (size_t)M * sizeof(double), &dD));
    RES_TRY(ws_get(op, "trm_design_E", (size_t)M * sizeof(cd), &dE));
    Etab = unit_circle(M);
    HIP_TRY(hipMemcpyAsync(dE, Etab.data(), Etab.size() * sizeof(cd), hipMemcpyHostToDevice, st));
  }
  double* scale = (double*)part + normalise_parts();
  op->trm_om.assign(omegas, omegas + nw);
  const std::vector<double>& om = op->trm_om;
  std::vector<double> hn((size_t)3 * nw), bnu, bgain;
  const cd& one = op->trm_one;
  HIP_TRY(hipMemcpyAsync(omd, om.data(), (size_t)nw * sizeof(double), hipMemcpyHostToDevice, st));
  // F = taper(f0) / ||taper(f0)||: the identity filter with the taper (with metrics, of W_f^{1/2} f0: the iteration
  // runs on the Euclidean R~)
  ModesRole role(op);
  HIP_TRY(hipMemcpyAsync(taps, &one, sizeof(cd), hipMemcpyHostToDevice, st));
  if (launch_fir((const cx<double>*)taps, 0, f0, F, n, ncols, pad, ramp, op->fp64(), st))
    return fail(RES_EINVAL, "taper launch");
  if (op->weighted)
    launch_node_scale(F, op->fp64(), F, op->fp64(), (const double*)op->d_wsc + (size_t)kWscSqrtWf * op->N, n * k,
                      op->N, st);
  launch_normalise(F, op->fp64(), count, (double*)part, scale, st);
  for (int it = 0; it < iters; ++it) {
    RES_TRY(signal_run_any(op, k, n, every, scheme, 0, F, Y, st));
    RES_TRY(signal_run_any(op, k, n, every, scheme, 1, Y, W, st));
    const void* ser[3] = {F, Y, W};
    {
      TimedLaunch tl(op, RES_TIMING_PROJECTION, st);
      for (int q = 0; q < 3; ++q) {
        if (launch_series_dft(ser[q], op->fp64(), n, ncols, (const double*)omd, nw, dt, dpart, hat, st))
          return fail(RES_EINVAL, "series too long for the transform's chunk grid");
        launch_row_norms(hat, nw, ncols, (double*)nrm + (size_t)q * nw, st);
      }
    }
    HIP_TRY(hipMemcpyAsync(hn.data(), nrm, hn.size() * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));  // also retires the host-side copies issued before
    for (int j = 0; j < nw; ++j) {
      gains[(size_t)it * nw + j] = hn[(size_t)nw + j] / hn[j];
      if (amps) amps[(size_t)it * nw + j] = hn[j];
    }
    if (it + 1 == iters) {  // modes of the last iteration: the spectra of F and Y normalised per frequency
      void* mo[2] = {V, U};
      for (int q = 0; q < 2; ++q) {
        if (!mo[q]) continue;
        if (launch_series_dft(ser[q], op->fp64(), n, ncols, (const double*)omd, nw, dt, dpart, hat, st))
          return fail(RES_EINVAL, "series too long for the transform's chunk grid");
        launch_scale_rows(hat, (const double*)nrm + (size_t)q * nw, nw, ncols, mo[q], op->fp64(), st);
      }
      if (op->weighted) RES_TRY(modes_to_problem(op, nw, k, V, U, st));  // W_f^{-1/2} V~, W_y^{-1/2} U~
    }
    if (it + 1 == iters && !f_out) break;
    if (passes == 0) {
      HIP_TRY(hipMemcpyAsync(taps, &one, sizeof(cd), hipMemcpyHostToDevice, st));
    } else {
      std::vector<double> wn(hn.begin() + 2 * nw, hn.end());
      RES_TRY(flattening_breakpoints(om, wn, dt, margin, passes, &bnu, &bgain));
      RES_TRY(fir_response_samples(order, (int)bnu.size(), bnu.data(), bgain.data(), &Dq));
      HIP_TRY(hipMemcpyAsync(dD, Dq.data(), Dq.size() * sizeof(double), hipMemcpyHostToDevice, st));
      TimedLaunch tl(op, RES_TIMING_QR, st);
      if (launch_fir_taps((const double*)dD, dE, (int64_t)Dq.size(), order, taps, st))
        return fail(RES_EINVAL, "FIR design launch");
    }
    {
      TimedLaunch tl(op, RES_TIMING_QR, st);
      if (passes == 0) {
        if (launch_fir((const cx<double>*)taps, 0, W, F, n, ncols, pad, ramp, op->fp64(), st))
          return fail(RES_EINVAL, "taper launch");
      } else {
        const void* src = W;
        for (int p = 0; p < passes; ++p) {
          const bool last = p + 1 == passes;
          void* dst = last ? F : (src == W ? Tm : W);
          if (launch_fir((const cx<double>*)taps, order, src, dst, n, ncols, last ? pad : -1, ramp, op->fp64(), st))
            return fail(RES_EINVAL, "FIR launch");
          src = dst;
        }
      }
      launch_normalise(F, op->fp64(), count, (double*)part, scale, st);
    }
  }
  if (f_out) HIP_TRY(hipMemcpyAsync(f_out, F, (size_t)count * ws, hipMemcpyDeviceToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));  // the host taps and frequencies must outlive their copies
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

}  // namespace

namespace {

// Workspace sizes of one direct run in a fixed arena of `cap` bytes (the no-allocation apply): the slots a run takes
// from ws_get, with the flexible buffers (pre-filter blocks, snapshot rows, forcing tiles, projection partials)
// sized from what the fixed ones leave.  RES_EINVAL with the byte counts when even the smallest layout does not fit.
int arena_sizes(const resolvent_op* op, const Plan& pl, int k, size_t cap, ArenaSizes* out) {
  const double ws = (double)op->wsize();
  const double ncols = (double)k * (double)op->N;
  const int M = run_power(op, pl);
  const int nw = pl.nw;
  auto al = [](double b) { return std::ceil(b / 256.0) * 256.0; };
  double fixed = al(nw * ncols * ws)                                   // G
                 + al((double)pl.P * ws)                               // phase table
                 + 2 * al(ncols * ws);                                 // state0, state1
  if (!op->fp64()) fixed += al(nw * ncols * 16.0);                     // FP64 accumulator of the complex64 output
  if (op->weighted) fixed += al(nw * ncols * 16.0);                    // scaled input block
  if (is_grid(op) && op->ncomp == 3) fixed += al(ncols * ws);          // third-stage input of the 3-D step
  if (!is_grid(op)) fixed += al((double)k * op->segs.size() * sizeof(Seg1D));
  const double room = (double)cap - fixed;
  const int nbuf = M > 2 ? 3 : 2;
  const double snap_ld = ncols + 1;
  const int64_t table_rows = std::min<int64_t>(pl.P, pl.forced_end) / M;
  ArenaSizes z;
  z.horner_chunk = (int)std::max<int64_t>(1, std::min<int64_t>(nw, (int64_t)(room / 8 / (nbuf * ncols * 16.0))));
  z.snap_rows = std::min<int64_t>(pl.pcount, std::max<int64_t>(64, (int64_t)(room / 8 / (snap_ld * ws))));
  z.table = (double)table_rows * ncols * ws <= room / 4;
  z.tile_rows = std::max<int64_t>(64, (int64_t)(room / 8 / (ncols * ws)));
  z.max_nsplit = std::max<int64_t>(1, (int64_t)(room / 8 / (nw * ncols * 16.0)));
  double total = fixed + nbuf * al(z.horner_chunk * ncols * 16.0) + al((double)z.snap_rows * snap_ld * ws) +
                 (z.table ? al((double)table_rows * ncols * ws) : al((double)(z.tile_rows + 16) * ncols * ws)) +
                 (z.max_nsplit > 1 ? al((double)z.max_nsplit * nw * ncols * 16.0) : 0.0);
  if (total > (double)cap)
    return fail(RES_EINVAL, "resolvent_apply_noalloc: this run needs at least " + std::to_string((long long)total) +
                            " bytes of workspace and the no-allocation scratch holds " + std::to_string(cap) +
                            "; use resolvent_apply");
  z.total = (size_t)total;
  *out = z;
  return RES_OK;
}

}  // namespace

// resolvent_apply with every workspace buffer carved from [base, base + cap) (device memory the caller keeps for
// the process): see resolvent_apply_noalloc in noalloc.hip.
int res_apply_in_scratch(resolvent_op* op, const resolvent_grid* g, const resolvent_run* r, int32_t k,
                         const void* f_hat, void* u_hat, void* base, size_t cap, void* stream) {
  g_last_error.clear();
  if (!op || !g || !r || !f_hat || !u_hat || !base) return fail(RES_EINVAL, "NULL argument");
  if (k < 1) return fail(RES_EINVAL, "k must be >= 1");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev != op->device) return fail(RES_EINVAL, "the current device is not the one the handle was created on");
  Plan pl;
  RES_TRY(make_plan(op, g, r, &pl));
  ArenaSizes z;
  RES_TRY(arena_sizes(op, pl, k, cap, &z));
  Arena a;
  a.base = (char*)base;
  a.cap = cap;
  a.sz = z;
  op->arena = &a;
  op->arena_stream = (hipStream_t)stream;
  const int rc = apply_common(op, g, r, k, f_hat, u_hat, +1, (hipStream_t)stream);
  op->arena = nullptr;
  op->arena_stream = nullptr;
  return rc;
}

int res_fail(int code, const char* msg) { return fail(code, msg); }

// =====================================================================================================
// C ABI
// =====================================================================================================
extern "C" {

const char* resolvent_strerror(int s) {
  switch (s) {
    case RES_OK: return "success";
    case RES_EINVAL: return "invalid argument";
    case RES_EGRID: return "frequency grid not commensurate with the time step";
    case RES_ESTEP: return "RK4 step unstable for this operator";
    case RES_EUNSTABLE: return "operator is not stable (decay probe did not decay)";
    case RES_ENONFINITE: return "non-finite values in a result";
    case RES_ENOMEM: return "device allocation failed";
    case RES_EHIP: return "HIP runtime error";
    case RES_ENOTSUP: return "not supported for this operator";
    default: return "unknown status";
  }
}

const char* resolvent_last_error(void) { return g_last_error.c_str(); }

int resolvent_op_create(const resolvent_op_desc* d, void* stream, resolvent_op** out) {
  g_last_error.clear();
  if (!out) return fail(RES_EINVAL, "out is NULL");
  *out = nullptr;
  if (!d) return fail(RES_EINVAL, "desc is NULL");
  if (!(d->h > 0) || !std::isfinite(d->h)) return fail(RES_EINVAL, "h must be positive");
  if (d->precision != RES_FP64 && d->precision != RES_MIXED) return fail(RES_EINVAL, "bad precision");
  hipStream_t st = (hipStream_t)stream;
  resolvent_op* op = new resolvent_op();
  if (hipGetDevice(&op->device) != hipSuccess) {
    delete op;
    return fail(RES_EHIP, "hipGetDevice failed");
  }
  op->kind = d->kind;
  op->prec = d->precision;
  op->h = d->h;
  auto bail = [&](int rc) {
    resolvent_op_destroy(op);
    return rc;
  };
  if (d->kind == RES_OP_TRIDIAG) {
    if (!d->lower || !d->diag || !d->upper) return bail(fail(RES_EINVAL, "tridiagonal arrays are NULL"));
    op->ninst = d->ninst < 1 ? 1 : d->ninst;
    if (d->inst_offsets) {
      op->off.assign(d->inst_offsets, d->inst_offsets + op->ninst + 1);
    } else {
      if (op->ninst != 1) return bail(fail(RES_EINVAL, "inst_offsets required when ninst > 1"));
      op->off = {0, d->nx};
    }
    if (op->off[0] != 0) return bail(fail(RES_EINVAL, "inst_offsets[0] must be 0"));
    for (int m = 0; m < op->ninst; ++m)
      if (op->off[m + 1] <= op->off[m]) return bail(fail(RES_EINVAL, "instances must be non-empty"));
    op->N = op->off[op->ninst];
    const int64_t n = op->N;
    op->zl.resize(n);
    op->zd.resize(n);
    op->zu.resize(n);
    std::vector<char> first(n, 0), last(n, 0);
    for (int m = 0; m < op->ninst; ++m) {
      first[op->off[m]] = 1;
      last[op->off[m + 1] - 1] = 1;
    }
    for (int64_t i = 0; i < n; ++i) {
      const cd l(d->lower[2 * i], d->lower[2 * i + 1]), c(d->diag[2 * i], d->diag[2 * i + 1]),
          u(d->upper[2 * i], d->upper[2 * i + 1]);
      if (!std::isfinite(l.real()) || !std::isfinite(l.imag()) || !std::isfinite(c.real()) ||
          !std::isfinite(c.imag()) || !std::isfinite(u.real()) || !std::isfinite(u.imag()))
        return bail(fail(RES_EINVAL, "non-finite operator coefficient"));
      op->zl[i] = first[i] ? cd(0, 0) : d->h * l;
      op->zd[i] = d->h * c;
      op->zu[i] = last[i] ? cd(0, 0) : d->h * u;
    }
    int rc = plan_1d_default(op);
    if (rc) return bail(rc);
    rc = build_1d_stencils(op);
    if (rc) return bail(rc);
  } else if (d->kind == RES_OP_ADR2D || d->kind == RES_OP_ADR3D3C) {
    const bool three = d->kind == RES_OP_ADR3D3C;
    op->ncomp = three ? 3 : 1;
    op->nx = d->nx;
    op->ny = d->ny;
    op->nz = three ? d->nz : 1;
    if (op->nx < 1 || op->ny < 1 || op->nz < 1) return bail(fail(RES_EINVAL, "grid sizes must be >= 1"));
    if (!d->cxm || !d->cxp || !d->cym || !d->cyp || !d->dfield || (three && (!d->czm || !d->czp)))
      return bail(fail(RES_EINVAL, "grid coefficient arrays are NULL"));
    const int64_t nl = op->ny * op->nz, nn = nl * op->nx;
    const double* src[6] = {d->cxm, d->cxp, d->cym, d->cyp, three ? d->czm : nullptr, three ? d->czp : nullptr};
    for (int a = 0; a < 6; ++a) {
      op->gx[a].assign(nl, 0.0);
      if (src[a])
        for (int64_t l = 0; l < nl; ++l) op->gx[a][l] = d->h * src[a][l];
    }
    op->gd.resize(nn);
    for (int64_t i = 0; i < nn; ++i) op->gd[i] = d->h * d->dfield[i];
    if (three && d->coupling) {
      op->gK.resize(nl * 9);
      for (int64_t i = 0; i < nl * 9; ++i) op->gK[i] = d->h * d->coupling[i];
    }
    for (int a = 0; a < 6; ++a)
      for (double v : op->gx[a])
        if (!std::isfinite(v)) return bail(fail(RES_EINVAL, "non-finite operator coefficient"));
    op->N = (int64_t)op->ncomp * nn;
    op->ninst = 1;
    op->off = {0, op->N};
    int rc = build_grid_coefficients(op);
    if (rc) return bail(rc);
  } else {
    return bail(fail(RES_ENOTSUP, "operator kind not supported"));
  }
  if (upload((void**)&op->d_off, op->off.data(), op->off.size() * sizeof(int64_t))) return bail(RES_EHIP);
  if (hipMalloc(&op->d_flag, sizeof(int)) != hipSuccess) return bail(fail(RES_ENOMEM, "flag"));
  if (hipMemset(op->d_flag, 0, sizeof(int)) != hipSuccess) return bail(fail(RES_EHIP, "flag memset"));
  if (d->probe) {
    int rc = decay_probe(op, d, st);
    if (rc) return bail(rc);
  }
  *out = op;
  return RES_OK;
}

void resolvent_op_destroy(resolvent_op* op) {
  if (!op) return;
  (void)hipDeviceSynchronize();
  for (auto& kv : op->ws)
    if (kv.second.p) (void)hipFree(kv.second.p);
  for (auto& kv : op->btab)
    if (kv.second) (void)hipFree(kv.second);
  for (auto& kv : op->btab64)
    if (kv.second) (void)hipFree(kv.second);
  for (int s = 0; s < 2; ++s) {
    if (op->d_tri[s]) (void)hipFree(op->d_tri[s]);
    if (op->d_band[s]) (void)hipFree(op->d_band[s]);
    if (op->d_band64[s]) (void)hipFree(op->d_band64[s]);
    if (op->d_bandm[s]) (void)hipFree(op->d_bandm[s]);
  }
  if (op->d_wsc) (void)hipFree(op->d_wsc);
  if (op->cap_stream) (void)hipStreamDestroy(op->cap_stream);
  if (op->side_stream) (void)hipStreamDestroy(op->side_stream);
  for (hipEvent_t e : op->side_ev) (void)hipEventDestroy(e);
  if (op->d_off) (void)hipFree(op->d_off);
  if (op->xch) retired_exchange_areas().push_back(op->xch);  // uncached memory is not freed (see march_1d)
  for (void* b : op->gbufs) (void)hipFree(b);
  for (int c = 0; c < 4; ++c)
    for (auto& e : op->tev[c]) {
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
  if (op->d_flag) (void)hipFree(op->d_flag);
  delete op;
}

int64_t resolvent_op_size(const resolvent_op* op) { return op ? op->N : -1; }
double resolvent_op_decay_time(const resolvent_op* op) { return op ? op->decay_time : -1; }

int resolvent_op_set_diagonal(resolvent_op* op, const double* values, int32_t on_device, void* stream) {
  if (!op || !values) return fail(RES_EINVAL, "NULL argument");
  hipStream_t st = (hipStream_t)stream;
  if (op->kind == RES_OP_TRIDIAG) {
    std::vector<double> hv(2 * op->N);
    if (on_device) {
      HIP_TRY(hipMemcpyAsync(hv.data(), values, hv.size() * sizeof(double), hipMemcpyDeviceToHost, st));
      HIP_TRY(hipStreamSynchronize(st));
    } else {
      std::memcpy(hv.data(), values, hv.size() * sizeof(double));
    }
    for (int64_t i = 0; i < op->N; ++i) op->zd[i] = op->h * cd(hv[2 * i], hv[2 * i + 1]);
    HIP_TRY(hipStreamSynchronize(st));  // kernels in flight may still read the old stencils
    return build_1d_stencils(op);
  }
  if (is_grid(op)) {
    const int64_t nn = op->nx * op->ny * op->nz;
    std::vector<double> hv(nn);
    if (on_device) {
      HIP_TRY(hipMemcpyAsync(hv.data(), values, nn * sizeof(double), hipMemcpyDeviceToHost, st));
    } else {
      std::memcpy(hv.data(), values, nn * sizeof(double));
    }
    HIP_TRY(hipStreamSynchronize(st));
    for (int64_t i = 0; i < nn; ++i) op->gd[i] = op->h * hv[i];
    return build_grid_coefficients(op);
  }
  return fail(RES_ENOTSUP, "operator kind not supported");
}

int resolvent_apply(resolvent_op* op, const resolvent_grid* grid, const resolvent_run* run, int32_t k,
                    const void* f_hat, void* u_hat, void* stream) {
  g_last_error.clear();
  return apply_common(op, grid, run, k, f_hat, u_hat, +1, (hipStream_t)stream);
}

int resolvent_adjoint_apply(resolvent_op* op, const resolvent_grid* grid, const resolvent_run* run, int32_t k,
                            const void* g_hat, void* z_hat, void* stream) {
  g_last_error.clear();
  return apply_common(op, grid, run, k, g_hat, z_hat, -1, (hipStream_t)stream);
}

static int modes_body(resolvent_op* op, const resolvent_grid* grid, const resolvent_run* run, int32_t k,
                      int32_t iters, const void* f0_hat, double* gains, void* V, void* U, double* hist,
                    void* stream) {
  g_last_error.clear();
  if (!op || !f0_hat || !gains) return fail(RES_EINVAL, "NULL argument");
  if (k < 1 || k > 8) return fail(RES_EINVAL, "k must be in 1..8");
  if (iters < 1) return fail(RES_EINVAL, "iters must be >= 1");
  hipStream_t st = (hipStream_t)stream;
  {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      return fail(RES_EINVAL, "resolvent_modes returns host data and cannot be captured (capture resolvent_apply, or "
                              "let the library replay its iterations: resolvent_op_set_graphs)");
  }
  Plan pl;
  RES_TRY(make_plan(op, grid, run, &pl));
  const int nw = pl.nw;
  const int64_t count = (int64_t)nw * k * op->N;
  const size_t mats = (size_t)nw * op->ninst * 64 * sizeof(cd);
  void *Fh, *Y, *Z, *rY, *phi, *psi, *apsi, *dg, *dh = nullptr;
  RES_TRY(ws_get(op, "modes_F", count * sizeof(cd), &Fh));
  RES_TRY(ws_get(op, "modes_Y", count * sizeof(cd), &Y));
  RES_TRY(ws_get(op, "modes_Z", count * sizeof(cd), &Z));
  RES_TRY(ws_get(op, "modes_rY", mats, &rY));
  RES_TRY(ws_get(op, "modes_phi", mats, &phi));
  RES_TRY(ws_get(op, "modes_psi", mats, &psi));
  RES_TRY(ws_get(op, "modes_apsi", mats, &apsi));
  const size_t gcount = (size_t)op->ninst * nw * k;
  RES_TRY(ws_get(op, "modes_gains", gcount * sizeof(double), &dg));
  if (hist) RES_TRY(ws_get(op, "modes_hist", (size_t)iters * gcount * 2 * sizeof(double), &dh));
  ModesRole role(op);
  launch_convert(f0_hat, op->fp64(), Fh, 1, count, 1.0, st);
  if (op->weighted)  // start forcings in the problem's coordinates: to the Euclidean R~'s (times W_f^{1/2})
    launch_node_scale(Fh, 1, Fh, 1, (const double*)op->d_wsc + (size_t)kWscSqrtWf * op->N, (int64_t)nw * k, op->N, st);
  // Amplitude weights (iterations after the first): every run marches all frequencies superposed in one state, so
  // in the working precision the rounding of the large responses lands on the small ones.  The runs therefore
  // march frequency j with its input scaled by 1/sqrt(sigma_1(j)) from the previous iteration and unscale the
  // result, which balances the response amplitudes (large gains) against the forcing amplitudes (small gains)
  // across frequencies -- the frequency normalisation of Sec. 2.2, applied between iterations.  Exact in exact
  // arithmetic (the runs are linear); the QR and SVD see unscaled blocks.  Only for the periodic method: there
  // each frequency's response depends on its own forcing alone (the run applies R_d(w_j) block by block), while
  // the transient method's truncated tail leaks every frequency into its neighbours, so scaling frequency j's input
  // by its own weight and unscaling the output by the weight of j' would change the leakage terms and with them
  // the iterated map (by 2e-7 relative on the N = 200 transient workload, where the ratio of the largest to the
  // smallest gain is 100).
  const bool weigh = pl.method == RES_PERIODIC;
  void* fac;
  RES_TRY(ws_get(op, "modes_fac", (size_t)op->ninst * nw * sizeof(double), &fac));
  // Weighted run: the input block is scaled in place (restored afterwards when keep_input) and the output unscaled.
  auto weighted_run = [&](bool weighted, bool keep_input, void* in, double* out, int sigma, hipStream_t s) -> int {
    if (!weighted) return run_any(op, pl, k, in, 1, out, sigma, s);
    launch_freq_scale(in, in, op->N, k, nw, op->d_off, op->ninst, (const double*)fac, 0, s);
    RES_TRY(run_any(op, pl, k, in, 1, out, sigma, s));
    if (keep_input) launch_freq_scale(in, in, op->N, k, nw, op->d_off, op->ninst, (const double*)fac, 1, s);
    launch_freq_scale(out, out, op->N, k, nw, op->d_off, op->ninst, (const double*)fac, 1, s);
    HIP_TRY(hipGetLastError());
    return RES_OK;
  };
  // One iteration on stream s; hprev receives the norm estimate of the previous iteration, hcur the gains.
  auto iteration = [&](bool last, bool weighted, double* hprev, double* hcur, hipStream_t s) -> int {
    // 1. F = Q(QR(F_hat))
    RES_TRY(cholqr2(op, nw, k, (double*)Fh, rY, hprev, s));
    // 2. Y = R_d F
    RES_TRY(weighted_run(weighted, last && V, Fh, (double*)Y, +1, s));  // F_hat is needed again only for V
    // 3. Y = Q_Y R_Y, R_Y = Phi Sigma Psi^H
    RES_TRY(cholqr2(op, nw, k, (double*)Y, rY, nullptr, s));
    launch_svd(rY, k, nw, op->ninst, phi, psi, apsi, (double*)dg, hcur, s);
    if (last) {
      if (U) launch_rmul(Y, 1, U, op->fp64(), op->N, k, op->d_off, op->ninst, nw, nsplit_for(max_instance_len(op)), phi, s);
      if (V) launch_rmul(Fh, 1, V, op->fp64(), op->N, k, op->d_off, op->ninst, nw, nsplit_for(max_instance_len(op)), psi, s);
    }
    // 4. Z = R_d^H Q_Y (with the weights of the previous iteration, as the direct run)
    RES_TRY(weighted_run(weighted, false, Y, (double*)Z, -1, s));
    launch_freq_weights((const double*)dg, (double*)fac, op->ninst, nw, k, s);  // for the next iteration
    // 5. F_hat = Z R_Y Psi
    launch_rmul(Z, 1, Fh, 1, op->N, k, op->d_off, op->ninst, nw, nsplit_for(max_instance_len(op)), apsi, s);
    HIP_TRY(hipGetLastError());
    return RES_OK;
  };
  auto hslot = [&](int it) -> double* { return hist ? (double*)dh + (size_t)it * gcount * 2 : nullptr; };
  // Graph mode: the first iteration runs eagerly (it sizes every workspace), the middle ones replay one captured
  // iteration (history slots are fixed scratch rows copied out after each replay), the last runs eagerly (modes).
  const bool graphs = op->use_graphs && iters >= 3;
  int it = 0;
  RES_TRY(iteration(iters == 1, false, nullptr, hslot(0), st));
  ++it;
  if (graphs) {
    void* hs = nullptr;
    if (hist) RES_TRY(ws_get(op, "modes_hist_slots", gcount * 4 * sizeof(double), &hs));
    double* hs_prev = hist ? (double*)hs : nullptr;
    double* hs_cur = hist ? (double*)hs + gcount * 2 : nullptr;
    if (!op->cap_stream) HIP_TRY(hipStreamCreateWithFlags(&op->cap_stream, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    HIP_TRY(hipStreamBeginCapture(op->cap_stream, hipStreamCaptureModeThreadLocal));
    op->capturing = true;
    int rc = iteration(false, weigh, hs_prev, hs_cur, op->cap_stream);
    op->capturing = false;
    const hipError_t ec = hipStreamEndCapture(op->cap_stream, &graph);
    if (rc == RES_OK && ec != hipSuccess) rc = fail(RES_EHIP, std::string("graph capture: ") + hipGetErrorString(ec));
    if (rc == RES_OK && hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) != hipSuccess)
      rc = fail(RES_EHIP, "graph instantiation failed");
    for (; rc == RES_OK && it < iters - 1; ++it) {
      // history rows interleave (gain, norm estimate); the replay writes the estimate of it - 1 into hs_prev and
      // the gains of it into hs_cur, so hs_prev first takes the row of it - 1 to keep its gains
      if (hist && hipMemcpyAsync(hs_prev, hslot(it - 1), gcount * 2 * sizeof(double), hipMemcpyDeviceToDevice, st) !=
                      hipSuccess) {
        rc = fail(RES_EHIP, "history copy");
        break;
      }
      if (hipGraphLaunch(exec, st) != hipSuccess) {
        rc = fail(RES_EHIP, "graph launch failed");
        break;
      }
      if (hist) {
        if (hipMemcpyAsync(hslot(it - 1), hs_prev, gcount * 2 * sizeof(double), hipMemcpyDeviceToDevice, st) !=
                hipSuccess ||
            hipMemcpyAsync(hslot(it), hs_cur, gcount * 2 * sizeof(double), hipMemcpyDeviceToDevice, st) != hipSuccess)
          rc = fail(RES_EHIP, "history copy");
      }
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipGetLastError();
    RES_TRY(rc);
  }
  for (; it < iters; ++it) RES_TRY(iteration(it == iters - 1, weigh, hslot(it - 1), hslot(it), st));
  if (hist) {
    // norm estimate of the last iteration from the Gram of the final F_hat
    const int nsplit = nsplit_for(max_instance_len(op));
    const int km = gram_km(k);
    void *part, *r1, *r1i;
    RES_TRY(ws_get(op, "gram_part", (size_t)nw * op->ninst * nsplit * km * (km + 1) / 2 * sizeof(cd), &part));
    RES_TRY(ws_get(op, "qr_r1", mats, &r1));
    RES_TRY(ws_get(op, "qr_r1i", mats, &r1i));
    launch_gram(Fh, 1, op->N, k, op->d_off, op->ninst, nw, nsplit, part, op->d_flag, st);
    launch_chol(part, nsplit, k, nw, op->ninst, r1, r1i, nullptr, nullptr,
                (double*)dh + (size_t)(iters - 1) * gcount * 2, op->d_flag, st);
    HIP_TRY(hipMemcpyAsync(hist, dh, (size_t)iters * gcount * 2 * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  if (op->weighted) RES_TRY(modes_to_problem(op, nw, k, V, U, st));
  HIP_TRY(hipMemcpyAsync(gains, dg, gcount * sizeof(double), hipMemcpyDeviceToHost, st));
  return resolvent_op_check(op, stream);
}

// Block Arnoldi (Appendix A): basis blocks B_0 = Q(QR(f0)), B_{i+1} = Q(QR(W_i - sum_b B_b C_b)) with
// W_i = R_d^H R_d B_i and the coefficients C_b = B_b^H W_i taken twice (classical Gram-Schmidt, two passes).  The
// first-pass coefficients fill the upper block triangle of H = B^H R_d^H R_d B; the estimates come from the
// eigen-decomposition of its Hermitian completion: gains sqrt(lambda), V = B psi, U = R_d B psi / gain.
static int krylov_body(resolvent_op* op, const resolvent_grid* grid, const resolvent_run* run, int32_t k,
                       int32_t blocks, const void* f0_hat, double* gains, void* V, void* U, double* hist,
                     void* stream) {
  g_last_error.clear();
  if (!op || !f0_hat || !gains) return fail(RES_EINVAL, "NULL argument");
  if (k < 1 || k > 8) return fail(RES_EINVAL, "k must be in 1..8");
  if (blocks < 1 || blocks * k > 40) return fail(RES_EINVAL, "blocks must be >= 1 with blocks * k <= 40");
  for (int i = 0; i < op->ninst; ++i)
    if (op->off[i + 1] - op->off[i] < (int64_t)blocks * k)
      return fail(RES_EINVAL, "blocks * k exceeds the unknowns of an instance");
  hipStream_t st = (hipStream_t)stream;
  {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
      return fail(RES_EINVAL, "resolvent_krylov returns host data and cannot be captured");
  }
  Plan pl;
  RES_TRY(make_plan(op, grid, run, &pl));
  const int nw = pl.nw, ninst = op->ninst;
  const int64_t N = op->N;
  const int64_t bsz = (int64_t)nw * k * N;  // complex values per block
  const int nmax = blocks * k;
  const int nsplit = nsplit_for(max_instance_len(op));
  const int km = gram_km(k);
  const size_t gcount = (size_t)ninst * nw * k;
  void *B, *Yb, *H, *C, *part, *psi, *dg, *dh = nullptr, *rq, *one;
  RES_TRY(ws_get(op, "kry_basis", (size_t)(blocks + 1) * bsz * sizeof(cd), &B));
  RES_TRY(ws_get(op, "kry_y", (size_t)blocks * bsz * sizeof(cd), &Yb));
  RES_TRY(ws_get(op, "kry_h", (size_t)nw * ninst * nmax * nmax * sizeof(cd), &H));
  RES_TRY(ws_get(op, "kry_c", (size_t)nw * ninst * nmax * k * sizeof(cd), &C));
  RES_TRY(ws_get(op, "kry_part", (size_t)blocks * nw * ninst * nsplit * km * km * sizeof(cd), &part));
  RES_TRY(ws_get(op, "kry_psi", (size_t)nw * ninst * nmax * k * sizeof(cd), &psi));
  RES_TRY(ws_get(op, "kry_gains", gcount * sizeof(double), &dg));
  RES_TRY(ws_get(op, "kry_one", gcount * sizeof(double), &one));
  RES_TRY(ws_get(op, "kry_rq", (size_t)nw * ninst * 64 * sizeof(cd), &rq));
  RES_TRY(ws_get(op, "kry_hist", (size_t)blocks * gcount * sizeof(double), &dh));
  // Mixed precision: amplitude weights from the second block on, as in resolvent_modes.  Every run superposes all
  // frequencies in one FP32 state, so the direct run takes B_i scaled by sigma_1^{-1/2} and the adjoint run takes
  // R B_i (amplitude sigma) scaled by sigma_1^{-3/2} (sigma_1 from the previous block's estimates), and their
  // outputs are unscaled.  FP64 runs are not weighted: the later basis blocks come from strongly cancelling
  // differences, which would turn the rescaling's rounding into differences of 1e-9 in the estimates.  Transient
  // runs are not weighted either (their tail couples the frequencies; see resolvent_modes).
  const bool weigh = !op->fp64() && pl.method == RES_PERIODIC;
  void *fd, *fa, *tmp;
  RES_TRY(ws_get(op, "kry_fd", (size_t)ninst * nw * sizeof(double), &fd));
  RES_TRY(ws_get(op, "kry_fa", (size_t)ninst * nw * sizeof(double), &fa));
  RES_TRY(ws_get(op, "kry_tmp", (size_t)bsz * sizeof(cd), &tmp));
  auto blk = [&](void* base, int i) { return (double*)base + (size_t)2 * i * bsz; };
  auto weighted = [&](bool w, const void* fac, double* in, double* out, int sigma) -> int {
    if (!w) return run_any(op, pl, k, in, 1, out, sigma, st);
    launch_freq_scale(in, tmp, N, k, nw, op->d_off, ninst, (const double*)fac, 0, st);
    RES_TRY(run_any(op, pl, k, tmp, 1, out, sigma, st));
    launch_freq_scale(out, out, N, k, nw, op->d_off, ninst, (const double*)fac, 1, st);
    HIP_TRY(hipGetLastError());
    return RES_OK;
  };
  RES_TRY(zero_device(H, (size_t)nw * ninst * nmax * nmax * sizeof(cd), st));
  {
    std::vector<double> ones(gcount, 1.0);
    HIP_TRY(hipMemcpyAsync(one, ones.data(), gcount * sizeof(double), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));  // the host vector goes out of scope
  }
  ModesRole role(op);
  launch_convert(f0_hat, op->fp64(), blk(B, 0), 1, bsz, 1.0, st);
  if (op->weighted)  // start forcings in the problem's coordinates: to the Euclidean R~'s (times W_f^{1/2})
    launch_node_scale(blk(B, 0), 1, blk(B, 0), 1, (const double*)op->d_wsc + (size_t)kWscSqrtWf * N, (int64_t)nw * k, N,
                      st);
  RES_TRY(cholqr2(op, nw, k, blk(B, 0), rq, nullptr, st));
  for (int i = 0; i < blocks; ++i) {
    double* W = blk(B, i + 1);  // the next block is built in place (the spare slot after the last one)
    RES_TRY(weighted(weigh && i > 0, fd, blk(B, i), blk(Yb, i), +1));
    RES_TRY(weighted(weigh && i > 0, fa, blk(Yb, i), W, -1));
    {
      TimedLaunch tl(op, RES_TIMING_QR, st);
      // first pass: coefficients of every basis block, recorded as column block i of H
      if (launch_xgram(B, bsz, i + 1, W, N, k, op->d_off, ninst, nw, nsplit, part, st))
        return fail(RES_EINVAL, "Krylov Gram launch");
      launch_xgram_reduce(part, nsplit, k, i + 1, nw, ninst, C, H, nmax, i * k, st);
      double* est = (double*)dh + (size_t)i * gcount;  // estimates after this block (history, weights)
      if (launch_heig(H, nmax, (i + 1) * k, k, nw, ninst, est, nullptr, 0, st))
        return fail(RES_EINVAL, "Krylov eigen-decomposition launch");
      launch_freq_weights(est, (double*)fd, ninst, nw, k, st, 0.5);
      launch_freq_weights(est, (double*)fa, ninst, nw, k, st, 1.5);
      if (i + 1 < blocks) {
        for (int pass = 0; pass < 2; ++pass) {
          if (pass == 1) {
            launch_xgram(B, bsz, i + 1, W, N, k, op->d_off, ninst, nw, nsplit, part, st);
            launch_xgram_reduce(part, nsplit, k, i + 1, nw, ninst, C, nullptr, 0, 0, st);
          }
          if (launch_combine(W, 1, 1, B, bsz, i + 1, N, k, k, op->d_off, ninst, nw, nsplit, C, (i + 1) * k,
                             nullptr, st))
            return fail(RES_EINVAL, "Krylov update launch");
        }
      }
      HIP_TRY(hipGetLastError());
    }
    if (i + 1 < blocks) RES_TRY(cholqr2(op, nw, k, W, rq, nullptr, st));
  }
  {
    TimedLaunch tl(op, RES_TIMING_QR, st);
    if (launch_heig(H, nmax, nmax, k, nw, ninst, (double*)dg, psi, nmax, st))
      return fail(RES_EINVAL, "Krylov eigen-decomposition launch");
    if (V && launch_combine(V, op->fp64(), 0, B, bsz, blocks, N, k, k, op->d_off, ninst, nw, nsplit, psi, nmax,
                            (const double*)one, st))
      return fail(RES_EINVAL, "Krylov mode launch");
    if (U) {
      // U = R_d B psi / gain: the same combination of the stored responses, scaled by the reciprocal gains
      void* inv;
      RES_TRY(ws_get(op, "kry_inv", gcount * sizeof(double), &inv));
      launch_recip_gains((const double*)dg, (double*)inv, ninst, nw, k, st);
      if (launch_combine(U, op->fp64(), 0, Yb, bsz, blocks, N, k, k, op->d_off, ninst, nw, nsplit, psi, nmax,
                         (const double*)inv, st))
        return fail(RES_EINVAL, "Krylov mode launch");
    }
    HIP_TRY(hipGetLastError());
  }
  if (hist) HIP_TRY(hipMemcpyAsync(hist, dh, (size_t)blocks * gcount * sizeof(double), hipMemcpyDeviceToHost, st));
  if (op->weighted) RES_TRY(modes_to_problem(op, nw, k, V, U, st));
  HIP_TRY(hipMemcpyAsync(gains, dg, gcount * sizeof(double), hipMemcpyDeviceToHost, st));
  return resolvent_op_check(op, stream);
}

int resolvent_apply_backward(resolvent_op* op, const resolvent_grid* grid, const resolvent_run* run, int32_t k,
                             const void* f_hat, const void* g_hat, void* f_grad, double* mu_grad,
                             int32_t checkpoint_every, void* stream) {
  g_last_error.clear();
  if (!op || !f_hat || !g_hat) return fail(RES_EINVAL, "NULL argument");
  if (k < 1) return fail(RES_EINVAL, "k must be >= 1");
  if (checkpoint_every < 0) return fail(RES_EINVAL, "checkpoint_every must be >= 0");
  Plan pl;
  RES_TRY(make_plan(op, grid, run, &pl));
  if (!f_grad && !mu_grad) return RES_OK;
  hipStream_t st = (hipStream_t)stream;
  CaptureScope cap(op, st);
  if (!op->weighted) return backward(op, pl, k, f_hat, g_hat, f_grad, mu_grad, checkpoint_every, st);
  // y = C R B f with real diagonal B, C: the reverse mode of R at the input B f with the cotangent C g; the forcing
  // gradient is B R^H C g (the metrics do not enter a Euclidean vector-Jacobian product)
  const double* w = (const double*)op->d_wsc;
  const int64_t blocks = (int64_t)pl.nw * k;
  const int fp = op->fp64();
  void *fb, *gc;
  RES_TRY(ws_get(op, "bw_wsc_f", (size_t)blocks * op->N * op->wsize(), &fb));
  RES_TRY(ws_get(op, "bw_wsc_g", (size_t)blocks * op->N * op->wsize(), &gc));
  launch_node_scale(f_hat, fp, fb, fp, w + (size_t)kWscB * op->N, blocks, op->N, st);
  launch_node_scale(g_hat, fp, gc, fp, w + (size_t)kWscC * op->N, blocks, op->N, st);
  RES_TRY(backward(op, pl, k, fb, gc, f_grad, mu_grad, checkpoint_every, st));
  if (f_grad) launch_node_scale(f_grad, fp, f_grad, fp, w + (size_t)kWscB * op->N, blocks, op->N, st);
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

int resolvent_signal_run(resolvent_op* op, int32_t k, int64_t n_samples, int32_t every, int32_t scheme,
                         int32_t adjoint, const void* f, void* y, void* stream) {
  g_last_error.clear();
  if (!op || !f || !y) return fail(RES_EINVAL, "NULL argument");
  if (f == y) return fail(RES_EINVAL, "the forcing and the response must not alias");
  RES_TRY(signal_args(op, k, n_samples, every, scheme));
  hipStream_t st = (hipStream_t)stream;
  CaptureScope cap(op, st);
  RES_TRY(signal_run_any(op, k, n_samples, every, scheme, adjoint ? 1 : 0, f, y, st));
  launch_finite(y, op->fp64(), n_samples * k * op->N, op->d_flag, st);
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

int resolvent_grid_from_omegas(const double* omega, int32_t n_omega, double h, int64_t stride,
                               resolvent_grid* out, int64_t* P_out) {
  g_last_error.clear();
  if (!omega || !out) return fail(RES_EINVAL, "NULL argument");
  if (!(h > 0) || !std::isfinite(h)) return fail(RES_EINVAL, "h must be positive");
  if (stride < 1) return fail(RES_EINVAL, "stride must be >= 1");
  if (n_omega < 2) return fail(RES_EGRID, "an array of fewer than two frequencies fixes no spacing");
  for (int32_t j = 0; j < n_omega; ++j)
    if (!std::isfinite(omega[j])) return fail(RES_EGRID, "non-finite frequency");
  const double dw_nom = (omega[n_omega - 1] - omega[0]) / (double)(n_omega - 1);
  if (dw_nom == 0) return fail(RES_EGRID, "equal end frequencies");
  for (int32_t j = 0; j < n_omega; ++j)
    if (std::fabs(omega[j] - (omega[0] + j * dw_nom)) > 1e-9 * std::fabs(dw_nom))
      return fail(RES_EGRID, "frequency " + std::to_string(j) + " is off the uniform grid of its end points");
  // the period P h of the time grid must be 2 pi / |domega|: P is the multiple of the stride nearest that
  const double per = 2.0 * M_PI / (std::fabs(dw_nom) * h * (double)stride);
  if (!(per < 4e18)) return fail(RES_EGRID, "spacing too small for the time step");
  const int64_t P = stride * std::max<int64_t>(1, std::llround(per));
  if (P < n_omega) return fail(RES_EGRID, "more frequencies than steps per period (aliasing)");
  out->omega0 = omega[0];
  out->domega = std::copysign(2.0 * M_PI / ((double)P * h), dw_nom);
  out->n_omega = n_omega;
  if (P_out) *P_out = P;
  return RES_OK;
}

int resolvent_workspace_size(resolvent_op* op, const resolvent_grid* g, const resolvent_run* r, int32_t k,
                             size_t* bytes) {
  g_last_error.clear();
  if (!op || !g || !r || !bytes) return fail(RES_EINVAL, "NULL argument");
  if (k < 1) return fail(RES_EINVAL, "k must be >= 1");
  Plan pl;
  RES_TRY(make_plan(op, g, r, &pl));
  // The no-allocation apply fits its flexible buffers (forcing tiles, snapshot rows, pre-filter chunks) to the
  // capacity it is given and refuses a capacity below the smallest layout: find the smallest capacity (to 256
  // bytes) it accepts, by doubling and then bisection.
  ArenaSizes z;
  size_t lo = 0, hi = (size_t)1 << 20;
  while (arena_sizes(op, pl, k, hi, &z) != RES_OK) {
    if (hi >= ((size_t)1 << 52)) return fail(RES_EINVAL, "workspace size out of range");
    lo = hi;
    hi *= 2;
  }
  while (hi - lo > 256) {
    size_t mid = lo + (hi - lo) / 2;
    mid -= mid % 256;
    if (mid <= lo) break;
    if (arena_sizes(op, pl, k, mid, &z) == RES_OK) hi = mid; else lo = mid;
  }
  g_last_error.clear();
  *bytes = hi;
  return RES_OK;
}

int resolvent_fir_design(int32_t order, int32_t npts, const double* nu, const double* gain, double* taps) {
  g_last_error.clear();
  if (!taps) return fail(RES_EINVAL, "NULL argument");
  std::vector<cd> b;
  RES_TRY(fir_design_host(order, npts, nu, gain, &b));
  std::memcpy(taps, b.data(), b.size() * sizeof(cd));
  return RES_OK;
}

int resolvent_fir_apply(int32_t fp64, int64_t n_t, int64_t ncols, int32_t order, const double* taps, const void* x,
                        void* y, void* stream) {
  g_last_error.clear();
  if (!taps || !x || !y) return fail(RES_EINVAL, "NULL argument");
  if (x == y) return fail(RES_EINVAL, "the input and the output must not alias");
  if (n_t < 1 || ncols < 1) return fail(RES_EINVAL, "need n_t >= 1 and ncols >= 1");
  if (order < 0 || order % 2 || order > fir_max_order())
    return fail(RES_EINVAL, "FIR order must be even, >= 0 and <= " + std::to_string(fir_max_order()));
  if (launch_fir((const cx<double>*)taps, order, x, y, n_t, ncols, -1, 0, fp64 ? 1 : 0, (hipStream_t)stream))
    return fail(RES_EINVAL, "FIR launch");
  HIP_TRY(hipGetLastError());
  return RES_OK;
}

static int trm_modes_body(resolvent_op* op, int32_t k, int64_t n_samples, int32_t every, int32_t scheme,
                        const void* f0, int32_t n_omega, const double* omegas, int32_t iters, int32_t order,
                        int32_t passes, int64_t pad, int64_t ramp, double margin, double* gains, double* amps,
                        void* f_out, void* V, void* U, void* stream) {
  g_last_error.clear();
  if (!op || !f0 || !omegas || !gains) return fail(RES_EINVAL, "NULL argument");
  RES_TRY(signal_args(op, k, n_samples, every, scheme));
  if (n_omega < 1 || iters < 1 || passes < 0) return fail(RES_EINVAL, "need n_omega >= 1, iters >= 1, passes >= 0");
  if (passes > 0 && (order < 2 || order % 2 || order > fir_max_order()))
    return fail(RES_EINVAL, "FIR order must be even, >= 2 and <= " + std::to_string(fir_max_order()));
  if (pad < 0 || ramp < 0 || 2 * (pad + ramp) >= n_samples)
    return fail(RES_EINVAL, "the taper (pad, ramp) must leave samples at one");
  if (!(margin >= 0) || !std::isfinite(margin)) return fail(RES_EINVAL, "margin must be finite and >= 0");
  const double dt = (double)every * op->h;
  for (int j = 0; j < n_omega; ++j)
    if (!std::isfinite(omegas[j]) || std::fabs(omegas[j]) * dt > M_PI)
      return fail(RES_EINVAL, "analysis frequencies must be finite and within the sampling's Nyquist frequency");
  hipStream_t st = (hipStream_t)stream;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (hipStreamIsCapturing(st, &cs) == hipSuccess && cs != hipStreamCaptureStatusNone)
    return fail(RES_EINVAL, "resolvent_trm_modes synchronises its stream and cannot be captured");
  return trm_modes(op, k, n_samples, every, scheme, f0, n_omega, omegas, iters, order, passes, pad, ramp, margin,
                   gains, amps, f_out, V, U, st);
}

int resolvent_op_set_graphs(resolvent_op* op, int32_t enable) {
  if (!op) return fail(RES_EINVAL, "NULL op");
  op->use_graphs = enable != 0;
  return RES_OK;
}

int resolvent_op_set_backward_rows(resolvent_op* op, int32_t fp64) {
  if (!op) return fail(RES_EINVAL, "NULL op");
  op->rev_rows64 = fp64 != 0;
  return RES_OK;
}

int resolvent_op_get_plan(const resolvent_op* op, int32_t plan[4]) {
  if (!op || !plan) return fail(RES_EINVAL, "NULL argument");
  if (is_grid(op)) return fail(RES_ENOTSUP, "grid operators have no stepper plan");
  plan[0] = op->step_cfg;
  plan[1] = (int32_t)op->step_chunk;
  plan[2] = (int32_t)op->step_block;
  plan[3] = op->step_persist ? 1 : 0;
  return RES_OK;
}

int resolvent_op_set_plan(resolvent_op* op, const int32_t plan[4]) {
  g_last_error.clear();
  if (!op || !plan) return fail(RES_EINVAL, "NULL argument");
  if (is_grid(op)) return fail(RES_ENOTSUP, "grid operators have no stepper plan");
  RES_TRY(apply_plan(op, plan[0], plan[1], plan[2], plan[3]));
  op->plan_default = false;
  return RES_OK;
}

int resolvent_op_set_weights(resolvent_op* op, const double* b, const double* c, const double* wf,
                             const double* wy) {
  g_last_error.clear();
  if (!op) return fail(RES_EINVAL, "NULL op");
  if (op->capturing) return fail(RES_EINVAL, "weights cannot change during graph capture");
  const int64_t n = op->N;
  if (!b && !c && !wf && !wy) {
    op->weighted = false;
    return RES_OK;
  }
  std::vector<double> h((size_t)kWscRows * n);
  for (int64_t i = 0; i < n; ++i) {
    const double bi = b ? b[i] : 1.0, ci = c ? c[i] : 1.0, fi = wf ? wf[i] : 1.0, yi = wy ? wy[i] : 1.0;
    if (!std::isfinite(bi) || !std::isfinite(ci) || !(fi > 0) || !(yi > 0) || !std::isfinite(fi) ||
        !std::isfinite(yi))
      return fail(RES_EINVAL, "weights: b and c must be finite, wf and wy finite and positive");
    h[(size_t)kWscB * n + i] = bi;
    h[(size_t)kWscC * n + i] = ci;
    h[(size_t)kWscCWy * n + i] = ci * yi;
    h[(size_t)kWscBInvWf * n + i] = bi / fi;
    h[(size_t)kWscBInvSqrtWf * n + i] = bi / std::sqrt(fi);
    h[(size_t)kWscCSqrtWy * n + i] = ci * std::sqrt(yi);
    h[(size_t)kWscInvSqrtWf * n + i] = 1.0 / std::sqrt(fi);
    h[(size_t)kWscInvSqrtWy * n + i] = 1.0 / std::sqrt(yi);
    h[(size_t)kWscSqrtWf * n + i] = std::sqrt(fi);
  }
  if (!op->d_wsc) HIP_TRY(hipMalloc(&op->d_wsc, h.size() * sizeof(double)));
  HIP_TRY(hipMemcpy(op->d_wsc, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice));
  op->weighted = true;
  return RES_OK;
}

int resolvent_op_set_step_power(resolvent_op* op, int32_t m) {
  g_last_error.clear();
  if (!op) return fail(RES_EINVAL, "NULL op");
  if (is_grid(op)) return fail(RES_ENOTSUP, "grid operators march one RK4 step per kernel step");
  if (m != 1 && m != 2 && m != 4) return fail(RES_EINVAL, "step power must be 1, 2 or 4");
  if (op->capturing) return fail(RES_EINVAL, "step power cannot change during graph capture");
  if (m == op->step_power) return RES_OK;
  op->step_power = m;
  RES_TRY(build_power_bands(op));
  return op->plan_default ? plan_1d_default(op) : RES_OK;  // a default plan follows the step power
}

int resolvent_op_get_step_power(const resolvent_op* op, int32_t* m) {
  if (!op || !m) return fail(RES_EINVAL, "NULL argument");
  *m = op->step_power;
  return RES_OK;
}

int resolvent_op_tune(resolvent_op* op, int32_t k, int32_t steps, int32_t plan_out[4], double* us_per_step,
                      void* stream) {
  g_last_error.clear();
  if (!op) return fail(RES_EINVAL, "NULL op");
  if (is_grid(op)) return fail(RES_ENOTSUP, "grid operators have no stepper plan");
  if (k < 1 || steps < 16) return fail(RES_EINVAL, "k must be >= 1 and steps >= 16");
  PlanCand best{};
  double us = 0;
  RES_TRY(tune_1d(op, k, steps, &best, &us, (hipStream_t)stream));
  op->plan_default = false;
  if (plan_out) RES_TRY(resolvent_op_get_plan(op, plan_out));
  if (us_per_step) *us_per_step = us;
  return RES_OK;
}

int resolvent_op_set_timing(resolvent_op* op, int32_t enable) {
  if (!op) return fail(RES_EINVAL, "NULL op");
  op->timing = enable != 0;
  return RES_OK;
}

int resolvent_op_get_timing(resolvent_op* op, int32_t kind, double* total_ms, int64_t* launches) {
  if (!op || kind < 0 || kind > 3 || !total_ms || !launches) return fail(RES_EINVAL, "bad argument");
  double tot = 0;
  for (auto& e : op->tev[kind]) {
    HIP_TRY(hipEventSynchronize(e.second));
    float ms = 0;
    HIP_TRY(hipEventElapsedTime(&ms, e.first, e.second));
    tot += ms;
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  *total_ms = tot;
  *launches = (int64_t)op->tev[kind].size();
  op->tev[kind].clear();
  return RES_OK;
}

int resolvent_op_check(resolvent_op* op, void* stream) {
  if (!op) return fail(RES_EINVAL, "NULL op");
  int flag = 0;
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  HIP_TRY(hipMemcpy(&flag, op->d_flag, sizeof(int), hipMemcpyDeviceToHost));
  if (flag) {
    int zero = 0;
    HIP_TRY(hipMemcpy(op->d_flag, &zero, sizeof(int), hipMemcpyHostToDevice));
    if (flag & 8) return fail(RES_EHIP, "persistent stepper: neighbour synchronisation timed out");
    if (flag & 2) return fail(RES_ENONFINITE, "rank-deficient or non-finite block in the per-frequency QR");
    return fail(RES_ENONFINITE, "non-finite values in a result");
  }
  return RES_OK;
}

// The iterations return host data and synchronise their stream anyway, so they report what the device flagged
// during the call (non-finite values, a rank-deficient QR block, an abandoned neighbour exchange) themselves.
int resolvent_modes(resolvent_op* op, const resolvent_grid* grid, const resolvent_run* run, int32_t k,
                    int32_t iters, const void* f0_hat, double* gains, void* V, void* U, double* hist,
                    void* stream) {
  const int rc = modes_body(op, grid, run, k, iters, f0_hat, gains, V, U, hist, stream);
  return rc == RES_OK ? resolvent_op_check(op, stream) : rc;
}

int resolvent_krylov(resolvent_op* op, const resolvent_grid* grid, const resolvent_run* run, int32_t k,
                     int32_t blocks, const void* f0_hat, double* gains, void* V, void* U, double* hist,
                     void* stream) {
  const int rc = krylov_body(op, grid, run, k, blocks, f0_hat, gains, V, U, hist, stream);
  return rc == RES_OK ? resolvent_op_check(op, stream) : rc;
}

int resolvent_trm_modes(resolvent_op* op, int32_t k, int64_t n_samples, int32_t every, int32_t scheme,
                        const void* f0, int32_t n_omega, const double* omegas, int32_t iters, int32_t order,
                        int32_t passes, int64_t pad, int64_t ramp, double margin, double* gains, double* amps,
                        void* f_out, void* V, void* U, void* stream) {
  const int rc = trm_modes_body(op, k, n_samples, every, scheme, f0, n_omega, omegas, iters, order, passes, pad,
                                ramp, margin, gains, amps, f_out, V, U, stream);
  return rc == RES_OK ? resolvent_op_check(op, stream) : rc;
}

}  // extern "C"
