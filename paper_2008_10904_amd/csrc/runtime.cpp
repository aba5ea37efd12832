// Host runtime of the resolvent library: operator set-up (the RK4 step stencils of L and L^H, the stepper plan),
// the handle's workspace, the per-frequency QR, the decay probe, the stepper autotuner, the no-allocation layout
// and the C ABI of the handle (create, settings, apply, check).  Run scheduling is in runs.cpp, the iterations in
// iterations.cpp, the reverse mode in backward.cpp and the transient-response method's host side in
// trm_host.cpp.  All device work is stream-ordered on the caller's stream.
#include "runtime_state.h"

namespace rt {

thread_local std::string g_last_error;

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

}  // namespace rt

namespace rt {

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

}  // namespace rt

namespace rt {

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

}  // namespace rt

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
  const double steps = 2.0 * M_PI / (std::fabs(dw_nom) * h);  // the array's own period in steps
  if (!(steps < 1e15)) return fail(RES_EGRID, "spacing too small for the time step");
  const int64_t P = stride * std::max<int64_t>(1, std::llround(steps / (double)stride));
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

int resolvent_op_set_graphs(resolvent_op* op, int32_t enable) {
  if (!op) return fail(RES_EINVAL, "NULL op");
  op->use_graphs = enable != 0;
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

}  // extern "C"
