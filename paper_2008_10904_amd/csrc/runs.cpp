// Run scheduling of the host runtime (Sec. 2.1 to 2.3): the schedule of one run (make_plan), the forcing
// pre-filter and its synthesis as a phase GEMM, the 1-D and grid marches, the streaming projection onto the
// frequencies, and the direct and adjoint applies that combine them.
#include "runtime_state.h"

namespace rt {

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


// March n kernel steps of mstep RK4 steps each (op->march_band holds P(Z)^mstep; forcing rows and snapshot
// positions count kernel steps) for all k columns from the current state buffer.  With halo regions the march is
// cut into launches of op->step_block RK4 steps, the state ping-ponging between two buffers; otherwise one launch.
int march_1d(resolvent_op* op, int k, int64_t n, const ForceSpec& fs, const SnapSpec& ss, const void* dsegs,
             int64_t nseg, hipStream_t st, int mstep) {
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
  auto force_row = [&](int64_t t) -> const void* {
    if (fs.frc == nullptr) return nullptr;
    int64_t row = fs.row0 + t;
    if (fs.period > 0) row %= fs.period;
    return (const char*)fs.frc + (size_t)row * ncols * ws;
  };
  auto snap_row = [&](int64_t t) -> void* {  // consumes the snapshot of step t if it is sampled
    if (t != next) return nullptr;
    void* p = (char*)ss.snap + (size_t)(ss.row0 + m) * ss.ld * ws;
    ++m;
    next = m < ss.count ? next + ss.stride : -1;
    return p;
  };
  // FP32 2-D steps go in pairs, two per launch (window rows 64, or 48; RESOLVENT_STEP2D_PAIR = 0 keeps one step
  // per launch): the same bits, half the launches and half the state's trips through memory.
  const long pair_wy = fused && !op->fp64() ? env_long("RESOLVENT_STEP2D_PAIR", 64) : 0;
  for (int64_t t = 0; t < n; ++t) {
    const void* frow = force_row(t);
    void* srow = snap_row(t);
    void* uin = sb[op->cur_state];
    void* uout = sb[1 - op->cur_state];
    if (pair_wy != 0 && t + 1 < n) {
      const void* frow2 = force_row(t + 1);
      void* srow2 = snap_row(t + 1);
      if (launch_grid_step2d_pair(g, k, uin, uout, frow, frow2, fs.phi.real(), fs.phi.imag(), srow, srow2,
                                  (int)pair_wy, st))
        return fail(RES_EINVAL, "2-D step pair launch (window rows must be 48 or 64)");
      ++t;
    } else if (fused) {
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
              hipStream_t st, int out_fp64) {
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

}  // namespace rt
