// Transient-response method with time-domain hand-off on the host side (Sec. 2.2, App. B, App. C): the signal runs
// of the direct and adjoint systems, the FIR design of the flattening filter and the TRM iteration, and their C ABI
// entry points.
#include "runtime_state.h"

namespace rt {

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

}  // namespace rt

extern "C" {

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

int resolvent_trm_modes(resolvent_op* op, int32_t k, int64_t n_samples, int32_t every, int32_t scheme,
                        const void* f0, int32_t n_omega, const double* omegas, int32_t iters, int32_t order,
                        int32_t passes, int64_t pad, int64_t ramp, double margin, double* gains, double* amps,
                        void* f_out, void* V, void* U, void* stream) {
  const int rc = trm_modes_body(op, k, n_samples, every, scheme, f0, n_omega, omegas, iters, order, passes, pad,
                                ramp, margin, gains, amps, f_out, V, U, stream);
  return rc == RES_OK ? resolvent_op_check(op, stream) : rc;
}

}  // extern "C"
