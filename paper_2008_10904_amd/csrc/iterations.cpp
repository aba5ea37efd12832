// The iterations of the host runtime (App. A): the block power iteration (eqs. iteration, powerMethod, arDec, with
// the per-frequency normalisation of Sec. 2.3) and the block Arnoldi estimates (eqs. RRFi, arDec, freqOrt), each a
// sequence of direct and adjoint runs with per-frequency QR and small SVD or eigen-decompositions between them.
#include "runtime_state.h"

extern "C" {

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

}  // extern "C"
